"""Writes the stored expected values under tests/golden/ by calling only the oracle.

medium_game_expl.json: on the medium two-round game (6 ranks x 2 suits, 100,981 nodes),
the exploitability of the average strategy after 1,000 iterations of vanilla CFR and of
CFR+, computed by the recursive FP64 oracle; plus the same runs made to carry fp32-sized
rounding: every iteration's instantaneous regrets perturbed by seeded relative noise of one
fp32 unit roundoff (2^-24) and the cumulative regrets and weights rounded to fp32. The
spread of those runs measures how far rounding at fp32 level alone moves the result after
1,000 iterations (regret matching switches strategies where regrets cross zero, so tiny
differences grow over the run). Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import games  # noqa: E402
from oracle import br, cfr  # noqa: E402
from oracle.tree import Tree  # noqa: E402

ITERS = 1000
SEEDS = list(range(1, 17))


def run(args):
    variant, seed = args
    g = games.leduc_like(6, 2, deal="joint")
    t = Tree(g)
    rng = np.random.default_rng(seed) if seed else None
    st = cfr.State.zeros(t)
    t0 = time.time()
    for _ in range(ITERS):
        prev = st
        st, info = cfr.iterate(t, st, variant)
        if rng is not None:
            rt = np.asarray(info["rtilde"])
            noisy = np.asarray(prev.R) + rt * (1.0 + 2.0 ** -24 * rng.standard_normal(len(rt)))
            if variant == cfr.CFR_PLUS:
                noisy = np.maximum(noisy, 0.0)
            st.R = noisy.astype(np.float32).astype(np.float64).tolist()
            st.S = np.asarray(st.S).astype(np.float32).astype(np.float64).tolist()
    e = br.exploitability(t, cfr.average_strategy(t, st.S))
    return variant, seed, e, time.time() - t0


def main():
    jobs = [(v, s) for v in ("vanilla", "cfr+") for s in [0] + SEEDS]
    with Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        results = pool.map(run, jobs)
    g = games.leduc_like(6, 2, deal="joint")
    out = {"game": "leduc_like(6, 2, deal='joint')", "nodes": g.n_nodes}
    for variant in ("vanilla", "cfr+"):
        exact = [r for r in results if r[0] == variant and r[1] == 0][0]
        pert = [r[2]["expl"] for r in results if r[0] == variant and r[1] != 0]
        out[variant] = {"iterations": ITERS, "expl": exact[2]["expl"], "br1": exact[2]["br1"],
                        "br2": exact[2]["br2"], "value": exact[2]["value"],
                        "oracle_seconds": exact[3], "expl_fp32_noise": pert,
                        "noise_spread": max(abs(p - exact[2]["expl"]) for p in pert)}
        print(variant, out[variant], flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "medium_game_expl.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
