"""Writes the stored expected values under tests/golden/ by calling only the oracle.

medium_game_expl.json: on the medium two-round game (6 ranks x 2 suits, 100,981 nodes,
D = 10 levels), the exploitability of the average strategy at checkpoints up to 1,000
iterations of vanilla CFR and of CFR+, computed by the recursive FP64 oracle; plus the same
runs made to carry fp32-sized rounding, one run per seed:
* each iteration's instantaneous regret r~(h, a) gets seeded noise D * 2^-24 * N(0, 1) times
  the magnitude it is summed from (sum over the infoset's nodes of |pi_-i| (|w_a| + |u|)):
  the size of the rounding that D levels of fp32 products (reaches) and sums (values, and
  the regret's own sum over members) leave in it;
* each iteration's increment of the strategy sums gets relative noise D * 2^-24 * N(0, 1)
  (its player reach and strategy come out of the same fp32 products);
* the cumulative regrets and strategy sums are rounded to fp32 after every iteration.
The spread of those runs around the exact one measures how far rounding at fp32 level alone
moves the result (regret matching switches strategies where regrets cross zero, so tiny
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
CHECKPOINTS = [25, 50, 100, 150, 200, 300, 400, 600, 800, 1000]
SEEDS = list(range(1, 25))
DEPTH = 10  # levels of the medium game
U = 2.0 ** -24


def run(args):
    variant, seed = args
    g = games.leduc_like(6, 2, deal="joint")
    t = Tree(g)
    rng = np.random.default_rng(seed) if seed else None
    st = cfr.State.zeros(t)
    t0 = time.time()
    out = {}
    for it in range(1, ITERS + 1):
        prev = st
        st, info = cfr.iterate(t, st, variant)
        if rng is not None:
            rt = np.asarray(info["rtilde"])
            scale = np.asarray(info["rtilde_scale"])
            noisy = np.asarray(prev.R) + rt + DEPTH * U * scale * rng.standard_normal(len(rt))
            if variant == cfr.CFR_PLUS:
                noisy = np.maximum(noisy, 0.0)
            st.R = noisy.astype(np.float32).astype(np.float64).tolist()
            inc = np.asarray(st.S) - np.asarray(prev.S)
            S = np.asarray(prev.S) + inc * (1.0 + DEPTH * U * rng.standard_normal(len(inc)))
            st.S = S.astype(np.float32).astype(np.float64).tolist()
        if it in CHECKPOINTS:
            out[it] = br.exploitability(t, cfr.average_strategy(t, st.S))
    return variant, seed, out, time.time() - t0


def main():
    jobs = [(v, s) for v in ("vanilla", "cfr+") for s in [0] + SEEDS]
    with Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        results = pool.map(run, jobs)
    g = games.leduc_like(6, 2, deal="joint")
    out = {"game": "leduc_like(6, 2, deal='joint')", "nodes": g.n_nodes,
           "noise_model": "r~ + D 2^-24 |scale| N(0,1); S increments x (1 + D 2^-24 N(0,1)); R, S "
                          "rounded to fp32 each iteration; D = 10"}
    for variant in ("vanilla", "cfr+"):
        exact = [r for r in results if r[0] == variant and r[1] == 0][0]
        pert = [r for r in results if r[0] == variant and r[1] != 0]
        cps = {}
        for T in CHECKPOINTS:
            e = exact[2][T]["expl"]
            ens = [p[2][T]["expl"] for p in pert]
            cps[str(T)] = {"expl": e, "ensemble": ens,
                           "spread": max(abs(x - e) for x in ens),
                           "mean": float(np.mean(ens)), "std": float(np.std(ens, ddof=1))}
        fin = exact[2][ITERS]
        out[variant] = {"iterations": ITERS, "expl": fin["expl"], "br1": fin["br1"],
                        "br2": fin["br2"], "value": fin["value"], "oracle_seconds": exact[3],
                        "checkpoints": cps}
        print(variant, {T: (c["expl"], c["spread"]) for T, c in cps.items()}, flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "medium_game_expl.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
