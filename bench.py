"""Benchmark: CFR node-updates/s on the large synthetic poker game, one MI355X.

One step is one full CFR+ iteration over the 21,509,281-node game (13 private
ranks, 3 betting rounds, fold / call / pot-raise / all-in, at most 3 raises per
round, stack 400): top-down reach, bottom-up values fused with the regret
reductions, and the infoset pass (regret update, average-strategy accumulation,
regret matching). The game is built on the host and resident in HBM before the
timed region starts.

Prints one JSON line (rank 0) with the throughput, the roofline of the dominant
kernel (bytes it must move per launch / its event-timed average duration) and
the FP64 oracle timed on a bounded sample of the same game on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CFR node-updates/s + %HBM peak; wall time to exploitability 1e-3 (plain vs warm)"
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(lay: dict, kernel: str) -> float:
    """Bytes one average launch of `kernel` must move, from the layout's level counts.

    value_level (per level, internal parent p with children c): child_begin 4, node_player 1
    for every node of the level, value write 4 per internal node, reach 12 + infoset 4 per
    player node; per child c: node_edge 4, value 4, sigma gather 4, and for a player child
    the regret accumulation 8 (read + write); pibar 8 per player node.
    reach_level (per level): node_player 1 per node; per decision node: parent 4, edge 4,
    sigma gather 4, parent reach 12, reach write 12.
    infoset_update: per pair R 8, S 8, rtilde 8, sigma 8; per infoset q_offset 4, pibar 8.
    """
    lo = lay["level_offset"]
    player = lay["node_player"]
    D = len(lo) - 2
    if kernel == "value_level":
        tot = 0.0
        for l in range(D):
            a, b = lo[l], lo[l + 1]
            pl = player[a:b]
            n_int = int((pl >= 0).sum())
            n_play = int((pl >= 1).sum())
            ca, cb = lo[l + 1], lo[l + 2]
            par_pl = player[lay["parent"][ca:cb]]
            n_ch = cb - ca
            n_pch = int((par_pl >= 1).sum())
            tot += (b - a) * 1 + n_int * (4 + 4) + n_play * (12 + 4 + 8) + n_ch * 12 + n_pch * 8
        return tot / max(D, 1)
    if kernel == "reach_level":
        tot = 0.0
        for l in range(1, D):
            a, b = lo[l], lo[l + 1]
            n_dec = int((player[a:b] >= 0).sum())
            tot += (b - a) * 1 + n_dec * (4 + 4 + 4 + 12 + 12)
        return tot / max(D - 1, 1)
    if kernel == "infoset_update":
        Hp = len(lay["q_offset"]) - 1
        Qp = int(lay["q_offset"][-1])
        return Qp * 32 + Hp * 12
    return 0.0


def cpu_baseline(seconds_cap: float = 30.0) -> dict:
    """The FP64 oracle (single-threaded Python) on the first 16 of the 156 deals."""
    import games
    from oracle import cfr
    from oracle.tree import Tree

    g = games.poker_game(13, 3, 3, 400, max_deals=16)
    t = Tree(g)
    st = cfr.State.zeros(t)
    t0 = time.perf_counter()
    iters = 0
    while iters < 3 and time.perf_counter() - t0 < seconds_cap:
        st, _ = cfr.iterate(t, st, cfr.CFR_PLUS)
        iters += 1
    dt = time.perf_counter() - t0
    return {"value": g.n_nodes * iters / dt, "unit": "node-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{iters} CFR+ iterations of the recursive FP64 oracle on the first 16 of "
                      f"156 deals of the same game ({g.n_nodes} nodes); host "
                      f"{platform.processor() or platform.machine()}, os.cpu_count()="
                      f"{os.cpu_count()}"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--timed-kernel-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exploitability", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not part of this build.", file=sys.stderr)
        return 2

    import torch

    import games
    from paper_2408_14778_amd import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g = games.large_game()
    log(f"game built: {g.n_nodes} nodes in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    s = Solver(g, "cfr+", device="cuda:0")
    torch.cuda.synchronize()
    log(f"solver built (flatten + upload + graph capture) in {time.perf_counter() - t0:.1f}s; "
        f"workspace {s.info['workspace_bytes'] / 2**30:.2f} GiB")
    s.iterate(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = g.n_nodes * args.steps / dt
    log(f"timed {args.steps} iterations: {ms_per_step:.4f} ms/iteration, {value:.4e} node-updates/s")

    # per-kernel durations, hipEvents around every launch on the solver's stream
    kt = s.iterate_timed(args.timed_kernel_steps)
    lay = {k: s.layout(k) for k in ("level_offset", "node_player", "parent", "q_offset")}
    dom = max(kt, key=lambda k: kt[k][1])
    launches, total_ms = kt[dom]
    avg_s = total_ms / launches * 1e-3
    bytes_per_launch = algorithmic_bytes(lay, dom)
    achieved = bytes_per_launch / avg_s / 1e9
    kernels = {k: {"launches": n, "avg_us": ms / n * 1e3,
                   "share": ms / sum(v[1] for v in kt.values())} for k, (n, ms) in kt.items()}
    log(f"kernels: {json.dumps(kernels)}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large poker game: 13 ranks, 3 rounds, fold/call/pot/all-in, "
                               "cap 3, stack 400, CFR+ (linear averaging), seed 2",
                   "nodes": g.n_nodes, "infosets": s.info["n_infosets"], "q": s.info["n_q"],
                   "depth": s.info["depth"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_s * 1e6},
        "kernels": kernels,
    }
    if not args.no_exploitability:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = s.exploitability()
        out["exploitability"] = {"iterations": args.warmup + args.steps + args.timed_kernel_steps,
                                 "expl": e["expl"], "seconds": time.perf_counter() - t0}
        log(f"exploitability {e['expl']:.6g} after {out['exploitability']['iterations']} iterations")
    s.close()
    del s
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample (host)")
        out["cpu_baseline"] = cpu_baseline()
        log(f"oracle: {out['cpu_baseline']['value']:.4e} node-updates/s")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
