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


def level_counts(lay: dict) -> list:
    """Per level: nodes, decision nodes, player nodes (members), chance nodes, children of
    player nodes, children of chance nodes, infosets, infoset-action pairs, and the number
    of distinct parents of the level's decision nodes."""
    lo = lay["level_offset"]
    player = lay["node_player"]
    cb = lay["child_begin"].astype(np.int64)
    nch = np.diff(cb)
    mo = lay["member_offset"]
    first = lay["members"][mo[:-1]] if len(mo) > 1 else np.zeros(0, dtype=np.int64)
    hlev = np.searchsorted(lo, first, side="right") - 1
    qo = lay["q_offset"].astype(np.int64)
    qk = np.diff(qo)
    parent = lay["parent"]
    out = []
    for l in range(len(lo) - 1):
        a, b = lo[l], lo[l + 1]
        pl = player[a:b]
        dec = pl >= 0
        out.append({
            "nodes": b - a, "decision": int(dec.sum()), "player": int((pl >= 1).sum()),
            "chance": int((pl == 0).sum()),
            "player_children": int(nch[a:b][pl >= 1].sum()),
            "chance_children": int(nch[a:b][pl == 0].sum()),
            "infosets": int((hlev == l).sum()), "q": int(qk[hlev == l].sum()),
            "parents": int(len(np.unique(parent[a:b][dec]))) if l > 0 else 0,
        })
    return out


def algorithmic_bytes(lay: dict, kernel: str, counts: list) -> float:
    """Bytes one average launch of `kernel` must move (each distinct datum once).

    block_reach (level l, one thread per node): node kind 1 B per node; per decision node
    the parent index 4, edge index 4, edge probability 4 and its reach write 12; the
    parents' reach 12 per distinct parent.
    block_up (level l, one thread per infoset or chance node): per infoset its pair offset
    4, player 1 and member offset 4; per pair sigma 4, R read+write 8, S read+write 8 and
    the next sigma 4; per member its index 4, child begin 4, child stride 4, reach 12, value
    write 4 and one value 4 per child; per chance node its index, base and count 12, value
    write 4 and per child a listed index 4, probability 4 and value 4.
    value_level / reach_level / infoset_update: the breadth-first node engine's kernels,
    counted the same way (its regret and player-reach accumulation add 8 B per player child
    and 8 B per player node).
    """
    D = len(counts) - 1
    if kernel in ("block_reach", "reach_level"):
        tot = sum(c["nodes"] + c["decision"] * 24 + c["parents"] * 12 for c in counts[1:D])
        return tot / max(D - 1, 1)
    if kernel == "block_up":
        levels = [c for c in counts if c["infosets"] + c["chance"] > 0]
        tot = sum(c["infosets"] * 9 + c["q"] * 24 + c["player"] * 28 + c["player_children"] * 4
                  + c["chance"] * 16 + c["chance_children"] * 12 for c in levels)
        return tot / max(len(levels), 1)
    if kernel == "value_level":
        tot = sum(c["nodes"] + c["decision"] * 8 + c["player"] * (12 + 4 + 8)
                  + (c["player_children"] + c["chance_children"]) * 12
                  + c["player_children"] * 8 for c in counts[:D])
        return tot / max(D, 1)
    if kernel == "infoset_update":
        Qp = sum(c["q"] for c in counts)
        Hp = sum(c["infosets"] for c in counts)
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
    ap.add_argument("--engine", choices=["auto", "node"], default="auto")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device 3 times (a known-size kernel for "
                         "scaling hardware byte counters)")
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
    if args.calibrate_copy:
        src = torch.ones(2**28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB device-to-device copies done")
    t0 = time.perf_counter()
    g = games.large_game()
    log(f"game built: {g.n_nodes} nodes in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    s = Solver(g, "cfr+", device="cuda:0", engine=args.engine)
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
    lay = {k: s.layout(k) for k in ("level_offset", "node_player", "parent", "q_offset",
                                     "child_begin", "member_offset", "members")}
    counts = level_counts(lay)
    dom = max(kt, key=lambda k: kt[k][1])
    launches, total_ms = kt[dom]
    avg_s = total_ms / launches * 1e-3
    bytes_per_launch = algorithmic_bytes(lay, dom, counts)
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
                   "depth": s.info["depth"],
                   "engine": ["node", "public-block"][s.info["engine"]]},
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
