"""Autotuner for the public-block engine's launch shapes.

Each iteration is a sequence of launches, one per tree level and direction; a launch has
some number of work items (nodes for the top-down pass, infoset members for the bottom-up
pass), and those counts span six orders of magnitude between the first and the deepest
levels and between small and large (sub)games. A shape is a workgroup size and a number of
items per thread. The tuner times every launch of an iteration under each candidate shape
(hipEvents around each launch, through the library's per-launch profile), groups launches
by kernel and log2 bucket of work items, and keeps the fastest shape per bucket. The table is
a JSON file keyed by architecture; the solvers load it when it exists. Each infoset sums its
members' contributions in member order whatever the shape, so results are bit-identical for
any table (up to infosets larger than a chunk).

    python -m paper_2408_14778_amd.autotune --out paper_2408_14778_amd/tuning/gfx950.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

N_BUCKETS = 32
# (threads per workgroup, items per thread); run i sets UP[i] and REACH[i] together
UP_CANDIDATES = ((64, 1), (128, 1), (256, 1), (512, 1), (64, 2), (128, 2), (256, 2), (512, 2))
REACH_CANDIDATES = ((128, 1), (256, 1), (512, 1), (1024, 1), (128, 2), (256, 2), (256, 4),
                    (512, 2))
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.json")


def bucket(units: int) -> int:
    return 0 if units < 2 else min(N_BUCKETS - 1, int(math.floor(math.log2(units))))


def measure(solver, iters: int = 5, up=UP_CANDIDATES, reach=REACH_CANDIDATES) -> dict:
    """{kernel: {bucket: {(threads, items): ms per iteration}}}; the solver's state is
    restored. Launches of the single-workgroup first levels (level -1) take no shape."""
    T, R, S = solver.get_state()
    out: dict = {}
    for (ut, um), (rt, rn) in zip(up, reach):
        solver.set_launch_shape(up_threads=ut, up_members=um, reach_threads=rt, reach_nodes=rn)
        solver.iterate_profile(1)                        # warm the new shape
        for rec in solver.iterate_profile(iters):
            if rec["level"] < 0:
                continue
            shape = (ut, um) if rec["kernel"] == "block_up" else (rt, rn)
            slot = out.setdefault(rec["kernel"], {}).setdefault(bucket(rec["units"]), {})
            slot[shape] = slot.get(shape, 0.0) + rec["ms"]
    solver.set_launch_shape()
    solver.set_state(T, R, S)
    return out


def merge(measurements: list) -> dict:
    tot: dict = {}
    for m in measurements:
        for k, bks in m.items():
            for b, by_c in bks.items():
                for c, ms in by_c.items():
                    s = tot.setdefault(k, {}).setdefault(b, {})
                    s[c] = s.get(c, 0.0) + ms
    return tot


def choose(measured: dict) -> dict:
    """Fastest shape per (kernel, bucket); buckets never seen take the nearest seen one."""
    table = {}
    for kernel, keys, default in (("block_up", ("up_threads", "up_members"), (256, 1)),
                                  ("block_reach", ("reach_threads", "reach_nodes"), (256, 1))):
        seen = {b: min(by_c, key=by_c.get) for b, by_c in measured.get(kernel, {}).items()}
        rows = ([], [])
        for b in range(N_BUCKETS):
            shape = default
            if seen:
                shape = seen[min(seen, key=lambda x: (abs(x - b), -x))]
            rows[0].append(int(shape[0]))
            rows[1].append(int(shape[1]))
        table[keys[0]], table[keys[1]] = rows
    return table


def load(path: str = TABLE_PATH):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def apply(solver, table) -> None:
    if table is None or solver.info.get("engine") != 1:
        return
    solver.set_launch_shape(up_threads=table["up_threads"], up_members=table["up_members"],
                            reach_threads=table["reach_threads"], reach_nodes=table["reach_nodes"])


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--iters", type=int, default=5)
    ap.add_argument("--batch", type=int, default=128, help="subgames in the batched workload")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import torch

    import games
    from paper_2408_14778_amd import BatchSolver, Solver

    torch.cuda.set_device(0)
    meas = []
    t0 = time.time()
    s = Solver(games.large_game(), "cfr+", tuned=False)
    s.iterate(3)
    meas.append(measure(s, iters=args.iters))
    print(f"[autotune] large game measured in {time.time() - t0:.1f}s", flush=True)
    s.close()
    del s
    t0 = time.time()
    b = BatchSolver([games.subgame(100 + i) for i in range(args.batch)], "cfr+", tuned=False)
    b.iterate(3)
    meas.append(measure(b, iters=args.iters))
    print(f"[autotune] batch of {args.batch} subgames measured in {time.time() - t0:.1f}s",
          flush=True)
    b.close()
    merged = merge(meas)
    table = choose(merged)
    table["arch"] = "gfx950"
    table["candidates"] = {"up": [list(c) for c in UP_CANDIDATES],
                           "reach": [list(c) for c in REACH_CANDIDATES]}
    table["measured_ms"] = {k: {str(bk): {f"{c[0]}x{c[1]}": round(v, 5) for c, v in by_c.items()}
                                for bk, by_c in sorted(bks.items())} for k, bks in merged.items()}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({k: table[k] for k in ("up_threads", "up_members", "reach_threads",
                                            "reach_nodes")}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
