"""Autotuner for the public-block engine's launch shapes.

Each iteration is a sequence of launches, one per tree level and direction; a launch has
some number of work items (nodes for the top-down pass, infosets and chance nodes for the
bottom-up pass), and those counts span six orders of magnitude between the first and the
deepest levels and between small and large (sub)games. The tuner times every launch of an
iteration under each candidate workgroup size (hipEvents around each launch, through the
library's per-launch profile), groups launches by kernel and log2 bucket of work items,
and keeps the fastest size per bucket. The table is a JSON file keyed by architecture; the
solvers load it when it exists. Work per item does not depend on the workgroup size, so
results are bit-identical for any table.

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
CANDIDATES = (64, 128, 256, 512)
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.json")


def bucket(units: int) -> int:
    return 0 if units < 2 else min(N_BUCKETS - 1, int(math.floor(math.log2(units))))


def measure(solver, candidates=CANDIDATES, iters: int = 5) -> dict:
    """{kernel: {bucket: {threads: ms per iteration}}}; the solver's state is restored."""
    T, R, S = solver.get_state()
    out: dict = {}
    for c in candidates:
        solver.set_launch_shape([c] * N_BUCKETS, [c] * N_BUCKETS)
        solver.iterate_profile(1)                        # warm the new shape
        for rec in solver.iterate_profile(iters):
            b = bucket(rec["units"])
            slot = out.setdefault(rec["kernel"], {}).setdefault(b, {})
            slot[c] = slot.get(c, 0.0) + rec["ms"]
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
    """Fastest size per (kernel, bucket); buckets never seen take the nearest seen one."""
    table = {}
    for kernel, key in (("block_up", "up_threads"), ("block_reach", "reach_threads")):
        seen = {b: min(by_c, key=by_c.get) for b, by_c in measured.get(kernel, {}).items()}
        row = []
        for b in range(N_BUCKETS):
            if not seen:
                row.append(256)
                continue
            near = min(seen, key=lambda x: (abs(x - b), -x))
            row.append(int(seen[near]))
        table[key] = row
    return table


def load(path: str = TABLE_PATH):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def apply(solver, table) -> None:
    if table is None or solver.info.get("engine") != 1:
        return
    solver.set_launch_shape(table["up_threads"], table["reach_threads"])


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
    table["candidates"] = list(CANDIDATES)
    table["measured_ms"] = {k: {str(bk): {str(c): round(v, 5) for c, v in by_c.items()}
                                for bk, by_c in sorted(bks.items())} for k, bks in merged.items()}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({"up_threads": table["up_threads"], "reach_threads": table["reach_threads"]}),
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
