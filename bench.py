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
            "nodes": int(b - a), "decision": int(dec.sum()), "player": int((pl >= 1).sum()),
            "chance": int((pl == 0).sum()),
            "player_children": int(nch[a:b][pl >= 1].sum()),
            "chance_children": int(nch[a:b][pl == 0].sum()),
            "infosets": int((hlev == l).sum()), "q": int(qk[hlev == l].sum()),
            "parents": int(len(np.unique(parent[a:b][dec]))) if l > 0 else 0,
        })
    return out


def algorithmic_bytes(kernel: str, counts: list, reach_launch=None, real: int = 4) -> float:
    """Bytes `kernel` must move per iteration under the two-sweep streaming model (values of
    `real` bytes, 4 or 8; int32 indices; N_int = internal nodes, chance included; only internal
    nodes need reach). With r = real: top-down, per internal non-root node, parent index and
    edge label 8, the parent's two reach factors 2r and its own 2r (24 B in fp32); bottom-up,
    per node read as a child its value r with its structure 8, per internal node its value write
    and the acting player's reach 2r, per pair 9r (R and S read and written, the instantaneous
    regret, sigma read and written, sigma gathers: 36 B in fp32) and per infoset 2r. A level
    whose reach its bottom-up launch computes (reach_launch[l] == 4, the solver's reach_launch
    layout) needs no reach written and read back: its bottom-up launch moves 8 + r more per
    internal node (parent index, edge label and parent reach, less the reach read) and the
    top-down pass nothing for it. A kernel's launches over one iteration move the sum of the
    levels they process; the per-launch figure is that sum divided by the launches.
    block_reach / reach_level: top-down; block_up: bottom-up (values, regrets and the infoset
    update fused); value_level and infoset_update: the node engine's split of the bottom-up
    terms.
    """
    r = real
    D = len(counts) - 1
    fused = [l for l in range(D + 1) if reach_launch is not None and reach_launch[l] == 4]
    reach = sum((8 + 4 * r) * counts[l]["decision"] for l in range(1, D) if l not in fused)
    values = sum((8 + r) * counts[l + 1]["nodes"] + 2 * r * counts[l]["decision"]
                 for l in range(D))
    values += sum((8 + r) * counts[l]["decision"] for l in fused)
    infoset = sum(9 * r * c["q"] + 2 * r * c["infosets"] for c in counts)
    return float({"block_reach": reach, "reach_level": reach, "block_up": values + infoset,
                  "value_level": values, "infoset_update": infoset}.get(kernel, 0.0))


def algorithmic_bytes_n(kernel: str, counts: list, players: int, real: int = 4) -> float:
    """The same streaming model for a general-sum game of `players` rational players on the node
    engine, which keeps one value column per player and players + 1 reach planes: top-down, per
    internal non-root node, parent index and edge label 8, the parent's planes and its own
    2 (players + 1) r; bottom-up, per node read as a child its players values and its structure
    8, per internal node its players values written and its players + 1 reach planes read; per
    pair 9r and per infoset 2r as for two players."""
    r, P = real, players
    D = len(counts) - 1
    reach = sum((8 + 2 * (P + 1) * r) * counts[l]["decision"] for l in range(1, D))
    values = sum((8 + P * r) * counts[l + 1]["nodes"] + (2 * P + 1) * r * counts[l]["decision"]
                 for l in range(D))
    infoset = sum(9 * r * c["q"] + 2 * r * c["infosets"] for c in counts)
    return float({"reach_level": reach, "value_level": values,
                  "infoset_update": infoset}.get(kernel, 0.0))


LAYOUT_FOR_COUNTS = ["level_offset", "node_player", "parent", "q_offset", "child_begin",
                     "member_offset", "members"]


def game_level_counts(game) -> list:
    """level_counts of one game from its canonical layout, flattened on the host."""
    from paper_2408_14778_amd.solver import host_layout
    return level_counts(host_layout(game, LAYOUT_FOR_COUNTS))


def forest_level_counts(game_list) -> list:
    """level_counts of a batch's forest: level l of the forest is level l of every game, so the
    counts add up level by level."""
    total: list = []
    for g in game_list:
        for l, c in enumerate(game_level_counts(g)):
            if l == len(total):
                total.append({k: 0 for k in c})
            for k, v in c.items():
                total[l][k] += v
    return total


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when the kernels have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_large_game.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, rec["kernel_source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["kernel_source_sha256"]:
            return None
    return rec.get(kernel, {}).get("bytes_per_launch")


def write_traffic(fetch_csv: str, write_csv: str) -> dict:
    """profiles/traffic_large_game.txt from two rocprofv3 counter runs of this script with
    --calibrate-copy (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch): each counter is scaled
    so that the calibration copy (2^28 floats read and written, 1 GiB each way) reads 1 GiB, then
    averaged over the dispatches of each kernel family (block_reach: the top-down launches;
    block_up: the bottom-up ones), with the SHA-256 of the kernel source they were taken on."""
    import collections
    import csv
    import hashlib

    def family(name):
        if "k_x_up_level" in name or "k_x_up_top" in name:
            return "block_up"
        if "k_x_reach" in name and "k_x_reach_full" not in name:
            return "block_reach"
        return None

    def read(path, counter):
        per, calib = collections.defaultdict(list), []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if "AUnaryFunctor" in r["Kernel_Name"] and int(r["Grid_Size"]) == 2**26:
                    calib.append(v)
                per[r["Kernel_Name"]].append(v)
        if not calib:
            raise SystemExit(f"{path}: no calibration copy (run with --calibrate-copy)")
        return per, (2**30 / 1024) / (sum(calib) / len(calib))

    fetch, fscale = read(fetch_csv, "FETCH_SIZE")
    write, wscale = read(write_csv, "WRITE_SIZE")
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0])
    for name in set(fetch) | set(write):
        k = family(name)
        if k is None:
            continue
        f, w = fetch.get(name, []), write.get(name, [])
        a = agg[k]
        a[0] += max(len(f), len(w))
        a[1] += sum(f) * 1024 * fscale
        a[2] += sum(w) * 1024 * wscale
    src = "paper_2408_14778_amd/csrc/xkernels.hip"
    with open(os.path.join(ROOT, src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    out = {k: {"dispatches": d, "bytes_per_launch": (fb + wb) / d, "fetch_bytes_per_launch": fb / d,
               "write_bytes_per_launch": wb / d} for k, (d, fb, wb) in agg.items()}
    out.update({"kernel_source": src, "kernel_source_sha256": sha,
                "calibration": {"fetch_scale": fscale, "write_scale": wscale}})
    with open(os.path.join(ROOT, "profiles", "traffic_large_game.txt"), "w") as f:
        json.dump(out, f, indent=1)
    return out


def copy_bandwidth(mbytes: int = 1024, copies: int = 3, reps: int = 12) -> float:
    """GB/s of a plain elementwise copy (dst = src * 1) moving `mbytes` MB per launch (half read,
    half written), timed with hipEvents: the attainable bandwidth the roofline is read against.
    Successive launches rotate over `copies` disjoint buffer pairs (3 GB in all by default), so no
    launch finds its operands in the 256 MB last-level cache: the figure is an HBM figure."""
    import torch
    n = mbytes * 2**20 // 8
    pairs = [(torch.ones(n, device="cuda"), torch.empty(n, device="cuda")) for _ in range(copies)]
    for i in range(copies):
        torch.mul(pairs[i][0], 1.0, out=pairs[i][1])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        src, dst = pairs[r % copies]
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del pairs
    torch.cuda.empty_cache()
    return mbytes * 2**20 / (ms * 1e-3) / 1e9


def bench_batch(args, gl) -> dict:
    """The batched workload: 512 subgames (seeds 100-611) as one forest, CFR+, with the
    roofline of its dominant kernel measured as for the large game."""
    import torch

    from paper_2408_14778_amd import BatchSolver

    nodes = sum(g.n_nodes for g in gl)
    t0 = time.perf_counter()
    counts = forest_level_counts(gl)
    log(f"forest level counts from the host layouts in {time.perf_counter() - t0:.1f}s")
    b = BatchSolver(gl, "cfr+")
    b.iterate(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    assert b.stream == torch.cuda.current_stream()
    t0 = time.perf_counter()
    ev0.record(b.stream)
    b.iterate(args.steps)
    ev1.record(b.stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gpu_iter_s = ev0.elapsed_time(ev1) * 1e-3 / args.steps
    kt = b.iterate_timed(args.timed_kernel_steps)
    rl = b.layout("reach_launch")
    dom = max(kt, key=lambda k: kt[k][1])
    launches, total_ms = kt[dom]
    share = total_ms / sum(v[1] for v in kt.values())
    avg_s = gpu_iter_s * share / (launches / args.timed_kernel_steps)
    bytes_per_launch = algorithmic_bytes(dom, counts, rl) * args.timed_kernel_steps / launches
    achieved = bytes_per_launch / avg_s / 1e9
    iter_bytes = float(sum(algorithmic_bytes(k, counts, rl) for k in ("block_reach", "block_up")))
    br_s = []  # the first best response also writes the terminal values once
    for _ in range(3):
        t1 = time.perf_counter()
        e = b.exploitability()
        torch.cuda.synchronize()
        br_s.append(time.perf_counter() - t1)
    return {"metric": METRIC, "value": nodes * args.steps / dt, "unit": "node-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "batch of 512 subgames (seeds 100-611), CFR+, one forest",
                       "nodes": nodes},
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": None, "bytes_per_launch": bytes_per_launch,
                         "avg_launch_us": avg_s * 1e6, "iteration_us_events": gpu_iter_s * 1e6,
                         "iteration_bytes": iter_bytes,
                         "iteration_gbs": iter_bytes / gpu_iter_s / 1e9},
            "kernels": {k: {"launches": n, "avg_us": ms / n * 1e3} for k, (n, ms) in kt.items()},
            "exploitability": {"max": float(np.max(e["expl"])), "median": float(np.median(e["expl"])),
                               "seconds_first": br_s[0], "seconds": min(br_s[1:])}}


PCIE_PEAK_GBS = 64.0  # PCIe 5.0 x16 host link, per direction (nominal)
NPLAYER_GAME = dict(seed=6, n_players=3, n_types=12, depth=9, max_actions=3, p_terminal=0.15)


def _timed(solver, steps: int):
    """steps iterations between hipEvents on the solver's stream (torch's current stream):
    (wall seconds, event seconds) per iteration."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    assert solver.stream == torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(solver.stream)
    solver.iterate(steps)
    ev1.record(solver.stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, ev0.elapsed_time(ev1) * 1e-3 / steps


def bench_nplayer(args, g) -> dict:
    """A three-player general-sum game (games.random_game_n, NPLAYER_GAME) on the node engine's
    general-sum kernels (cfr_build_n), CFR+: node-updates/s and the roofline of the dominant
    kernel under algorithmic_bytes_n."""
    from paper_2408_14778_amd import NPlayerSolver

    real = 8 if args.precision == "f64" else 4
    s = NPlayerSolver(g, "cfr+", precision=args.precision, schedule=args.schedule)
    # a node-update is one node processed once: the alternating schedule makes a pass per player
    passes = g.n_players if args.schedule == "alternating" else 1
    s.iterate(args.warmup)
    wall_s, gpu_s = _timed(s, args.steps)
    kt = s.iterate_timed(args.timed_kernel_steps)
    lay = {k: s.layout(k) for k in LAYOUT_FOR_COUNTS}
    counts = level_counts(lay)
    dom = max(kt, key=lambda k: kt[k][1])
    launches, total_ms = kt[dom]
    share = total_ms / sum(v[1] for v in kt.values())
    avg_s = gpu_s * share / (launches / args.timed_kernel_steps)
    P = g.n_players
    bytes_per_launch = (algorithmic_bytes_n(dom, counts, P, real) * passes *
                        args.timed_kernel_steps / launches)
    achieved = bytes_per_launch / avg_s / 1e9
    iter_bytes = passes * float(sum(algorithmic_bytes_n(k, counts, P, real)
                                    for k in ("reach_level", "value_level", "infoset_update")))
    s.close()
    return {"metric": METRIC, "value": g.n_nodes * passes / wall_s, "unit": "node-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall_s * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
            "config": {"workload": "three-player general-sum random game (private types 12 per "
                                   "player, public depth 9), CFR+, node engine" +
                                   (", alternating updates" if passes > 1 else ""),
                       "game": NPLAYER_GAME, "nodes": g.n_nodes, "q": s.n_q, "players": P,
                       "passes_per_iteration": passes},
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": None, "bytes_per_launch": bytes_per_launch,
                         "avg_launch_us": avg_s * 1e6, "iteration_us_events": gpu_s * 1e6,
                         "iteration_bytes": iter_bytes, "iteration_gbs": iter_bytes / gpu_s / 1e9},
            "kernels": {k: {"launches": n, "avg_us": ms / n * 1e3} for k, (n, ms) in kt.items()}}


def bench_partitioned(args, g) -> dict:
    """The large game through the subtree-partitioned, out-of-core iteration (cut at level 8,
    windows of at most 2^21 nodes), CFR+: node-updates/s, and the host link it is bound by:
    every iteration streams each partition's window (the pinned bytes) host to device."""
    from paper_2408_14778_amd import PartitionedSolver

    s = PartitionedSolver(g, "cfr+", cut_level=8, max_window_nodes=1 << 21,
                          precision=args.precision)
    s.iterate(args.warmup)
    wall_s, gpu_s = _timed(s, args.steps)
    achieved = s.host_bytes / gpu_s / 1e9
    out = {"metric": METRIC, "value": g.n_nodes / wall_s, "unit": "node-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": wall_s * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
           "config": {"workload": "large poker game, subtree-partitioned out-of-core iteration "
                                  "(cut level 8, windows <= 2^21 nodes), CFR+",
                      "nodes": g.n_nodes, "partitions": s.n_partitions,
                      "device_workspace_bytes": int(s.info["workspace_bytes"]),
                      "pinned_host_bytes": s.host_bytes},
           "roofline": {"bound": "pcie", "achieved": achieved, "peak": PCIE_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / PCIE_PEAK_GBS, "traffic": None,
                        "bytes_per_iteration": s.host_bytes, "iteration_us_events": gpu_s * 1e6}}
    s.close()
    return out


def warm_start_eval(game_list) -> dict:
    """Wall time until every one of the 512 held-out subgames reaches exploitability 1e-3: CFR+
    from zero regrets against the stored warm-start network (same solver, same checks)."""
    import numpy as np

    from paper_2408_14778_amd import warmstart as ws
    from paper_2408_14778_amd import warmstart_pipeline as wp

    meta_path = os.path.splitext(wp.WEIGHTS_PATH)[0] + ".json"
    if not (os.path.exists(wp.WEIGHTS_PATH) and os.path.exists(meta_path)):
        return {"skipped": "no trained network"}
    with open(meta_path) as f:
        meta = json.load(f)
    weight = meta["weight"]
    net = ws.WarmStartNet(max_batch=65536)
    net.set_params(np.load(wp.WEIGHTS_PATH))
    log("warm start: evaluating plain vs warm on 512 held-out subgames")
    r = wp.evaluate(game_list, net, weight)
    net.close()
    res = {"target": 1e-3, "subgames": len(game_list), "seeds": [100, 99 + len(game_list)],
           "plain_seconds": r["plain"]["seconds"], "warm_seconds": r["warm"]["seconds"],
           "speedup": r["plain"]["seconds"] / r["warm"]["seconds"],
           "plain_mean_iterations": r["paired"]["mean_iterations_plain"],
           "warm_mean_iterations": r["paired"]["mean_iterations_warm"],
           "warm_faster_subgames": r["paired"]["warm_faster"],
           "warm_slower_subgames": r["paired"]["warm_slower"],
           "paired_iteration_ratio": {k: r["paired"][f"{k}_iteration_ratio"]
                                      for k in ("geomean", "median", "p10", "p90")},
           "seconds_until_solved_fraction": {"plain": r["plain"]["seconds_until_solved_fraction"],
                                             "warm": r["warm"]["seconds_until_solved_fraction"]},
           "targets": meta.get("targets", "strategy"), "weight": weight}
    log(f"warm start: {json.dumps(res)}")
    return res


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), else what platform reports."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(seconds_min: float = 10.0) -> dict:
    """The FP64 oracle (single-threaded Python) on the first 16 of the 156 deals: whole CFR+
    iterations until at least `seconds_min` of them have run (about 10-15 s)."""
    import games
    from oracle import cfr
    from oracle.tree import Tree

    g = games.poker_game(13, 3, 3, 400, max_deals=16)
    t = Tree(g)
    st = cfr.State.zeros(t)
    t0 = time.perf_counter()
    iters = 0
    while iters < 1 or (time.perf_counter() - t0 < seconds_min and iters < 50):
        st, _ = cfr.iterate(t, st, cfr.CFR_PLUS)
        iters += 1
    dt = time.perf_counter() - t0
    return {"value": g.n_nodes * iters / dt, "unit": "node-updates/s", "cores": 1,
            "kind": "oracle", "sampled": True, "cpu": cpu_model(),
            "sample": f"{iters} CFR+ iterations of the recursive FP64 oracle on the first 16 of "
                      f"156 deals of the same game ({g.n_nodes} nodes); host {cpu_model()}, "
                      f"os.cpu_count()={os.cpu_count()}"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--timed-kernel-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exploitability", action="store_true")
    ap.add_argument("--engine", choices=["auto", "packs", "node"], default="auto",
                    help="auto: the public-block engine (the reported line); packs: the same with "
                         "subtree packs; node: the breadth-first node engine")
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32",
                    help="f64: the node engine in double precision (CFR_FLAG_FP64)")
    ap.add_argument("--variant", choices=["cfr+", "vanilla", "dcfr"], default="cfr+",
                    help="update rule of the large-game line (the reported workload is CFR+; "
                         "dcfr: discounted CFR with exponents 1.5, 0, 2)")
    ap.add_argument("--schedule", choices=["simultaneous", "alternating"], default="simultaneous",
                    help="alternating: an iteration is a player-1 pass and a player-2 pass")
    ap.add_argument("--workload", choices=["large", "batch", "partitioned", "nplayer"],
                    default="large",
                    help="large: the large single game (the reported line); batch: 512 "
                         "subgames; partitioned: the large game out of core; nplayer: a "
                         "three-player general-sum game")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the second half of the metric: wall time to exploitability 1e-3 on "
                         "the 512 held-out subgames, zero start vs the stored warm-start network")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_large_game.txt from two rocprofv3 counter "
                         "collections of this script run with --calibrate-copy, then exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain elementwise copy of 1 GiB (dst = src * 1) 3 times: a "
                         "kernel of known size for scaling hardware byte counters")
    args = ap.parse_args()
    if args.write_traffic:
        print(json.dumps(write_traffic(*args.write_traffic), indent=1))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not part of this build.", file=sys.stderr)
        return 2

    ws_pool = ws_games = None
    if args.workload == "large" and not args.no_warm_start:
        # the held-out subgames are built by worker processes (forked before this process
        # touches the GPU) while the large game is timed
        from multiprocessing import Pool

        from paper_2408_14778_amd.warmstart_pipeline import _subgame
        ws_pool = Pool(16)
        ws_games = ws_pool.map_async(_subgame, list(range(100, 612)), chunksize=4)
    gl = None
    if args.workload == "batch":
        # the subgames are built by worker processes before this process touches the GPU
        from paper_2408_14778_amd.warmstart_pipeline import build_games
        t0 = time.perf_counter()
        gl = build_games(range(100, 612), 16)
        log(f"512 subgames built: {sum(g.n_nodes for g in gl)} nodes in "
            f"{time.perf_counter() - t0:.1f}s")

    import torch

    import games
    from paper_2408_14778_amd import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(2**28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # 1 GiB read + 1 GiB written per launch
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x (1 GiB read + 1 GiB written) elementwise copies done")
    if gl is not None:
        print(json.dumps(bench_batch(args, gl)), flush=True)
        return 0
    if args.workload in ("nplayer", "partitioned"):
        t0 = time.perf_counter()
        g = games.random_game_n(**NPLAYER_GAME) if args.workload == "nplayer" else games.large_game()
        log(f"game built: {g.n_nodes} nodes in {time.perf_counter() - t0:.1f}s")
        run = bench_nplayer if args.workload == "nplayer" else bench_partitioned
        print(json.dumps(run(args, g)), flush=True)
        return 0
    t0 = time.perf_counter()
    g = games.large_game()
    log(f"game built: {g.n_nodes} nodes in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    s = Solver(g, args.variant, device="cuda:0", engine=args.engine, schedule=args.schedule,
               precision=args.precision)
    real = 8 if args.precision == "f64" else 4
    torch.cuda.synchronize()
    log(f"solver built (flatten + upload + graph capture) in {time.perf_counter() - t0:.1f}s; "
        f"workspace {s.info['workspace_bytes'] / 2**30:.2f} GiB")
    s.iterate(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    # the K timed iterations run as 10 consecutive groups (a synchronisation after each) so that
    # the per-iteration time comes with its standard error over the groups
    groups = [args.steps // 10 + (1 if i < args.steps % 10 else 0) for i in range(10)]
    group_s = []
    # hipEvents on the solver's stream (torch's current stream) around the whole timed region
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    assert s.stream == torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(s.stream)
    for n in groups:
        if n == 0:
            continue
        tg = time.perf_counter()
        s.iterate(n)
        torch.cuda.synchronize()
        group_s.append(((time.perf_counter() - tg) / n))
    ev1.record(s.stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gpu_iter_s = ev0.elapsed_time(ev1) * 1e-3 / args.steps
    ms_per_step = dt * 1e3 / args.steps
    per = np.array(group_s) * 1e3
    sem_ms = float(per.std(ddof=1) / np.sqrt(len(per))) if len(per) > 1 else 0.0
    # a node-update is one node processed once: the alternating schedule makes two passes
    passes = 2 if args.schedule == "alternating" else 1
    value = g.n_nodes * passes * args.steps / dt
    log(f"timed {args.steps} iterations: {ms_per_step:.4f} +- {sem_ms:.4f} ms/iteration (SEM over "
        f"{len(per)} groups), {value:.4e} node-updates/s")

    # per-kernel durations, hipEvents around every launch on the solver's stream
    kt = s.iterate_timed(args.timed_kernel_steps)
    lay = {k: s.layout(k) for k in ("level_offset", "node_player", "parent", "q_offset",
                                     "child_begin", "member_offset", "members")}
    counts = level_counts(lay)
    rl = s.layout("reach_launch")
    dom = max(kt, key=lambda k: kt[k][1])
    launches, total_ms = kt[dom]
    # per-launch duration of the dominant kernel in the timed graph replays: the event-timed
    # iteration split by the kernels' shares of the per-launch event times (each launch timed
    # between two events, outside the graph, which also counts its dispatch gap)
    share = total_ms / sum(v[1] for v in kt.values())
    avg_s = gpu_iter_s * share / (launches / args.timed_kernel_steps)
    avg_direct_s = total_ms / launches * 1e-3
    bytes_per_launch = (algorithmic_bytes(dom, counts, rl, real) * passes * args.timed_kernel_steps /
                        launches)
    achieved = bytes_per_launch / avg_s / 1e9
    iter_bytes = passes * float(sum(algorithmic_bytes(k, counts, rl, real) for k in (
        ("block_reach", "block_up") if s.info["engine"] == 1 else
        ("reach_level", "value_level", "infoset_update"))))
    attainable = copy_bandwidth()
    # rocprofv3 HBM bytes per launch of the same kernel (taken on the default FP32 line)
    traffic = measured_traffic(dom) if (args.precision, args.engine) == ("f32", "auto") else None
    log(f"plain copy: {attainable:.0f} GB/s")
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
        "ms_per_step_sem": sem_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "large poker game: 13 ranks, 3 rounds, fold/call/pot/all-in, "
                               "cap 3, stack 400, " + {
                                   "cfr+": "CFR+ (linear averaging)", "vanilla": "vanilla CFR",
                                   "dcfr": "discounted CFR (1.5, 0, 2)"}[args.variant] +
                               (", alternating updates" if args.schedule == "alternating" else "") +
                               ", seed 2",
                   "nodes": g.n_nodes, "infosets": s.info["n_infosets"], "q": s.info["n_q"],
                   "depth": s.info["depth"],
                   "engine": ["node", "public-block"][s.info["engine"]] +
                             (" with subtree packs" if args.engine == "packs" else ""),
                   "passes_per_iteration": passes},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbs": None if traffic is None else traffic / avg_s / 1e9,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_s * 1e6,
                     "avg_launch_us_direct": avg_direct_s * 1e6,
                     "iteration_us_events": gpu_iter_s * 1e6,
                     "iteration_bytes": iter_bytes, "attainable_copy_gbs": attainable,
                     "iteration_gbs": iter_bytes / (ms_per_step * 1e-3) / 1e9},
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
    if ws_games is not None:
        out["warm_start"] = warm_start_eval(ws_games.get())
        ws_pool.close()
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample (host)")
        out["cpu_baseline"] = cpu_baseline()
        log(f"oracle: {out['cpu_baseline']['value']:.4e} node-updates/s")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
