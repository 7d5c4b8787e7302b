"""Training and evaluation of the learned warm start on the batched subgame family.

    python -m paper_2408_14778_amd.warmstart_pipeline --train-games 20000 --out-weights W.npy

1. Data: seeded subgames (training seeds from 10,000 up, disjoint from the evaluation seeds
   100-611) are solved in batches by GPU CFR+ for K iterations; each infoset gets two targets
   over its legal action slots: the average strategy (the equilibrium estimate), and the
   normalised positive regrets (the current CFR+ strategy, what regret matching plays next).
   One network is trained on each (`--targets`), and the one whose chosen weight gives the
   lower validation wall time is kept.
2. Training: minibatch Adam on the masked softmax cross-entropy, all on the GPU with the
   library's BF16-MFMA kernels (features, forward, backward, optimiser).
3. Weight: the warm-start weight (how strongly the initial regrets commit to the network's
   strategy) is chosen per network on validation seeds 9000..: the least wall time among the
   weights that speed up the typical game (see select_weight).
4. Evaluation: on the held-out batch, plain CFR+ from zero regrets against the warm start,
   both checked with the best-response pass every `check_every` iterations; a game is solved
   at its first check with exploitability at most the target, and the batch when every game
   is. Wall time includes the network's inference and the warm start's own checks; per-game
   iteration counts are compared pairwise.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
VAL_SEED = 9000   # validation seeds 9000.. (training 10000.., evaluation 100-611)
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning",
                            "warmstart_gfx950.npy")


def log(msg):
    # progress goes to stderr: a caller's stdout (bench.py's one JSON line) stays clean
    print(f"[warmstart] {msg}", file=sys.stderr, flush=True)


def _subgame(seed):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import games
    return games.subgame(seed)


def build_games(seeds, workers: int = 16):
    with Pool(workers) as pool:
        return pool.map(_subgame, list(seeds), chunksize=4)


def _batches(total: int, size: int, first_seed: int):
    return [range(first_seed + s, first_seed + min(total, s + size)) for s in range(0, total, size)]


def solve_targets(game_list, iterations: int, per_game: int, rng) -> dict:
    """Solve a batch with GPU CFR+ and sample up to per_game infosets per game."""
    from . import warmstart as ws
    from .solver import BatchSolver
    b = BatchSolver(game_list, "cfr+")
    b.iterate(iterations)
    avg = b.average_strategy()
    cur = b.current_strategy()  # CFR+: the positive regrets normalised (uniform where none)
    expl = b.exploitability()["expl"]
    b.close()
    desc, bel, qoff = ws.descriptors(game_list)
    target, mask = ws.slot_targets(desc, avg, qoff)
    rtarget, _ = ws.slot_targets(desc, cur, qoff)
    keep = []
    gidx = desc[:, 15].astype(np.int64)
    starts = np.searchsorted(gidx, np.arange(len(game_list)))
    ends = np.searchsorted(gidx, np.arange(len(game_list)), side="right")
    for s, e in zip(starts, ends):
        n = e - s
        keep.append(s + (np.arange(n) if n <= per_game else rng.choice(n, per_game, replace=False)))
    keep = np.concatenate(keep)
    return {"desc": desc[keep], "beliefs": bel, "target": target[keep],
            "rtarget": rtarget[keep], "mask": mask[keep], "expl": expl}


def train(net, data: dict, epochs: int, batch: int, lr: float, seed: int = 0,
          key: str = "target") -> list:
    import torch
    from . import warmstart as ws
    dev = net.device
    x = ws.features(torch.from_numpy(data["desc"]).to(dev), torch.from_numpy(data["beliefs"]).to(dev),
                    net.shape[0])
    t = torch.from_numpy(data[key]).to(dev)
    m = torch.from_numpy(data["mask"]).to(dev)
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            tot += net.train_step(x[idx].contiguous(), t[idx].contiguous(), m[idx].contiguous(), lr)
            cnt += 1
        losses.append(tot / max(cnt, 1))
        log(f"{key} epoch {ep}: loss {losses[-1]:.5f}")
    return losses


def run_to_target(solver, target: float, check_every: int, max_iters: int, done: int = 0,
                  t0: float = None, game_list=None, variant: str = "cfr+",
                  compact: float = 0.05):
    """Iterate with best-response checks every `check_every` iterations. A game is solved at
    the first check where its exploitability is at most `target` (a batched solver keeps that
    game's average strategy from then on). With `game_list`, the batch is compacted: once the
    unsolved games hold at most `compact` of the current forest's nodes, the forest is rebuilt
    from them alone and their state (T, R, S) carried over, so the last, slow games do not keep
    the whole batch iterating. Returns, per game, the iteration and the wall time (from t0) at
    which it was solved (-1 / inf if it never was), the exploitability then, and the solver
    left at the end (the caller closes it; `solver` itself is closed if it was replaced)."""
    import torch
    from .solver import BatchSolver
    t0 = time.perf_counter() if t0 is None else t0
    n = solver.n_games
    solved_it = np.full(n, -1, dtype=np.int64)
    solved_s = np.full(n, np.inf)
    solved_e = np.full(n, np.nan)
    idx = np.arange(n)  # original index of each game of the current solver
    sizes = None if game_list is None else np.array([g.n_nodes for g in game_list])
    it = done
    while it < max_iters:
        solver.iterate(check_every)
        it += check_every
        e = solver.exploitability()["expl"]
        now = time.perf_counter() - t0
        new = (solved_it[idx] < 0) & (e <= target)
        solved_it[idx[new]], solved_s[idx[new]], solved_e[idx[new]] = it, now, e[new]
        active = solved_it[idx] < 0
        if not active.any():
            break
        if (it // check_every) % 50 == 0:
            log(f"  iteration {it}: {n - int(active.sum())}/{n} solved, "
                f"max exploitability {float(np.max(e[active])):.3e}")
        if sizes is not None and active.sum() < len(idx) and \
                sizes[idx[active]].sum() <= compact * sizes[idx].sum():
            T, R, S = solver.get_state()
            keep = np.flatnonzero(active)
            Rs, Ss = solver.split(R), solver.split(S)
            smaller = BatchSolver([game_list[i] for i in idx[keep]], variant)
            smaller.set_state(T, np.concatenate([Rs[k] for k in keep]),
                              np.concatenate([Ss[k] for k in keep]))
            solver.close()
            solver, idx = smaller, idx[keep]
            log(f"  iteration {it}: continuing with the {len(idx)} unsolved games "
                f"({int(sizes[idx].sum())} nodes)")
    torch.cuda.synchronize()
    return solved_it, solved_s, solved_e, solver


def _arm(solved_it, solved_s) -> dict:
    ok = solved_it >= 0
    ts = np.sort(solved_s)
    return {"iterations": int(solved_it.max()) if ok.all() else -1,
            "seconds": float(solved_s.max()),
            "solved": int(ok.sum()),
            "seconds_until_solved_fraction": {
                str(f): float(ts[max(0, int(np.ceil(f * len(ts))) - 1)])
                for f in (0.5, 0.9, 0.99, 1.0)},
            "per_game_iterations": {"mean": float(solved_it[ok].mean()),
                                    "median": float(np.median(solved_it[ok])),
                                    "p90": float(np.percentile(solved_it[ok], 90)),
                                    "max": int(solved_it[ok].max())}}


def plain_arm(game_list, target: float = 1e-3, check_every: int = 10, max_iters: int = 20000,
              compact: float = 0.05) -> tuple:
    """Zero-start CFR+ on the batch: per game the iteration and wall time it was solved at."""
    import torch
    from .solver import BatchSolver
    b = BatchSolver(game_list, "cfr+")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p_it, p_s, _, b = run_to_target(b, target, check_every, max_iters, t0=t0,
                                    game_list=game_list, compact=compact)
    b.close()
    return p_it, p_s


def _slowest(solved_it, k: int = 3) -> list:
    """The k games solved last (never-solved first): [index in the batch, iterations]."""
    key = np.where(solved_it < 0, np.iinfo(np.int64).max, solved_it)
    return [[int(i), int(solved_it[i])] for i in np.argsort(-key, kind="stable")[:k]]


def evaluate(game_list, net, weight: float, target: float = 1e-3, check_every: int = 10,
             max_iters: int = 20000, compact: float = 0.05, plain: tuple = None) -> dict:
    """Plain zero-start CFR+ against the warm start on the same batch, both with the same
    compaction rule: wall time until every game is solved (the batch's time to the target), and
    per game the iterations to it. `plain` takes a plain_arm result of the same batch and
    settings, so that a weight sweep runs the plain arm once."""
    import torch
    from . import warmstart as ws
    from .solver import BatchSolver
    out = {}
    p_it, p_s = plain_arm(game_list, target, check_every, max_iters, compact) if plain is None \
        else plain
    out["plain"] = _arm(p_it, p_s)
    out["plain"]["slowest"] = _slowest(p_it)
    # warm start (one zero-start iteration, network inference, fallback check, then CFR+)
    b = BatchSolver(game_list, "cfr+")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ws.warm_start(b, net, game_list, weight)
    w_it, w_s, _, b = run_to_target(b, target, check_every, max_iters, done=2, t0=t0,
                                    game_list=game_list, compact=compact)
    out["warm"] = _arm(w_it, w_s)
    out["warm"]["slowest"] = _slowest(w_it)
    out["warm"].update({"warm_start_seconds": info["seconds"],
                        "fallback_games": info["fallback_games"],
                        "first_expl_zero_max": float(np.max(info["expl_zero_start"])),
                        "first_expl_warm_max": float(np.max(info["expl_warm_start"]))})
    b.close()
    both = (p_it >= 0) & (w_it >= 0)
    ratio = w_it[both] / np.maximum(p_it[both], 1)
    out["paired"] = {"games": int(both.sum()),
                     "warm_faster": int(np.sum(w_it[both] < p_it[both])),
                     "warm_slower": int(np.sum(w_it[both] > p_it[both])),
                     "geomean_iteration_ratio": float(np.exp(np.mean(np.log(ratio)))),
                     "median_iteration_ratio": float(np.median(ratio)),
                     "p10_iteration_ratio": float(np.percentile(ratio, 10)),
                     "p90_iteration_ratio": float(np.percentile(ratio, 90)),
                     "mean_iterations_plain": float(p_it[both].mean()),
                     "mean_iterations_warm": float(w_it[both].mean())}
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16


def mlp_throughput(infer, trainer, rows: int = 65536, batch: int = 4096, reps: int = 20) -> dict:
    """Achieved TFLOP/s of the network's forward pass (`rows` infosets) and of one training step
    (`batch` infosets: forward, backward, Adam), hipEvent-timed. Multiply-adds per row: forward
    F H + H H + H A; training step 2 F H + 3 H H + 3 H A (no input gradient)."""
    import torch
    F, H, A = infer.shape
    dev = infer.device
    x = torch.randn(rows, F, device=dev).to(torch.bfloat16)
    xb = x[:batch].contiguous()
    t = torch.full((batch, A), 1.0 / A, device=dev)
    m = torch.ones(batch, A, device=dev)
    p0 = trainer.params()
    out = {}
    for name, fn, macs in (("forward", lambda: infer.forward(x), rows * (F * H + H * H + H * A)),
                           ("train_step", lambda: trainer.train_step(xb, t, m, 0.0),
                            batch * (2 * F * H + 3 * H * H + 3 * H * A))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2.0 * macs / (ms * 1e-3) / 1e12
        out[name] = {"ms": ms, "tflops": tf, "frac_of_bf16_peak": tf / MFMA_BF16_PEAK_TFLOPS}
    trainer.set_params(p0)
    return out


def eval_only(args) -> int:
    pool = Pool(args.workers)  # forked before this process touches the GPU
    pending = pool.map_async(_subgame, list(range(100, 100 + args.eval_games)), chunksize=4)
    import torch
    from . import warmstart as ws
    torch.cuda.set_device(0)
    with open(os.path.splitext(args.out_weights)[0] + ".json") as f:
        weight = json.load(f)["weight"]
    net = ws.WarmStartNet(max_batch=65536)
    net.set_params(np.load(args.out_weights))
    gl = pending.get()
    pool.close()
    res = evaluate(gl, net, weight)
    res.update({"weight": weight, "eval_games": args.eval_games,
                "eval_seeds": [100, 99 + args.eval_games]})
    log(json.dumps(res))
    if args.out_json:
        with open(args.out_json, "w") as f:
            json.dump(res, f, indent=1)
    return 0


def select_weight(val, infer, weights, by: str = "seconds") -> tuple:
    """Evaluates each warm-start weight on the validation games; returns (the chosen weight, the
    sweep). A weight qualifies when the warm start speeds up the typical game (paired geometric
    mean of warm / plain iterations below 1); if none does, all do. by='seconds': among those,
    the least wall time until every validation game reaches the target (the metric itself);
    by='iterations': the fewest mean per-game iterations to it (less noisy, but blind to the
    slowest games that set the batch's time). The wall time alone favours weights that commit
    hard enough to speed up the slowest games while slowing most of the others."""
    sweep = {}
    plain = plain_arm(val)
    for w in weights:
        r = evaluate(val, infer, w, plain=plain)
        sweep[w] = r
        log(f"validation weight {w}: plain {r['plain']['seconds']:.3f}s, mean "
            f"{r['paired']['mean_iterations_plain']:.0f} it; warm {r['warm']['seconds']:.3f}s, "
            f"mean {r['paired']['mean_iterations_warm']:.0f} it, geomean ratio "
            f"{r['paired']['geomean_iteration_ratio']:.3f}")
    ok = [w for w in sweep if sweep[w]["paired"]["geomean_iteration_ratio"] < 1.0] or list(sweep)
    if by == "iterations":
        return min(ok, key=lambda w: sweep[w]["paired"]["mean_iterations_warm"]), sweep
    return min(ok, key=lambda w: sweep[w]["warm"]["seconds"]), sweep


def _validation_summary(sweep) -> dict:
    return {str(w): {"plain_s": r["plain"]["seconds"], "warm_s": r["warm"]["seconds"],
                     "plain_mean_it": r["paired"]["mean_iterations_plain"],
                     "warm_mean_it": r["paired"]["mean_iterations_warm"],
                     "geomean_ratio": r["paired"]["geomean_iteration_ratio"],
                     "warm_faster": r["paired"]["warm_faster"]}
            for w, r in sweep.items()}


def select_only(args) -> int:
    """Re-chooses the weight of the stored network on the validation games and re-evaluates it
    on the held-out games (no training); rewrites the weight in the sidecar."""
    pool = Pool(args.workers)  # forked before this process touches the GPU
    pend_val = pool.map_async(_subgame, list(range(VAL_SEED, VAL_SEED + args.val_games)), chunksize=4)
    pend_test = pool.map_async(_subgame, list(range(100, 100 + args.eval_games)), chunksize=4)
    import torch
    from . import warmstart as ws
    torch.cuda.set_device(0)
    side = os.path.splitext(args.out_weights)[0] + ".json"
    with open(side) as f:
        meta = json.load(f)
    net = ws.WarmStartNet(max_batch=65536)
    net.set_params(np.load(args.out_weights))
    weight, sweep = select_weight(pend_val.get(), net, [float(v) for v in args.weights.split(",")],
                                  args.select_by)
    gl = pend_test.get()
    pool.close()
    res = evaluate(gl, net, weight)
    res.update({"weight": weight, "eval_games": args.eval_games,
                "eval_seeds": [100, 99 + args.eval_games], "val_games": args.val_games,
                "validation": _validation_summary(sweep)})
    log(json.dumps(res))
    meta["weight"] = weight
    meta["selection"] = res
    with open(side, "w") as f:
        json.dump(meta, f, indent=1)
    if args.out_json:
        with open(args.out_json, "w") as f:
            json.dump(res, f, indent=1)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-games", type=int, default=20000)
    ap.add_argument("--batch-games", type=int, default=512)
    ap.add_argument("--solve-iters", type=int, default=2000)
    ap.add_argument("--per-game", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weights", default="10,15,20,30,45,60,100",
                    help="warm-start weights tried on the validation games; the best is used")
    ap.add_argument("--select-by", choices=["seconds", "iterations"], default="seconds",
                    help="validation criterion for the weight (see select_weight)")
    ap.add_argument("--targets", choices=["both", "strategy", "regret"], default="both",
                    help="training targets: the average strategy after --solve-iters CFR+ "
                         "iterations, the normalised positive regrets then, or a network for "
                         "each with the better one on the validation games kept")
    ap.add_argument("--val-games", type=int, default=256)
    ap.add_argument("--eval-games", type=int, default=512)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out-weights", default=WEIGHTS_PATH)
    ap.add_argument("--out-json", default=None)
    ap.add_argument("--eval-only", action="store_true",
                    help="evaluate the stored network (weights and chosen weight next to "
                         "--out-weights) on the held-out games, without training")
    ap.add_argument("--select-only", action="store_true",
                    help="choose the weight of the stored network again on the validation games "
                         "(--weights, --val-games), then evaluate it on the held-out games")
    ap.add_argument("--throughput-only", action="store_true",
                    help="time the network's forward pass (65,536 rows) and one training step "
                         "(4,096 rows) with random weights and print them as JSON")
    args = ap.parse_args()
    if args.throughput_only:
        import torch
        from . import warmstart as ws
        torch.cuda.set_device(0)
        net = ws.WarmStartNet(max_batch=4096, seed=1)
        infer = ws.WarmStartNet(max_batch=65536, seed=1)
        print(json.dumps(mlp_throughput(infer, net)), flush=True)
        return 0
    if args.eval_only:
        return eval_only(args)
    if args.select_only:
        return select_only(args)
    sys.path.insert(0, ROOT)
    # the worker processes are forked before this process touches the GPU
    pool = Pool(args.workers)
    import torch
    from . import warmstart as ws

    torch.cuda.set_device(0)
    rng = np.random.default_rng(0)
    parts = []
    t0 = time.time()
    batches = _batches(args.train_games, args.batch_games, 10000)
    n_games = 0
    # the host builds batch i + 1 while the GPU solves batch i
    pending = pool.map_async(_subgame, list(batches[0]), chunksize=4)
    for i, seeds in enumerate(batches):
        gl = pending.get()
        if i + 1 < len(batches):
            pending = pool.map_async(_subgame, list(batches[i + 1]), chunksize=4)
        else:
            pending = pool.map_async(_subgame, list(range(VAL_SEED, VAL_SEED + args.val_games)),
                                     chunksize=4)
        d = solve_targets(gl, args.solve_iters, args.per_game, rng)
        log(f"solved training seeds {seeds.start}-{seeds.stop - 1}: {len(d['desc'])} samples, "
            f"median expl {np.median(d['expl']):.2e} ({time.time() - t0:.0f}s)")
        d["desc"] = d["desc"].copy()
        d["desc"][:, 15] += n_games  # global game index into the stacked beliefs
        n_games += len(gl)
        parts.append(d)
        del gl
    data = {"desc": np.concatenate([p["desc"] for p in parts]),
            "beliefs": np.concatenate([p["beliefs"] for p in parts]),
            "target": np.concatenate([p["target"] for p in parts]),
            "rtarget": np.concatenate([p["rtarget"] for p in parts]),
            "mask": np.concatenate([p["mask"] for p in parts])}
    del parts
    kinds = {"strategy": "target", "regret": "rtarget"}
    names = list(kinds) if args.targets == "both" else [args.targets]
    nets, losses = {}, {}
    for name in names:
        net = ws.WarmStartNet(max_batch=4096, seed=1)
        t1 = time.time()
        losses[name] = train(net, data, args.epochs, 4096, args.lr, key=kinds[name])
        log(f"{name} targets: trained on {len(data['desc'])} samples in {time.time() - t1:.1f}s")
        nets[name] = net
    # each network's weight is chosen on validation games (seeds disjoint from training and
    # evaluation); the network kept is the one whose chosen weight is faster there
    val = pending.get()
    pending = pool.map_async(_subgame, list(range(100, 100 + args.eval_games)), chunksize=4)
    infer = ws.WarmStartNet(max_batch=65536)
    chosen = {}
    for name in names:
        infer.set_params(nets[name].params())
        w, sweep = select_weight(val, infer, [float(v) for v in args.weights.split(",")],
                                 args.select_by)
        chosen[name] = {"weight": w, "validation": _validation_summary(sweep),
                        "validation_warm_s": sweep[w]["warm"]["seconds"],
                        "validation_paired": sweep[w]["paired"]}
        log(f"{name} targets: weight {w}, validation warm {sweep[w]['warm']['seconds']:.3f}s")
    best = min(names, key=lambda n: chosen[n]["validation_warm_s"])
    del val
    gl = pending.get()
    pool.close()
    # every trained network is reported on the held-out games; the kept one was chosen above
    plain = plain_arm(gl)
    results = {}
    for name in names:
        infer.set_params(nets[name].params())
        results[name] = evaluate(gl, infer, chosen[name]["weight"], plain=plain)
        results[name].update(chosen[name])
        results[name]["losses"] = losses[name]
    net = nets[best]
    infer.set_params(net.params())
    res = dict(results[best])
    res["mlp"] = mlp_throughput(infer, net)
    log(f"network throughput: {json.dumps(res['mlp'])}")
    res.update({"targets": best, "train_games": args.train_games,
                "solve_iters": args.solve_iters, "samples": int(len(data["desc"])),
                "eval_games": args.eval_games, "eval_seeds": [100, 99 + args.eval_games],
                "val_games": args.val_games,
                "alternatives": {n: results[n] for n in names if n != best}})
    log(json.dumps(res))
    os.makedirs(os.path.dirname(args.out_weights), exist_ok=True)
    stem = os.path.splitext(args.out_weights)[0]
    np.save(args.out_weights, net.params())
    log(f"{best}-target weights written to {args.out_weights}")
    with open(stem + ".json", "w") as f:
        json.dump({"weight": chosen[best]["weight"], "targets": best, "shape": list(net.shape),
                   "results": res}, f, indent=1)
    # the other networks beside it (usable with --eval-only --out-weights STEM_NAME.npy)
    for name in names:
        if name != best:
            np.save(f"{stem}_{name}.npy", nets[name].params())
            with open(f"{stem}_{name}.json", "w") as f:
                json.dump({"weight": chosen[name]["weight"], "targets": name,
                           "shape": list(nets[name].shape), "results": results[name]}, f, indent=1)
            log(f"{name}-target weights written to {stem}_{name}.npy")
    if args.out_json:
        with open(args.out_json, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
