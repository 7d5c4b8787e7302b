"""Training and evaluation of the learned warm start on the batched subgame family.

    python -m paper_2408_14778_amd.warmstart_pipeline --train-games 20000 --out-weights W.npy

1. Data: seeded subgames (training seeds from 10,000 up, disjoint from the evaluation seeds
   100-611) are solved in batches by GPU CFR+; each infoset's target is the average strategy
   GPU CFR+ reaches after K iterations, over its legal action slots.
2. Training: minibatch Adam on the masked softmax cross-entropy, all on the GPU with the
   library's BF16-MFMA kernels (features, forward, backward, optimiser).
3. Evaluation: on the held-out batch, plain CFR+ from zero regrets against the warm start,
   both checked with the best-response pass every `check_every` iterations until the largest
   exploitability in the batch is at most the target; wall time includes the network's
   inference and the warm start's own checks.
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
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning",
                            "warmstart_gfx950.npy")


def log(msg):
    print(f"[warmstart] {msg}", flush=True)


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
    expl = b.exploitability()["expl"]
    b.close()
    desc, bel, qoff = ws.descriptors(game_list)
    target, mask = ws.slot_targets(desc, avg, qoff)
    keep = []
    gidx = desc[:, 15].astype(np.int64)
    starts = np.searchsorted(gidx, np.arange(len(game_list)))
    ends = np.searchsorted(gidx, np.arange(len(game_list)), side="right")
    for s, e in zip(starts, ends):
        n = e - s
        keep.append(s + (np.arange(n) if n <= per_game else rng.choice(n, per_game, replace=False)))
    keep = np.concatenate(keep)
    return {"desc": desc[keep], "beliefs": bel, "target": target[keep], "mask": mask[keep],
            "expl": expl}


def train(net, data: dict, epochs: int, batch: int, lr: float, seed: int = 0) -> list:
    import torch
    from . import warmstart as ws
    dev = net.device
    x = ws.features(torch.from_numpy(data["desc"]).to(dev), torch.from_numpy(data["beliefs"]).to(dev),
                    net.shape[0])
    t = torch.from_numpy(data["target"]).to(dev)
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
        log(f"epoch {ep}: loss {losses[-1]:.5f}")
    return losses


def run_to_target(solver, target: float, check_every: int, max_iters: int, done: int = 0):
    """Iterate with best-response checks until max exploitability <= target."""
    import torch
    it = done
    worst = float("inf")
    while it < max_iters:
        solver.iterate(check_every)
        it += check_every
        worst = float(np.max(solver.exploitability()["expl"]))
        if worst <= target:
            break
        if (it // check_every) % 50 == 0:
            log(f"  iteration {it}: max exploitability {worst:.3e}")
    torch.cuda.synchronize()
    return it, worst


def evaluate(game_list, net, weight: float, target: float = 1e-3, check_every: int = 10,
             max_iters: int = 4000) -> dict:
    import torch
    from . import warmstart as ws
    from .solver import BatchSolver
    out = {}
    # plain CFR+ from zero regrets
    b = BatchSolver(game_list, "cfr+")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, worst = run_to_target(b, target, check_every, max_iters)
    out["plain"] = {"iterations": iters, "seconds": time.perf_counter() - t0, "max_expl": worst}
    b.close()
    del b
    # warm start (one zero-start iteration, network inference, fallback check, then CFR+)
    b = BatchSolver(game_list, "cfr+")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ws.warm_start(b, net, game_list, weight)
    iters, worst = run_to_target(b, target, check_every, max_iters, done=2)
    out["warm"] = {"iterations": iters, "seconds": time.perf_counter() - t0, "max_expl": worst,
                   "warm_start_seconds": info["seconds"],
                   "fallback_games": info["fallback_games"],
                   "first_expl_zero": float(np.max(info["expl_zero_start"])),
                   "first_expl_warm": float(np.max(info["expl_warm_start"]))}
    b.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-games", type=int, default=20000)
    ap.add_argument("--batch-games", type=int, default=512)
    ap.add_argument("--solve-iters", type=int, default=300)
    ap.add_argument("--per-game", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weight", type=float, default=10.0)
    ap.add_argument("--eval-games", type=int, default=512)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out-weights", default=WEIGHTS_PATH)
    ap.add_argument("--out-json", default=None)
    args = ap.parse_args()
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
            pending = pool.map_async(_subgame, list(range(100, 100 + args.eval_games)), chunksize=4)
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
            "mask": np.concatenate([p["mask"] for p in parts])}
    del parts
    net = ws.WarmStartNet(max_batch=4096, seed=1)
    t1 = time.time()
    losses = train(net, data, args.epochs, 4096, args.lr)
    log(f"trained on {len(data['desc'])} samples in {time.time() - t1:.1f}s")
    os.makedirs(os.path.dirname(args.out_weights), exist_ok=True)
    np.save(args.out_weights, net.params())
    log(f"weights written to {args.out_weights}")
    gl = pending.get()
    pool.close()
    infer = ws.WarmStartNet(max_batch=65536)
    infer.set_params(net.params())
    res = evaluate(gl, infer, args.weight)
    res.update({"train_games": args.train_games, "solve_iters": args.solve_iters,
                "samples": int(len(data["desc"])), "losses": losses, "weight": args.weight,
                "eval_games": args.eval_games})
    log(json.dumps(res))
    side = os.path.splitext(args.out_weights)[0] + ".json"
    with open(side, "w") as f:
        json.dump({"weight": args.weight, "shape": list(net.shape), "results": res}, f, indent=1)
    if args.out_json:
        with open(args.out_json, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
