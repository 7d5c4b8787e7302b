"""GPU checks of the warm-start network and pipeline against the FP64 reference (oracle/mlp.py).

BF16 storage of weights and activations bounds the agreement: the forward pass is compared
with a numpy evaluation that rounds the same tensors to bf16 (tight), and the gradients with
the plain FP64 reference (about 2e-2 relative, the bf16 unit roundoff times a few layers)."""
import numpy as np
import pytest

import games
from oracle import mlp

pytestmark = pytest.mark.gpu


def bf16(a):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _flat(p):
    return np.concatenate([p[k].ravel() for k in mlp.PARAMS]).astype(np.float32)


def _unflat(v, F, H, A):
    out, o = {}, 0
    for k, shape in (("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, A)),
                     ("b3", (A,))):
        n = int(np.prod(shape))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def _net(F, H, A, B, seed):
    from paper_2408_14778_amd.warmstart import WarmStartNet
    return WarmStartNet(F, H, A, max_batch=B, seed=seed)


@pytest.mark.parametrize("F,H,A,B", [(96, 256, 4, 300), (40, 64, 4, 77), (96, 256, 4, 4096),
                                     (72, 128, 4, 333), (96, 256, 4, 65536), (48, 128, 4, 333),
                                     (64, 64, 8, 100)])
def test_forward_matches_bf16_emulation(F, H, A, B):
    import torch
    rng = np.random.default_rng(F + H + B)
    p = mlp.init(F, H, A, seed=3)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    net = _net(F, H, A, B, 0)
    net.set_params(_flat(p))
    X = bf16(rng.standard_normal((B, F)))
    xt = torch.from_numpy(X.astype(np.float32)).to("cuda").to(torch.bfloat16)
    Z = net.forward(xt).cpu().numpy().astype(np.float64)
    W1, W2, W3 = (bf16(p["W1"]), bf16(p["W2"]), bf16(p["W3"]))
    b1, b2, b3 = (np.asarray(p[k], np.float32).astype(np.float64) for k in ("b1", "b2", "b3"))
    A1 = bf16(np.maximum(X @ W1 + b1, 0))
    A2 = bf16(np.maximum(A1 @ W2 + b2, 0))
    Zref = A2 @ W3 + b3
    err = np.abs(Z - Zref).max() / np.abs(Zref).max()
    assert err < 2e-3, err


@pytest.mark.parametrize("F,H,A,B", [(96, 256, 4, 16384), (96, 256, 4, 37), (48, 128, 4, 1000),
                                     (64, 64, 8, 333), (32, 256, 1, 4097)])
def test_fused_forward_equals_per_layer_gemms(F, H, A, B):
    """cfr_mlp_forward runs the three layers in one kernel for these shapes; the allocation-free
    entry point runs them as three GEMMs through its device array. Every element is computed in
    the same order (the same BF16 operands, the same 16-wide MFMA steps, the same rounding of the
    hidden layers, the same order of the last layer's sums), so the logits agree bit for bit;
    ragged last tiles included."""
    import torch
    net = _net(F, H, A, B, 7)
    rng = np.random.default_rng(F * H + B)
    p = mlp.init(F, H, A, seed=9)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    net.set_params(_flat(p))
    x = torch.from_numpy(rng.standard_normal((B, F)).astype(np.float32)).to("cuda")
    x = x.to(torch.bfloat16)
    ref = net.forward(x)
    out = torch.full((B, A), float("nan"), dtype=torch.float32, device="cuda")
    net.forward_noalloc(x, out)
    torch.cuda.synchronize()
    a, b = ref.cpu().numpy(), out.cpu().numpy()
    assert np.isfinite(a).all()
    assert np.array_equal(a, b), float(np.abs(a - b).max())


def test_gradients_match_fp64_reference():
    import torch
    F, H, A, B = 96, 256, 4, 512
    rng = np.random.default_rng(11)
    p = mlp.init(F, H, A, seed=5)
    p = {k: bf16(v) for k, v in p.items()}   # parameters exactly representable on both sides
    net = _net(F, H, A, B, 0)
    net.set_params(_flat(p))
    X = bf16(rng.standard_normal((B, F)))
    mask = (rng.random((B, A)) < 0.8).astype(np.float64)
    mask[:, 1] = 1.0
    T = rng.random((B, A)) * mask
    T /= T.sum(axis=1, keepdims=True)
    dev = "cuda"
    xt = torch.from_numpy(X.astype(np.float32)).to(dev).to(torch.bfloat16)
    tt = torch.from_numpy(T.astype(np.float32)).to(dev)
    mt = torch.from_numpy(mask.astype(np.float32)).to(dev)
    loss = net.train_step(xt, tt, mt, lr=0.0)
    g = _unflat(net.grads(), F, H, A)
    cache = mlp.forward(p, X)
    ref_loss = mlp.loss(cache["Z3"], T, mask)
    ref = mlp.backward(p, cache, T, mask)
    assert abs(loss - ref_loss) <= 2e-2 * abs(ref_loss)
    for k in mlp.PARAMS:
        rel = np.abs(g[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-12)
        assert rel < 5e-2, (k, rel)


def test_training_reduces_loss():
    import torch
    F, H, A, B = 96, 256, 4, 2048
    rng = np.random.default_rng(2)
    X = bf16(rng.standard_normal((B, F)))
    Wt = rng.standard_normal((F, A))
    mask = np.ones((B, A))
    T = mlp.masked_softmax(X @ Wt, mask)
    net = _net(F, H, A, B, 1)
    xt = torch.from_numpy(X.astype(np.float32)).to("cuda").to(torch.bfloat16)
    tt = torch.from_numpy(T.astype(np.float32)).to("cuda")
    mt = torch.from_numpy(mask.astype(np.float32)).to("cuda")
    first = net.train_step(xt, tt, mt, lr=1e-3)
    for _ in range(200):
        last = net.train_step(xt, tt, mt, lr=1e-3)
    entropy = float(-(T * np.log(T)).sum() / B)
    assert last < first and last - entropy < 0.5 * (first - entropy)


def test_adam_matches_fp64_reference_over_steps():
    """Six training steps with lr > 0: after each, the GPU's FP32 master parameters equal the
    FP64 Adam of the oracle applied to the GPU's own gradient of that step, with the oracle's
    moments carried over from step to step (b1 0.9, b2 0.999, eps 1e-8, bias corrections by
    the step count). The parameters are compared at FP32 rounding of their magnitude plus
    1e-5 of the step size."""
    import torch
    F, H, A, B = 40, 64, 4, 256
    rng = np.random.default_rng(17)
    X = bf16(rng.standard_normal((B, F)))
    mask = (rng.random((B, A)) < 0.8).astype(np.float64)
    mask[:, 0] = 1.0
    T = rng.random((B, A)) * mask
    T /= T.sum(axis=1, keepdims=True)
    net = _net(F, H, A, B, 3)
    xt = torch.from_numpy(X.astype(np.float32)).to("cuda").to(torch.bfloat16)
    tt = torch.from_numpy(T.astype(np.float32)).to("cuda")
    mt = torch.from_numpy(mask.astype(np.float32)).to("cuda")
    lr = 3e-3
    state = {}
    for step in range(6):
        before = _unflat(net.params(), F, H, A)
        net.train_step(xt, tt, mt, lr=lr)
        g = _unflat(net.grads(), F, H, A)
        after = _unflat(net.params(), F, H, A)
        ref = mlp.adam_step({k: v.copy() for k, v in before.items()}, g, state, lr=lr)
        for k in mlp.PARAMS:
            tol = 2.0 ** -23 * np.abs(ref[k]) + 1e-5 * lr
            err = np.abs(after[k] - ref[k])
            assert np.all(err <= tol), (step, k, float((err / tol).max()))
            moved = np.abs(after[k] - before[k]).max()
            assert moved > 0.1 * lr, (step, k, moved)  # every tensor takes real steps
    net.close()


def test_features_match_definition():
    import torch
    from paper_2408_14778_amd import warmstart as ws
    gl = [games.subgame(s) for s in (102, 104, 107)]
    desc, bel, qoff = ws.descriptors(gl)
    x = ws.features(torch.from_numpy(desc).cuda(), torch.from_numpy(bel).cuda()).float().cpu().numpy()
    assert x.shape == (len(desc), 96)
    for i in np.random.default_rng(0).choice(len(desc), 50, replace=False):
        d = desc[i]
        player, own, rnd = int(d[0]), int(d[1]), int(d[2])
        row = x[i]
        assert row[own] == 1 and row[:13].sum() == 1
        assert row[13 + (0 if player == 1 else 1)] == 1
        assert row[15 + rnd] == 1
        board = [c for c in d[3:6] if c >= 0]
        assert sorted(np.flatnonzero(row[18:31]).tolist()) == sorted(set(int(c) for c in board))
        mask = int(d[11])
        assert [row[31 + 4 + 5 + 4 + s] for s in range(4)] == [float((mask >> s) & 1) for s in range(4)]
        # layout: own 13, player 2, round 3, board 13, raises 4, last 5, pot 4, slots 4,
        # depth/cap/stack/ranks 4 (= 52), opponent range 13, own range 13, win/lose 2, bias 1
        bop = bel[d[15], 2 - player]
        bme = bel[d[15], player - 1]
        np.testing.assert_allclose(row[52:65], bf16(bop), rtol=0, atol=1e-6)
        np.testing.assert_allclose(row[65:78], bf16(bme), rtol=0, atol=1e-6)
        np.testing.assert_allclose(row[78], bf16(bop[:own].sum()), atol=4e-3)
        np.testing.assert_allclose(row[79], bf16(bop[own + 1:].sum()), atol=4e-3)
        assert row[80] == 1.0 and np.all(row[81:] == 0)


def test_warm_start_sets_scaled_regrets():
    import torch
    from paper_2408_14778_amd import BatchSolver
    from paper_2408_14778_amd import warmstart as ws
    gl = [games.subgame(s) for s in (102, 103)]
    b = BatchSolver(gl, "cfr+")
    b.iterate(1)
    _, R1, _ = b.get_state()
    desc, bel, qoff = ws.descriptors(gl)
    net = ws.WarmStartNet(max_batch=4096, seed=3)
    x = ws.features(torch.from_numpy(desc).cuda(), torch.from_numpy(bel).cuda())
    logits = net.forward(x)
    probs = ws.probs_to_pairs(logits, torch.from_numpy(desc).cuda(), torch.from_numpy(qoff).cuda(),
                              b.n_q)
    pr = probs.cpu().numpy()
    # probabilities per infoset sum to one over its actions
    k = np.diff(np.concatenate([qoff, [b.n_q]]))
    sums = np.add.reduceat(pr, qoff)
    np.testing.assert_allclose(sums, 1.0, atol=1e-5)
    import ctypes
    from paper_2408_14778_amd import _native as N
    N.check(ws._lib().cfr_warm_start(b._h, ctypes.c_void_p(probs.data_ptr()), b.n_q, 7.0))
    T, R, S = b.get_state()
    assert T == 0 and np.all(S == 0)
    m = np.add.reduceat(np.maximum(R1, 0), qoff)
    expect = 7.0 * np.repeat(m, k) * pr
    np.testing.assert_allclose(R, expect, rtol=1e-5, atol=1e-7)
    sig = b.current_strategy()
    np.testing.assert_allclose(np.where(np.repeat(m, k) > 0, sig, pr), pr, atol=1e-5)


def test_trained_network_reduces_iterations_to_target():
    """The committed network (trained by warmstart_pipeline on seeds 10000-29999) against
    zero-start CFR+ on 64 held-out subgames: iterations until each game's exploitability first
    reaches 1e-3 (best-response check every 10 iterations)."""
    import json
    import os
    from paper_2408_14778_amd import warmstart as ws
    from paper_2408_14778_amd import warmstart_pipeline as wp
    if not os.path.exists(wp.WEIGHTS_PATH):
        pytest.skip("no trained weights (run paper_2408_14778_amd.warmstart_pipeline)")
    with open(os.path.splitext(wp.WEIGHTS_PATH)[0] + ".json") as f:
        weight = json.load(f)["weight"]
    net = ws.WarmStartNet(max_batch=65536)
    net.set_params(np.load(wp.WEIGHTS_PATH))
    gl = [games.subgame(s) for s in range(100, 164)]
    res = wp.evaluate(gl, net, weight, max_iters=8000)
    paired = res["paired"]
    assert paired["games"] >= 60
    assert paired["mean_iterations_warm"] < 0.95 * paired["mean_iterations_plain"], paired
    assert paired["geomean_iteration_ratio"] < 0.95, paired
    assert res["warm"]["first_expl_warm_max"] < res["warm"]["first_expl_zero_max"]
