"""Pin for the FP64 warm-start network reference: backward equals central finite
differences of the loss; the masked softmax ignores illegal slots; Adam matches its
closed form on the first step (update = -lr * sign(g) up to eps)."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, B=7, F=5, A=4):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, F))
    mask = (rng.random((B, A)) < 0.75).astype(float)
    mask[:, 0] = 1.0
    T = rng.random((B, A)) * mask
    T /= T.sum(axis=1, keepdims=True)
    return X, T, mask


@pytest.mark.parametrize("seed", range(3))
def test_backward_matches_finite_differences(seed):
    X, T, mask = _data(seed)
    p = mlp.init(5, 6, 4, seed)
    for k in mlp.PARAMS:  # nonzero biases so every path is exercised
        if k.startswith("b"):
            p[k] = np.random.default_rng(seed + 9).standard_normal(p[k].shape) * 0.1
    g = mlp.backward(p, mlp.forward(p, X), T, mask)
    h = 1e-6
    for k in mlp.PARAMS:
        num = np.zeros_like(p[k])
        it = np.nditer(p[k], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            old = p[k][i]
            p[k][i] = old + h
            lp = mlp.loss(mlp.forward(p, X)["Z3"], T, mask)
            p[k][i] = old - h
            lm = mlp.loss(mlp.forward(p, X)["Z3"], T, mask)
            p[k][i] = old
            num[i] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(g[k], num, atol=1e-7, rtol=1e-5)


def test_masked_softmax_ignores_illegal_slots():
    Z = np.array([[1.0, 2.0, 300.0, -1.0]])
    mask = np.array([[1.0, 1.0, 0.0, 1.0]])
    P = mlp.masked_softmax(Z, mask)
    assert P[0, 2] == 0.0 and abs(P.sum() - 1.0) < 1e-15
    e = np.exp([1.0, 2.0, -1.0])
    np.testing.assert_allclose(P[0, [0, 1, 3]], e / e.sum(), rtol=1e-15)


def test_adam_first_step_is_signed_lr():
    X, T, mask = _data(5)
    p = mlp.init(5, 6, 4, 5)
    g = mlp.backward(p, mlp.forward(p, X), T, mask)
    q = {k: v.copy() for k, v in p.items()}
    with np.errstate(invalid="ignore"):   # eps = 0: zero-gradient entries divide 0 by 0
        mlp.adam_step(q, g, {}, lr=1e-3, eps=0.0)
    for k in mlp.PARAMS:
        nz = g[k] != 0
        np.testing.assert_allclose((q[k] - p[k])[nz], -1e-3 * np.sign(g[k][nz]), rtol=1e-9)


def _const_grads(values):
    return {k: np.full((2, 3), v) for k, v in zip(mlp.PARAMS, values)}


def test_adam_constant_gradient_moves_by_lr_every_step():
    """A gradient that never changes gives m_t = g (1 - b1^t) and v_t = g^2 (1 - b2^t), so the
    bias-corrected step is exactly -lr * sign(g) at every t (eps = 0). A step counter that
    does not advance, or a correction with another power of beta, fails from t = 2 on."""
    vals = [0.5, -2.0, 3e-3, -7.0, 1.0, -0.25]
    g = _const_grads(vals)
    p = {k: np.zeros((2, 3)) for k in mlp.PARAMS}
    state = {}
    for t in range(1, 8):
        before = {k: v.copy() for k, v in p.items()}
        mlp.adam_step(p, g, state, lr=1e-2, eps=0.0)
        assert state["t"] == t
        for k, v in zip(mlp.PARAMS, vals):
            np.testing.assert_allclose(p[k] - before[k], -1e-2 * np.sign(v), rtol=1e-12)


def test_adam_alternating_gradient_closed_form():
    """Gradients g, -g, g, ... : v_t = g^2 (1 - b2^t) so the corrected second moment is g^2,
    and m_t = (1 - b1) g (-1)^(t-1) sum_{j<t} (-b1)^j, so the step at t is
    -lr (-1)^(t-1) sign(g) (1 - b1)(1 - (-b1)^t) / ((1 + b1)(1 - b1^t)) (eps = 0). This pins the
    momentum recursion (which past gradient gets which power of b1) on steps 1-6."""
    b1, b2, lr = 0.8, 0.99, 1e-2
    vals = [1.5, -0.5, 2.0, -3.0, 0.25, 4.0]
    p = {k: np.zeros((2, 3)) for k in mlp.PARAMS}
    state = {}
    for t in range(1, 7):
        sgn = (-1.0) ** (t - 1)
        g = _const_grads([sgn * v for v in vals])
        before = {k: v.copy() for k, v in p.items()}
        mlp.adam_step(p, g, state, lr=lr, beta1=b1, beta2=b2, eps=0.0)
        frac = (1 - b1) * (1 - (-b1) ** t) / ((1 + b1) * (1 - b1 ** t))
        for k, v in zip(mlp.PARAMS, vals):
            np.testing.assert_allclose(p[k] - before[k], -lr * sgn * np.sign(v) * frac,
                                       rtol=1e-12)
