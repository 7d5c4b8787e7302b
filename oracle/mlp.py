"""FP64 reference of the warm-start network: forward, backward, loss and Adam.

Test infrastructure (oracle): not part of the product path. The warm start is not in the
paper; this is the plain definition of a three-layer perceptron trained with a masked
softmax cross-entropy, written out with numpy.

    Z1 = X W1 + b1,  A1 = relu(Z1)
    Z2 = A1 W2 + b2, A2 = relu(Z2)
    Z3 = A2 W3 + b3                              (logits, one per action slot)
    p  = softmax over the legal slots (mask = 1) of Z3
    L  = -(1/B) sum_b sum_a mask[b,a] * target[b,a] * log p[b,a]

Backward by the chain rule; Adam with the usual bias corrections.
"""
from __future__ import annotations

import numpy as np

PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3")


def init(in_features: int, hidden: int, outputs: int, seed: int) -> dict:
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)

    def he(fan_in, fan_out):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=(fan_in, fan_out))

    return {"W1": he(in_features, hidden), "b1": np.zeros(hidden),
            "W2": he(hidden, hidden), "b2": np.zeros(hidden),
            "W3": he(hidden, outputs), "b3": np.zeros(outputs)}


def forward(p: dict, X: np.ndarray) -> dict:
    Z1 = X @ p["W1"] + p["b1"]
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ p["W2"] + p["b2"]
    A2 = np.maximum(Z2, 0.0)
    Z3 = A2 @ p["W3"] + p["b3"]
    return {"X": X, "Z1": Z1, "A1": A1, "Z2": Z2, "A2": A2, "Z3": Z3}


def masked_softmax(Z: np.ndarray, mask: np.ndarray) -> np.ndarray:
    Zm = np.where(mask > 0, Z, -np.inf)
    m = Zm.max(axis=1, keepdims=True)
    e = np.where(mask > 0, np.exp(Zm - m), 0.0)
    return e / e.sum(axis=1, keepdims=True)


def loss(Z3: np.ndarray, target: np.ndarray, mask: np.ndarray) -> float:
    P = masked_softmax(Z3, mask)
    logp = np.log(np.where(mask > 0, P, 1.0))
    return float(-(mask * target * logp).sum() / Z3.shape[0])


def backward(p: dict, cache: dict, target: np.ndarray, mask: np.ndarray) -> dict:
    B = cache["X"].shape[0]
    P = masked_softmax(cache["Z3"], mask)
    tsum = (mask * target).sum(axis=1, keepdims=True)
    dZ3 = mask * (P * tsum - target) / B
    g = {"W3": cache["A2"].T @ dZ3, "b3": dZ3.sum(axis=0)}
    dA2 = dZ3 @ p["W3"].T
    dZ2 = dA2 * (cache["Z2"] > 0)
    g["W2"] = cache["A1"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dA1 = dZ2 @ p["W2"].T
    dZ1 = dA1 * (cache["Z1"] > 0)
    g["W1"] = cache["X"].T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(p: dict, g: dict, state: dict, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in PARAMS:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] ** 2
        mhat = m / (1 - beta1 ** t)
        vhat = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return p
