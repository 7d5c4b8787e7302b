"""Learned warm start for batched subgame solving (gfx950 kernels behind include/cfr_warmstart.h).

A three-layer perceptron (96 inputs -> 256 -> 256 -> 4 action slots, ReLU; BF16 weights on
MFMA, FP32 accumulation, Adam on FP32 master weights) maps each infoset's features to a
distribution over its legal actions. The warm start sets the initial cumulative regrets to
R0(h, a) = w * m(h) * p(h, a), with m(h) the size of h's regrets after one CFR+ iteration
from zero, so the first strategies played are the network's. Training targets are the
average strategies that GPU CFR+ itself reaches on seeded subgames. Plain CFR from zero
regrets is the fallback: a warm start whose first average strategy is more exploitable
than the uniform one is undone.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import _native as N
from .solver import BatchSolver, _ptr

IN_FEATURES, HIDDEN, SLOTS = 96, 256, 4


def _lib():
    lib = N.load()
    if not getattr(lib, "_warm_bound", False):
        sig = {
            "cfr_mlp_num_params": (ctypes.c_int64, [ctypes.c_int32] * 3),
            "cfr_mlp_workspace_bytes": (ctypes.c_int64, [ctypes.c_int32] * 4),
            "cfr_mlp_create": (ctypes.c_int, [ctypes.c_int32] * 4 + [ctypes.c_void_p, ctypes.c_size_t,
                                                                     ctypes.c_void_p,
                                                                     ctypes.POINTER(ctypes.c_void_p)]),
            "cfr_mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                                  ctypes.c_int64]),
            "cfr_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                                  ctypes.c_int64]),
            "cfr_mlp_get_grads": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                                 ctypes.c_int64]),
            "cfr_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_void_p]),
            "cfr_mlp_forward_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.c_int32, ctypes.c_void_p]),
            "cfr_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_int32, ctypes.c_float,
                                                  ctypes.POINTER(ctypes.c_float)]),
            "cfr_mlp_destroy": (ctypes.c_int, [ctypes.c_void_p]),
            "cfr_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
            "cfr_probs_to_pairs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                                  ctypes.c_void_p]),
            "cfr_warm_start": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_float]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        lib._warm_bound = True
    return lib


def descriptors(game_list):
    """Concatenated infoset descriptors (int16 [H, 16], game index filled in), per-game root
    beliefs (float32 [G, 2, 13]) and each infoset's first pair in the batch order (int64)."""
    descs, bels, qoff = [], [], []
    base = 0
    for g_i, g in enumerate(game_list):
        d = np.array(g.meta["infoset_desc"], dtype=np.int16, copy=True)
        d[:, 15] = g_i
        descs.append(d)
        bel = g.meta.get("beliefs")
        if bel is None:
            bel = np.zeros((2, 13), dtype=np.float32)
            bel[:, :g.meta["n_ranks"]] = 1.0 / g.meta["n_ranks"]
        bels.append(np.asarray(bel, dtype=np.float32))
        rational = g.infoset_player != 0
        k = g.infoset_num_actions[rational].astype(np.int64)
        qoff.append(base + np.concatenate([[0], np.cumsum(k)[:-1]]))
        base += int(k.sum())
    return np.concatenate(descs), np.stack(bels), np.concatenate(qoff)


def slot_targets(desc: np.ndarray, pair_probs: np.ndarray, qoff: np.ndarray):
    """Per infoset: target distribution over the 4 slots and the legal-slot mask."""
    n = desc.shape[0]
    target = np.zeros((n, SLOTS), dtype=np.float32)
    mask = np.zeros((n, SLOTS), dtype=np.float32)
    amask = desc[:, 11].astype(np.int64)
    a = np.zeros(n, dtype=np.int64)
    for s in range(SLOTS):
        legal = (amask >> s) & 1 == 1
        mask[legal, s] = 1.0
        target[legal, s] = pair_probs[qoff[legal] + a[legal]]
        a += legal
    return target, mask


def he_uniform_params(in_features: int, hidden: int, outputs: int, seed: int) -> np.ndarray:
    """Initial parameters, flat FP32 in the library's order (W1, b1, W2, b2, W3, b3):
    weights uniform in +-sqrt(6 / fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((in_features, hidden), (hidden, hidden), (hidden, outputs)):
        lim = np.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, size=(fi, fo)).astype(np.float32).ravel())
        parts.append(np.zeros(fo, dtype=np.float32))
    return np.concatenate(parts)


class WarmStartNet:
    """The network on one GPU; device buffers come from torch, all math from the library."""

    def __init__(self, in_features=IN_FEATURES, hidden=HIDDEN, outputs=SLOTS, max_batch=65536,
                 seed=0, device="cuda", stream=None):
        import torch

        self.lib = _lib()
        self.shape = (in_features, hidden, outputs)
        self.max_batch = max_batch
        self.n_params = int(self.lib.cfr_mlp_num_params(in_features, hidden, outputs))
        nbytes = int(self.lib.cfr_mlp_workspace_bytes(in_features, hidden, outputs, max_batch))
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        N.check(self.lib.cfr_mlp_create(in_features, hidden, outputs, max_batch,
                                        ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.set_params(he_uniform_params(in_features, hidden, outputs, seed))

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        N.check(self.lib.cfr_mlp_set_params(self._h, _ptr(p, ctypes.c_float), p.size))

    def params(self) -> np.ndarray:
        p = np.empty(self.n_params, dtype=np.float32)
        N.check(self.lib.cfr_mlp_get_params(self._h, _ptr(p, ctypes.c_float), p.size))
        return p

    def grads(self) -> np.ndarray:
        g = np.empty(self.n_params, dtype=np.float32)
        N.check(self.lib.cfr_mlp_get_grads(self._h, _ptr(g, ctypes.c_float), g.size))
        return g

    def forward(self, x):
        """x: bf16 device tensor [B, in_features] -> fp32 logits [B, outputs] (device)."""
        import torch
        B = int(x.shape[0])
        out = torch.empty((B, self.shape[2]), dtype=torch.float32, device=self.device)
        for s in range(0, B, self.max_batch):
            e = min(B, s + self.max_batch)
            N.check(self.lib.cfr_mlp_forward(self._h, ctypes.c_void_p(x[s:e].data_ptr()), e - s,
                                             ctypes.c_void_p(out[s:e].data_ptr())))
        return out

    def forward_noalloc(self, x, out) -> None:
        """The allocation-free forward pass into an existing fp32 device tensor out [B, outputs]
        (activations in the library's own device array; see cfr_mlp_forward_noalloc)."""
        assert out.dtype.itemsize == 4 and out.is_cuda and out.shape[0] == x.shape[0]
        N.check(self.lib.cfr_mlp_forward_noalloc(self._h, ctypes.c_void_p(x.data_ptr()),
                                                 int(x.shape[0]), ctypes.c_void_p(out.data_ptr())))

    def train_step(self, x, target, mask, lr: float) -> float:
        loss = ctypes.c_float()
        N.check(self.lib.cfr_mlp_train_step(self._h, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(target.data_ptr()),
                                            ctypes.c_void_p(mask.data_ptr()), int(x.shape[0]),
                                            float(lr), ctypes.byref(loss)))
        return float(loss.value)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.cfr_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(desc_dev, beliefs_dev, in_features=IN_FEATURES, stream=None):
    """Device descriptors (int16 [n, 16]) and beliefs (float32 [G, 2, 13]) -> bf16 [n, F]."""
    import torch
    n = int(desc_dev.shape[0])
    x = torch.empty((n, in_features), dtype=torch.bfloat16, device=desc_dev.device)
    st = stream if stream is not None else torch.cuda.current_stream(desc_dev.device)
    N.check(_lib().cfr_features(ctypes.c_void_p(desc_dev.data_ptr()),
                                ctypes.c_void_p(beliefs_dev.data_ptr()), n, in_features,
                                ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
    return x


def probs_to_pairs(logits, desc_dev, qoff_dev, n_q, stream=None):
    import torch
    probs = torch.zeros(n_q, dtype=torch.float32, device=logits.device)
    st = stream if stream is not None else torch.cuda.current_stream(logits.device)
    N.check(_lib().cfr_probs_to_pairs(ctypes.c_void_p(logits.data_ptr()),
                                      ctypes.c_void_p(desc_dev.data_ptr()),
                                      ctypes.c_void_p(qoff_dev.data_ptr()), int(desc_dev.shape[0]),
                                      int(logits.shape[1]), ctypes.c_void_p(probs.data_ptr()),
                                      ctypes.c_void_p(st.cuda_stream)))
    return probs


def warm_start(solver: BatchSolver, net: WarmStartNet, game_list, weight: float,
               fallback: bool = True) -> dict:
    """One zero-start iteration, then R0 = weight * m * p from the network (all on the GPU).
    With ``fallback``, keep zero-start CFR where the warm strategy is more exploitable than
    the first uniform one. Returns timings and exploitabilities of both starts."""
    import torch
    t0 = time.perf_counter()
    desc, bel, qoff = descriptors(game_list)
    dev = solver.device
    desc_d = torch.from_numpy(desc).to(dev)
    bel_d = torch.from_numpy(bel).to(dev)
    qoff_d = torch.from_numpy(qoff).to(dev)
    solver.iterate(1)
    base = solver.exploitability()["expl"] if fallback else None
    x = features(desc_d, bel_d, net.shape[0], solver.stream)
    logits = net.forward(x)
    probs = probs_to_pairs(logits, desc_d, qoff_d, solver.n_q, solver.stream)
    if fallback:
        T, R, S = solver.get_state()
    N.check(_lib().cfr_warm_start(solver._h, ctypes.c_void_p(probs.data_ptr()), solver.n_q,
                                  float(weight)))
    out = {"seconds": 0.0, "fallback_games": 0}
    if fallback:
        solver.iterate(1)
        warm = solver.exploitability()["expl"]
        out["expl_zero_start"] = base
        out["expl_warm_start"] = warm
        bad = warm > base
        if bad.all():
            solver.set_state(T, R, S)
            out["fallback_games"] = int(len(bad))
        elif bad.any():
            # per-game fallback: restore those games' pairs to the zero-start state
            T2, R2, S2 = solver.get_state()
            for g in np.flatnonzero(bad):
                a, b = solver.pair_offsets[g], solver.pair_offsets[g + 1]
                R2[a:b], S2[a:b] = R[a:b], S[a:b]
            solver.set_state(T2, R2, S2)
            out["fallback_games"] = int(bad.sum())
    torch.cuda.synchronize()
    out["seconds"] = time.perf_counter() - t0
    return out
