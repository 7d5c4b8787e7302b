"""ctypes binding of the C ABI in include/cfr.h: argument marshalling only.

Every step of the computation runs in the gfx950 library; if the library is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcfr_mi355x.so")

CFR_OK = 0
ERRORS = {
    -1: "CFR_EINVAL", -2: "CFR_ENOTTREE", -3: "CFR_EACTION", -4: "CFR_ECHANCE",
    -5: "CFR_EZEROSUM", -6: "CFR_ELEVEL", -7: "CFR_ENOMEM", -8: "CFR_ESTATE", -9: "CFR_EHIP",
}
CFR_VANILLA, CFR_PLUS, CFR_DCFR = 0, 1, 2
CFR_AVG_DEFAULT, CFR_AVG_UNIFORM, CFR_AVG_LINEAR = -1, 0, 1
CFR_FLAG_NO_GRAPH = 1
CFR_FLAG_NODE_ENGINE = 2
CFR_FLAG_ALTERNATING = 4
CFR_FLAG_KEEP_NODE_VALUES = 8
CFR_FLAG_SUBTREE_PACKS = 16
CFR_FLAG_FP64 = 32

_i32p = ctypes.POINTER(ctypes.c_int32)
_i8p = ctypes.POINTER(ctypes.c_int8)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)


class CfrGame(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64),
        ("parent", _i32p),
        ("node_infoset", _i32p),
        ("node_action", _i32p),
        ("n_infosets", ctypes.c_int32),
        ("infoset_player", _i8p),
        ("infoset_num_actions", _i32p),
        ("chance_prob", _f64p),
        ("payoff_u1", _f64p),
        ("payoff_u2", _f64p),
    ]


class CfrConfig(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("averaging", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("dcfr_alpha", ctypes.c_float),
        ("dcfr_beta", ctypes.c_float),
        ("dcfr_gamma", ctypes.c_float),
        ("reserved", ctypes.c_int32 * 2),
    ]


class CfrPlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64),
        ("n_terminals", ctypes.c_int64),
        ("n_infosets", ctypes.c_int64),
        ("n_q", ctypes.c_int64),
        ("n_chance_infosets", ctypes.c_int64),
        ("n_chance_q", ctypes.c_int64),
        ("max_actions", ctypes.c_int32),
        ("depth", ctypes.c_int32),
        ("level_pure", ctypes.c_int32),
        ("engine", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_int64),
    ]


class CfrLaunchShape(ctypes.Structure):
    """cfr_launch_shape: per log2 bucket of work items (32 buckets)."""
    _fields_ = [("up_threads", ctypes.c_int32 * 32), ("up_members", ctypes.c_int32 * 32),
                ("reach_threads", ctypes.c_int32 * 32), ("reach_nodes", ctypes.c_int32 * 32)]


# name -> (restype, argtypes); exactly the entry points declared in include/cfr.h
SIGNATURES = {
    "cfr_plan": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.POINTER(CfrConfig),
                                ctypes.POINTER(CfrPlanInfo)]),
    "cfr_build": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.POINTER(CfrConfig),
                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "cfr_plan_n": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.c_int32, _f64p,
                                  ctypes.POINTER(CfrConfig), ctypes.POINTER(CfrPlanInfo)]),
    "cfr_build_n": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.c_int32, _f64p,
                                   ctypes.POINTER(CfrConfig), ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "cfr_get_node_values_n": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p, ctypes.c_int64]),
    "cfr_iterate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cfr_iterate_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p, _i64p,
                                         ctypes.c_int32]),
    "cfr_kernel_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "cfr_iterate_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p, _i32p, _i32p,
                                           _i64p, ctypes.c_int32, _i32p]),
    "cfr_default_launch_shape": (None, [ctypes.POINTER(CfrLaunchShape)]),
    "cfr_set_launch_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CfrLaunchShape)]),
    "cfr_average_strategy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_int]),
    "cfr_current_strategy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_int]),
    "cfr_average_strategy_f64": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_int]),
    "cfr_current_strategy_f64": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_int]),
    "cfr_exploitability": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p]),
    "cfr_get_state": (ctypes.c_int, [ctypes.c_void_p, _i64p, _f32p, _f32p, ctypes.c_int64]),
    "cfr_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _f32p, _f32p,
                                     ctypes.c_int64]),
    "cfr_get_state_f64": (ctypes.c_int, [ctypes.c_void_p, _i64p, _f64p, _f64p, ctypes.c_int64]),
    "cfr_set_state_f64": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _f64p, _f64p,
                                         ctypes.c_int64]),
    "cfr_layout_bytes": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_char_p]),
    "cfr_get_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p,
                                      ctypes.c_int64]),
    "cfr_get_node_values": (ctypes.c_int, [ctypes.c_void_p, _f32p, _f32p, ctypes.c_int64]),
    "cfr_get_node_values_f64": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p, ctypes.c_int64]),
    "cfr_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "cfr_host_layout_create": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.c_uint32,
                                              ctypes.POINTER(ctypes.c_void_p)]),
    "cfr_host_layout_bytes": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_char_p]),
    "cfr_host_layout_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p,
                                           ctypes.c_int64]),
    "cfr_host_layout_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "cfr_host_layout_create_batch": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.c_int32,
                                                    ctypes.c_uint32,
                                                    ctypes.POINTER(ctypes.c_void_p)]),
    "cfr_plan_batch": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.c_int32,
                                      ctypes.POINTER(CfrConfig), ctypes.POINTER(CfrPlanInfo)]),
    "cfr_build_batch": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.c_int32,
                                       ctypes.POINTER(CfrConfig), ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "cfr_exploitability_batch": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p, ctypes.c_int32]),
    "cfr_plan_partitioned": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.POINTER(CfrConfig),
                                            ctypes.c_int32, ctypes.c_int64,
                                            ctypes.POINTER(CfrPlanInfo), _i32p, _i64p]),
    "cfr_build_partitioned": (ctypes.c_int, [ctypes.POINTER(CfrGame), ctypes.POINTER(CfrConfig),
                                             ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p,
                                             ctypes.POINTER(ctypes.c_void_p)]),
    "cfr_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load the library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_2408_14778_amd.build.build() "
                "(hipcc, gfx950). There is no fallback path.")
        # torch's HIP runtime first: the library then binds to that same runtime (both carry
        # the soname libamdhip64.so.7) instead of loading a second one that the device memory
        # torch allocates is foreign to
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class CfrError(RuntimeError):
    def __init__(self, code: int, message: str):
        self.code = code
        super().__init__(f"{ERRORS.get(code, code)}: {message}")


def check(code: int) -> None:
    if code != CFR_OK:
        msg = load().cfr_last_error()
        raise CfrError(code, msg.decode() if msg else "")
