"""Python face of the library: a CFR solver over one game on one GPU.

PyTorch supplies only the workspace (a uint8 device tensor) and the stream;
every step of the computation runs in the gfx950 library behind the C ABI.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native as N

VARIANTS = {"vanilla": N.CFR_VANILLA, "cfr+": N.CFR_PLUS, "dcfr": N.CFR_DCFR}
# discounted CFR's (alpha, beta, gamma) unless the caller gives others
DCFR_DEFAULT = (1.5, 0.0, 2.0)
AVERAGING = {None: N.CFR_AVG_DEFAULT, "uniform": N.CFR_AVG_UNIFORM, "linear": N.CFR_AVG_LINEAR}

LAYOUT_DTYPES = {
    "level_offset": np.int32, "node_id": np.int32, "parent": np.int32, "child_begin": np.int32,
    "node_player": np.int8, "node_infoset": np.int32, "node_edge": np.int32,
    "infoset_id": np.int32, "infoset_player": np.int8, "q_offset": np.int32,
    "chance_id": np.int32, "cq_offset": np.int32, "member_offset": np.int32,
    "members": np.int32, "chance_prob": np.float32, "payoff": np.float32, "q_input": np.int32,
}
# per-solver launch facts exported by the same call (not part of the canonical layout)
SOLVER_LAYOUT_DTYPES = {"reach_launch": np.int32}


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class GameArgs:
    """Holds contiguous copies of a game's arrays and the ctypes struct pointing at them."""

    def __init__(self, game):
        self.parent = np.ascontiguousarray(game.parent, dtype=np.int32)
        self.node_infoset = np.ascontiguousarray(game.node_infoset, dtype=np.int32)
        self.node_action = np.ascontiguousarray(game.node_action, dtype=np.int32)
        self.infoset_player = np.ascontiguousarray(game.infoset_player, dtype=np.int8)
        self.infoset_num_actions = np.ascontiguousarray(game.infoset_num_actions, dtype=np.int32)
        self.chance_prob = np.ascontiguousarray(game.chance_prob, dtype=np.float64)
        if self.chance_prob.size == 0:
            self.chance_prob = np.zeros(1, dtype=np.float64)
        self.payoff_u1 = np.ascontiguousarray(game.payoff_u1, dtype=np.float64)
        self.payoff_u2 = (None if game.payoff_u2 is None
                          else np.ascontiguousarray(game.payoff_u2, dtype=np.float64))
        self.struct = N.CfrGame(
            n_nodes=self.parent.shape[0],
            parent=_ptr(self.parent, ctypes.c_int32),
            node_infoset=_ptr(self.node_infoset, ctypes.c_int32),
            node_action=_ptr(self.node_action, ctypes.c_int32),
            n_infosets=self.infoset_player.shape[0],
            infoset_player=_ptr(self.infoset_player, ctypes.c_int8),
            infoset_num_actions=_ptr(self.infoset_num_actions, ctypes.c_int32),
            chance_prob=_ptr(self.chance_prob, ctypes.c_double),
            payoff_u1=_ptr(self.payoff_u1, ctypes.c_double),
            payoff_u2=(None if self.payoff_u2 is None else _ptr(self.payoff_u2, ctypes.c_double)),
        )


def make_config(variant: str = "vanilla", averaging=None, graph: bool = True,
                engine: str = "auto", dcfr=None, schedule: str = "simultaneous",
                keep_node_values: bool = False, precision: str = "f32") -> N.CfrConfig:
    if variant not in VARIANTS:
        raise ValueError(f"variant must be one of {list(VARIANTS)}")
    if engine not in ("auto", "packs", "node"):
        raise ValueError("engine must be 'auto' (the public-block engine where it applies), "
                         "'packs' (the same with subtree packs) or 'node'")
    cfg = N.CfrConfig()
    cfg.variant = VARIANTS[variant]
    cfg.averaging = AVERAGING[averaging]
    if dcfr is not None and variant != "dcfr":
        raise ValueError("dcfr exponents apply to variant 'dcfr' only")
    cfg.dcfr_alpha, cfg.dcfr_beta, cfg.dcfr_gamma = (dcfr if dcfr is not None else DCFR_DEFAULT)
    if schedule not in ("simultaneous", "alternating"):
        raise ValueError("schedule must be 'simultaneous' or 'alternating'")
    if precision not in ("f32", "f64"):
        raise ValueError("precision must be 'f32' or 'f64'")
    cfg.flags = ((0 if graph else N.CFR_FLAG_NO_GRAPH) |
                 (N.CFR_FLAG_FP64 if precision == "f64" else 0) |
                 (N.CFR_FLAG_NODE_ENGINE if engine == "node" else 0) |
                 (N.CFR_FLAG_SUBTREE_PACKS if engine == "packs" else 0) |
                 (N.CFR_FLAG_ALTERNATING if schedule == "alternating" else 0) |
                 (N.CFR_FLAG_KEEP_NODE_VALUES if keep_node_values else 0))
    return cfg


def plan(game, variant: str = "vanilla", averaging=None, engine: str = "auto", dcfr=None,
         schedule: str = "simultaneous", precision: str = "f32") -> dict:
    lib = N.load()
    args = GameArgs(game)
    cfg = make_config(variant, averaging, engine=engine, dcfr=dcfr, schedule=schedule,
                      precision=precision)
    info = N.CfrPlanInfo()
    N.check(lib.cfr_plan(ctypes.byref(args.struct), ctypes.byref(cfg), ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in N.CfrPlanInfo._fields_ if f != "reserved"}


PLAN_DTYPES = {
    "x_canon_of": np.int32, "x_parent": np.int32, "x_edge": np.int32, "x_meta": np.int8,
    "x_child_begin": np.int32, "x_child_stride": np.int32, "x_child_list": np.int32,
    "x_infoset_canon": np.int32, "x_q_offset": np.int32, "x_member_offset": np.int32,
    "x_members": np.int32, "x_h_level_offset": np.int32, "x_chance_nodes": np.int32,
    "x_c_level_offset": np.int32, "x_q_input": np.int32, "x_up_end": np.int32,
    "x_h_up_end": np.int32, "x_c_up_end": np.int32, "x_packs": np.int32,
    "x_pack_blob": np.int32, "x_tier_offset": np.int32,
}
# fields of one subtree pack in x_packs (int32 each; the per-level ranges have 9 entries)
PACK_LEVELS = 8
PACK_FIELDS = (["tier", "level0", "nlv", "n_dec", "n_mem", "n_ch", "n_root", "n_inf", "n_pairs",
                "n_kid", "off_root", "off_mem", "off_inf", "off_ch", "off_kid", "off_node"] +
               [f"{name}{i}" for name in ("mlo", "clo") for i in range(PACK_LEVELS + 1)])


def packs(lay: dict) -> list:
    """The subtree packs of a host layout (x_packs) as dicts; mlo and clo as lists."""
    raw = lay["x_packs"].reshape(-1, len(PACK_FIELDS))
    out = []
    for row in raw:
        pk = {name: int(v) for name, v in zip(PACK_FIELDS[:16], row[:16])}
        for j, name in enumerate(("mlo", "clo")):
            pk[name] = [int(v) for v in row[16 + j * 9:16 + (j + 1) * 9]]
        out.append(pk)
    return out


def host_layout(game, names=None, packs: bool = False) -> dict:
    """The canonical layout flattened on the host by the library (no GPU needed); the plan
    arrays with subtree packs if ``packs``."""
    lib = N.load()
    args = GameArgs(game)
    h = ctypes.c_void_p()
    N.check(lib.cfr_host_layout_create(ctypes.byref(args.struct),
                                       N.CFR_FLAG_SUBTREE_PACKS if packs else 0, ctypes.byref(h)))
    return _read_host_layout(lib, h, names or LAYOUT_DTYPES)


def host_batch_layout(game_list, names, packs: bool = False) -> dict:
    """The forest plan of a batch, built on the host by the library (plan arrays only)."""
    lib = N.load()
    args = [GameArgs(g) for g in game_list]
    arr = (N.CfrGame * len(args))(*[a.struct for a in args])
    h = ctypes.c_void_p()
    N.check(lib.cfr_host_layout_create_batch(arr, len(args),
                                             N.CFR_FLAG_SUBTREE_PACKS if packs else 0,
                                             ctypes.byref(h)))
    return _read_host_layout(lib, h, names)


def _read_host_layout(lib, h, names) -> dict:
    try:
        out = {}
        for name in names:
            nbytes = lib.cfr_host_layout_bytes(h, name.encode())
            if nbytes < 0:
                raise KeyError(name)
            dt = np.dtype(LAYOUT_DTYPES.get(name) or PLAN_DTYPES.get(name) or np.int32)
            arr = np.empty(nbytes // dt.itemsize, dtype=dt)
            N.check(lib.cfr_host_layout_get(h, name.encode(), arr.ctypes.data_as(ctypes.c_void_p),
                                            nbytes))
            out[name] = arr
        return out
    finally:
        lib.cfr_host_layout_destroy(h)


def default_launch_shape(lib=None) -> "N.CfrLaunchShape":
    """The library's default launch shapes (a cfr_launch_shape)."""
    sh = N.CfrLaunchShape()
    (lib or N.load()).cfr_default_launch_shape(ctypes.byref(sh))
    return sh


class Solver:
    """CFR (vanilla, CFR+ or discounted CFR) over one game, resident on one GPU. ``dcfr``:
    (alpha, beta, gamma) of variant 'dcfr' (default (1.5, 0, 2)); ``schedule``: 'simultaneous'
    (both players' updates in one pass) or 'alternating' (player 1's pass, then player 2's);
    ``keep_node_values``: the subtree-pack launch also stores every node's value and reach, so
    that node_values() can read them (off by default: the packs keep them on chip);
    ``precision``: 'f32' (default) or 'f64' (the node engine in double precision: strategies,
    state and node values come back as float64)."""

    def __init__(self, game, variant: str = "vanilla", averaging=None, device: str = "cuda",
                 graph: bool = True, stream=None, engine: str = "auto", tuned: bool = True,
                 dcfr=None, schedule: str = "simultaneous", keep_node_values: bool = False,
                 precision: str = "f32"):
        import torch

        self._lib = N.load()
        self.variant = variant
        self.precision = precision
        args = GameArgs(game)
        cfg = make_config(variant, averaging, graph, engine, dcfr, schedule, keep_node_values,
                          precision)
        info = N.CfrPlanInfo()
        N.check(self._lib.cfr_plan(ctypes.byref(args.struct), ctypes.byref(cfg),
                                   ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in N.CfrPlanInfo._fields_ if f != "reserved"}
        self.device = torch.device(device)
        self.workspace = torch.empty(int(info.workspace_bytes), dtype=torch.uint8,
                                     device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        N.check(self._lib.cfr_build(ctypes.byref(args.struct), ctypes.byref(cfg),
                                    ctypes.c_void_p(self.workspace.data_ptr()),
                                    ctypes.c_size_t(int(info.workspace_bytes)),
                                    ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(handle)))
        self._h = handle
        self.n_q = int(info.n_q)
        self.n_nodes = int(info.n_nodes)
        self._f64 = precision == "f64"
        self._rdt = np.float64 if self._f64 else np.float32
        self._sfx = "_f64" if self._f64 else ""
        if tuned and not self._f64:
            from . import autotune
            autotune.apply(self, autotune.load())

    # -- iteration ------------------------------------------------------------------
    def iterate(self, n: int = 1) -> None:
        N.check(self._lib.cfr_iterate(self._h, int(n)))

    def iterate_timed(self, n: int) -> dict:
        """n iterations with hipEvents around every kernel launch: {kernel: (launches, ms)}."""
        kinds = 16
        ms = np.zeros(kinds, dtype=np.float64)
        cnt = np.zeros(kinds, dtype=np.int64)
        N.check(self._lib.cfr_iterate_timed(self._h, int(n), _ptr(ms, ctypes.c_double),
                                            _ptr(cnt, ctypes.c_int64), kinds))
        out = {}
        for k in range(kinds):
            name = self._lib.cfr_kernel_name(k).decode()
            if name and cnt[k]:
                out[name] = (int(cnt[k]), float(ms[k]))
        return out

    def iterate_profile(self, n: int) -> list:
        """n iterations; per launch of one iteration: kernel, level, work items, mean ms."""
        cap = 4096
        ms = np.zeros(cap, dtype=np.float64)
        kind = np.zeros(cap, dtype=np.int32)
        level = np.zeros(cap, dtype=np.int32)
        units = np.zeros(cap, dtype=np.int64)
        nl = ctypes.c_int32()
        N.check(self._lib.cfr_iterate_profile(self._h, int(n), _ptr(ms, ctypes.c_double),
                                              _ptr(kind, ctypes.c_int32), _ptr(level, ctypes.c_int32),
                                              _ptr(units, ctypes.c_int64), cap, ctypes.byref(nl)))
        return [{"kernel": self._lib.cfr_kernel_name(int(kind[i])).decode(), "level": int(level[i]),
                 "units": int(units[i]), "ms": float(ms[i]) / n} for i in range(min(nl.value, cap))]

    def set_launch_shape(self, up_threads=None, reach_threads=None, up_members=None,
                         reach_nodes=None) -> None:
        """Launch shapes per log2 bucket of work items: bottom-up threads per workgroup and
        members per thread, top-down threads per workgroup and nodes per thread (a scalar or
        a list of up to 32 buckets, the last entry repeated). Arguments left None keep the
        library default; all None restores every default."""
        if all(v is None for v in (up_threads, reach_threads, up_members, reach_nodes)):
            N.check(self._lib.cfr_set_launch_shape(self._h, None))
            return
        sh = default_launch_shape(self._lib)
        for name, val in (("up_threads", up_threads), ("up_members", up_members),
                          ("reach_threads", reach_threads), ("reach_nodes", reach_nodes)):
            if val is None:
                continue
            vals = [int(val)] * 32 if np.isscalar(val) else [int(v) for v in val]
            vals = (vals + [vals[-1]] * 32)[:32]
            getattr(sh, name)[:] = vals
        N.check(self._lib.cfr_set_launch_shape(self._h, ctypes.byref(sh)))

    def synchronize(self) -> None:
        self.stream.synchronize()

    # -- results --------------------------------------------------------------------
    def _call(self, name: str):
        return getattr(self._lib, name + self._sfx)

    def average_strategy(self) -> np.ndarray:
        out = np.empty(self.n_q, dtype=self._rdt)
        N.check(self._call("cfr_average_strategy")(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                                   self.n_q, 0))
        return out

    def current_strategy(self) -> np.ndarray:
        """sigma^(T+1): the strategy the next iteration plays (input pair order)."""
        out = np.empty(self.n_q, dtype=self._rdt)
        N.check(self._call("cfr_current_strategy")(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                                   self.n_q, 0))
        return out

    def average_strategy_device(self, out) -> None:
        """Write the average strategy into a device tensor of n_q elements (float32, or
        float64 for precision 'f64')."""
        assert out.dtype.itemsize == np.dtype(self._rdt).itemsize
        assert out.numel() == self.n_q and out.is_cuda
        N.check(self._call("cfr_average_strategy")(self._h, ctypes.c_void_p(out.data_ptr()),
                                                   self.n_q, 1))

    def exploitability(self) -> dict:
        expl = ctypes.c_double()
        br = (ctypes.c_double * 2)()
        N.check(self._lib.cfr_exploitability(self._h, ctypes.byref(expl), br))
        return {"expl": expl.value, "br1": br[0], "br2": br[1], "nash_conv": br[0] + br[1]}

    def _cty(self):
        return ctypes.c_double if self._f64 else ctypes.c_float

    def get_state(self):
        T = ctypes.c_int64()
        R = np.empty(self.n_q, dtype=self._rdt)
        S = np.empty(self.n_q, dtype=self._rdt)
        N.check(self._call("cfr_get_state")(self._h, ctypes.byref(T), _ptr(R, self._cty()),
                                            _ptr(S, self._cty()), self.n_q))
        return int(T.value), R, S

    def set_state(self, T: int, R, S) -> None:
        R = np.ascontiguousarray(R, dtype=self._rdt)
        S = np.ascontiguousarray(S, dtype=self._rdt)
        N.check(self._call("cfr_set_state")(self._h, int(T), _ptr(R, self._cty()),
                                            _ptr(S, self._cty()), R.shape[0]))

    def layout(self, name: str) -> np.ndarray:
        nbytes = self._lib.cfr_layout_bytes(self._h, name.encode())
        if nbytes < 0:
            raise KeyError(name)
        dt = np.dtype(LAYOUT_DTYPES.get(name) or SOLVER_LAYOUT_DTYPES[name])
        out = np.empty(nbytes // dt.itemsize, dtype=dt)
        N.check(self._lib.cfr_get_layout(self._h, name.encode(),
                                          out.ctypes.data_as(ctypes.c_void_p), nbytes))
        return out

    def node_values(self):
        """(u1[N], reach[N, 3]) of the last iteration, canonical node order."""
        u1 = np.empty(self.n_nodes, dtype=self._rdt)
        reach = np.empty((self.n_nodes, 3), dtype=self._rdt)
        N.check(self._call("cfr_get_node_values")(self._h, _ptr(u1, self._cty()),
                                                  _ptr(reach, self._cty()), self.n_nodes))
        return u1, reach

    def close(self) -> None:
        if getattr(self, "_h", None):
            N.check(self._lib.cfr_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NPlayerSolver(Solver):
    """CFR over a general-sum game of n rational players (``game.payoff``: one payoff column
    per player, Section 3.1) on the node engine, through cfr_plan_n / cfr_build_n: vanilla,
    CFR+ or discounted, every player's infosets updated in one pass (``schedule``
    'simultaneous') or a pass per player in seat order ('alternating'), precision 'f32' or 'f64'.
    State, strategies and iteration work as in Solver; exploitability() raises (it is defined
    for two-player zero-sum games), and node_values() returns every player's value column."""

    def __init__(self, game, variant: str = "vanilla", averaging=None, device: str = "cuda",
                 graph: bool = True, stream=None, dcfr=None, precision: str = "f32",
                 schedule: str = "simultaneous"):
        import torch

        if game.payoff is None:
            raise ValueError("a general-sum game needs game.payoff (n_nodes x n_players)")
        self._lib = N.load()
        self.variant = variant
        self.precision = precision
        args = GameArgs(game)
        self._payoff = np.ascontiguousarray(game.payoff, dtype=np.float64)
        self.n_players = int(self._payoff.shape[1])
        cfg = make_config(variant, averaging, graph, "node", dcfr, schedule, precision=precision)
        info = N.CfrPlanInfo()
        pay = _ptr(self._payoff, ctypes.c_double)
        N.check(self._lib.cfr_plan_n(ctypes.byref(args.struct), self.n_players, pay,
                                     ctypes.byref(cfg), ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in N.CfrPlanInfo._fields_ if f != "reserved"}
        self.device = torch.device(device)
        self.workspace = torch.empty(int(info.workspace_bytes), dtype=torch.uint8,
                                     device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        N.check(self._lib.cfr_build_n(ctypes.byref(args.struct), self.n_players, pay,
                                      ctypes.byref(cfg),
                                      ctypes.c_void_p(self.workspace.data_ptr()),
                                      ctypes.c_size_t(int(info.workspace_bytes)),
                                      ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(handle)))
        self._h = handle
        self.n_q = int(info.n_q)
        self.n_nodes = int(info.n_nodes)
        self._f64 = precision == "f64"
        self._rdt = np.float64 if self._f64 else np.float32
        self._sfx = "_f64" if self._f64 else ""

    def node_values(self):
        """(values[N, n], reach[N, n + 1]) of the last iteration in canonical node order, as
        float64: every player's expected payoff, and every player's reach then chance's."""
        values = np.empty((self.n_nodes, self.n_players), dtype=np.float64)
        reach = np.empty((self.n_nodes, self.n_players + 1), dtype=np.float64)
        N.check(self._lib.cfr_get_node_values_n(self._h, _ptr(values, ctypes.c_double),
                                                _ptr(reach, ctypes.c_double), self.n_nodes))
        return values, reach


class PartitionedSolver(Solver):
    """The subtree-partitioned, out-of-core iteration (cfr_build_partitioned): levels
    0 .. cut_level resident on the device, the subtrees below grouped into partitions of at most
    max_window_nodes nodes held in pinned host memory and streamed through one device window per
    iteration. Same update rules, schedules and precisions as Solver (node engine arithmetic);
    exploitability and node values are not available (the device never holds the whole tree):
    move the state into a Solver of the same game to evaluate it."""

    def __init__(self, game, variant: str = "vanilla", cut_level: int = 1,
                 max_window_nodes: int = 1 << 20, averaging=None, device: str = "cuda",
                 stream=None, dcfr=None, schedule: str = "simultaneous", precision: str = "f32"):
        import torch

        self._lib = N.load()
        self.variant = variant
        self.precision = precision
        args = GameArgs(game)
        cfg = make_config(variant, averaging, False, "node", dcfr, schedule, False, precision)
        info = N.CfrPlanInfo()
        parts = ctypes.c_int32()
        host_bytes = ctypes.c_int64()
        N.check(self._lib.cfr_plan_partitioned(ctypes.byref(args.struct), ctypes.byref(cfg),
                                               int(cut_level), int(max_window_nodes),
                                               ctypes.byref(info), ctypes.byref(parts),
                                               ctypes.byref(host_bytes)))
        self.info = {f: getattr(info, f) for f, _ in N.CfrPlanInfo._fields_ if f != "reserved"}
        self.n_partitions = int(parts.value)
        self.host_bytes = int(host_bytes.value)
        self.device = torch.device(device)
        self.workspace = torch.empty(int(info.workspace_bytes), dtype=torch.uint8,
                                     device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        N.check(self._lib.cfr_build_partitioned(ctypes.byref(args.struct), ctypes.byref(cfg),
                                                int(cut_level), int(max_window_nodes),
                                                ctypes.c_void_p(self.workspace.data_ptr()),
                                                ctypes.c_size_t(int(info.workspace_bytes)),
                                                ctypes.c_void_p(self.stream.cuda_stream),
                                                ctypes.byref(handle)))
        self._h = handle
        self.n_q = int(info.n_q)
        self.n_nodes = int(info.n_nodes)
        self._f64 = precision == "f64"
        self._rdt = np.float64 if self._f64 else np.float32
        self._sfx = "_f64" if self._f64 else ""


def plan_partitioned(game, cut_level: int, max_window_nodes: int, variant: str = "vanilla",
                     precision: str = "f32", schedule: str = "simultaneous") -> dict:
    """cfr_plan_partitioned: the sizes, the device workspace, the partition count and the
    pinned host bytes of a partitioned solver (no GPU needed)."""
    lib = N.load()
    args = GameArgs(game)
    cfg = make_config(variant, None, False, "node", None, schedule, False, precision)
    info = N.CfrPlanInfo()
    parts = ctypes.c_int32()
    host_bytes = ctypes.c_int64()
    N.check(lib.cfr_plan_partitioned(ctypes.byref(args.struct), ctypes.byref(cfg), int(cut_level),
                                     int(max_window_nodes), ctypes.byref(info),
                                     ctypes.byref(parts), ctypes.byref(host_bytes)))
    out = {f: getattr(info, f) for f, _ in N.CfrPlanInfo._fields_ if f != "reserved"}
    out["partitions"] = int(parts.value)
    out["host_bytes"] = int(host_bytes.value)
    return out


class BatchSolver(Solver):
    """Many independent games solved together (one forest, one graph replay per iteration).

    Pair vectors (state, strategies) concatenate the games' input pair orders, game 0 first;
    ``pair_offsets[g]`` is where game g's pairs start."""

    def __init__(self, game_list, variant: str = "cfr+", averaging=None, device: str = "cuda",
                 graph: bool = True, stream=None, tuned: bool = True, dcfr=None,
                 schedule: str = "simultaneous", engine: str = "auto"):
        import torch

        self._lib = N.load()
        self.variant = variant
        self._args = [GameArgs(g) for g in game_list]
        n = len(self._args)
        arr = (N.CfrGame * n)(*[a.struct for a in self._args])
        if engine not in ("auto", "packs"):
            raise ValueError("a batch runs on the public-block engine: 'auto' or 'packs'")
        cfg = make_config(variant, averaging, graph, engine=engine, dcfr=dcfr, schedule=schedule)
        info = N.CfrPlanInfo()
        N.check(self._lib.cfr_plan_batch(arr, n, ctypes.byref(cfg), ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in N.CfrPlanInfo._fields_ if f != "reserved"}
        self.device = torch.device(device)
        self.workspace = torch.empty(int(info.workspace_bytes), dtype=torch.uint8,
                                     device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        N.check(self._lib.cfr_build_batch(arr, n, ctypes.byref(cfg),
                                          ctypes.c_void_p(self.workspace.data_ptr()),
                                          ctypes.c_size_t(int(info.workspace_bytes)),
                                          ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(handle)))
        self._args = None
        self._h = handle
        self.precision = "f32"
        self._f64 = False
        self._rdt = np.float32
        self._sfx = ""
        self.n_games = n
        self.n_q = int(info.n_q)
        self.n_nodes = int(info.n_nodes)
        qs = [int(np.sum(g.infoset_num_actions[g.infoset_player != 0])) for g in game_list]
        self.pair_offsets = np.concatenate([[0], np.cumsum(qs)]).astype(np.int64)
        if tuned:
            from . import autotune
            autotune.apply(self, autotune.load())

    def exploitability(self) -> dict:
        expl = np.empty(self.n_games, dtype=np.float64)
        br = np.empty(2 * self.n_games, dtype=np.float64)
        N.check(self._lib.cfr_exploitability_batch(self._h, _ptr(expl, ctypes.c_double),
                                                   _ptr(br, ctypes.c_double), self.n_games))
        return {"expl": expl, "br1": br[0::2], "br2": br[1::2]}

    def split(self, vec):
        """Per-game slices of a concatenated pair vector."""
        return [vec[self.pair_offsets[g]:self.pair_offsets[g + 1]] for g in range(self.n_games)]
