"""Host-side checks of the C ABI (no GPU): the library loads and exports every
entry point the header declares, validation reports the documented error
codes, and the host flattener emits the oracle's canonical layout bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import games
from oracle.layout import canonical_layout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2408_14778_amd import _native
    return _native.load()


def test_every_declared_symbol_is_exported():
    header = open(os.path.join(ROOT, "include", "cfr.h")).read()
    names = set(re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(cfr_\w+)\s*\(", header,
                           re.M))
    assert len(names) >= 25
    lib = _lib()
    from paper_2408_14778_amd import _native
    for n in sorted(names):
        assert hasattr(lib, n), n
        assert n in _native.SIGNATURES, f"{n} has no binding"


def test_default_launch_shape():
    from paper_2408_14778_amd.solver import default_launch_shape
    sh = default_launch_shape()
    for name, allowed in (("up_threads", {64, 128, 256, 512}), ("up_members", {1, 2}),
                          ("reach_threads", set(range(64, 1025, 64))), ("reach_nodes", {1, 2, 4})):
        assert set(getattr(sh, name)) <= allowed, name


def test_warmstart_symbols_are_exported():
    header = open(os.path.join(ROOT, "include", "cfr_warmstart.h")).read()
    names = set(re.findall(r"^\s*(?:int|int64_t)\s+(cfr_\w+)\s*\(", header, re.M))
    assert len(names) >= 11
    lib = _lib()
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_plan_sizes():
    from paper_2408_14778_amd import plan
    p = plan(games.kuhn_like(3, "joint"))
    assert (p["n_nodes"], p["n_terminals"], p["n_infosets"], p["n_q"], p["depth"]) == (55, 30, 12, 24, 4)
    assert p["level_pure"] == 1 and p["workspace_bytes"] > 0
    p = plan(games.leduc_like(6, 2, deal="joint"))
    assert (p["n_nodes"], p["n_terminals"], p["n_infosets"], p["n_q"]) == (100981, 59928, 4032, 9408)


def _copy(g):
    import copy
    return copy.deepcopy(g)


@pytest.mark.parametrize("mutate,code", [
    (lambda g: g.parent.__setitem__(0, 3), "CFR_ENOTTREE"),                 # two roots / cycle
    (lambda g: g.parent.__setitem__(5, 5), "CFR_ENOTTREE"),                 # self parent
    (lambda g: g.node_action.__setitem__(2, 1), "CFR_EACTION"),              # duplicate action
    (lambda g: g.node_action.__setitem__(2, 7), "CFR_EACTION"),              # out of range
    (lambda g: g.chance_prob.__setitem__(0, 0.5), "CFR_ECHANCE"),            # sum != 1
    (lambda g: g.chance_prob.__setitem__(0, -0.1), "CFR_ECHANCE"),
    (lambda g: setattr(g, "payoff_u2", g.payoff_u2 + 1.0), "CFR_EZEROSUM"),
    (lambda g: g.infoset_player.__setitem__(1, 5), "CFR_EINVAL"),
])
def test_validation_error_codes(mutate, code):
    from paper_2408_14778_amd import CfrError, plan
    g = _copy(games.kuhn_like(3, "joint"))
    mutate(g)
    with pytest.raises(CfrError) as e:
        plan(g)
    assert str(e.value).startswith(code)


def test_config_layout_and_discount_validation():
    """cfr_config stays 32 bytes; the discounted variant takes finite exponents in [-64, 64]
    and the default averaging only (its gamma sets the weights)."""
    import ctypes

    from paper_2408_14778_amd import CfrError, plan
    from paper_2408_14778_amd import _native as N
    assert ctypes.sizeof(N.CfrConfig) == 32
    assert N.CfrConfig.dcfr_alpha.offset == 12 and N.CfrConfig.reserved.offset == 24
    g = games.kuhn_like(3, "joint")
    assert plan(g, "dcfr")["n_q"] == 24
    assert plan(g, "dcfr", dcfr=(1.0, 1.0, 1.0))["n_q"] == 24
    for bad in [(float("nan"), 0.0, 2.0), (1.5, float("inf"), 2.0), (1.5, 0.0, 65.0)]:
        with pytest.raises(CfrError, match="CFR_EINVAL"):
            plan(g, "dcfr", dcfr=bad)
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        plan(g, "dcfr", averaging="linear")
    with pytest.raises(ValueError):
        plan(g, "cfr+", dcfr=(1.0, 1.0, 1.0))
    assert plan(g, "cfr+", schedule="alternating")["n_q"] == 24


def test_unknown_flag_bits_rejected():
    import ctypes

    from paper_2408_14778_amd import _native as N
    from paper_2408_14778_amd.solver import GameArgs, make_config
    lib = N.load()
    args = GameArgs(games.kuhn_like(3, "joint"))
    cfg = make_config("cfr+")
    cfg.flags |= 64
    info = N.CfrPlanInfo()
    assert lib.cfr_plan(ctypes.byref(args.struct), ctypes.byref(cfg), ctypes.byref(info)) != 0


def test_fp64_plan_and_flag_validation():
    """CFR_FLAG_FP64: the node engine with double-precision state (a larger workspace than the
    FP32 node engine's); not with subtree packs, nor for a batch."""
    import ctypes

    from paper_2408_14778_amd import CfrError, plan
    from paper_2408_14778_amd import _native as N
    from paper_2408_14778_amd.solver import GameArgs, make_config
    g = games.leduc_like(3, 2, deal="sequential")
    p64 = plan(g, "cfr+", precision="f64")
    p32 = plan(g, "cfr+", engine="node")
    assert p64["engine"] == 0 and plan(g, "cfr+")["engine"] == 1
    # per node 7 doubles instead of 7 floats, per pair 6 instead of 6 (R, S, r~, sigma, average,
    # two staging): at least 28 bytes per node more
    assert p64["workspace_bytes"] >= p32["workspace_bytes"] + 28 * p64["n_nodes"]
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        plan(g, "cfr+", engine="packs", precision="f64")
    with pytest.raises(ValueError):
        plan(g, "cfr+", precision="f16")
    lib = N.load()
    args = GameArgs(g)
    arr = (N.CfrGame * 1)(args.struct)
    cfg = make_config("cfr+", precision="f64")
    info = N.CfrPlanInfo()
    assert N.ERRORS[lib.cfr_plan_batch(arr, 1, ctypes.byref(cfg), ctypes.byref(info))] == "CFR_EINVAL"


def test_partition_plans():
    """cfr_plan_partitioned: one partition per nonempty level-cut subtree at window 1, one for the whole
    lower tree at an unbounded window; the device workspace shrinks with the window; invalid cut
    levels, windows and flags are refused."""
    from paper_2408_14778_amd import CfrError, plan, plan_partitioned
    from paper_2408_14778_amd.solver import host_layout
    g = games.leduc_like(3, 2, deal="sequential")
    D = plan(g)["depth"]
    lay = host_layout(g, ["level_offset", "node_player"])
    lo, player = lay["level_offset"], lay["node_player"]
    for cut in range(1, D):
        one = plan_partitioned(g, cut, 1)
        # every level-cut decision node opens a partition; terminal ones join the current one
        assert one["partitions"] == max(1, int((player[lo[cut]:lo[cut + 1]] >= 0).sum()))
        whole = plan_partitioned(g, cut, 1 << 40)
        assert whole["partitions"] == 1
        assert one["workspace_bytes"] <= whole["workspace_bytes"]
        assert one["host_bytes"] > 0 and one["n_nodes"] == g.n_nodes
    assert plan_partitioned(g, 3, 1)["workspace_bytes"] < plan(g, engine="node")["workspace_bytes"]
    for cut in (0, D, -1):
        with pytest.raises(CfrError, match="CFR_EINVAL"):
            plan_partitioned(g, cut, 100)
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        plan_partitioned(g, 2, 0)
    import ctypes

    from paper_2408_14778_amd import _native as N
    from paper_2408_14778_amd.solver import GameArgs, make_config
    lib = N.load()
    args = GameArgs(g)
    cfg = make_config("cfr+", engine="packs")
    info = N.CfrPlanInfo()
    assert N.ERRORS[lib.cfr_plan_partitioned(ctypes.byref(args.struct), ctypes.byref(cfg), 2, 100,
                                             ctypes.byref(info), None, None)] == "CFR_EINVAL"


def test_terminal_with_infoset_rejected():
    from paper_2408_14778_amd import CfrError, plan
    g = _copy(games.kuhn_like(3, "joint"))
    term = int(np.flatnonzero(g.node_infoset < 0)[0])
    g.node_infoset[term] = 0
    with pytest.raises(CfrError, match="CFR_ENOTTREE"):
        plan(g)


def test_non_level_pure_game_is_flagged():
    # one infoset whose two members sit at depths 1 and 2
    from paper_2408_14778_amd import plan
    b = games.GameBuilder("skew")
    root = b.node(-1, -1)
    b.decide(root, b.infoset_id("c", 0, 2, [0.5, 0.5]))
    x = b.node(root, 0)
    y = b.node(root, 1)
    hp = b.infoset_id("p1", 1, 2)
    b.decide(x, hp)
    b.decide(y, b.infoset_id("c2", 0, 1, [1.0]))
    z = b.node(y, 0)
    b.decide(z, hp)
    for v in (x, z):
        for a in range(2):
            b.terminal(b.node(v, a), float(a))
    p = plan(b.build())
    assert p["level_pure"] == 0


LAYOUT_GAMES = [
    lambda: games.kuhn_like(3, "joint"),
    lambda: games.kuhn_like(3, "sequential").permuted(4),
    lambda: games.leduc_like(3, 2, deal="sequential"),
    lambda: games.leduc_like(6, 2, deal="joint"),
    lambda: games.leduc_like(6, 2, deal="joint").permuted(9),
    lambda: games.random_game(11, deal="sequential", depth=5),
    lambda: games.random_game(12, deal="none", depth=6),
    lambda: games.rock_paper_scissors(),
    lambda: games.subgame(103),
]


@pytest.mark.parametrize("maker", LAYOUT_GAMES)
def test_host_layout_bit_exact(maker):
    from paper_2408_14778_amd import host_layout
    g = maker()
    a = host_layout(g)
    b = canonical_layout(g)
    for k, v in a.items():
        assert v.dtype == b[k].dtype, k
        assert np.array_equal(v, b[k]), k


def test_host_layout_bit_exact_large(large_game):
    from paper_2408_14778_amd import host_layout
    a = host_layout(large_game)
    b = canonical_layout(large_game)
    for k, v in a.items():
        assert np.array_equal(v, b[k]), k


def test_single_node_game():
    from paper_2408_14778_amd import host_layout, plan
    g = games.Game("single", np.array([-1], np.int32), np.array([-1], np.int32),
                   np.array([-1], np.int32), np.zeros(0, np.int8), np.zeros(0, np.int32),
                   np.zeros(0), np.array([0.25]))
    p = plan(g)
    assert p["n_nodes"] == 1 and p["depth"] == 0 and p["n_q"] == 0
    lay = host_layout(g)
    assert lay["level_offset"].tolist() == [0, 1] and lay["payoff"].tolist() == [0.25]


def test_nplayer_plan_validation():
    """cfr_plan_n (no device needed): a general-sum game plans on the node engine with n value
    columns and n + 1 reach planes (a larger workspace than the same tree's two-player plan);
    the player count, the payoff pointer and the subtree-pack flag are checked (the alternating
    schedule is accepted); the two-player call refuses a third player."""
    import ctypes

    import numpy as np

    from paper_2408_14778_amd import _native as N
    from paper_2408_14778_amd.solver import GameArgs, _ptr, make_config

    EINVAL = -1  # CFR_EINVAL
    lib = N.load()
    g = games.kuhn3()
    args = GameArgs(g)
    pay = np.ascontiguousarray(g.payoff)
    pp = _ptr(pay, ctypes.c_double)

    def plan_n(n, payoff=pp, cfg=None):
        info = N.CfrPlanInfo()
        rc = lib.cfr_plan_n(ctypes.byref(args.struct), n, payoff,
                            None if cfg is None else ctypes.byref(cfg), ctypes.byref(info))
        return rc, info

    rc, info = plan_n(3)
    assert rc == 0 and info.engine == 0 and info.n_nodes == 617 and info.n_q == 96
    # the same tree as a two-player game (players renamed 1, 2) needs fewer bytes
    g2 = games.kuhn3()
    g2.infoset_player[g2.infoset_player == 3] = 2
    a2 = GameArgs(g2)
    i2 = N.CfrPlanInfo()
    cfg2 = make_config("vanilla", engine="node")
    assert lib.cfr_plan(ctypes.byref(a2.struct), ctypes.byref(cfg2), ctypes.byref(i2)) == 0
    assert info.workspace_bytes > i2.workspace_bytes
    for bad in (1, 9):
        assert plan_n(bad)[0] == EINVAL
    assert plan_n(2)[0] == EINVAL  # an infoset of player 3
    assert plan_n(3, payoff=None)[0] == EINVAL
    assert plan_n(3, cfg=make_config("cfr+", engine="packs"))[0] == EINVAL
    assert plan_n(3, cfg=make_config("cfr+", engine="node", schedule="alternating"))[0] == 0
    info = N.CfrPlanInfo()
    assert lib.cfr_plan(ctypes.byref(args.struct), None, ctypes.byref(info)) == EINVAL


def test_nplayer_plan_edges():
    """cfr_plan_n at the edges: eight players (the most) plan, the same game as seven is refused
    (an infoset of player 8), a silent player (no infosets) is accepted, and a game of one
    terminal node plans with no infosets and depth 0."""
    import ctypes

    import numpy as np

    from paper_2408_14778_amd import _native as N
    from paper_2408_14778_amd.solver import GameArgs, _ptr

    lib = N.load()

    def plan_n(g, n):
        args = GameArgs(g)
        pay = np.ascontiguousarray(g.payoff)
        info = N.CfrPlanInfo()
        rc = lib.cfr_plan_n(ctypes.byref(args.struct), n, _ptr(pay, ctypes.c_double), None,
                            ctypes.byref(info))
        return rc, info

    g8 = games.random_game_n(seed=26, n_players=8, n_types=2, depth=6, max_actions=2,
                             p_terminal=0.15, p_chance=0.1)
    rc, info = plan_n(g8, 8)
    assert rc == 0 and info.engine == 0 and info.n_nodes == 9729
    assert plan_n(g8, 7)[0] == -1  # CFR_EINVAL
    rc, info = plan_n(games.with_silent_players(games.kuhn_like(3, "joint"), 6, seed=1), 8)
    assert rc == 0 and info.n_nodes == 55
    b = games.GameBuilder("single3")
    b.terminal_vec(b.node(-1, -1), [0.25, -0.5, 1.0])
    rc, info = plan_n(b.build(players=3), 3)
    assert rc == 0 and info.n_nodes == 1 and info.n_infosets == 0 and info.depth == 0
