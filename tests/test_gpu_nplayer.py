"""GPU parity of the general-sum path (cfr_build_n: the node engine with one value column per
rational player and n + 1 reach planes) against the n-player FP64 oracle (oracle/cfr_n.py).

Bounds are those of the two-player tests: one iteration from an identical seeded state within
1e-6 norm-wise in FP32 and 1e-12 in FP64 (max|gpu - oracle| / max|oracle|, for R', S', every
player's node values and every reach plane), the next strategy elementwise outside regret
matching's uniform-fallback discontinuity. After T iterations, where FP32 rounding decorrelates
the regret-matching switches, the FP64 path is held to 1e-9 on R and S and the FP32 path to
1e-3 on each player's expected payoff under the average strategy (payoff scale 1 to 2).
"""
import numpy as np
import pytest

import games
from oracle import cfr, cfr_n

pytestmark = pytest.mark.gpu


def _normal3():
    rng = np.random.default_rng(4)
    return games.normal_form_n(rng.integers(-64, 65, size=(3, 2, 4, 3)) / 64.0, name="nf3")


def _bimatrix():
    rng = np.random.default_rng(5)
    return games.normal_form_n(rng.integers(-64, 65, size=(4, 3, 2)) / 64.0, name="bimatrix")


def _normal8():
    rng = np.random.default_rng(8)
    return games.normal_form_n(rng.integers(-64, 65, size=(2,) * 8 + (8,)) / 64.0, name="nf8")


def _single_action():
    rng = np.random.default_rng(9)
    return games.normal_form_n(rng.integers(-64, 65, size=(1, 1, 3, 3)) / 64.0, name="nf_k1")


# eight players (the most), two private types each: a 256-way deal at the root and infosets of up
# to 128 members, every player owning infosets
RANDOM8 = dict(seed=26, n_players=8, n_types=2, depth=6, max_actions=2, p_terminal=0.15,
               p_chance=0.1)

GAMES = {
    "kuhn3": lambda: games.kuhn3(),
    "kuhn3_joint": lambda: games.kuhn3(deal="joint"),
    "rand3": lambda: games.random_game_n(3, 3),
    "rand4": lambda: games.random_game_n(7, 4, depth=5),
    "rand5": lambda: games.random_game_n(11, 5, depth=4, max_actions=4),
    "nf3": _normal3,
    "bimatrix": _bimatrix,
    "nf8": _normal8,
    "nf_k1": _single_action,
    "rand8": lambda: games.random_game_n(**RANDOM8),
    "rand3_t9": lambda: games.random_game_n(5, 3, n_types=9, depth=4),  # 81 members per infoset
    "silent3": lambda: games.with_silent_players(games.kuhn_like(3, "joint"), 1, seed=6),
    "silent8": lambda: games.with_silent_players(games.leduc_like(3, 2, deal="sequential"), 6,
                                                 seed=7),
}


def _rel(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(float(np.abs(ref).max()) if ref.size else 0.0, 1e-300)
    return float(np.abs(gpu - ref).max()) / scale if ref.size else 0.0


def _solver(g, variant, precision):
    from paper_2408_14778_amd import NPlayerSolver
    s = NPlayerSolver(g, variant, precision=precision)
    assert s.info["engine"] == 0 and s.n_players == g.n_players
    return s


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("name", sorted(GAMES))
def test_one_iteration_parity(name, variant, precision, tol):
    g = GAMES[name]()
    T, R, S = games.random_state(g, seed=len(name) + 2, nonnegative=(variant == "cfr+"))
    s = _solver(g, variant, precision)
    dt = np.float64 if precision == "f64" else np.float32
    s.set_state(T, R.astype(dt), S.astype(dt))
    s.iterate(1)
    T2, R2, S2 = s.get_state()
    sig2 = s.current_strategy()
    vals, reach = s.node_values()
    tree = cfr_n.TreeN(g)
    new, info = cfr_n.iterate(tree, cfr.State(T, [float(x) for x in R], [float(x) for x in S]),
                              variant, record=True)
    assert T2 == T + 1
    errs = {"R": _rel(R2, new.R), "S": _rel(S2, new.S)}
    nid = s.layout("node_id")
    ref_u = np.asarray([info["node_u"][v] for v in nid])
    for i in range(g.n_players):
        errs[f"u{i + 1}"] = _rel(vals[:, i], ref_u[:, i])
    dec = s.layout("node_player") >= 0
    ref_reach = np.asarray([info["node_reach"][v] for v in nid])
    for k in range(g.n_players + 1):
        errs[f"reach{k}"] = _rel(reach[dec, k], ref_reach[dec, k])
    print(name, variant, precision, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= tol, errs
    ref_sig = np.asarray(info["next_sigma"])
    scale = max(float(np.abs(new.R).max()), 1e-300)
    for h in tree.rational:
        o, k = tree.qoff[h], tree.nact[h]
        pos = sum(max(x, 0.0) for x in new.R[o:o + k])
        if 0.0 < pos < 1e3 * tol * scale:  # regret matching's uniform-fallback discontinuity
            continue
        np.testing.assert_allclose(sig2[o:o + k], ref_sig[o:o + k], rtol=0, atol=10 * tol)


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("name", ["kuhn3", "rand4", "rand5", "nf3", "rand8", "silent3"])
def test_alternating_one_iteration_parity(name, variant, precision, tol):
    """The alternating schedule: a pass per player in seat order, each under the strategies the
    earlier passes produced, against the oracle's n-pass iteration."""
    from paper_2408_14778_amd import NPlayerSolver
    g = GAMES[name]()
    T, R, S = games.random_state(g, seed=len(name) + 9, nonnegative=(variant == "cfr+"))
    s = NPlayerSolver(g, variant, precision=precision, schedule="alternating")
    dt = np.float64 if precision == "f64" else np.float32
    s.set_state(T, R.astype(dt), S.astype(dt))
    s.iterate(1)
    T2, R2, S2 = s.get_state()
    new, _ = cfr_n.iterate_alternating(
        cfr_n.TreeN(g), cfr.State(T, [float(x) for x in R], [float(x) for x in S]), variant)
    assert T2 == T + 1
    assert _rel(R2, new.R) <= tol and _rel(S2, new.S) <= tol, (_rel(R2, new.R), _rel(S2, new.S))


@pytest.mark.parametrize("name,variant,iters", [("kuhn3", "cfr+", 300), ("rand4", "vanilla", 200),
                                                ("nf3", "dcfr", 200)])
def test_fp64_after_T_iterations(name, variant, iters):
    g = GAMES[name]()
    s = _solver(g, variant, "f64")
    s.iterate(iters)
    T, R, S = s.get_state()
    ref = cfr_n.solve(cfr_n.TreeN(g), iters, variant)
    assert T == iters == ref.T
    assert _rel(R, ref.R) <= 1e-9 and _rel(S, ref.S) <= 1e-9


@pytest.mark.parametrize("name,variant,iters", [("kuhn3", "cfr+", 300), ("rand3", "cfr+", 300),
                                                ("nf3", "vanilla", 200)])
def test_fp32_expected_payoffs_after_T_iterations(name, variant, iters):
    g = GAMES[name]()
    s = _solver(g, variant, "f32")
    s.iterate(iters)
    tree = cfr_n.TreeN(g)
    got = cfr_n.expected_values(tree, [float(x) for x in s.average_strategy()])
    ref = cfr_n.expected_values(tree, cfr.average_strategy(tree, cfr_n.solve(tree, iters, variant).S))
    print(name, variant, got, ref, flush=True)
    assert np.abs(np.asarray(got) - np.asarray(ref)).max() <= 1e-3


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("name", ["rand8", "rand3_t9"])
def test_runs_are_bit_identical(name, precision):
    """No step of the general-sum path adds by atomics: two solvers of the same game from the
    same state agree bit for bit after T iterations."""
    g = GAMES[name]()
    T, R, S = games.random_state(g, seed=4, nonnegative=True)
    dt = np.float64 if precision == "f64" else np.float32
    runs = []
    for _ in range(2):
        s = _solver(g, "cfr+", precision)
        s.set_state(T, R.astype(dt), S.astype(dt))
        s.iterate(25)
        runs.append(s.get_state())
    assert runs[0][0] == runs[1][0] == T + 25
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])


def test_kuhn3_values_add_up_to_zero_on_the_gpu():
    g = GAMES["kuhn3"]()
    s = _solver(g, "cfr+", "f64")
    s.iterate(50)
    vals, _ = s.node_values()
    assert abs(vals[0].sum()) <= 1e-12  # the root (canonical node 0): a zero-sum game


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_single_terminal_game(precision):
    """A game of one terminal node: no infosets, depth 0; iterations only count, the root's value
    is its payoff vector and every reach plane is 1."""
    b = games.GameBuilder("single3")
    b.terminal_vec(b.node(-1, -1), [0.25, -0.5, 1.0])
    s = _solver(b.build(players=3), "cfr+", precision)
    s.iterate(3)
    T, R, S = s.get_state()
    assert T == 3 and R.size == 0 and S.size == 0
    vals, reach = s.node_values()
    assert vals.tolist() == [[0.25, -0.5, 1.0]] and reach.tolist() == [[1.0] * 4]


def test_non_finite_payoff_is_refused():
    """A payoff that is not finite at a terminal is refused before anything runs, in any column;
    the payoff rows of decision nodes are not read."""
    from dataclasses import replace

    from paper_2408_14778_amd import CfrError, NPlayerSolver
    g = GAMES["kuhn3"]()
    term = np.flatnonzero(g.node_infoset < 0)
    for col, bad in ((0, np.nan), (2, np.inf)):
        pay = g.payoff.copy()
        pay[term[5], col] = bad
        with pytest.raises(CfrError, match="CFR_EINVAL"):
            NPlayerSolver(replace(g, payoff=pay, payoff_u1=pay[:, 0].copy()), "cfr+")
    pay = g.payoff.copy()
    pay[np.flatnonzero(g.node_infoset >= 0)[3], 1] = np.nan
    s = NPlayerSolver(replace(g, payoff=pay), "cfr+")
    s.iterate(2)
    _, R, S = s.get_state()
    assert np.isfinite(R).all() and np.isfinite(S).all()
    ref = NPlayerSolver(g, "cfr+")
    ref.iterate(2)
    _, R0, S0 = ref.get_state()
    assert np.array_equal(R, R0) and np.array_equal(S, S0)


def test_two_player_calls_are_refused():
    from paper_2408_14778_amd import CfrError, Solver
    g = GAMES["kuhn3"]()
    s = _solver(g, "cfr+", "f32")
    s.iterate(2)
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        s.exploitability()
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        Solver.node_values(s)  # the two-player export
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        s.set_launch_shape(up_threads=128)
    # and a two-player zero-sum solver refuses the n-column export
    import ctypes

    from paper_2408_14778_amd import _native as N
    z = Solver(games.kuhn_like(3, "joint"), "cfr+", engine="node")
    buf = np.empty(2 * z.n_nodes, dtype=np.float64)
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        N.check(z._lib.cfr_get_node_values_n(z._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             None, z.n_nodes))


def _mean_members(g):
    """Members per rational infoset, rounded up: what picks the gather's workgroup (one
    wavefront up to 64, two up to 128, else four)."""
    rational = g.infoset_player[g.node_infoset[g.node_infoset >= 0]] > 0
    H = int((g.infoset_player > 0).sum())
    return -(-int(rational.sum()) // H)


def test_gather_workgroup_sizes_are_covered():
    assert _mean_members(GAMES["kuhn3"]()) <= 64
    assert 64 < _mean_members(GAMES["rand3_t9"]()) <= 128


_GATHER_CASES = [(t, v, p, s) for t in (40, 90) for v in ("vanilla", "cfr+")
                 for p in ("f32", "f64") for s in ("simultaneous", "alternating")] + \
                [(150, v, p, "simultaneous") for v in ("vanilla", "cfr+") for p in ("f32", "f64")]


@pytest.mark.parametrize("types,variant,precision,schedule", _GATHER_CASES)
def test_two_player_gather_path_parity(types, variant, precision, schedule):
    """A two-player zero-sum game whose infosets average 40, 90 or 150 members (the gather's
    workgroup of one, two or four wavefronts): the node engine stores the regret contributions
    and gathers them per infoset instead of adding them by atomics. One iteration against the
    two-player oracle, with both schedules (the alternating one gathers once per pass)."""
    from oracle.tree import Tree
    from paper_2408_14778_amd import Solver
    tol = 1e-6 if precision == "f32" else 1e-12
    g = games.random_game(47, n_types=(types, types), depth=4, deal="joint")
    assert _mean_members(g) == types
    T, R, S = games.random_state(g, seed=3, nonnegative=(variant == "cfr+"))
    s = Solver(g, variant, engine="node", precision=precision, schedule=schedule)
    dt = np.float64 if precision == "f64" else np.float32
    s.set_state(T, R.astype(dt), S.astype(dt))
    s.iterate(1)
    _, R2, S2 = s.get_state()
    step = cfr.iterate_alternating if schedule == "alternating" else cfr.iterate
    new, _ = step(Tree(g), cfr.State(T, [float(x) for x in R], [float(x) for x in S]), variant)
    assert _rel(R2, new.R) <= tol and _rel(S2, new.S) <= tol


@pytest.fixture(scope="module")
def bench_game():
    import bench
    return games.random_game_n(**bench.NPLAYER_GAME)


@pytest.mark.parametrize("precision,tol", [("f32", 1e-6), ("f64", 1e-12)])
def test_bench_game_one_iteration_full_size(bench_game, precision, tol):
    """The three-player game `bench.py --workload nplayer` times (2,127,169 nodes, a 1,728-way
    root, infosets of about 180 members: the wide-level kernels and the four-wavefront gather),
    CFR+ as timed, one iteration from a seeded state against the oracle over every pair and
    node."""
    g = bench_game
    T, R, S = games.random_state(g, seed=1, nonnegative=True)
    s = _solver(g, "cfr+", precision)
    dt = np.float64 if precision == "f64" else np.float32
    s.set_state(T, R.astype(dt), S.astype(dt))
    s.iterate(1)
    _, R2, S2 = s.get_state()
    vals, _ = s.node_values()
    tree = cfr_n.TreeN(g)
    new, info = cfr_n.iterate(tree, cfr.State(T, [float(x) for x in R], [float(x) for x in S]),
                              "cfr+", record=True)
    errs = {"R": _rel(R2, new.R), "S": _rel(S2, new.S)}
    nid = s.layout("node_id")
    ref_u = np.asarray([info["node_u"][v] for v in nid])
    for i in range(g.n_players):
        errs[f"u{i + 1}"] = _rel(vals[:, i], ref_u[:, i])
    print(precision, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= tol, errs
