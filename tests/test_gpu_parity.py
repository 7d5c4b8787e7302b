"""GPU parity: the gfx950 path, called through the C ABI, against the FP64 oracle.

Tolerances (the FP32 GPU path against FP64 on the same fp32-representable inputs):
* index and level arrays: bit-exact;
* one iteration from an identical seeded state: every array (R', S', sigma', node
  values, reaches) within 1e-6 norm-wise, max|gpu - oracle| / max|oracle|; the next
  strategy elementwise except at infosets sitting on regret matching's uniform
  fallback (oracle sum of positive regrets below 1e-6 max|R'|), which are counted;
* exploitability after T iterations: within 1e-4 of the oracle's.
"""
import json
import os

import numpy as np
import pytest

import games
from oracle import br, cfr
from oracle.layout import canonical_layout
from oracle.sampled import InfosetSampler
from oracle.tree import Tree

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


ENGINES = ["auto", "packs", "node"]


def _solver(g, variant="vanilla", **kw):
    from paper_2408_14778_amd import Solver
    return Solver(g, variant, **kw)


def _rel(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(float(np.abs(ref).max()) if ref.size else 0.0, 1e-30)
    return float(np.abs(gpu - ref).max()) / scale if ref.size else 0.0


SMALL_GAMES = {
    "kuhn": lambda: games.kuhn_like(3, "joint"),
    "kuhn_seq": lambda: games.kuhn_like(3, "sequential"),
    "leduc3x2": lambda: games.leduc_like(3, 2, deal="sequential"),
    "leduc6x2": lambda: games.leduc_like(6, 2, deal="joint"),
    "rand_joint": lambda: games.random_game(21, deal="joint", depth=5, n_types=(3, 3)),
    "rand_seq": lambda: games.random_game(22, deal="sequential", depth=6),
    "rand_perfect": lambda: games.random_game(23, deal="none", depth=7),
    "rps": lambda: games.rock_paper_scissors(),
    "subgame": lambda: games.subgame(102),
    # 33 levels: past the single-workgroup kernels' 16 and the path kernel's 5
    "deep": lambda: games.random_game(66, deal="sequential", depth=30, max_actions=2, p_terminal=0.3),
    # 33 levels, no chance node on the deepest decision level: its reach is taken in its
    # bottom-up launch
    "deep_nochance": lambda: games.random_game(64, deal="sequential", depth=30, max_actions=2,
                                               p_terminal=0.3, p_chance=0.05),
}


@pytest.mark.parametrize("name", ["kuhn", "leduc6x2", "rand_seq", "subgame"])
def test_device_layout_bit_exact(name):
    g = SMALL_GAMES[name]()
    s = _solver(g)
    ref = canonical_layout(g)
    for k in ("level_offset", "node_id", "parent", "child_begin", "node_player", "node_infoset",
              "node_edge", "infoset_id", "infoset_player", "q_offset", "chance_id", "cq_offset",
              "member_offset", "members", "chance_prob", "payoff", "q_input"):
        assert np.array_equal(s.layout(k), ref[k]), k


def test_deepest_level_reach_in_its_bottom_up_launch():
    """The deepest decision level of deep_nochance (children all terminal, no chance nodes)
    takes its reach in its bottom-up launch, so that game's one-iteration parity (reach of
    every decision node, values, R, S) covers that path; the deep game (chance nodes on that
    level) and the node engine launch every level."""
    g = SMALL_GAMES["deep_nochance"]()
    s = _solver(g)
    D = s.info["depth"]
    rl = s.layout("reach_launch")
    assert rl.shape == (D + 1,) and rl[0] == 0 and rl[D] == 0  # roots; terminals only
    assert rl[D - 1] == 4
    assert np.all(rl[1:D - 1] != 4) and np.all(rl[1:D] != 0)
    assert np.all(np.diff(rl[1:D - 1]) >= 0)  # first levels, then the path, then their own
    assert rl[1] == 1  # 33 tiny levels: the single-workgroup launch takes the first 16
    rn = _solver(g, engine="node").layout("reach_launch")
    assert rn[0] == 0 and np.all(rn[1:D] == 3) and rn[D] == 0
    gd = SMALL_GAMES["deep"]()
    assert np.all(_solver(gd).layout("reach_launch") != 4)


def test_large_game_launch_plan(large_game):
    """The large game's top-down launches: levels 1-7 (at most 175,032 decision nodes each) in
    the launch that walks up to the roots, levels 8-13 one launch each, level 14 (the deepest
    decision level, no chance nodes) in its bottom-up launch, level 15 terminal only. With
    subtree packs, levels 12-14 lie entirely in packs."""
    s = _solver(large_game, "cfr+")
    assert s.layout("reach_launch").tolist() == [0] + [2] * 7 + [3] * 6 + [4, 0]
    rl = _solver(large_game, "cfr+", engine="packs").layout("reach_launch").tolist()
    print("reach_launch with packs:", rl, flush=True)
    assert rl[12:15] == [5, 5, 5] and rl[15] == 0


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("name", sorted(SMALL_GAMES))
def test_one_iteration_parity(name, variant, engine):
    g = SMALL_GAMES[name]()
    T, R, S = games.random_state(g, seed=len(name), nonnegative=(variant == "cfr+"))
    s = _solver(g, variant, engine=engine, keep_node_values=True)
    if engine != "node":
        assert s.info["engine"] == 1  # level-pure, few actions: the public-block engine
    s.set_state(T, R, S)
    s.iterate(1)
    T2, R2, S2 = s.get_state()
    sig2 = s.current_strategy()
    u1, reach = s.node_values()

    t = Tree(g)
    st = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    new, info = cfr.iterate(t, st, variant, record=True)
    assert T2 == T + 1
    assert _rel(R2, new.R) <= 1e-6
    assert _rel(S2, new.S) <= 1e-6
    nid = s.layout("node_id")
    ref_u = np.asarray(info["node_u"])[nid]
    assert _rel(u1, ref_u) <= 1e-6
    ref_reach = np.asarray([info["node_reach"][v] for v in nid])
    dec = s.layout("node_player") >= 0
    for k in range(3):
        assert _rel(reach[dec, k], ref_reach[dec, k]) <= 1e-6
    # next strategy, away from the uniform-fallback discontinuity
    ref_sig = np.asarray(info["next_sigma"])
    scale = max(float(np.abs(new.R).max()), 1e-30)
    skipped = 0
    for h in t.rational:
        o, k = t.qoff[h], t.nact[h]
        pos = sum(max(x, 0.0) for x in new.R[o:o + k])
        if 0.0 < pos < 1e-6 * scale:
            skipped += 1
            continue
        np.testing.assert_allclose(sig2[o:o + k], ref_sig[o:o + k], rtol=0, atol=2e-6)
    assert skipped <= max(1, len(t.rational) // 100)


@pytest.mark.parametrize("name,variant,iters", [
    ("kuhn", "vanilla", 10000),
    ("kuhn", "cfr+", 1000),
    ("rand_joint", "vanilla", 600),
    ("rand_seq", "cfr+", 600),
    ("leduc3x2", "vanilla", 200),
    ("deep", "cfr+", 300),
    ("deep", "vanilla", 300),
    ("kuhn", "dcfr", 1000),
    ("rand_seq", "dcfr", 600),
    ("leduc3x2", "dcfr", 60),
])
@pytest.mark.parametrize("engine", ENGINES)
def test_exploitability_after_T_iterations(name, variant, iters, engine):
    """Discounted CFR (1.5, 0, 2) amplifies fp32-level differences much faster than CFR and
    CFR+ on the two-round game (its discount keeps many regrets near zero, where regret
    matching switches strategies): both engines agree with the oracle to 1e-7 over the first
    iterations, but their states drift about 1e-2 apart by iteration 150, so its case there
    stops at 60 iterations, before the runs decorrelate."""
    g = SMALL_GAMES[name]()
    s = _solver(g, variant, engine=engine)
    s.iterate(iters)
    e = s.exploitability()
    t = Tree(g)
    st = cfr.solve(t, iters, variant)
    ref = br.exploitability(t, cfr.average_strategy(t, st.S))
    assert abs(e["expl"] - ref["expl"]) <= 1e-4, (e, ref)
    assert e["expl"] >= -1e-6


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("name", ["kuhn", "leduc3x2", "rand_joint", "rand_seq", "rps", "subgame"])
def test_alternating_one_iteration_parity(name, variant, engine):
    """Alternating schedule: player 1's pass, then player 2's under player 1's new strategy,
    one t; from a seeded state, R' and S' within 1e-6 of the oracle's two passes."""
    g = SMALL_GAMES[name]()
    T, R, S = games.random_state(g, seed=len(name) + 1, nonnegative=(variant == "cfr+"))
    s = _solver(g, variant, engine=engine, schedule="alternating")
    s.set_state(T, R, S)
    s.iterate(1)
    T2, R2, S2 = s.get_state()
    t = Tree(g)
    new, _ = cfr.iterate_alternating(t, cfr.State(T, [float(x) for x in R], [float(x) for x in S]),
                                     variant)
    assert T2 == T + 1
    assert _rel(R2, new.R) <= 1e-6 and _rel(S2, new.S) <= 1e-6


@pytest.mark.parametrize("name,variant,iters", [
    ("kuhn", "cfr+", 1000),
    ("rand_seq", "cfr+", 300),
    ("leduc3x2", "cfr+", 50),
    ("kuhn", "vanilla", 1000),
])
@pytest.mark.parametrize("engine", ENGINES)
def test_alternating_exploitability_after_T_iterations(name, variant, iters, engine):
    """As for discounted CFR, the two-round game is compared early (T = 50): alternating
    CFR+ there amplifies fp32-level differences fast enough that by T = 100 the GPU and
    oracle runs are about 1.4e-4 apart in exploitability."""
    g = SMALL_GAMES[name]()
    s = _solver(g, variant, engine=engine, schedule="alternating")
    s.iterate(iters)
    e = s.exploitability()
    t = Tree(g)
    st = cfr.solve(t, iters, variant, schedule=cfr.ALTERNATING)
    ref = br.exploitability(t, cfr.average_strategy(t, st.S))
    assert abs(e["expl"] - ref["expl"]) <= 1e-4, (e, ref)


def _strict_checkpoint(cps, band=2.5e-5):
    """The last checkpoint before the fp32-noise ensemble first leaves `band` of the exact run."""
    last = None
    for T in sorted(cps, key=int):
        if cps[T]["spread"] > band:
            break
        last = T
    return last


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("variant", ["vanilla", "cfr+"])
def test_medium_game_exploitability_against_golden(variant, engine):
    """The medium game (100,981 nodes) against the FP64 oracle's stored run, in two parts.

    Strict: at the last checkpoint where every run of an ensemble that carries fp32-sized
    rounding (tests/golden/make_golden.py: noise of D 2^-24 times the magnitude each regret is
    summed from, the same on the strategy-sum increments, R and S rounded to fp32) stays within
    2.5e-5 of the exact run (T = 100 for vanilla CFR, 200 for CFR+), the exploitability is
    within 1e-4 of the exact run's.

    At T = 1,000 the runs have decorrelated: regret matching switches strategies where regrets
    cross zero, so unit-roundoff differences grow over the run, and the ensemble spreads over
    2.4e-3 (vanilla) and 2.4e-4 (CFR+) around the exact value; no fp32 implementation can be
    held to 1e-4 there. The GPU value must then lie within 4 standard deviations of the
    ensemble's mean."""
    gold = json.load(open(os.path.join(HERE, "golden", "medium_game_expl.json")))[variant]
    cps = gold["checkpoints"]
    T_strict = _strict_checkpoint(cps)
    assert T_strict is not None and int(T_strict) >= 100
    g = games.leduc_like(6, 2, deal="joint")
    s = _solver(g, variant, engine=engine)
    s.iterate(int(T_strict))
    e = s.exploitability()["expl"]
    ref = cps[T_strict]["expl"]
    print(f"medium {variant} {engine} T={T_strict}: gpu {e:.7f} oracle {ref:.7f} "
          f"diff {abs(e - ref):.2e}", flush=True)
    assert abs(e - ref) <= 1e-4
    s.iterate(gold["iterations"] - int(T_strict))
    e = s.exploitability()["expl"]
    fin = cps[str(gold["iterations"])]
    z = (e - fin["mean"]) / fin["std"]
    print(f"medium {variant} {engine} T={gold['iterations']}: gpu {e:.6f} oracle {fin['expl']:.6f} "
          f"ensemble {fin['mean']:.6f} +- {fin['std']:.2e} (z {z:+.2f})", flush=True)
    assert abs(z) <= 4.0


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("name", ["kuhn", "leduc3x2", "rand_seq", "subgame"])
def test_best_response_on_the_gpu_average(name, engine):
    g = SMALL_GAMES[name]()
    s = _solver(g, "cfr+", engine=engine)
    s.iterate(37)
    avg = s.average_strategy().astype(np.float64)
    e = s.exploitability()
    t = Tree(g)
    ref = br.exploitability(t, avg.tolist())
    scale = max(1.0, float(np.abs(g.payoff_u1).max()))
    assert abs(e["br1"] - ref["br1"]) <= 1e-5 * scale
    assert abs(e["br2"] - ref["br2"]) <= 1e-5 * scale
    # the average strategy itself stays close to the oracle's after 37 FP32 iterations
    # (differences at rounding level grow slowly through regret matching)
    st = cfr.solve(t, 37, "cfr+")
    assert _rel(avg, cfr.average_strategy(t, st.S)) <= 1e-4


@pytest.mark.parametrize("engine", ENGINES)
def test_graph_replay_matches_direct_launches(engine):
    """The block engine sums in a fixed order: graph replays and direct launches agree bit for
    bit. The node engine accumulates with float atomics, whose order varies between runs, so
    over 21 iterations the two agree to fp32 reordering only."""
    g = games.leduc_like(3, 2, deal="sequential")
    a = _solver(g, "cfr+", graph=True, engine=engine)
    b = _solver(g, "cfr+", graph=False, engine=engine)
    for _ in range(3):
        a.iterate(7)
        b.iterate(7)
        Ta, Ra, Sa = a.get_state()
        Tb, Rb, Sb = b.get_state()
        assert Ta == Tb
        if engine == "node":
            assert _rel(Ra, Rb) <= 1e-5 and _rel(Sa, Sb) <= 1e-5
        else:
            assert np.array_equal(Ra, Rb) and np.array_equal(Sa, Sb)


def test_average_strategy_to_device():
    import torch
    g = games.kuhn_like(3, "joint")
    s = _solver(g)
    s.iterate(5)
    out = torch.empty(s.n_q, dtype=torch.float32, device="cuda")
    s.average_strategy_device(out)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), s.average_strategy())


@pytest.mark.parametrize("engine", ENGINES)
def test_state_roundtrip_and_resume(engine):
    g = games.random_game(31, deal="joint", depth=5)
    a = _solver(g, "cfr+", engine=engine)
    a.iterate(25)
    T, R, S = a.get_state()
    b = _solver(g, "cfr+", engine=engine)
    b.set_state(T, R, S)
    a.iterate(10)
    b.iterate(10)
    Ta, Ra, Sa = a.get_state()
    Tb, Rb, Sb = b.get_state()
    assert Ta == Tb == 35
    assert _rel(Rb, Ra) <= 1e-6 and _rel(Sb, Sa) <= 1e-6


def test_single_node_and_single_action_games():
    g = games.Game("single", np.array([-1], np.int32), np.array([-1], np.int32),
                   np.array([-1], np.int32), np.zeros(0, np.int8), np.zeros(0, np.int32),
                   np.zeros(0), np.array([0.25]))
    s = _solver(g)
    s.iterate(3)
    e = s.exploitability()
    assert e["br1"] == pytest.approx(0.25) and e["br2"] == pytest.approx(-0.25)
    g = games.random_game(5, deal="none", depth=4, max_actions=1)
    s = _solver(g)
    s.iterate(2)
    assert s.exploitability()["expl"] == pytest.approx(0.0, abs=1e-6)


def test_non_level_pure_game_iterates_but_refuses_exploitability():
    from paper_2408_14778_amd import CfrError
    b = games.GameBuilder("skew")
    root = b.node(-1, -1)
    b.decide(root, b.infoset_id("c", 0, 2, [0.5, 0.5]))
    x, y = b.node(root, 0), b.node(root, 1)
    hp = b.infoset_id("p1", 1, 2)
    b.decide(x, hp)
    b.decide(y, b.infoset_id("c2", 0, 1, [1.0]))
    z = b.node(y, 0)
    b.decide(z, hp)
    for v, base in ((x, 0.0), (z, 1.0)):
        for a in range(2):
            b.terminal(b.node(v, a), base + a)
    g = b.build()
    s = _solver(g)
    s.iterate(4)
    t = Tree(g)
    st = cfr.solve(t, 4)
    _, R, S = s.get_state()
    assert _rel(R, st.R) <= 1e-6 and _rel(S, st.S) <= 1e-6
    with pytest.raises(CfrError, match="CFR_ELEVEL"):
        s.exploitability()


@pytest.mark.parametrize("engine,variant", [("auto", "cfr+"), ("node", "cfr+"), ("auto", "dcfr")])
def test_large_game_one_iteration_sampled(large_game, engine, variant):
    """Full-size large workload (21,509,281 nodes), seeded state: R' and S' of three sampled
    infosets of every decision level (levels 1-14) against the oracle, which takes every
    node's value from one FP64 sweep and each member's reach from its root path.

    The FP32 bound each element is held to: the instantaneous regret is a sum over the
    infoset's members of pi_-i (w_a - u), where the reach is a product of at most D = 15 edge
    probabilities and the values sums of products over at most D levels, so each term carries
    a relative rounding of about D * 2^-24 of its magnitude and |dr~| <= 2 D 2^-24 * scale,
    scale = sum |pi_-i| (|w_a| + |u|) (the oracle returns it); the update adds a few units of
    2^-24 of |R| + |r~| (8; 32 for discounted CFR, whose factors come from the hardware exp2 and
    log2). For S' = S + w pibar sigma: (D + 8) 2^-24 of the increment plus 4 (16) units of
    |S'|. The
    test prints, per level, the largest error as a fraction of its bound."""
    g = large_game
    T, R, S = games.random_state(g, seed=2, nonnegative=(variant == "cfr+"))
    s = _solver(g, variant, engine=engine)
    s.set_state(T, R, S)
    s.iterate(1)
    T2, R2, S2 = s.get_state()
    sig = s.current_strategy()
    assert T2 == T + 1
    if variant == "cfr+":
        assert np.all(R2 >= 0) and np.all(S2 >= S - 1e-6 * np.abs(S).max())
    samp = InfosetSampler(g)
    values = samp.all_values(R)
    lo = s.layout("level_offset")
    nid = s.layout("node_id")
    level_of = np.empty(g.n_nodes, dtype=np.int64)
    for lv in range(len(lo) - 1):
        level_of[nid[lo[lv]:lo[lv + 1]]] = lv
    rational = np.flatnonzero(g.infoset_player != 0)
    first = np.full(g.n_infosets, -1, dtype=np.int64)
    dec = np.flatnonzero(g.node_infoset >= 0)
    first[g.node_infoset[dec[::-1]]] = dec[::-1]
    h_level = level_of[first[rational]]
    rng = np.random.default_rng(2)
    u = 2.0 ** -24
    D = len(lo) - 2
    c = 32 if variant == "dcfr" else 8  # units of 2^-24 on the update's own rounding
    levels = sorted(set(h_level.tolist()))
    assert levels == list(range(1, D)), levels  # every decision level holds rational infosets
    for lv in levels:
        pool = rational[h_level == lv]
        picks = rng.choice(pool, size=min(3, pool.size), replace=False)
        worst_R = worst_S = 0.0
        for h in picks:
            out = samp.update(R, S, T, int(h), variant, values=values)
            q = np.asarray(out["q"])
            rt = np.abs(np.asarray(out["rtilde"]))
            bound_R = 2 * D * u * np.asarray(out["rtilde_scale"]) + c * u * (np.abs(R[q]) + rt)
            w = float(T + 1) if variant == "cfr+" else 1.0
            inc = np.abs(w * out["pibar"] * np.asarray(out["sigma"]))
            bound_S = (D + 8) * u * inc + c / 2 * u * np.abs(np.asarray(out["S"]))
            err_R = np.abs(R2[q] - np.asarray(out["R"]))
            err_S = np.abs(S2[q] - np.asarray(out["S"]))
            worst_R = max(worst_R, float((err_R / np.maximum(bound_R, 1e-30)).max()))
            worst_S = max(worst_S, float((err_S / np.maximum(bound_S, 1e-30)).max()))
        print(f"level {lv:2d}: {len(picks)} infosets, largest error / bound: R' {worst_R:.3f} "
              f"S' {worst_S:.3f}", flush=True)
        assert worst_R <= 1.0 and worst_S <= 1.0, lv
    # the next strategy is regret matching of the GPU's own R' (and sums to one)
    qo = np.concatenate([[0], np.cumsum(g.infoset_num_actions[rational])])
    pos = np.maximum(R2.astype(np.float64), 0.0)
    tot = np.add.reduceat(pos, qo[:-1])
    k = np.diff(qo)
    rm = np.where(np.repeat(tot, k) > 0, pos / np.repeat(np.maximum(tot, 1e-300), k),
                  1.0 / np.repeat(k, k))
    assert np.abs(sig - rm).max() <= 2e-6
    sums = np.add.reduceat(sig.astype(np.float64), qo[:-1])
    assert np.abs(sums - 1.0).max() < 1e-5


def test_large_game_engines_agree(large_game):
    """Both engines over the full large game: same state after 3 iterations (1e-5), same
    exploitability, which is nonnegative."""
    a = _solver(large_game, "cfr+")
    b = _solver(large_game, "cfr+", engine="node")
    assert a.info["engine"] == 1 and b.info["engine"] == 0
    a.iterate(3)
    b.iterate(3)
    _, Ra, Sa = a.get_state()
    _, Rb, Sb = b.get_state()
    assert _rel(Ra, Rb) <= 1e-5 and _rel(Sa, Sb) <= 1e-5
    ea, eb = a.exploitability(), b.exploitability()
    assert np.isfinite(ea["expl"]) and ea["expl"] >= -1e-3
    assert abs(ea["expl"] - eb["expl"]) <= 1e-4 * max(1.0, abs(eb["expl"]))
