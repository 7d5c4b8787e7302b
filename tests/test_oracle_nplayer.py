"""Pins of the n-player, general-sum FP64 oracle (oracle/cfr_n.py) against what the paper and
the mathematics fix, not against itself:

* the three-player Kuhn game's size is the row the paper's game table prints (nodes,
  terminals, infosets, actions, players);
* on two-player zero-sum games (u_2 = -u_1 as a second payoff column) it is the pinned
  two-player oracle, for all three update rules;
* on normal-form games of 2, 3 and 4 players, one iteration's regrets are the closed form
  E_{sigma_-i}[u_i(x, .)] - E_sigma[u_i] (tensor contractions), and the strategy sums grow by
  the weight times the number of the infoset's nodes times sigma;
* the root's payoff vector is the expected payoff summed over terminals by path probability;
* three-player Kuhn is zero-sum, so the players' values add up to 0 under any strategy;
* a strictly dominant action wins the average strategy;
* players who own no infoset change nothing for the others: the first two players' updates are
  the two-player oracle's on the same tree, at 3 and at 8 (the most) players;
* a game that is one terminal node has its payoff vector as the root's value and no state.
"""
import json
import os

import numpy as np
import pytest

import games
from oracle import cfr, cfr_n
from oracle.tree import Tree

HERE = os.path.dirname(os.path.abspath(__file__))

# eight players (the most the GPU path takes), each with two private types: a 256-way deal and
# infosets of up to 128 members; every player owns infosets
RANDOM8 = dict(seed=26, n_players=8, n_types=2, depth=6, max_actions=2, p_terminal=0.15,
               p_chance=0.1)


def test_kuhn3_matches_the_paper_table():
    with open(os.path.join(HERE, "golden", "game_properties.json")) as f:
        ref = json.load(f)["games"]
    for name, g in (("kuhn_poker", games.kuhn_like(3, "sequential")),
                    ("kuhn_poker(players=3)", games.kuhn3())):
        c = g.counts()
        branching = int(np.bincount(g.parent[g.parent >= 0]).max())
        got = {"nodes": c["nodes"], "terminals": c["terminals"], "infosets": c["infosets"],
               "actions": branching, "players": g.n_players}
        assert got == ref[name], (name, got)


def _as_general_sum(g):
    """The same two-player zero-sum game, its payoffs given as the two columns (u_1, -u_1)."""
    from dataclasses import replace
    pay = np.stack([g.payoff_u1, -g.payoff_u1], axis=1)
    return replace(g, payoff=pay, payoff_u2=None)


@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("make", [lambda: games.kuhn_like(3, "joint"),
                                  lambda: games.leduc_like(3, 2, deal="sequential"),
                                  lambda: games.random_game(22, deal="sequential", depth=6)])
def test_two_player_zero_sum_is_the_two_player_oracle(make, variant):
    g = make()
    t2, tn = Tree(g), cfr_n.TreeN(_as_general_sum(g))
    T, R, S = games.random_state(g, seed=5, nonnegative=(variant == "cfr+"))
    a = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    b = a.copy()
    for _ in range(3):
        a, ia = cfr.iterate(t2, a, variant)
        b, ib = cfr_n.iterate(tn, b, variant)
        assert ib["root_value"][0] == pytest.approx(ia["root_value"], abs=1e-12)
        assert ib["root_value"][1] == pytest.approx(-ia["root_value"], abs=1e-12)
    assert a.T == b.T
    scale = max(1.0, max(abs(x) for x in a.R + a.S))
    assert max(abs(x - y) for x, y in zip(a.R, b.R)) <= 1e-12 * scale
    assert max(abs(x - y) for x, y in zip(a.S, b.S)) <= 1e-12 * scale


def _normal_form_case(shape, seed):
    rng = np.random.default_rng(seed)
    n = len(shape)
    A = rng.integers(-64, 65, size=tuple(shape) + (n,)) / 64.0
    return A, games.normal_form_n(A)


@pytest.mark.parametrize("variant", ["vanilla", "cfr+"])
@pytest.mark.parametrize("shape", [(3, 4), (2, 3, 2), (2, 2, 3, 2), (1, 1, 3), (2,) * 8])
def test_normal_form_regrets_are_the_closed_form(shape, variant):
    A, g = _normal_form_case(shape, seed=len(shape) * 7 + shape[0])
    n = len(shape)
    tree = cfr_n.TreeN(g)
    T, R, S = games.random_state(g, seed=3, nonnegative=(variant == "cfr+"))
    st = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    new, info = cfr_n.iterate(tree, st, variant)
    # each player's strategy, from the oracle's own (pinned) regret matching
    sig = info["sigma"]
    offs = np.cumsum([0] + list(shape))
    strat = [np.asarray(sig[offs[i]:offs[i + 1]]) for i in range(n)]
    letters = "abcdefgh"[:n]
    full = ",".join(letters) + "," + letters + "z->z"
    ev = np.einsum(full, *strat, A)  # E_sigma[u], one entry per player
    assert info["root_value"] == pytest.approx(list(ev), abs=1e-12)
    wt = float(T + 1) if variant == "cfr+" else 1.0
    for i in range(n):
        others = [strat[j] if j != i else np.ones(shape[i]) for j in range(n)]
        spec = ",".join(letters) + "," + letters + "->" + letters[i]
        u_i = np.einsum(spec, *others, A[..., i])  # E_{sigma_-i}[u_i(x, .)] per action x
        r_expected = u_i - ev[i]
        got = np.asarray(info["rtilde"][offs[i]:offs[i + 1]])
        np.testing.assert_allclose(got, r_expected, atol=1e-12)
        members = int(np.prod(shape[:i]))  # player i's infoset holds one node per earlier path
        s_expected = np.asarray(S[offs[i]:offs[i + 1]], dtype=np.float64) + \
            wt * members * strat[i]
        np.testing.assert_allclose(new.S[offs[i]:offs[i + 1]], s_expected, rtol=1e-12)


@pytest.mark.parametrize("make", [lambda: games.kuhn3(), lambda: games.random_game_n(3, 3),
                                  lambda: games.random_game_n(7, 4, depth=5),
                                  lambda: games.random_game_n(**RANDOM8)])
def test_root_value_is_the_expected_payoff_by_enumeration(make):
    g = make()
    tree = cfr_n.TreeN(g)
    T, R, S = games.random_state(g, seed=9)
    st = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    _, info = cfr_n.iterate(tree, st, "vanilla", record=True)
    ev = cfr_n.expected_values(tree, info["sigma"])
    assert info["root_value"] == pytest.approx(ev, abs=1e-12)
    # every node's vector is its children's sigma-weighted sum (spot check at decision nodes)
    for v in range(0, tree.n, max(1, tree.n // 50)):
        ch = tree.children[v]
        if not ch:
            continue
        h = tree.infoset[v]
        probs = tree.sigma0[h] if tree.player[h] == 0 else \
            info["sigma"][tree.qoff[h]:tree.qoff[h] + len(ch)]
        for i in range(tree.n_players):
            want = sum(p * info["node_u"][c][i] for p, c in zip(probs, ch))
            assert info["node_u"][v][i] == pytest.approx(want, abs=1e-12)


def test_kuhn3_values_add_up_to_zero():
    g = games.kuhn3()
    assert np.abs(g.payoff.sum(axis=1)).max() == 0.0
    tree = cfr_n.TreeN(g)
    st = cfr.State.zeros(tree)
    for _ in range(20):
        st, info = cfr_n.iterate(tree, st, "cfr+")
        assert abs(sum(info["root_value"])) <= 1e-12
    avg = cfr.average_strategy(tree, st.S)
    assert abs(sum(cfr_n.expected_values(tree, avg))) <= 1e-12


def test_strictly_dominant_action_wins_the_average():
    # player 3's action 0 pays 1 more than action 1 whatever the others do
    rng = np.random.default_rng(11)
    A = rng.integers(-8, 9, size=(2, 3, 2, 3)) / 8.0
    A[:, :, 0, 2] = A[:, :, 1, 2] + 1.0
    g = games.normal_form_n(A)
    tree = cfr_n.TreeN(g)
    st = cfr_n.solve(tree, 200, "cfr+")
    avg = cfr.average_strategy(tree, st.S)
    o = tree.qoff[tree.rational[2]]
    assert avg[o] > 0.99


@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("make", [lambda: games.kuhn_like(3, "joint"),
                                  lambda: games.leduc_like(3, 2, deal="sequential")])
def test_two_player_alternating_is_the_two_player_oracle(make, variant):
    """The n-pass alternating schedule on two-player zero-sum games is the two-player oracle's
    alternating schedule."""
    g = make()
    t2, tn = Tree(g), cfr_n.TreeN(_as_general_sum(g))
    T, R, S = games.random_state(g, seed=8, nonnegative=(variant == "cfr+"))
    a = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    b = a.copy()
    for _ in range(3):
        a, _ = cfr.iterate_alternating(t2, a, variant)
        b, _ = cfr_n.iterate_alternating(tn, b, variant)
    assert a.T == b.T
    scale = max(1.0, max(abs(x) for x in a.R + a.S))
    assert max(abs(x - y) for x, y in zip(a.R, b.R)) <= 1e-12 * scale
    assert max(abs(x - y) for x, y in zip(a.S, b.S)) <= 1e-12 * scale


def test_alternating_passes_update_one_player_each():
    """On a three-player normal-form game, the first pass changes only player 1's regrets, the
    second sees player 1's new strategy, and the iteration counts once."""
    A, g = _normal_form_case((2, 3, 2), seed=5)
    tree = cfr_n.TreeN(g)
    T, R, S = games.random_state(g, seed=2)
    st = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    one, _ = cfr_n.iterate(tree, st, "vanilla", players=(1,), count=False)
    assert one.T == T and one.R[2:] == st.R[2:] and one.R[:2] != st.R[:2]
    full, _ = cfr_n.iterate_alternating(tree, st, "vanilla")
    assert full.T == T + 1 and full.R[:2] == one.R[:2]
    # the second pass plays player 1's updated strategy: its regrets for player 2 are those of a
    # simultaneous iteration from the state after the first pass
    two, _ = cfr_n.iterate(tree, one, "vanilla", players=(2,), count=False)
    assert full.R[2:5] == two.R[2:5]


@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("extra", [1, 6])
def test_silent_players_leave_the_two_player_game_unchanged(extra, variant):
    """A rational player who owns no infoset never multiplies an edge into anyone's reach (its
    plane stays 1), so with u_2 = -u_1 the first two players' regrets and strategy sums are the
    two-player oracle's on the same tree, exactly; every silent player's root value is its
    payoff's expectation under the profile (summed over terminals by path probability)."""
    g2 = games.kuhn_like(3, "joint")
    g = games.with_silent_players(g2, extra, seed=6)
    assert g.n_players == 2 + extra and set(g.infoset_player.tolist()) == {0, 1, 2}
    t2, tn = Tree(g2), cfr_n.TreeN(g)
    T, R, S = games.random_state(g2, seed=5, nonnegative=(variant == "cfr+"))
    a = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    b = a.copy()
    for _ in range(3):
        a, ia = cfr.iterate(t2, a, variant)
        b, ib = cfr_n.iterate(tn, b, variant)
        assert ib["root_value"][0] == pytest.approx(ia["root_value"], abs=1e-12)
        ev = cfr_n.expected_values(tn, ib["sigma"])
        assert ib["root_value"][2:] == pytest.approx(ev[2:], abs=1e-12)
    assert a.T == b.T
    scale = max(1.0, max(abs(x) for x in a.R + a.S))
    assert max(abs(x - y) for x, y in zip(a.R, b.R)) <= 1e-12 * scale
    assert max(abs(x - y) for x, y in zip(a.S, b.S)) <= 1e-12 * scale


def test_single_terminal_game():
    b = games.GameBuilder("single3")
    b.terminal_vec(b.node(-1, -1), [0.25, -0.5, 1.0])
    g = b.build(players=3)
    tree = cfr_n.TreeN(g)
    st, info = cfr_n.iterate(tree, cfr.State.zeros(tree), "cfr+", record=True)
    assert info["root_value"] == [0.25, -0.5, 1.0]
    assert st.T == 1 and st.R == [] and st.S == []
