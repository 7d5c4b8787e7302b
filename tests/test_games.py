"""Generator pins: node / terminal / infoset counts.

The paper's game-properties table (Appendix, Table tab:properties) lists
kuhn_poker with 58 nodes, 30 terminals and 12 infosets, and leduc_poker with
9,457 nodes, 5,520 terminals and 936 infosets. The Kuhn-shaped and Leduc-shaped
families reproduce those rows exactly when cards are dealt one player at a
time; the workloads use a single joint deal instead.
"""
import numpy as np
import pytest

import games


def test_kuhn_sequential_matches_paper_row():
    c = games.kuhn_like(3, "sequential").counts()
    assert (c["nodes"], c["terminals"], c["infosets"]) == (58, 30, 12)


def test_leduc_sequential_matches_paper_row():
    c = games.leduc_like(3, 2, deal="sequential").counts()
    assert (c["nodes"], c["terminals"], c["infosets"]) == (9457, 5520, 936)


def test_tiny_workload_counts():
    c = games.kuhn_like(3, "joint").counts()
    assert (c["nodes"], c["terminals"], c["infosets"], c["infoset_actions"]) == (55, 30, 12, 24)


def test_medium_workload_counts():
    c = games.leduc_like(6, 2, deal="joint").counts()
    assert (c["nodes"], c["terminals"], c["infosets"], c["infoset_actions"]) == (
        100981, 59928, 4032, 9408)


def test_large_workload_counts(large_game):
    c = large_game.counts()
    assert (c["nodes"], c["terminals"], c["infosets"], c["infoset_actions"]) == (
        21509281, 13476840, 793910, 2068430)
    # memoised count without building the template agrees
    assert 1 + 156 * games.template_size(13, 3, 3, 400) == 21509281


def test_large_game_payoffs_and_chance(large_game):
    g = large_game
    term = g.node_infoset < 0
    assert np.all(g.payoff_u1[~term] == 0)
    assert np.abs(g.payoff_u1[term]).max() == 400
    # chance probabilities sum to one per chance infoset
    off = 0
    for h in np.flatnonzero(g.infoset_player == 0)[:2000]:
        k = g.infoset_num_actions[h]
        assert abs(g.chance_prob[off:off + k].sum() - 1.0) < 1e-12
        off += k


@pytest.mark.parametrize("seed", [100, 101, 102, 103])
def test_subgame_family(seed):
    spec = games.subgame_spec(seed)
    g = games.subgame(seed)
    assert g.n_nodes == spec["size"]
    assert 1e3 / 2 <= g.n_nodes <= 2e6
    assert np.abs(g.payoff_u1).max() == pytest.approx(1.0)
    root = int(np.flatnonzero(g.parent < 0)[0])
    h = g.node_infoset[root]
    assert g.infoset_player[h] == 0
    assert abs(g.chance_prob[:g.infoset_num_actions[h]].sum() - 1.0) < 1e-12


def test_random_game_grid_probabilities_are_exact():
    for seed in range(10):
        g = games.random_game(seed, deal="joint")
        assert np.all(g.chance_prob * 64 == np.round(g.chance_prob * 64))
        assert np.all(g.payoff_u1 * 64 == np.round(g.payoff_u1 * 64))


def test_permuted_game_same_counts():
    g = games.leduc_like(3, 2, deal="sequential")
    p = g.permuted(7)
    assert p.counts() == g.counts()
    assert sorted(p.payoff_u1.tolist()) == sorted(g.payoff_u1.tolist())
