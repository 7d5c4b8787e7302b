"""Pins for the oracle's canonical layout: structural invariants that any
correct level-ordered flattening of the tree (Section 3.1) satisfies, and
independence from the input's node and infoset numbering."""
import numpy as np
import pytest

import games
from oracle.layout import canonical_layout
from oracle.tree import Tree

GAMES = [
    lambda: games.kuhn_like(3, "joint"),
    lambda: games.leduc_like(3, 2, deal="sequential"),
    lambda: games.random_game(3, deal="sequential", depth=5),
    lambda: games.random_game(4, deal="none", depth=5),
    lambda: games.rock_paper_scissors(),
]


def _check_invariants(g, lay):
    n = g.n_nodes
    t = Tree(g)
    node_id = lay["node_id"].astype(np.int64)
    assert sorted(node_id.tolist()) == list(range(n))
    canon = np.empty(n, dtype=np.int64)
    canon[node_id] = np.arange(n)
    lo = lay["level_offset"]
    depth = np.repeat(np.arange(len(lo) - 1), np.diff(lo))
    # depth matches the tree's own depth, parent is one level up
    assert np.array_equal(depth, np.asarray(t.depth)[node_id])
    par = lay["parent"].astype(np.int64)
    assert par[0] == -1 and np.all(depth[1:] == depth[par[1:]] + 1)
    # children contiguous, in action order
    cb = lay["child_begin"].astype(np.int64)
    assert np.all(np.diff(cb) >= 0) and cb[-1] == n
    for v in range(n):
        kids = list(range(cb[v], cb[v + 1]))
        assert [int(node_id[c]) for c in kids] == t.children[int(node_id[v])]
    # edge index decodes to (infoset, action) of the parent
    q_off = lay["q_offset"].astype(np.int64)
    Qp = q_off[-1]
    for v in range(1, n):
        p = par[v]
        a = v - cb[p]
        e = lay["node_edge"][v]
        if lay["node_player"][p] >= 1:
            h = lay["node_infoset"][p]
            assert e == q_off[h] + a
        else:
            c = lay["node_infoset"][p]
            assert e == Qp + lay["cq_offset"][c] + a
            assert lay["chance_prob"][e - Qp] == np.float32(t.sigma0[t.infoset[node_id[p]]][a])
    # members listed once, in ascending order, all at one level here
    mem = lay["members"]
    mo = lay["member_offset"]
    assert len(mem) == int((lay["node_player"] >= 1).sum())
    for h in range(len(mo) - 1):
        m = mem[mo[h]:mo[h + 1]]
        assert np.all(np.diff(m) > 0)
        assert np.all(lay["node_infoset"][m] == h)
    assert lay["level_pure"]
    # q_input maps onto the input's pair numbering
    assert sorted(lay["q_input"].tolist()) == list(range(int(Qp)))


@pytest.mark.parametrize("maker", GAMES)
def test_layout_invariants(maker):
    g = maker()
    _check_invariants(g, canonical_layout(g))


@pytest.mark.parametrize("maker", GAMES)
def test_layout_independent_of_input_numbering(maker):
    g = maker()
    a = canonical_layout(g)
    for seed in (1, 2):
        p = g.permuted(seed)
        b = canonical_layout(p)
        _check_invariants(p, b)
        for k in ("level_offset", "parent", "child_begin", "node_player", "node_infoset",
                  "node_edge", "infoset_player", "q_offset", "cq_offset", "member_offset",
                  "members", "chance_prob", "payoff"):
            assert np.array_equal(a[k], b[k]), k


def test_kuhn_levels_by_hand():
    lay = canonical_layout(games.kuhn_like(3, "joint"))
    # root, 6 deals, 12 player-2 nodes, 24 = 6 player-1 nodes + 18 terminals, 12 terminals
    assert lay["level_offset"].tolist() == [0, 1, 7, 19, 43, 55]
    assert lay["q_offset"][-1] == 24 and len(lay["q_offset"]) == 13
