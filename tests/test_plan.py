"""Host checks of the public-block execution plan: it is a relabelling of the canonical
layout that keeps every parent/child/edge relation, groups each infoset's members inside
one public block, and numbers infosets contiguously per level."""
import numpy as np
import pytest

import games
from oracle.layout import canonical_layout

GAMES = [
    lambda: games.kuhn_like(3, "joint"),
    lambda: games.kuhn_like(3, "sequential").permuted(2),
    lambda: games.leduc_like(3, 2, deal="sequential"),
    lambda: games.leduc_like(6, 2, deal="joint"),
    lambda: games.random_game(51, deal="sequential", depth=6, n_types=(3, 2)),
    lambda: games.random_game(52, deal="none", depth=6),
    lambda: games.rock_paper_scissors(),
    lambda: games.subgame(104),
]


def _plan(g):
    from paper_2408_14778_amd.solver import LAYOUT_DTYPES, PLAN_DTYPES, host_layout
    return host_layout(g, list(LAYOUT_DTYPES) + list(PLAN_DTYPES))


def _check(g, lay):
    ref = canonical_layout(g)
    n = g.n_nodes
    canon = lay["x_canon_of"].astype(np.int64)
    assert sorted(canon.tolist()) == list(range(n))
    exec_of = np.empty(n, dtype=np.int64)
    exec_of[canon] = np.arange(n)
    lo = ref["level_offset"]
    # exec order keeps levels
    for l in range(len(lo) - 1):
        seg = canon[lo[l]:lo[l + 1]]
        assert seg.min() >= lo[l] and seg.max() < lo[l + 1]
    par = ref["parent"].astype(np.int64)
    xpar = lay["x_parent"].astype(np.int64)
    assert xpar[0] == -1
    assert np.array_equal(xpar[1:], exec_of[par[canon[1:]]])
    # children in action order, through stride or list
    cb = ref["child_begin"].astype(np.int64)
    for x in range(n):
        c = canon[x]
        kids = exec_of[np.arange(cb[c], cb[c + 1])]
        if len(kids) == 0:
            assert (lay["x_meta"][x] & 3) == 0
            continue
        st = lay["x_child_stride"][x]
        b = lay["x_child_begin"][x]
        got = b + st * np.arange(len(kids)) if st != 0 else lay["x_child_list"][b:b + len(kids)]
        assert np.array_equal(got, kids)
    # exec infosets: a relabelling, members = exec positions of the canonical members
    xh = lay["x_infoset_canon"]
    assert sorted(xh.tolist()) == list(range(len(ref["q_offset"]) - 1))
    xq = lay["x_q_offset"]
    mo, mem = lay["x_member_offset"], lay["x_members"]
    for hx, h in enumerate(xh):
        cm = ref["members"][ref["member_offset"][h]:ref["member_offset"][h + 1]]
        assert np.array_equal(mem[mo[hx]:mo[hx + 1]], np.sort(exec_of[cm]))
        assert xq[hx + 1] - xq[hx] == ref["q_offset"][h + 1] - ref["q_offset"][h]
        assert np.array_equal(lay["x_q_input"][xq[hx]:xq[hx + 1]],
                              ref["q_input"][ref["q_offset"][h]:ref["q_offset"][h + 1]])
    # edges of player children use the parent's exec infoset
    Qp = int(ref["q_offset"][-1])
    for x in range(1, n):
        c = canon[x]
        p = par[c]
        e = lay["x_edge"][x]
        if ref["node_player"][p] >= 1:
            hx = int(np.flatnonzero(xh == ref["node_infoset"][p])[0])
            assert e == xq[hx] + (c - cb[p])
        else:
            assert e == ref["node_edge"][c] and e >= Qp
    # infosets of each level are contiguous and ordered by level
    hlo = lay["x_h_level_offset"]
    depth = np.repeat(np.arange(len(lo) - 1), np.diff(lo))
    for l in range(len(hlo) - 1):
        for hx in range(hlo[l], hlo[l + 1]):
            assert np.all(depth[canon[mem[mo[hx]:mo[hx + 1]]]] == l)


@pytest.mark.parametrize("maker", GAMES)
def test_plan_is_a_faithful_relabelling(maker):
    g = maker()
    _check(g, _plan(g))


def test_plan_locality_on_the_large_game(large_game):
    lay = _plan(large_game)
    mo, mem = lay["x_member_offset"], lay["x_members"]
    span = np.maximum.reduceat(mem, mo[:-1]) - np.minimum.reduceat(mem, mo[:-1])
    # every infoset's members lie within one public block of at most 156 deals
    assert span.max() < 156
    # only chance nodes (public cards) need explicit child lists
    n_chance = len(lay["x_chance_nodes"])
    listed = int((lay["x_child_stride"] == 0).sum() - (lay["x_meta"] & 3 == 0).sum())
    assert listed <= n_chance
