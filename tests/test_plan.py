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


def _plan(g, packs=False):
    from paper_2408_14778_amd.solver import LAYOUT_DTYPES, PLAN_DTYPES, host_layout
    return host_layout(g, list(LAYOUT_DTYPES) + list(PLAN_DTYPES), packs=packs)


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


def _f32(w):
    return float(np.array([w], dtype=np.int32).view(np.float32)[0])


def _check_packs(g, lay, sample=None):
    """Subtree packs: every decision node outside the upper prefixes lies in exactly one pack;
    a pack's records reproduce the tree (each member's children are the pack's own decision
    nodes, terminals with their payoffs, or roots of a lower tier's packs), its infosets are
    whole, and the caps hold."""
    from paper_2408_14778_amd.solver import packs as get_packs
    ref = canonical_layout(g)
    lo = ref["level_offset"]
    n = g.n_nodes
    meta = lay["x_meta"]
    par = lay["x_parent"].astype(np.int64)
    edge = lay["x_edge"]
    cb, cs, cl = lay["x_child_begin"], lay["x_child_stride"], lay["x_child_list"]
    mo, mem, qo = lay["x_member_offset"], lay["x_members"], lay["x_q_offset"]
    hlo, cnodes, clo = lay["x_h_level_offset"], lay["x_chance_nodes"], lay["x_c_level_offset"]
    up, hup, cup = lay["x_up_end"], lay["x_h_up_end"], lay["x_c_up_end"]
    payoff = lay["payoff"][lay["x_canon_of"]]
    B = lay["x_pack_blob"]
    to = lay["x_tier_offset"]
    nkids = np.bincount(par[par >= 0], minlength=n)
    level = np.repeat(np.arange(len(lo) - 1), np.diff(lo))
    h_of = np.full(n, -1)
    for h in range(len(mo) - 1):
        h_of[mem[mo[h]:mo[h + 1]]] = h

    def kids(x):
        k = nkids[x]
        return cb[x] + cs[x] * np.arange(k) if cs[x] != 0 else cl[cb[x]:cb[x] + k]

    P = get_packs(lay)
    owner = np.full(n, -1)
    tier_of = np.zeros(n, dtype=np.int64)
    root_tier = {}
    # records checked in full for every pack, or for `sample` packs picked at random (the
    # coverage and caps for all)
    full = set(range(len(P))) if sample is None else set(
        np.random.default_rng(0).choice(len(P), min(sample, len(P)), replace=False).tolist())
    for p, pk in enumerate(P):
        for i in range(pk["n_root"]):
            w = B[pk["off_root"] + 4 * i:pk["off_root"] + 4 * i + 4]
            root_tier[w[3]] = pk["tier"]
    for p, pk in enumerate(P):
        nodes = B[pk["off_node"]:pk["off_node"] + pk["n_dec"]]
        assert np.all(owner[nodes] == -1)
        owner[nodes] = p
        if p not in full:
            assert pk["n_dec"] <= 512 and pk["n_pairs"] <= 384 and 1 <= pk["nlv"] <= 8
            continue
        owner[nodes] = -1
        assert pk["n_dec"] <= 512 and pk["n_pairs"] <= 384 and 1 <= pk["nlv"] <= 8
        assert to[pk["tier"] - 1] <= p < to[pk["tier"]]
        nodes = B[pk["off_node"]:pk["off_node"] + pk["n_dec"]]
        assert np.all(owner[nodes] == -1) and np.all((meta[nodes] & 3) != 0)
        owner[nodes] = p
        tier_of[nodes] = pk["tier"]
        assert np.all(np.diff(level[nodes]) >= 0)
        assert level[nodes[0]] == pk["level0"] and level[nodes[-1]] < pk["level0"] + pk["nlv"]
        for i in range(pk["n_root"]):
            w = B[pk["off_root"] + 4 * i:pk["off_root"] + 4 * i + 4]
            x = w[3]
            assert nodes[w[0] & 0xffff] == x and level[x] == pk["level0"]
            assert w[1] == par[x] and (w[1] < 0 or w[2] == edge[x])
            assert ((w[0] >> 16) & 3) == ((meta[x] >> 2) & 3)
            root_tier[x] = pk["tier"]
        # infosets: whole, with their pairs; members in infoset order, level by level
        ql = 0
        mi = 0
        for h in range(pk["n_inf"]):
            w = B[pk["off_inf"] + 4 * h:pk["off_inf"] + 4 * h + 4]
            hx = int(np.searchsorted(qo, w[0], side="right") - 1)
            k = w[3] & 255
            assert qo[hx] == w[0] and qo[hx + 1] - qo[hx] == k and w[1] == ql
            first, end = w[2] & 0xffff, w[2] >> 16
            assert first == mi and end - first == mo[hx + 1] - mo[hx]
            for m in range(first, end):
                mw = B[pk["off_mem"] + 6 * m:pk["off_mem"] + 6 * m + 6]
                x = nodes[mw[0] & 0xffff]
                assert h_of[x] == hx and mw[1] == ql and ((mw[0] >> 16) & 7) == k
                assert x == mem[mo[hx] + m - first]
                ext = False
                for a, c in enumerate(kids(x)):
                    kind = (mw[0] >> (24 + 2 * a)) & 3
                    if kind == 0:
                        assert nodes[mw[2 + a]] == c
                    elif kind == 1:
                        assert (meta[c] & 3) == 0 and _f32(mw[2 + a]) == payoff[c]
                    else:
                        assert kind == 2 and mw[2 + a] == c and (meta[c] & 3) != 0
                        ext = True
                assert bool((mw[0] >> 20) & 1) == ext
            ql += k
            mi = end
        assert ql == pk["n_pairs"] and mi == pk["n_mem"]
        # chance nodes and their children
        for ci in range(pk["n_ch"]):
            w = B[pk["off_ch"] + 4 * ci:pk["off_ch"] + 4 * ci + 4]
            x = nodes[w[0] & 0xffff]
            assert (meta[x] & 3) == 1 and w[1] == nkids[x]
            for a, c in enumerate(kids(x)):
                kw = B[pk["off_kid"] + 3 * (w[2] + a):pk["off_kid"] + 3 * (w[2] + a) + 3]
                assert kw[2] in (0, 1, 2)
                if kw[2] == 0:
                    assert nodes[kw[0]] == c
                elif kw[2] == 1:
                    assert _f32(kw[0]) == payoff[c]
                else:
                    assert kw[0] == c
    # external children are roots of packs of lower tiers; every decision node past the upper
    # prefix is in a pack
    for p, pk in enumerate(P):
        if p not in full:
            continue
        for m in range(pk["n_mem"]):
            mw = B[pk["off_mem"] + 6 * m:pk["off_mem"] + 6 * m + 6]
            for a in range((mw[0] >> 16) & 7):
                if ((mw[0] >> (24 + 2 * a)) & 3) == 2:
                    assert root_tier[mw[2 + a]] < pk["tier"]
    for l in range(len(lo) - 1):
        dec = (meta[lo[l]:lo[l + 1]] & 3) != 0
        inside = owner[lo[l]:lo[l + 1]] >= 0
        x = np.arange(lo[l], lo[l + 1])
        assert np.all(inside[dec] == (x[dec] >= up[l]))
        first = mem[mo[hlo[l]:hlo[l + 1]]]
        assert np.all((first < up[l]) == (np.arange(hlo[l], hlo[l + 1]) < hup[l]))
        cn = cnodes[clo[l]:clo[l + 1]]
        assert np.all((cn < up[l]) == (np.arange(clo[l], clo[l + 1]) < cup[l]))
    return P, owner


@pytest.mark.parametrize("maker", GAMES)
def test_subtree_packs_hold_whole_subtrees(maker):
    g = maker()
    lay = _plan(g, packs=True)
    _check(g, lay)  # still a faithful relabelling
    _check_packs(g, lay)


def test_subtree_packs_of_the_large_game(large_game):
    """Packs of the large game: every decision node below level 11 lies in a pack, most of
    them in tier 1; the levels above keep their per-level launches."""
    lay = _plan(large_game, packs=True)
    packs, owner = _check_packs(large_game, lay, sample=200)
    dec = (lay["x_meta"] & 3) != 0
    lo = lay["level_offset"]
    to = lay["x_tier_offset"]
    print(f"{len(packs)} packs in {len(to) - 1} tiers", flush=True)
    assert np.all(owner[lo[12]:][dec[lo[12]:]] >= 0) and len(to) - 1 <= 8
    t1 = sum(p["n_dec"] for p in packs[:to[1]])
    assert t1 > 0.75 * dec.sum()
