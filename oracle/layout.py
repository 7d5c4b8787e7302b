"""Independent implementation of the canonical level-ordered layout.

Test infrastructure (oracle): not part of the product path. The GPU library's
host flattener must emit these arrays bit for bit.

The layout replaces each constant matrix of Section 3.1 by index arrays, which
is possible because each matrix has at most one nonzero per column: G and the
level graphs L^(l) become ``parent``/``child_begin``/``level_offset``,
M^(Q+,V) becomes ``node_edge`` plus the member lists, M^(H+,Q+) becomes
``q_offset``, M^(V,I+) becomes the player of the parent, and s^(sigma0)
becomes ``chance_prob`` indexed through ``node_edge``.

Specification
-------------
* Level 0 is the root. Level l+1 holds the children of level l sorted by
  (canonical index of the parent, action index). A node's canonical index is
  its position in the concatenation of the levels, so each parent's children
  are contiguous and in action order. D is the deepest level.
* ``level_offset[l]`` .. ``level_offset[l+1]`` is level l (D + 2 entries).
* ``node_id[v]``: input id of canonical node v. ``parent[v]``: canonical parent
  (-1 at the root). ``child_begin[v]`` = 1 + number of non-root nodes whose
  parent is < v, so the children of v are child_begin[v] .. child_begin[v+1]-1;
  child_begin[N] = N.
* ``node_player[v]``: -1 terminal, 0 chance, 1 or 2.
* Rational infosets are numbered 0..H+-1 by first appearance in canonical node
  order; chance infosets 0..H0-1 likewise, separately. ``node_infoset[v]`` is
  that number for decision nodes (rational or chance id by ``node_player``), -1
  at terminals. ``infoset_id`` / ``chance_id``: their input ids.
* ``q_offset`` (H+ + 1) and ``cq_offset`` (H0 + 1): prefix sums of action
  counts. ``node_edge[v]`` for a child of a rational node in infoset h by
  action a is q_offset[h] + a; for a child of a chance node in chance infoset c
  it is Q+ + cq_offset[c] + a; -1 at the root.
* ``members`` / ``member_offset``: each rational infoset's nodes, ascending.
* ``chance_prob`` (Q0, fp32) and ``payoff`` (N, fp32: u_1 at terminals, else 0)
  are the input doubles rounded to nearest fp32.
* ``q_input[q]``: the input's infoset-action index of canonical pair q.
"""
from __future__ import annotations

import numpy as np


def canonical_layout(game) -> dict:
    n = game.n_nodes
    parent_in = game.parent.astype(np.int64)
    action_in = game.node_action.astype(np.int64)
    roots = np.flatnonzero(parent_in < 0)
    assert roots.size == 1
    root = int(roots[0])
    nonroot = np.flatnonzero(parent_in >= 0)
    order = nonroot[np.lexsort((action_in[nonroot], parent_in[nonroot]))]
    nchild = np.bincount(parent_in[nonroot], minlength=n)
    ptr = np.concatenate([[0], np.cumsum(nchild)])

    levels = [np.array([root], dtype=np.int64)]
    while True:
        cur = levels[-1]
        cnt = nchild[cur]
        if cnt.sum() == 0:
            break
        starts = np.repeat(ptr[cur], cnt)
        within = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        levels.append(order[starts + within])
    node_id = np.concatenate(levels)
    D = len(levels) - 1
    level_offset = np.concatenate([[0], np.cumsum([len(x) for x in levels])])
    canon = np.empty(n, dtype=np.int64)
    canon[node_id] = np.arange(n)

    parent = np.where(parent_in[node_id] < 0, -1, canon[np.maximum(parent_in[node_id], 0)])
    nch_c = nchild[node_id]
    # child_begin[v] = 1 + number of children of the nodes before v
    child_begin = np.concatenate([1 + np.concatenate([[0], np.cumsum(nch_c)[:-1]]), [n]])

    h_in = game.node_infoset.astype(np.int64)[node_id]
    iplayer_in = game.infoset_player.astype(np.int64)
    is_dec = h_in >= 0
    node_player = np.full(n, -1, dtype=np.int64)
    node_player[is_dec] = iplayer_in[h_in[is_dec]]

    def first_appearance(mask):
        hs = h_in[mask]
        uniq, first = np.unique(hs, return_index=True)
        ids_in_order = uniq[np.argsort(first)]
        remap = {int(h): i for i, h in enumerate(ids_in_order)}
        return ids_in_order, remap

    rat_mask = node_player >= 1
    ch_mask = node_player == 0
    infoset_id, rmap = first_appearance(rat_mask)
    chance_id, cmap = first_appearance(ch_mask)
    node_infoset = np.full(n, -1, dtype=np.int64)
    lut_r = np.full(game.n_infosets, -1, dtype=np.int64)
    lut_r[infoset_id] = np.arange(len(infoset_id))
    lut_c = np.full(game.n_infosets, -1, dtype=np.int64)
    lut_c[chance_id] = np.arange(len(chance_id))
    node_infoset[rat_mask] = lut_r[h_in[rat_mask]]
    node_infoset[ch_mask] = lut_c[h_in[ch_mask]]

    nact_in = game.infoset_num_actions.astype(np.int64)
    infoset_player = iplayer_in[infoset_id]
    infoset_num_actions = nact_in[infoset_id]
    q_offset = np.concatenate([[0], np.cumsum(infoset_num_actions)])
    chance_num_actions = nact_in[chance_id]
    cq_offset = np.concatenate([[0], np.cumsum(chance_num_actions)])
    Qp = int(q_offset[-1])

    act_c = action_in[node_id]
    par = parent
    node_edge = np.full(n, -1, dtype=np.int64)
    nr = np.flatnonzero(par >= 0)
    pp = par[nr]
    pl = node_player[pp]
    hi = node_infoset[pp]
    node_edge[nr] = np.where(pl >= 1, q_offset[np.where(pl >= 1, hi, 0)] + act_c[nr],
                             Qp + cq_offset[np.where(pl == 0, hi, 0)] + act_c[nr])

    # members
    rat_nodes = np.flatnonzero(rat_mask)
    mo = np.argsort(node_infoset[rat_nodes], kind="stable")
    members = rat_nodes[mo]
    member_offset = np.concatenate([[0], np.cumsum(np.bincount(node_infoset[rat_nodes],
                                                               minlength=len(infoset_id)))])

    # chance probabilities in canonical chance-pair order
    cp_in = game.chance_prob.astype(np.float64)
    in_off = {}
    pos = 0
    for h in range(game.n_infosets):
        if iplayer_in[h] == 0:
            in_off[h] = pos
            pos += int(nact_in[h])
    chance_prob = np.concatenate(
        [cp_in[in_off[int(h)]:in_off[int(h)] + int(nact_in[h])] for h in chance_id]
    ) if len(chance_id) else np.zeros(0)

    payoff = np.where(node_player < 0, game.payoff_u1.astype(np.float64)[node_id], 0.0)

    # input q of each canonical q
    in_qoff = np.zeros(game.n_infosets, dtype=np.int64)
    q = 0
    for h in range(game.n_infosets):
        if iplayer_in[h] != 0:
            in_qoff[h] = q
            q += int(nact_in[h])
    q_input = np.concatenate([in_qoff[h] + np.arange(k) for h, k in
                              zip(infoset_id, infoset_num_actions)]) if len(infoset_id) else \
        np.zeros(0, dtype=np.int64)

    depth = np.repeat(np.arange(D + 1), np.diff(level_offset))
    mdepth = depth[members]
    lo = np.minimum.reduceat(mdepth, member_offset[:-1]) if len(members) else np.zeros(0)
    hi_ = np.maximum.reduceat(mdepth, member_offset[:-1]) if len(members) else np.zeros(0)
    level_pure = bool(np.all(lo == hi_))

    i32 = np.int32
    return {
        "D": D,
        "level_offset": level_offset.astype(i32),
        "node_id": node_id.astype(i32),
        "parent": parent.astype(i32),
        "child_begin": child_begin.astype(i32),
        "node_player": node_player.astype(np.int8),
        "node_infoset": node_infoset.astype(i32),
        "node_edge": node_edge.astype(i32),
        "infoset_id": infoset_id.astype(i32),
        "infoset_player": infoset_player.astype(np.int8),
        "q_offset": q_offset.astype(i32),
        "chance_id": chance_id.astype(i32),
        "cq_offset": cq_offset.astype(i32),
        "member_offset": member_offset.astype(i32),
        "members": members.astype(i32),
        "chance_prob": chance_prob.astype(np.float32),
        "payoff": payoff.astype(np.float32),
        "q_input": q_input.astype(i32),
        "level_pure": level_pure,
    }
