"""Sequence-form linear program for two-player zero-sum games.

Test infrastructure (oracle): not part of the product path.

The value v* = max_x min_y x^T A y over realization plans (Koller, Megiddo and
von Stengel): x >= 0 with E x = e for player 1, y >= 0 with F y = f for player
2, where each player's sequences are the empty sequence and its (infoset,
action) pairs, row 0 fixes the empty sequence to 1, and each infoset's row says
that its actions' realizations sum to the realization of its parent sequence.
A[s1, s2] sums chance-reach x u_1 over the terminals whose last player-1 and
player-2 sequences are s1 and s2. Dualising the inner minimisation gives
    max_{x >= 0, z} f^T z  s.t.  E x = e,  F^T z <= A^T x
and symmetrically for player 2. Solved with scipy's HiGHS.

This is the independent check on the CFR oracle's convergence target (the
paper fixes the game value only through the Nash definition of Section 2.2).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog
from scipy.sparse import lil_matrix

from .tree import Tree


def _sequences(tree: Tree):
    """Per player: sequence index of each (h, a), parent sequence of each infoset,
    and the (last P1 sequence, last P2 sequence, chance reach) of each terminal."""
    seq = {1: {}, 2: {}}
    nseq = {1: 1, 2: 1}
    for h in tree.rational:
        p = tree.player[h]
        for a in range(tree.nact[h]):
            seq[p][(h, a)] = nseq[p]
            nseq[p] += 1
    parent_seq = {}
    leaves = []
    stack = [(tree.root, 0, 0, 1.0)]
    while stack:
        v, s1, s2, pc = stack.pop()
        ch = tree.children[v]
        if not ch:
            leaves.append((s1, s2, pc, tree.u1[v]))
            continue
        h = tree.infoset[v]
        pl = tree.player[h]
        if pl != 0:
            own = s1 if pl == 1 else s2
            if h in parent_seq:
                assert parent_seq[h] == own, "game lacks perfect recall"
            parent_seq[h] = own
        for a, c in enumerate(ch):
            if pl == 0:
                stack.append((c, s1, s2, pc * tree.sigma0[h][a]))
            elif pl == 1:
                stack.append((c, seq[1][(h, a)], s2, pc))
            else:
                stack.append((c, s1, seq[2][(h, a)], pc))
    return seq, nseq, parent_seq, leaves


def _constraints(tree, seq, nseq, parent_seq, p):
    hs = [h for h in tree.rational if tree.player[h] == p]
    E = lil_matrix((1 + len(hs), nseq[p]))
    E[0, 0] = 1.0
    for r, h in enumerate(hs, start=1):
        E[r, parent_seq.get(h, 0)] = -1.0
        for a in range(tree.nact[h]):
            E[r, seq[p][(h, a)]] = 1.0
    e = np.zeros(1 + len(hs))
    e[0] = 1.0
    return E.tocsr(), e, hs


def solve(tree: Tree):
    """Returns (value, profile) where profile is an equilibrium over Q_+."""
    seq, nseq, parent_seq, leaves = _sequences(tree)
    A = np.zeros((nseq[1], nseq[2]))
    for s1, s2, pc, u in leaves:
        A[s1, s2] += pc * u
    E, e, h1 = _constraints(tree, seq, nseq, parent_seq, 1)
    F, f, h2 = _constraints(tree, seq, nseq, parent_seq, 2)
    n1, n2 = nseq[1], nseq[2]
    m1, m2 = E.shape[0], F.shape[0]

    # player 1: variables [x (n1), z (m2)]; maximise f^T z
    c = np.concatenate([np.zeros(n1), -f])
    A_ub = np.hstack([-A.T, F.T.toarray()])
    A_eq = np.hstack([E.toarray(), np.zeros((m1, m2))])
    bounds = [(0, None)] * n1 + [(None, None)] * m2
    r1 = linprog(c, A_ub=A_ub, b_ub=np.zeros(n2), A_eq=A_eq, b_eq=e, bounds=bounds,
                 method="highs")
    assert r1.status == 0, r1.message
    x = r1.x[:n1]
    value = float(f @ r1.x[n1:])

    # player 2: variables [y (n2), w (m1)]; minimise e^T w s.t. A y - E^T w <= 0
    c2 = np.concatenate([np.zeros(n2), e])
    A_ub2 = np.hstack([A, -E.T.toarray()])
    A_eq2 = np.hstack([F.toarray(), np.zeros((m2, m1))])
    bounds2 = [(0, None)] * n2 + [(None, None)] * m1
    r2 = linprog(c2, A_ub=A_ub2, b_ub=np.zeros(n1), A_eq=A_eq2, b_eq=f, bounds=bounds2,
                 method="highs")
    assert r2.status == 0, r2.message
    y = r2.x[:n2]

    profile = [0.0] * tree.Q
    for p, plan, hs in ((1, x, h1), (2, y, h2)):
        for h in hs:
            o, k = tree.qoff[h], tree.nact[h]
            par = plan[parent_seq.get(h, 0)]
            vals = [max(plan[seq[p][(h, a)]], 0.0) for a in range(k)]
            tot = sum(vals)
            if par > 1e-12 and tot > 0.0:
                profile[o:o + k] = [v / tot for v in vals]
            else:
                profile[o:o + k] = [1.0 / k] * k
    return value, profile
