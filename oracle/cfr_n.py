"""Recursive FP64 CFR for games of n rational players with general-sum payoffs.

Test infrastructure (oracle): not part of the product path.

Section 3.1 of the paper writes the game for any set I+ of rational players: the payoff matrix
and the expected-payoff recurrence carry one column per rational player, and the excepted
reach of a node for player i is the product of the edge probabilities of everyone but i
(chance included). Nothing in the iteration needs zero sum; only the exploitability of
Section 2.2 does, so it is not defined here.

State and strategies are those of the two-player oracle (``oracle.cfr``): T, R[q], S[q] over
the rational infosets' pairs in input order, regret matching with the exact-zero uniform
fallback, and the same three update rules (vanilla, CFR+ with linear averaging, discounted).
One iteration with the simultaneous schedule:

1. sigma = regret matching of R; chance plays sigma_0.
2. A recursive walk carries the reach vector (pi_1, ..., pi_n, pi_c) and returns the node's
   payoff vector u(d) in R^n (Eq. expected_payoff per player: the sigma-weighted sum of the
   children's vectors, the terminal's payoffs at a leaf). At a node d of player i in infoset
   h, with child vectors w_a and node vector u:
       r~(h, a) += pi_{-i}(d) * (w_a[i] - u[i]),  pi_{-i}(d) = pi_c * prod_{j != i} pi_j
       pibar(h)  += pi_i(d)
   (the multiplied-out instantaneous regret and the own-reach player reach, as in the
   two-player oracle, where u_2 = -u_1 turns w_a[2] - u[2] into -(w_a[1] - u[1])).
3.-5. The regret and average updates and T += 1, as in ``oracle.cfr.iterate``.

The alternating schedule (``iterate_alternating``) makes a pass per player in seat order, each
updating that player's infosets only, under the strategies the earlier passes produced.
"""
from __future__ import annotations

from .cfr import (CFR_PLUS, DCFR, DCFR_DEFAULT, VANILLA, State, current_strategy,
                  dcfr_factors)
from .tree import Tree


class TreeN(Tree):
    """Tree with one payoff per rational player at each terminal (game.payoff[v, i - 1])."""

    def __init__(self, game):
        super().__init__(game)
        assert game.payoff is not None, "a general-sum game needs its payoff matrix"
        self.n_players = int(game.payoff.shape[1])
        self.u = [[float(x) for x in row] for row in game.payoff.tolist()]
        assert all(0 <= p <= self.n_players for p in self.player)


def iterate(tree: TreeN, state: State, variant: str = VANILLA, record: bool = False,
            dcfr=DCFR_DEFAULT, players=None, count: bool = True):
    """One simultaneous iteration. Returns (new_state, info) with sigma, r~, pibar, the root's
    payoff vector and, if ``record``, per node its payoff vector and reach vector. ``players``:
    whose infosets the call updates (default all; the others keep R and S); ``count``: whether
    it ends the iteration (T += 1)."""
    n_pl = tree.n_players
    sigma = current_strategy(tree, state.R)
    rt = [0.0] * tree.Q
    pibar = {h: 0.0 for h in tree.rational}
    node_u = [None] * tree.n if record else None
    node_reach = [None] * tree.n if record else None

    def walk(v, reach):
        # reach[0 .. n_pl - 1]: the players' products; reach[n_pl]: chance's
        if record:
            node_reach[v] = tuple(reach)
        ch = tree.children[v]
        if not ch:
            u = list(tree.u[v])
            if record:
                node_u[v] = u
            return u
        h = tree.infoset[v]
        pl = tree.player[h]
        if pl == 0:
            probs = tree.sigma0[h]
            slot = n_pl
        else:
            o = tree.qoff[h]
            probs = sigma[o:o + len(ch)]
            slot = pl - 1
        w = []
        for a, c in enumerate(ch):
            r2 = list(reach)
            r2[slot] *= probs[a]
            w.append(walk(c, r2))
        u = [0.0] * n_pl
        for a in range(len(ch)):
            for i in range(n_pl):
                u[i] += probs[a] * w[a][i]
        if pl != 0:
            i = pl - 1
            cf = reach[n_pl]
            for j in range(n_pl):
                if j != i:
                    cf *= reach[j]
            o = tree.qoff[h]
            for a in range(len(ch)):
                rt[o + a] += cf * (w[a][i] - u[i])
            pibar[h] += reach[i]
        if record:
            node_u[v] = u
        return u

    root_u = walk(tree.root, [1.0] * (n_pl + 1))
    R, S = list(state.R), list(state.S)
    wt = float(state.T + 1) if variant == CFR_PLUS else 1.0
    if variant == DCFR:
        d_pos, d_neg, d_avg = dcfr_factors(state.T + 1, dcfr)
    for h in tree.rational:
        if players is not None and tree.player[h] not in players:
            continue
        o, k = tree.qoff[h], tree.nact[h]
        for a in range(k):
            q = o + a
            if variant == VANILLA:
                R[q] += rt[q]
            elif variant == CFR_PLUS:
                R[q] = max(R[q] + rt[q], 0.0)
            elif variant == DCFR:
                x = R[q] + rt[q]
                R[q] = x * (d_pos if x > 0.0 else d_neg)
            else:
                raise ValueError(variant)
            S[q] += wt * pibar[h] * sigma[q]
            if variant == DCFR:
                S[q] *= d_avg
    info = {"sigma": sigma, "rtilde": rt, "pibar": pibar, "root_value": root_u,
            "next_sigma": current_strategy(tree, R)}
    if record:
        info["node_u"] = node_u
        info["node_reach"] = node_reach
    return State(state.T + (1 if count else 0), R, S), info


def iterate_alternating(tree: TreeN, state: State, variant: str = VANILLA, dcfr=DCFR_DEFAULT):
    """One iteration of the alternating schedule for n players: a pass per player in seat order,
    each updating only that player's infosets and seeing the strategies the earlier passes
    produced, all with t = T + 1 (the two-player schedule of ``oracle.cfr`` extended to every
    rational player). Returns (new_state, info of the last pass)."""
    st = state
    info = None
    for i in range(1, tree.n_players + 1):
        st, info = iterate(tree, st, variant, dcfr=dcfr, players=(i,),
                           count=(i == tree.n_players))
    return st, info


def solve(tree: TreeN, iterations: int, variant: str = VANILLA, state: State | None = None,
          dcfr=DCFR_DEFAULT) -> State:
    st = state.copy() if state is not None else State.zeros(tree)
    for _ in range(iterations):
        st, _info = iterate(tree, st, variant, dcfr=dcfr)
    return st


def expected_values(tree: TreeN, profile: list) -> list:
    """Each rational player's expected payoff under `profile` (over Q_+), summed over the
    terminals: the probability of reaching t times u(t, i) (Section 2.2, per player)."""
    out = [0.0] * tree.n_players
    stack = [(tree.root, 1.0)]
    while stack:
        v, p = stack.pop()
        ch = tree.children[v]
        if not ch:
            for i in range(tree.n_players):
                out[i] += p * tree.u[v][i]
            continue
        h = tree.infoset[v]
        if tree.player[h] == 0:
            probs = tree.sigma0[h]
        else:
            o = tree.qoff[h]
            probs = profile[o:o + len(ch)]
        for a, c in enumerate(ch):
            stack.append((c, p * probs[a]))
    return out
