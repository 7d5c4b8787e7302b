"""One infoset at a time: the regret and average-strategy update of a single
infoset of a game too large for the recursive oracle's full walk.

Test infrastructure (oracle): not part of the product path.

For an infoset h of player i with members d, the definitions of Section 2.3
give, for one iteration from state (T, R, S) with sigma = regret matching of R:
    r~(h, a)   = sum_d pi_{-i}(d) * sgn_i * (u(child(d, a)) - u(d))
    pibar(h)   = sum_d pi_i(d)
    R'(h, a)   = R + r~ (vanilla) or max(R + r~, 0) (CFR+)
    S'(h, a)   = S + w * pibar(h) * sigma(h, a),  w = 1 or T + 1
Reach probabilities are products along the root-to-node path (Section 2.2);
u is the expected payoff of Eq. (expected_payoff) by a recursive walk of the
member's subtree. Only the members' paths and subtrees are visited, so deep
infosets of a 2e7-node game cost milliseconds. For shallow infosets, whose
subtrees hold most of the game, all_values() gives every node's u in one
vectorised sweep (a few seconds at 2e7 nodes), passed to update() as values.
"""
from __future__ import annotations

import numpy as np


class InfosetSampler:
    def __init__(self, game):
        self.g = game
        n = game.n_nodes
        parent = game.parent.astype(np.int64)
        action = game.node_action.astype(np.int64)
        nonroot = np.flatnonzero(parent >= 0)
        self.order = nonroot[np.lexsort((action[nonroot], parent[nonroot]))]
        cnt = np.bincount(parent[nonroot], minlength=n)
        self.ptr = np.concatenate([[0], np.cumsum(cnt)])
        self.parent = parent
        self.action = action
        nact = game.infoset_num_actions.astype(np.int64)
        pl = game.infoset_player.astype(np.int64)
        is_ch = pl == 0
        self.coff = np.concatenate([[0], np.cumsum(np.where(is_ch, nact, 0))])[:-1]
        self.qoff = np.concatenate([[0], np.cumsum(np.where(is_ch, 0, nact))])[:-1]
        self.nact = nact
        self.player = pl
        self._members = None

    def members(self, h: int) -> np.ndarray:
        return np.flatnonzero(self.g.node_infoset == h)

    def children(self, v: int) -> list:
        return [int(x) for x in self.order[self.ptr[v]:self.ptr[v + 1]]]

    def strategy(self, R, h: int) -> list:
        o, k = int(self.qoff[h]), int(self.nact[h])
        r = [float(x) for x in R[o:o + k]]
        pos = [x if x > 0.0 else 0.0 for x in r]
        tot = sum(pos)
        return [x / tot for x in pos] if tot > 0.0 else [1.0 / k] * k

    def edge_prob(self, R, p: int, a: int) -> float:
        h = int(self.g.node_infoset[p])
        if self.player[h] == 0:
            return float(self.g.chance_prob[self.coff[h] + a])
        return self.strategy(R, h)[a]

    def reach(self, R, v: int):
        """(pi_1, pi_2, pi_c) of node v: products of edge probabilities by who acted."""
        prods = [1.0, 1.0, 1.0]          # chance, player 1, player 2
        x = v
        while self.parent[x] >= 0:
            p = int(self.parent[x])
            who = int(self.player[self.g.node_infoset[p]])
            prods[who] *= self.edge_prob(R, p, int(self.action[x]))
            x = p
        return prods[1], prods[2], prods[0]

    def value(self, R, v: int) -> float:
        kids = self.children(v)
        if not kids:
            return float(self.g.payoff_u1[v])
        return sum(self.edge_prob(R, v, a) * self.value(R, c) for a, c in enumerate(kids))

    def edge_probs(self, R) -> np.ndarray:
        """Probability of the edge into every node (1 at the root): sigma_0 below chance nodes,
        regret matching of R below player nodes (uniform where the positive regrets sum to 0)."""
        g = self.g
        Rf = np.asarray(R, dtype=np.float64)
        rat = np.flatnonzero(self.player != 0)
        pos = np.maximum(Rf, 0.0)
        sigma = np.empty_like(Rf)
        for h in rat:  # per infoset, as Eq. (next_strategy_profile) states it
            o, k = int(self.qoff[h]), int(self.nact[h])
            tot = pos[o:o + k].sum()
            sigma[o:o + k] = pos[o:o + k] / tot if tot > 0.0 else 1.0 / k
        prob = np.ones(g.n_nodes)
        nonroot = np.flatnonzero(self.parent >= 0)
        hp = g.node_infoset[self.parent[nonroot]].astype(np.int64)
        a = self.action[nonroot]
        ch = self.player[hp] == 0
        prob[nonroot[ch]] = g.chance_prob[self.coff[hp[ch]] + a[ch]]
        prob[nonroot[~ch]] = sigma[self.qoff[hp[~ch]] + a[~ch]]
        return prob

    def all_values(self, R) -> np.ndarray:
        """Expected payoff u_1 of every node (Eq. expected_payoff) in one sweep: a node's value
        is the probability-weighted sum of its children's values, and repeating that step as
        many times as the tree is deep makes every value final (payoffs at terminals)."""
        g = self.g
        prob = self.edge_probs(R)
        internal = np.flatnonzero(np.diff(self.ptr) > 0)
        u = np.where(np.diff(self.ptr) > 0, 0.0, g.payoff_u1.astype(np.float64))
        depth = 0
        x = np.flatnonzero(self.parent < 0)
        while x.size:  # tree depth by levels from the root
            x = np.concatenate([self.order[self.ptr[v]:self.ptr[v + 1]] for v in x]) \
                if x.size < 64 else self._kids(x)
            depth += 1
        for _ in range(depth):
            contrib = prob[self.order] * u[self.order]
            u[internal] = np.add.reduceat(contrib, self.ptr[internal])
        return u

    def _kids(self, x: np.ndarray) -> np.ndarray:
        cnt = self.ptr[x + 1] - self.ptr[x]
        starts = np.repeat(self.ptr[x], cnt)
        offs = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        return self.order[starts + offs]

    def update(self, R, S, T: int, h: int, variant: str = "vanilla", dcfr=(1.5, 0.0, 2.0),
               values=None) -> dict:
        i = int(self.player[h])
        k = int(self.nact[h])
        o = int(self.qoff[h])
        sigma = self.strategy(R, h)
        rt = [0.0] * k
        scale = [0.0] * k
        pibar = 0.0
        for d in self.members(h):
            d = int(d)
            p1, p2, pc = self.reach(R, d)
            kids = self.children(d)
            w = [float(values[c]) if values is not None else self.value(R, c) for c in kids]
            u = sum(sigma[a] * w[a] for a in range(k))
            cf = (p2 if i == 1 else p1) * pc
            sgn = 1.0 if i == 1 else -1.0
            for a in range(k):
                rt[a] += cf * sgn * (w[a] - u)
                scale[a] += abs(cf) * (abs(w[a]) + abs(u))
            pibar += p1 if i == 1 else p2
        wt = float(T + 1) if variant == "cfr+" else 1.0
        if variant == "dcfr":  # the discount factors of iteration T + 1 (see oracle.cfr)
            t = float(T + 1)
            ta, tb = t ** dcfr[0], t ** dcfr[1]
            d_pos, d_neg, d_avg = ta / (ta + 1.0), tb / (tb + 1.0), (t / (t + 1.0)) ** dcfr[2]
        Rn, Sn = [], []
        for a in range(k):
            r = float(R[o + a]) + rt[a]
            sn = float(S[o + a]) + wt * pibar * sigma[a]
            if variant == "cfr+":
                r = max(r, 0.0)
            elif variant == "dcfr":
                r *= d_pos if r > 0.0 else d_neg
                sn *= d_avg
            elif variant != "vanilla":
                raise ValueError(variant)
            Rn.append(r)
            Sn.append(sn)
        return {"q": list(range(o, o + k)), "rtilde": rt, "rtilde_scale": scale, "pibar": pibar,
                "R": Rn, "S": Sn, "sigma": sigma}
