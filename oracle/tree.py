"""The game tuple of Definition 1 (Section 2.1) as a tree with ordered children.

Test infrastructure (oracle): not part of the product path.

Input numbering is kept as is: node ids, infoset ids and the infoset-action
index q, which enumerates the rational-player infosets in increasing id order
and, inside each, the actions in index order (the set Q_+ of Section 2.1).
"""
from __future__ import annotations


class Tree:
    def __init__(self, game):
        n = game.n_nodes
        parent = game.parent.tolist()
        action = game.node_action.tolist()
        self.n = n
        self.parent = parent
        self.infoset = game.node_infoset.tolist()
        self.player = [int(p) for p in game.infoset_player.tolist()]
        self.nact = [int(k) for k in game.infoset_num_actions.tolist()]
        self.u1 = [float(x) for x in game.payoff_u1.tolist()]
        roots = [v for v in range(n) if parent[v] < 0]
        assert len(roots) == 1, "exactly one root"
        self.root = roots[0]
        self.children: list[list[int]] = [[] for _ in range(n)]
        slots: list[dict] = [dict() for _ in range(n)]
        for v in range(n):
            p = parent[v]
            if p >= 0:
                assert action[v] not in slots[p], "f_a must be a bijection"
                slots[p][action[v]] = v
        for v in range(n):
            if slots[v]:
                k = len(slots[v])
                assert sorted(slots[v]) == list(range(k)), "actions must be 0..k-1"
                self.children[v] = [slots[v][a] for a in range(k)]
                assert self.infoset[v] >= 0 and self.nact[self.infoset[v]] == k
            else:
                assert self.infoset[v] < 0, "a decision node needs children"
        # sigma_0 per chance infoset
        self.sigma0: dict[int, list[float]] = {}
        pos = 0
        cp = [float(x) for x in game.chance_prob.tolist()]
        for h, pl in enumerate(self.player):
            if pl == 0:
                self.sigma0[h] = cp[pos:pos + self.nact[h]]
                pos += self.nact[h]
        assert pos == len(cp)
        # Q_+ : infoset-action pairs of rational players
        self.qoff: dict[int, int] = {}
        q = 0
        for h, pl in enumerate(self.player):
            if pl != 0:
                self.qoff[h] = q
                q += self.nact[h]
        self.Q = q
        self.rational = [h for h, pl in enumerate(self.player) if pl != 0]
        # members of each infoset and node depths
        self.members: dict[int, list[int]] = {h: [] for h in range(len(self.player))}
        self.depth = [0] * n
        order = [self.root]
        for v in order:
            for c in self.children[v]:
                self.depth[c] = self.depth[v] + 1
                order.append(c)
        self.bfs = order
        for v in range(n):
            if self.infoset[v] >= 0:
                self.members[self.infoset[v]].append(v)

    def is_terminal(self, v: int) -> bool:
        return not self.children[v]

    def node_player(self, v: int) -> int:
        return -1 if not self.children[v] else self.player[self.infoset[v]]

    def q_pairs(self):
        """(h, a) for q = 0..Q-1."""
        out = []
        for h in self.rational:
            out.extend((h, a) for a in range(self.nact[h]))
        return out
