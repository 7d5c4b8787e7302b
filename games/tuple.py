"""The finite extensive-form game of Definition 1 (Section 2.1) as flat arrays.

A game is the tuple <T, H, f_h, A, f_a, I, f_i, sigma_0, u>:

* the tree T is the parent function ``parent`` (-1 at the unique root v_0);
  a node with no children is terminal;
* the information partition f_h is ``node_infoset`` (-1 at terminals);
* the action partition f_a is ``node_action``: the index, inside A(f_h(parent)),
  of the edge that leads into the node (-1 at the root), so that for every
  decision node d the map from its children to A(f_h(d)) is a bijection onto
  ``range(infoset_num_actions[f_h(d)])``;
* the player partition f_i is ``infoset_player`` (0 = chance, 1, 2);
* sigma_0 is ``chance_prob``: the chance infosets in increasing id order, each
  contributing ``infoset_num_actions[h]`` probabilities in action order;
* the utility u is ``payoff_u1`` (player 1) and, optionally, ``payoff_u2``;
  only terminal entries are meaningful.

Node ids and infoset ids are arbitrary; the consumers canonicalise them.
This module holds input plumbing only: no part of the regret computation.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Game:
    name: str
    parent: np.ndarray
    node_infoset: np.ndarray
    node_action: np.ndarray
    infoset_player: np.ndarray
    infoset_num_actions: np.ndarray
    chance_prob: np.ndarray
    payoff_u1: np.ndarray
    payoff_u2: np.ndarray | None = None
    meta: dict = field(default_factory=dict)
    # general-sum games of n rational players: u(t, i) at payoff[t, i - 1] (terminals; 0
    # elsewhere), payoff_u1 its first column and payoff_u2 None
    payoff: np.ndarray | None = None

    @property
    def n_players(self) -> int:
        return 2 if self.payoff is None else int(self.payoff.shape[1])

    @property
    def n_nodes(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_infosets(self) -> int:
        return int(self.infoset_player.shape[0])

    def counts(self) -> dict:
        """Sizes in the columns of the paper's game-properties table (Appendix)."""
        is_term = self.node_infoset < 0
        rational = self.infoset_player != 0
        return {
            "nodes": self.n_nodes,
            "terminals": int(is_term.sum()),
            "infosets": int(rational.sum()),
            "infoset_actions": int(self.infoset_num_actions[rational].sum()),
        }

    def permuted(self, seed: int) -> "Game":
        """The same game with node ids shuffled (root moved too) and infosets relabelled.

        Used to check that consumers do not depend on the input's numbering.
        """
        rng = np.random.default_rng(seed)
        n = self.n_nodes
        perm = rng.permutation(n)            # new id of old node i is perm[i]
        inv = np.empty(n, dtype=np.int64)
        inv[perm] = np.arange(n)
        hperm = rng.permutation(self.n_infosets)
        hinv = np.empty_like(hperm)
        hinv[hperm] = np.arange(self.n_infosets)
        old_parent = self.parent[inv]
        parent = np.where(old_parent < 0, -1, perm[np.maximum(old_parent, 0)]).astype(np.int32)
        old_h = self.node_infoset[inv]
        node_infoset = np.where(old_h < 0, -1, hperm[np.maximum(old_h, 0)]).astype(np.int32)
        # chance probabilities are packed in infoset-id order: repack
        offs = {}
        pos = 0
        for h in range(self.n_infosets):
            if self.infoset_player[h] == 0:
                k = int(self.infoset_num_actions[h])
                offs[h] = self.chance_prob[pos:pos + k]
                pos += k
        chance = [offs[int(hinv[h_new])] for h_new in range(self.n_infosets)
                  if self.infoset_player[hinv[h_new]] == 0]
        return Game(
            name=self.name + f"/perm{seed}",
            parent=parent,
            node_infoset=node_infoset,
            node_action=self.node_action[inv].astype(np.int32),
            infoset_player=self.infoset_player[hinv].astype(np.int8),
            infoset_num_actions=self.infoset_num_actions[hinv].astype(np.int32),
            chance_prob=(np.concatenate(chance) if chance else np.zeros(0)).astype(np.float64),
            payoff_u1=self.payoff_u1[inv].astype(np.float64),
            payoff_u2=None if self.payoff_u2 is None else self.payoff_u2[inv].astype(np.float64),
            meta=dict(self.meta),
            payoff=None if self.payoff is None else self.payoff[inv].astype(np.float64),
        )


class GameBuilder:
    """Incremental construction of a small game, one node at a time."""

    def __init__(self, name: str):
        self.name = name
        self.parent: list[int] = []
        self.infoset: list[int] = []
        self.action: list[int] = []
        self.u1: list[float] = []
        self.keys: dict = {}
        self.iplayer: list[int] = []
        self.inact: list[int] = []
        self.cprob: dict[int, list[float]] = {}
        self.uvec: dict[int, list[float]] = {}  # general-sum terminals: one payoff per player

    def node(self, parent: int, action: int) -> int:
        self.parent.append(parent)
        self.infoset.append(-1)
        self.action.append(action)
        self.u1.append(0.0)
        return len(self.parent) - 1

    def infoset_id(self, key, player: int, num_actions: int, probs=None) -> int:
        h = self.keys.get(key)
        if h is None:
            h = len(self.iplayer)
            self.keys[key] = h
            self.iplayer.append(player)
            self.inact.append(num_actions)
            if player == 0:
                assert probs is not None and len(probs) == num_actions
                self.cprob[h] = [float(p) for p in probs]
        else:
            assert self.iplayer[h] == player and self.inact[h] == num_actions, key
        return h

    def decide(self, v: int, h: int) -> None:
        self.infoset[v] = h

    def terminal(self, v: int, u1: float) -> None:
        self.u1[v] = float(u1)

    def terminal_vec(self, v: int, u) -> None:
        """A terminal of a general-sum game: u[i - 1] is player i's payoff."""
        self.uvec[v] = [float(x) for x in u]
        self.u1[v] = float(u[0])

    def build(self, **meta) -> Game:
        chance = [self.cprob[h] for h in range(len(self.iplayer)) if self.iplayer[h] == 0]
        flat = [p for ps in chance for p in ps]
        u1 = np.asarray(self.u1, dtype=np.float64)
        if self.uvec:
            n_players = len(next(iter(self.uvec.values())))
            pay = np.zeros((len(self.parent), n_players), dtype=np.float64)
            for v, u in self.uvec.items():
                assert len(u) == n_players
                pay[v] = u
            return Game(
                name=self.name,
                parent=np.asarray(self.parent, dtype=np.int32),
                node_infoset=np.asarray(self.infoset, dtype=np.int32),
                node_action=np.asarray(self.action, dtype=np.int32),
                infoset_player=np.asarray(self.iplayer, dtype=np.int8),
                infoset_num_actions=np.asarray(self.inact, dtype=np.int32),
                chance_prob=np.asarray(flat, dtype=np.float64),
                payoff_u1=pay[:, 0].copy(),
                payoff_u2=None,
                meta=meta,
                payoff=pay,
            )
        return Game(
            name=self.name,
            parent=np.asarray(self.parent, dtype=np.int32),
            node_infoset=np.asarray(self.infoset, dtype=np.int32),
            node_action=np.asarray(self.action, dtype=np.int32),
            infoset_player=np.asarray(self.iplayer, dtype=np.int8),
            infoset_num_actions=np.asarray(self.inact, dtype=np.int32),
            chance_prob=np.asarray(flat, dtype=np.float64),
            payoff_u1=u1,
            payoff_u2=-u1,
            meta=meta,
        )
