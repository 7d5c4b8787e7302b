"""Synthetic games of n rational players with general-sum payoffs (Definition 1 of Section 2.1
with I+ = {1, ..., n}; Section 3.1 gives the payoff matrix one column per rational player).

* ``normal_form_n``: an n-player normal-form game written as a tree: player 1 moves at the
  root, player 2 moves without seeing it, ..., player n last; the terminal reached by actions
  (a_1, ..., a_n) pays payoff[a_1, ..., a_n, i - 1] to player i;
* ``kuhn3``: three-player Kuhn poker (the shape of the three-player Kuhn row of the paper's
  game table): four ranks, one card to each player, ante 1, one betting round in which the
  players act in seat order with check or bet 1 until someone bets, after which every other
  player, in seat order from the bettor, calls or folds; the highest rank among the players
  still in takes the pot. Zero-sum (the payoffs of a terminal add up to 0);
* ``with_silent_players``: a two-player zero-sum game's tree with its payoffs as the columns
  (u_1, -u_1) and one seeded column per extra player who owns no infoset (a rational player
  who never moves: only the payoff recurrence carries that player's column);
* ``random_game_n``: chance deals every player a private type (one joint chance node), then a
  random public tree of player, chance and terminal nodes follows; an infoset is (player, own
  type, public history), so the game has perfect recall and level-pure infosets. Every
  player's payoff is an independent multiple of 1/64 in [-1, 1], so the game is general-sum
  and every payoff is exact in fp32.
"""
from __future__ import annotations

import itertools

import numpy as np

from .small import _grid
from .tuple import Game, GameBuilder


def normal_form_n(payoff, name: str = "normal_form") -> Game:
    """payoff: array of shape (k_1, ..., k_n, n)."""
    a = np.asarray(payoff, dtype=np.float64)
    n = a.ndim - 1
    assert n >= 2 and a.shape[-1] == n
    ks = a.shape[:-1]
    b = GameBuilder(name)
    hs = [b.infoset_id(("move", i), i + 1, ks[i]) for i in range(n)]

    def walk(v, i, acts):
        if i == n:
            b.terminal_vec(v, a[tuple(acts)])
            return
        b.decide(v, hs[i])
        for x in range(ks[i]):
            walk(b.node(v, x), i + 1, acts + [x])

    walk(b.node(-1, -1), 0, [])
    return b.build(kind="normal_form_n", players=n)


def kuhn3(ranks: int = 4, deal: str = "sequential") -> Game:
    """Three-player Kuhn poker over `ranks` ranks (one card each, ranks >= 3).
    ``deal='sequential'``: a chance node for player 1's card, then one for player 2's, then one
    for player 3's (uniform over the cards left); ``'joint'``: one chance node over the ordered
    deals."""
    n = 3
    b = GameBuilder(f"kuhn3_{ranks}_{deal}")
    root = b.node(-1, -1)

    def settle(cards, put, folded):
        pot = sum(put)
        live = [i for i in range(n) if not folded[i]]
        win = max(live, key=lambda i: cards[i])
        return [(pot if i == win else 0.0) - put[i] for i in range(n)]

    def walk(v, cards, hist, put, folded, bettor, to_act):
        # to_act: the seats still to act, in order
        if not to_act:
            b.terminal_vec(v, settle(cards, put, folded))
            return
        seat = to_act[0]
        b.decide(v, b.infoset_id((seat, cards[seat], hist), seat + 1, 2))
        if bettor < 0:
            # action 0 check, 1 bet
            walk(b.node(v, 0), cards, hist + ("k",), put, folded, -1, to_act[1:])
            put2 = list(put)
            put2[seat] += 1
            others = [(seat + j) % n for j in range(1, n)]
            walk(b.node(v, 1), cards, hist + ("b",), put2, folded, seat, others)
        else:
            # action 0 fold, 1 call
            f2 = list(folded)
            f2[seat] = True
            walk(b.node(v, 0), cards, hist + ("f",), put, f2, bettor, to_act[1:])
            put2 = list(put)
            put2[seat] += 1
            walk(b.node(v, 1), cards, hist + ("c",), put2, folded, bettor, to_act[1:])

    def start(v, cards):
        walk(v, cards, (), [1.0] * n, [False] * n, -1, list(range(n)))

    if deal == "joint":
        deals = list(itertools.permutations(range(ranks), n))
        b.decide(root, b.infoset_id(("deal",), 0, len(deals), [1.0 / len(deals)] * len(deals)))
        for a, cards in enumerate(deals):
            start(b.node(root, a), cards)
    elif deal == "sequential":
        def deal_to(v, cards):
            if len(cards) == n:
                start(v, tuple(cards))
                return
            left = [r for r in range(ranks) if r not in cards]
            b.decide(v, b.infoset_id(("deal", tuple(cards)), 0, len(left),
                                     [1.0 / len(left)] * len(left)))
            for a, r in enumerate(left):
                deal_to(b.node(v, a), cards + [r])

        deal_to(root, [])
    else:
        raise ValueError(deal)
    return b.build(kind="kuhn3", ranks=ranks, deal=deal, players=n)


def with_silent_players(game: Game, extra: int, seed: int) -> Game:
    """The tree of the two-player zero-sum ``game`` as a general-sum game of 2 + ``extra``
    players: columns u_1, -u_1, then ``extra`` columns of multiples of 1/64 in [-1, 1] at the
    terminals (0 at decision nodes). Players 3 .. 2 + extra own no infoset."""
    from dataclasses import replace
    rng = np.random.default_rng(seed)
    n = len(game.parent)
    term = game.node_infoset < 0
    cols = [game.payoff_u1, -game.payoff_u1]
    for _ in range(extra):
        cols.append(np.where(term, rng.integers(-64, 65, size=n) / 64.0, 0.0))
    meta = dict(game.meta, players=2 + extra)
    return replace(game, name=f"{game.name}_silent{extra}", payoff=np.stack(cols, axis=1),
                   payoff_u2=None, meta=meta)


def random_game_n(seed: int, n_players: int = 3, n_types: int = 2, depth: int = 4,
                  max_actions: int = 3, p_terminal: float = 0.25, p_chance: float = 0.15) -> Game:
    """Random general-sum game of n_players with private types and perfect recall."""
    rng = np.random.default_rng(seed)
    n = n_players
    b = GameBuilder(f"random_n{n}_{seed}")
    public: dict = {}

    def public_node(hist):
        if hist not in public:
            d = len(hist)
            if d >= depth or (d > 0 and rng.random() < p_terminal):
                public[hist] = ("T",)
            elif rng.random() < p_chance:
                k = int(rng.integers(2, max_actions + 1))
                public[hist] = ("C", k, _grid(rng, k))
            else:
                public[hist] = ("P", int(rng.integers(1, n + 1)),
                                int(rng.integers(1, max_actions + 1)))
        return public[hist]

    pay: dict = {}

    def payoff(hist, types):
        key = (hist, types)
        if key not in pay:
            pay[key] = [float(x) / 64.0 for x in rng.integers(-64, 65, size=n)]
        return pay[key]

    def walk(v, hist, types):
        node = public_node(hist)
        if node[0] == "T":
            b.terminal_vec(v, payoff(hist, types))
            return
        if node[0] == "C":
            _, k, probs = node
            b.decide(v, b.infoset_id(("C", hist), 0, k, probs))
        else:
            _, player, k = node
            b.decide(v, b.infoset_id((player, types[player - 1], hist), player, k))
        for a in range(node[-1] if node[0] == "P" else node[1]):
            walk(b.node(v, a), hist + (a,), types)

    root = b.node(-1, -1)
    combos = list(itertools.product(range(n_types), repeat=n))
    b.decide(root, b.infoset_id(("deal",), 0, len(combos), _grid(rng, len(combos))))
    for a, types in enumerate(combos):
        walk(b.node(root, a), (), types)
    return b.build(kind="random_n", seed=seed, players=n)
