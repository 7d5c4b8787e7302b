"""Small synthetic games built node by node (Definition 1, Section 2.1).

* ``matrix_game``: a two-player normal-form game written as a one-level tree
  (player 1 moves, player 2 moves without seeing it);
* ``rock_paper_scissors``: the 3x3 instance of the above;
* ``kuhn_like``: a Kuhn-shaped poker with ``ranks`` private ranks, pass/bet,
  ante 1 and bet 1 (the shape of the paper's kuhn_poker row);
* ``leduc_like``: a two-round poker with ranks x suits cards, fold/call/raise,
  at most ``cap`` raises per round, raise sizes per round, and one public card
  between the rounds (the shape of the paper's leduc_poker row);
* ``random_game``: random private types dealt by chance, followed by a random
  public tree of player and chance nodes; an infoset is (player, own type,
  public history), so the game has perfect recall and level-pure infosets.

Common poker readings: players alternate with player 1 first in every round; a
round ends on a call of a bet or on check-check; fold is legal only when
facing a bet; at showdown the higher hand wins the opponent's commitment and
equal hands split.
"""
from __future__ import annotations

import numpy as np

from .tuple import Game, GameBuilder


def matrix_game(payoff, name: str = "matrix") -> Game:
    """Player 1 picks a row, player 2 a column without seeing it; u1 = payoff[row][col]."""
    a = np.asarray(payoff, dtype=np.float64)
    m, n = a.shape
    b = GameBuilder(name)
    root = b.node(-1, -1)
    b.decide(root, b.infoset_id(("row",), 1, m))
    hc = b.infoset_id(("col",), 2, n)
    for i in range(m):
        v = b.node(root, i)
        b.decide(v, hc)
        for j in range(n):
            t = b.node(v, j)
            b.terminal(t, a[i, j])
    return b.build(kind="matrix", payoff=a.tolist())


def rock_paper_scissors() -> Game:
    # rows/cols: rock, paper, scissors
    return matrix_game([[0, -1, 1], [1, 0, -1], [-1, 1, 0]], name="rps")


# --------------------------------------------------------------------------- Kuhn-shaped

def kuhn_like(ranks: int = 3, deal: str = "joint") -> Game:
    """Kuhn-shaped poker. ``deal='joint'``: one chance node over the ordered deals;
    ``deal='sequential'``: a chance node for player 1's rank, then one for player 2's."""
    b = GameBuilder(f"kuhn{ranks}_{deal}")
    root = b.node(-1, -1)
    deals = [(r1, r2) for r1 in range(ranks) for r2 in range(ranks) if r1 != r2]

    def showdown(r1, r2, amount):
        return amount if r1 > r2 else -amount

    def betting(v, r1, r2, hist):
        if hist == "pp":
            b.terminal(v, showdown(r1, r2, 1)); return
        if hist in ("bb", "pbb"):
            b.terminal(v, showdown(r1, r2, 2)); return
        if hist == "bp":
            b.terminal(v, 1.0); return
        if hist == "pbp":
            b.terminal(v, -1.0); return
        player = 1 if hist in ("", "pb") else 2
        own = r1 if player == 1 else r2
        b.decide(v, b.infoset_id(("kuhn", player, own, hist), player, 2))
        for a, ch in enumerate("pb"):
            betting(b.node(v, a), r1, r2, hist + ch)

    if deal == "joint":
        b.decide(root, b.infoset_id(("deal",), 0, len(deals), [1.0 / len(deals)] * len(deals)))
        for a, (r1, r2) in enumerate(deals):
            betting(b.node(root, a), r1, r2, "")
    elif deal == "sequential":
        b.decide(root, b.infoset_id(("deal1",), 0, ranks, [1.0 / ranks] * ranks))
        for r1 in range(ranks):
            c = b.node(root, r1)
            others = [r for r in range(ranks) if r != r1]
            b.decide(c, b.infoset_id(("deal2", r1), 0, len(others), [1.0 / len(others)] * len(others)))
            for a, r2 in enumerate(others):
                betting(b.node(c, a), r1, r2, "")
    else:
        raise ValueError(deal)
    return b.build(kind="kuhn", ranks=ranks, deal=deal)


# --------------------------------------------------------------------------- Leduc-shaped

def leduc_like(ranks: int = 6, suits: int = 2, raise_sizes=(2, 4), cap: int = 2,
               deal: str = "joint") -> Game:
    """Two-round poker over ranks x suits cards (card id = rank * suits + suit).

    Round 1 (raise ``raise_sizes[0]``), one public card from the remaining deck,
    round 2 (raise ``raise_sizes[1]``). Ante 1. Pairing the public card's rank
    beats a high card; otherwise the higher rank wins; equal ranks split.
    Infosets are keyed by card identity and the public betting history.
    """
    ncards = ranks * suits
    b = GameBuilder(f"leduc{ranks}x{suits}_{deal}")
    root = b.node(-1, -1)

    def rank(c):
        return c // suits

    def showdown(c1card, c2card, pub, amount):
        r1, r2, rp = rank(c1card), rank(c2card), rank(pub)
        p1, p2 = r1 == rp, r2 == rp
        if p1 != p2:
            return amount if p1 else -amount
        if r1 == r2:
            return 0.0
        return amount if r1 > r2 else -amount

    def betting(v, rnd, c1, c2, hist, h1, cards, pub):
        player = 1 if len(hist) % 2 == 0 else 2
        facing = c1 != c2
        acts = (["f"] if facing else []) + ["c"] + (["r"] if hist.count("r") < cap else [])
        own = cards[0] if player == 1 else cards[1]
        key = ("leduc", player, own, h1, pub, hist)
        b.decide(v, b.infoset_id(key, player, len(acts)))
        for a, act in enumerate(acts):
            ch = b.node(v, a)
            if act == "f":
                b.terminal(ch, -c1 if player == 1 else c2)
            elif act == "c":
                if facing or player == 2:
                    m = max(c1, c2)
                    if rnd == 1:
                        public_card(ch, m, hist + "c", cards)
                    else:
                        b.terminal(ch, showdown(cards[0], cards[1], pub, m))
                else:
                    betting(ch, rnd, c1, c2, hist + "c", h1, cards, pub)
            else:
                m = max(c1, c2) + raise_sizes[rnd - 1]
                n1, n2 = (m, c2) if player == 1 else (c1, m)
                betting(ch, rnd, n1, n2, hist + "r", h1, cards, pub)

    def public_card(v, c, h1, cards):
        rest = [x for x in range(ncards) if x not in cards]
        b.decide(v, b.infoset_id(("pub", v), 0, len(rest), [1.0 / len(rest)] * len(rest)))
        for a, pc in enumerate(rest):
            betting(b.node(v, a), 2, c, c, "", h1, cards, pc)

    if deal == "joint":
        deals = [(x, y) for x in range(ncards) for y in range(ncards) if x != y]
        b.decide(root, b.infoset_id(("deal",), 0, len(deals), [1.0 / len(deals)] * len(deals)))
        for a, cards in enumerate(deals):
            betting(b.node(root, a), 1, 1, 1, "", None, cards, None)
    elif deal == "sequential":
        b.decide(root, b.infoset_id(("deal1",), 0, ncards, [1.0 / ncards] * ncards))
        for x in range(ncards):
            c = b.node(root, x)
            others = [y for y in range(ncards) if y != x]
            b.decide(c, b.infoset_id(("deal2", x), 0, len(others), [1.0 / len(others)] * len(others)))
            for a, y in enumerate(others):
                betting(b.node(c, a), 1, 1, 1, "", None, (x, y), None)
    else:
        raise ValueError(deal)
    return b.build(kind="leduc", ranks=ranks, suits=suits, deal=deal)


# --------------------------------------------------------------------------- random games

def _grid(rng, k: int, denom: int = 64) -> list[float]:
    """k probabilities that are multiples of 1/denom and sum to exactly 1 (some may be 0)."""
    cuts = np.sort(rng.integers(0, denom + 1, size=k - 1))
    parts = np.diff(np.concatenate([[0], cuts, [denom]]))
    return [float(p) / denom for p in parts]


def random_game(seed: int, n_types=(2, 2), depth: int = 4, max_actions: int = 3,
                p_terminal: float = 0.25, p_chance: float = 0.15, deal: str = "joint",
                allow_single_action: bool = True) -> Game:
    """Random two-player zero-sum game with perfect recall.

    Chance first deals private types (t1, t2) with random grid probabilities
    (``deal='joint'``: one chance node; ``'sequential'``: two levels; ``'none'``:
    no private information, a perfect-information game). A public tree follows:
    every public node is a player-1, player-2, chance or terminal node, with 1..
    ``max_actions`` actions. Payoffs are multiples of 1/64 in [-1, 1] and depend
    on the public leaf and both types, so every value is exact in fp32.
    """
    rng = np.random.default_rng(seed)
    b = GameBuilder(f"random{seed}_{deal}")
    t1n, t2n = n_types if deal != "none" else (1, 1)
    public: dict = {}

    def public_node(hist):
        if hist not in public:
            d = len(hist)
            if d >= depth or (d > 0 and rng.random() < p_terminal):
                public[hist] = ("T",)
            else:
                kind = "C" if rng.random() < p_chance else ("P1" if rng.random() < 0.5 else "P2")
                lo = 1 if (allow_single_action and kind != "C") else 2
                k = int(rng.integers(lo, max_actions + 1))
                if kind == "C":
                    public[hist] = ("C", k, _grid(rng, k))
                else:
                    public[hist] = (kind, k)
        return public[hist]

    payoff_cache: dict = {}

    def payoff(hist, t1, t2):
        key = (hist, t1, t2)
        if key not in payoff_cache:
            payoff_cache[key] = float(rng.integers(-64, 65)) / 64.0
        return payoff_cache[key]

    def walk(v, hist, t1, t2):
        node = public_node(hist)
        if node[0] == "T":
            b.terminal(v, payoff(hist, t1, t2))
            return
        if node[0] == "C":
            _, k, probs = node
            b.decide(v, b.infoset_id(("C", hist), 0, k, probs))
        else:
            player = 1 if node[0] == "P1" else 2
            own = t1 if player == 1 else t2
            b.decide(v, b.infoset_id((player, own, hist), player, node[1]))
        for a in range(node[1]):
            walk(b.node(v, a), hist + (a,), t1, t2)

    root = b.node(-1, -1)
    if deal == "none":
        walk(root, (), 0, 0)
    elif deal == "joint":
        probs = _grid(rng, t1n * t2n)
        b.decide(root, b.infoset_id(("deal",), 0, t1n * t2n, probs))
        for a in range(t1n * t2n):
            walk(b.node(root, a), (), a // t2n, a % t2n)
    elif deal == "sequential":
        b.decide(root, b.infoset_id(("deal1",), 0, t1n, _grid(rng, t1n)))
        for t1 in range(t1n):
            c = b.node(root, t1)
            b.decide(c, b.infoset_id(("deal2", t1), 0, t2n, _grid(rng, t2n)))
            for t2 in range(t2n):
                walk(b.node(c, t2), (), t1, t2)
    else:
        raise ValueError(deal)
    return b.build(kind="random", seed=seed, deal=deal)
