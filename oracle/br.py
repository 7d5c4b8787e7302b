"""Best response and exploitability (Section 2.2: Nash and epsilon-Nash).

Test infrastructure (oracle): not part of the product path.

The paper uses exploitability without defining it; it is read here as
NashConv / 2 with NashConv = BR_1 + BR_2, where BR_i is the best value player i
can reach against the others' strategies in the profile. In a two-player
zero-sum game u_1 + u_2 = 0, so NashConv is the sum of both players' gains from
deviating, and the profile is an epsilon-Nash equilibrium with
epsilon = NashConv (each gain is at most NashConv).

``best_response_value`` works for any perfect-recall game: at each infoset h of
the responding player it picks
    a*(h) = argmax_a  sum_{d in h} pi_{-i}(d) V(child(d, a))
(lowest action index on ties), where pi_{-i} is the product of chance and
opponent edge probabilities and V is the expected payoff of player i with the
opponent and chance playing the profile and player i playing a* below.
``brute_force_br`` enumerates every pure strategy of player i instead.
"""
from __future__ import annotations

import itertools

from .tree import Tree


def _utility(tree: Tree, v: int, i: int) -> float:
    return tree.u1[v] if i == 1 else -tree.u1[v]


def _probs(tree: Tree, profile: list, v: int) -> list:
    h = tree.infoset[v]
    if tree.player[h] == 0:
        return tree.sigma0[h]
    o = tree.qoff[h]
    return profile[o:o + tree.nact[h]]


def best_response(tree: Tree, profile: list, i: int):
    """Returns (value, {h: best action}) for player i against ``profile``."""
    n = tree.n
    reach = [0.0] * n          # pi_{-i}: chance and opponent probabilities only
    reach[tree.root] = 1.0
    for v in tree.bfs:
        ch = tree.children[v]
        if not ch:
            continue
        h = tree.infoset[v]
        if tree.player[h] == i:
            for c in ch:
                reach[c] = reach[v]
        else:
            probs = _probs(tree, profile, v)
            for a, c in enumerate(ch):
                reach[c] = reach[v] * probs[a]
    best: dict[int, int] = {}
    memo: dict[int, float] = {}

    def choose(h):
        if h not in best:
            k = tree.nact[h]
            totals = [0.0] * k
            for d in tree.members[h]:
                for a in range(k):
                    totals[a] += reach[d] * val(tree.children[d][a])
            a_star = 0
            for a in range(1, k):
                if totals[a] > totals[a_star]:
                    a_star = a
            best[h] = a_star
        return best[h]

    def val(v):
        if v in memo:
            return memo[v]
        ch = tree.children[v]
        if not ch:
            out = _utility(tree, v, i)
        else:
            h = tree.infoset[v]
            if tree.player[h] == i:
                out = val(ch[choose(h)])
            else:
                probs = _probs(tree, profile, v)
                out = 0.0
                for a, c in enumerate(ch):
                    out += probs[a] * val(c)
        memo[v] = out
        return out

    return val(tree.root), best


def best_response_value(tree: Tree, profile: list, i: int) -> float:
    return best_response(tree, profile, i)[0]


def exploitability(tree: Tree, profile: list) -> dict:
    """{'br1', 'br2', 'nash_conv', 'expl', 'value'} for a full profile over Q_+."""
    from .cfr import expected_value
    br1 = best_response_value(tree, profile, 1)
    br2 = best_response_value(tree, profile, 2)
    return {"br1": br1, "br2": br2, "nash_conv": br1 + br2, "expl": 0.5 * (br1 + br2),
            "value": expected_value(tree, profile)}


def brute_force_br(tree: Tree, profile: list, i: int) -> float:
    """Maximum over all pure strategies of player i of its expected payoff."""
    hs = [h for h in tree.rational if tree.player[h] == i]
    best = None
    for choice in itertools.product(*[range(tree.nact[h]) for h in hs]):
        prof = list(profile)
        for h, a in zip(hs, choice):
            o = tree.qoff[h]
            for b in range(tree.nact[h]):
                prof[o + b] = 1.0 if b == a else 0.0
        def val(v):
            ch = tree.children[v]
            if not ch:
                return _utility(tree, v, i)
            probs = _probs(tree, prof, v)
            return sum(probs[a] * val(c) for a, c in enumerate(ch))
        x = val(tree.root)
        best = x if best is None else max(best, x)
    return best
