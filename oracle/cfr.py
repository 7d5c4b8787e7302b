"""Recursive FP64 counterfactual regret minimisation (vanilla CFR, CFR+ and discounted CFR).

Test infrastructure (oracle): not part of the product path.

State: ``T`` (iterations done), ``R[q]`` cumulative counterfactual regret and
``S[q]`` cumulative weighted strategy, q indexing Q_+ in input order. These are
the paper's running means written as sums: the average regret of Eq.
(average_counterfactual_regret) is R / T, and the average strategy of Eq.
(average_strategy_profile) is S normalised per infoset. Regret matching is
scale invariant, so R and R / T give the same next strategy.

One iteration, with every infoset using the same strategy sigma^(T+1) (the
simultaneous schedule of Section 3.2):

1. sigma = regret matching of R (Eq. next_strategy_profile): positive parts
   normalised, or uniform when their sum is exactly 0; chance plays sigma_0.
2. A recursive walk carries (pi_1, pi_2, pi_c), the products of each player's
   and chance's edge probabilities from the root, and returns the node's
   expected payoff for player 1 (Eq. expected_payoff; u_2 = -u_1).
   At a node d of player i in infoset h, with child values w_a and node value
   u = sum_a sigma(h,a) w_a, it adds
       r~(h,a) += pi_{-i}(d) * sgn_i * (w_a - u)
   where pi_{-i}(d) is the excepted reach of Eq. (excepted_reach_probability)
   and sgn_1 = +1, sgn_2 = -1: summed over d in h this is the instantaneous
   counterfactual regret of Eq. (instantaneous_counterfactual_regret) with the
   division by the counterfactual reach multiplied out; and it adds
       pibar(h) += pi_i(d)
   the player reach of Eq. (player_reach_probability), read with the own-reach
   recursion (the printed recursion multiplies the excepted reach; the matrix
   form with the hatted strategies matrix confirms the own-reach reading).
3. Regret update: vanilla R += r~; CFR+ R = max(R + r~, 0).
4. Average update: S(h,a) += w * pibar(h) * sigma(h,a), with w = 1 (vanilla,
   Eq. average_strategy_profile) or w = T + 1 (CFR+ linear averaging).
5. T += 1.

CFR+ is only cited by the paper; it is read here as regret matching on
cumulative regrets clipped at zero after each update, linear averaging with no
delay, the same simultaneous schedule and the same uniform fallback.

Discounted CFR (DCFR with parameters alpha, beta, gamma) is the discounting of
the cited weighting work, which the paper's discussion (Section 5) says enters
only through the average-regret and average-strategy equations. Read here, for
iteration t = T + 1 (1-based) and the same r~, pibar and sigma as above:
   R(h,a) <- (R + r~) * t^alpha / (t^alpha + 1)   where R + r~ > 0,
             (R + r~) * t^beta / (t^beta + 1)     elsewhere;
   S(h,a) <- (S + pibar(h) * sigma(h,a)) * (t / (t + 1))^gamma.
Each iteration's strategy then carries weight proportional to t^gamma in the
normalised average, and with alpha = beta every iteration's regret carries a
weight that grows as t^alpha; alpha = beta = gamma = 1 is linear CFR up to a
positive scale, which the tests use as an independent pin.

Alternating updates (the schedule of the CFR+ work the paper cites, which the
discussion of Section 5 names as applicable to the matrix formulation): one
iteration is two passes of steps 1-4 with the same t. The first updates only
player 1's infosets (R, S, and so its strategy); the second, which sees player
1's new strategy, updates only player 2's; then T += 1.
"""
from __future__ import annotations

from dataclasses import dataclass

from .tree import Tree

VANILLA, CFR_PLUS, DCFR = "vanilla", "cfr+", "dcfr"
SIMULTANEOUS, ALTERNATING = "simultaneous", "alternating"
# the weighting work's recommended parameters (alpha, beta, gamma)
DCFR_DEFAULT = (1.5, 0.0, 2.0)


def dcfr_factors(t: int, params=DCFR_DEFAULT):
    """The discount factors of iteration t (1-based): on positive and on other cumulative
    regrets, and on the cumulative strategy."""
    alpha, beta, gamma = params
    ta, tb = float(t) ** alpha, float(t) ** beta
    return ta / (ta + 1.0), tb / (tb + 1.0), (t / (t + 1.0)) ** gamma


@dataclass
class State:
    T: int
    R: list
    S: list

    @staticmethod
    def zeros(tree: Tree) -> "State":
        return State(0, [0.0] * tree.Q, [0.0] * tree.Q)

    def copy(self) -> "State":
        return State(self.T, list(self.R), list(self.S))


def regret_matching(r: list) -> list:
    """Eq. (next_strategy_profile) for one infoset."""
    pos = [x if x > 0.0 else 0.0 for x in r]
    total = sum(pos)
    if total > 0.0:
        return [x / total for x in pos]
    return [1.0 / len(r)] * len(r)


def current_strategy(tree: Tree, R: list) -> list:
    """sigma over Q_+ from cumulative regrets."""
    sigma = [0.0] * tree.Q
    for h in tree.rational:
        o, k = tree.qoff[h], tree.nact[h]
        sigma[o:o + k] = regret_matching(R[o:o + k])
    return sigma


def average_strategy(tree: Tree, S: list) -> list:
    """S normalised per infoset; uniform where the infoset's weights sum to 0."""
    out = [0.0] * tree.Q
    for h in tree.rational:
        o, k = tree.qoff[h], tree.nact[h]
        tot = sum(S[o:o + k])
        out[o:o + k] = [x / tot for x in S[o:o + k]] if tot > 0.0 else [1.0 / k] * k
    return out


def iterate(tree: Tree, state: State, variant: str = VANILLA, record: bool = False,
            dcfr=DCFR_DEFAULT, players=(1, 2), count: bool = True):
    """One CFR iteration. Returns (new_state, info); ``info`` holds sigma, r~,
    pibar and, if ``record``, per-node expected payoff u1 and reaches. ``dcfr`` holds
    (alpha, beta, gamma) for the discounted variant. ``players``: whose infosets the
    call updates (the others keep R and S); ``count``: whether it ends the iteration.
    ``info["rtilde_scale"]`` is, per pair, the sum of the magnitudes the regret is summed from,
    |pi_{-i}(d)| (|w_a| + |u|) over the infoset's nodes d: the size that rounding errors in
    r~ scale with (r~ itself can be much smaller, by cancellation)."""
    sigma = current_strategy(tree, state.R)
    rt = [0.0] * tree.Q
    rt_scale = [0.0] * tree.Q  # sum of |cf| (|w_a| + |u|): the magnitude r~ is summed from
    pibar = {h: 0.0 for h in tree.rational}
    n = tree.n
    node_u = [0.0] * n if record else None
    node_reach = [None] * n if record else None
    children, infoset, player = tree.children, tree.infoset, tree.player
    qoff, sigma0, u1 = tree.qoff, tree.sigma0, tree.u1

    def walk(v, p1, p2, pc):
        if record:
            node_reach[v] = (p1, p2, pc)
        ch = children[v]
        if not ch:
            if record:
                node_u[v] = u1[v]
            return u1[v]
        h = infoset[v]
        pl = player[h]
        if pl == 0:
            probs = sigma0[h]
            u = 0.0
            for a, c in enumerate(ch):
                u += probs[a] * walk(c, p1, p2, pc * probs[a])
        else:
            o = qoff[h]
            w = []
            for a, c in enumerate(ch):
                s = sigma[o + a]
                if pl == 1:
                    w.append(walk(c, p1 * s, p2, pc))
                else:
                    w.append(walk(c, p1, p2 * s, pc))
            u = 0.0
            for a in range(len(ch)):
                u += sigma[o + a] * w[a]
            if pl == 1:
                cf, own, sgn = p2 * pc, p1, 1.0
            else:
                cf, own, sgn = p1 * pc, p2, -1.0
            for a in range(len(ch)):
                rt[o + a] += cf * sgn * (w[a] - u)
                rt_scale[o + a] += abs(cf) * (abs(w[a]) + abs(u))
            pibar[h] += own
        if record:
            node_u[v] = u
        return u

    root_value = walk(tree.root, 1.0, 1.0, 1.0)

    R = list(state.R)
    S = list(state.S)
    w = float(state.T + 1) if variant == CFR_PLUS else 1.0
    if variant == DCFR:
        d_pos, d_neg, d_avg = dcfr_factors(state.T + 1, dcfr)
    for h in tree.rational:
        if player[h] not in players:
            continue
        o, k = qoff[h], tree.nact[h]
        for a in range(k):
            q = o + a
            if variant == VANILLA:
                R[q] = R[q] + rt[q]
            elif variant == CFR_PLUS:
                R[q] = max(R[q] + rt[q], 0.0)
            elif variant == DCFR:
                x = R[q] + rt[q]
                R[q] = x * (d_pos if x > 0.0 else d_neg)
            else:
                raise ValueError(variant)
            S[q] = S[q] + w * pibar[h] * sigma[q]
            if variant == DCFR:
                S[q] = S[q] * d_avg
    info = {"sigma": sigma, "rtilde": rt, "rtilde_scale": rt_scale, "pibar": pibar,
            "root_value": root_value,
            "next_sigma": current_strategy(tree, R)}
    if record:
        info["node_u"] = node_u
        info["node_reach"] = node_reach
    return State(state.T + (1 if count else 0), R, S), info


def iterate_alternating(tree: Tree, state: State, variant: str = VANILLA, dcfr=DCFR_DEFAULT):
    """One iteration of the alternating schedule: a pass updating player 1, then one updating
    player 2 under player 1's new strategy, both with t = T + 1. Returns (new_state, info of
    the second pass)."""
    st, _ = iterate(tree, state, variant, dcfr=dcfr, players=(1,), count=False)
    return iterate(tree, st, variant, dcfr=dcfr, players=(2,), count=True)


def solve(tree: Tree, iterations: int, variant: str = VANILLA, state: State | None = None,
          callback=None, dcfr=DCFR_DEFAULT, schedule: str = SIMULTANEOUS) -> State:
    st = state.copy() if state is not None else State.zeros(tree)
    for _ in range(iterations):
        if schedule == ALTERNATING:
            st, _info = iterate_alternating(tree, st, variant, dcfr=dcfr)
        else:
            st, _info = iterate(tree, st, variant, dcfr=dcfr)
        if callback is not None:
            callback(st)
    return st


def expected_value(tree: Tree, profile: list) -> float:
    """u_hat(sigma, 1) = sum over terminals of pi(sigma, t) u(t, 1) (Section 2.2)."""
    def val(v):
        ch = tree.children[v]
        if not ch:
            return tree.u1[v]
        h = tree.infoset[v]
        if tree.player[h] == 0:
            probs = tree.sigma0[h]
        else:
            o = tree.qoff[h]
            probs = profile[o:o + len(ch)]
        return sum(probs[a] * val(c) for a, c in enumerate(ch))
    return val(tree.root)
