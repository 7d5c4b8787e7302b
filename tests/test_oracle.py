"""Pins for the FP64 oracle against facts that do not come from the oracle itself.

* closed forms: rock-paper-scissors stays exactly uniform with value 0; a 2x2
  zero-sum game without a saddle point has p* = (d-c)/(a-b-c+d) and value
  (ad-bc)/(a-b-c+d); Kuhn-shaped poker has value -1/18 (Kuhn, 1950);
* a matrix game written as a tree reduces CFR to normal-form regret matching
  (and CFR+ to RM+), which the tests write with numpy matrix products;
* the sequence-form LP (scipy HiGHS) on random tiny games;
* brute-force best responses over all pure strategies;
* reach probabilities and expected payoffs recomputed by enumerating
  root-to-node paths (the definitions of Section 2.2 read directly);
* the paper's own dense-matrix formulation (Section 3), evaluated literally;
* invariants: strategies are distributions, CFR+ regrets are nonnegative,
  exploitability is nonnegative and bounded by the regret bounds of the CFR
  convergence theorem behind the 2-epsilon statement of Section 2.3;
* discounted CFR: with alpha = beta = 1 it is linear CFR (iteration s's regret
  weighted by s and its strategy by s^gamma, accumulated without discounting)
  up to the positive scales (t+1) and (t+1)^gamma, which the tests accumulate
  separately; with beta far below 0 no cumulative regret stays negative.
"""
import math

import numpy as np
import pytest

import games
from oracle import br, cfr, literal, lp
from oracle.tree import Tree


def _tree(g):
    return Tree(g)


# ---------------------------------------------------------------- closed forms

def test_rps_stays_uniform_exactly():
    t = _tree(games.rock_paper_scissors())
    st = cfr.State.zeros(t)
    for _ in range(25):
        st, info = cfr.iterate(t, st)
        assert info["rtilde"] == [0.0] * t.Q
        assert info["sigma"] == [1.0 / 3] * t.Q
    avg = cfr.average_strategy(t, st.S)
    e = br.exploitability(t, avg)
    assert abs(e["value"]) < 1e-15 and abs(e["expl"]) < 1e-15


def test_2x2_mixed_equilibrium_closed_form():
    a, b, c, d = 2.0, -1.0, -1.0, 1.0
    den = a - b - c + d
    p_star, v_star = (d - c) / den, (a * d - b * c) / den
    t = _tree(games.matrix_game([[a, b], [c, d]]))
    value, prof = lp.solve(t)
    assert value == pytest.approx(v_star, abs=1e-9)
    assert prof[0] == pytest.approx(p_star, abs=1e-7)
    st = cfr.solve(t, 4000)
    avg = cfr.average_strategy(t, st.S)
    assert avg[0] == pytest.approx(p_star, abs=2e-2)
    e = br.exploitability(t, avg)
    assert 0.0 <= e["expl"] < 3e-2
    st = cfr.solve(t, 2000, cfr.CFR_PLUS)
    avg = cfr.average_strategy(t, st.S)
    assert avg[0] == pytest.approx(p_star, abs=2e-2)
    e = br.exploitability(t, avg)
    assert 0.0 <= e["expl"] < 3e-2
    assert e["value"] == pytest.approx(v_star, abs=2e-2)


def test_kuhn_value_is_minus_one_eighteenth():
    t = _tree(games.kuhn_like(3, "joint"))
    value, prof = lp.solve(t)
    assert value == pytest.approx(-1.0 / 18.0, abs=1e-9)
    assert br.exploitability(t, prof)["expl"] < 1e-9
    st = cfr.solve(t, 3000)
    e = br.exploitability(t, cfr.average_strategy(t, st.S))
    assert e["expl"] < 5e-3
    assert e["value"] == pytest.approx(-1.0 / 18.0, abs=5e-3)


# ---------------------------------------------------------------- normal-form reductions

def _normal_form(seed, m=3, n=4):
    rng = np.random.default_rng(seed)
    A = rng.integers(-8, 9, size=(m, n)) / 4.0
    return A, _tree(games.matrix_game(A))


@pytest.mark.parametrize("seed", range(5))
def test_one_iteration_equals_normal_form_regrets(seed):
    A, t = _normal_form(seed)
    m, n = A.shape
    T, R, S = games.random_state(games.matrix_game(A), seed)
    st = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    new, info = cfr.iterate(t, st)

    def rm(r):
        p = np.maximum(r, 0)
        return p / p.sum() if p.sum() > 0 else np.full(len(r), 1.0 / len(r))
    x = rm(np.asarray(st.R[:m]))
    y = rm(np.asarray(st.R[m:]))
    v = x @ A @ y
    r1 = A @ y - v                 # row player's regrets
    r2 = -(x @ A) + v              # column player's regrets (u2 = -u1)
    np.testing.assert_allclose(info["rtilde"], np.concatenate([r1, r2]), rtol=0, atol=1e-14)
    # player reach of an infoset sums own reach over its members (Eq.
    # player_reach_probability): 1 at the root, m (one per row node) for player 2
    np.testing.assert_allclose(new.S, np.asarray(st.S) + np.concatenate([x, m * y]), atol=1e-14)
    assert info["root_value"] == pytest.approx(v, abs=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_cfr_plus_equals_rm_plus_on_matrix_game(seed):
    A, t = _normal_form(seed + 10)
    m, n = A.shape
    R1, R2 = np.zeros(m), np.zeros(n)
    S1, S2 = np.zeros(m), np.zeros(n)

    def rm(r):
        p = np.maximum(r, 0)
        return p / p.sum() if p.sum() > 0 else np.full(len(r), 1.0 / len(r))
    st = cfr.State.zeros(t)
    for it in range(1, 40):
        x, y = rm(R1), rm(R2)
        v = x @ A @ y
        R1 = np.maximum(R1 + A @ y - v, 0)
        R2 = np.maximum(R2 - x @ A + v, 0)
        S1 += it * x
        S2 += it * m * y          # player 2's infoset has m member nodes of own reach 1
        st, _ = cfr.iterate(t, st, cfr.CFR_PLUS)
    np.testing.assert_allclose(st.R, np.concatenate([R1, R2]), atol=1e-12)
    np.testing.assert_allclose(st.S, np.concatenate([S1, S2]), atol=1e-10)


@pytest.mark.parametrize("seed", range(3))
def test_alternating_cfr_plus_equals_alternating_rm_plus_on_matrix_game(seed):
    """Alternating RM+ written with numpy matrix products: the row player updates against the
    column strategy, then the column player against the row player's new strategy."""
    A, t = _normal_form(seed + 20)
    m, n = A.shape
    R1, R2 = np.zeros(m), np.zeros(n)
    S1, S2 = np.zeros(m), np.zeros(n)

    def rm(r):
        p = np.maximum(r, 0)
        return p / p.sum() if p.sum() > 0 else np.full(len(r), 1.0 / len(r))
    st = cfr.State.zeros(t)
    for it in range(1, 40):
        x, y = rm(R1), rm(R2)
        R1 = np.maximum(R1 + A @ y - x @ A @ y, 0)
        S1 += it * x
        x = rm(R1)
        R2 = np.maximum(R2 - x @ A + x @ A @ y, 0)
        S2 += it * m * y
        st, _ = cfr.iterate_alternating(t, st, cfr.CFR_PLUS)
        assert st.T == it
    np.testing.assert_allclose(st.R, np.concatenate([R1, R2]), atol=1e-12)
    np.testing.assert_allclose(st.S, np.concatenate([S1, S2]), atol=1e-10)


@pytest.mark.parametrize("maker,passes,factor", [
    (lambda: games.kuhn_like(3, "joint"), 200, 4.0),
    (lambda: games.leduc_like(3, 2, deal="sequential"), 600, 2.0),
])
def test_alternating_cfr_plus_converges_faster_per_pass(maker, passes, factor):
    """The CFR+ work's observation: at equal numbers of tree passes the alternating schedule
    ends closer to equilibrium than the simultaneous one."""
    t = _tree(maker())
    sim = cfr.solve(t, passes, cfr.CFR_PLUS)
    alt = cfr.solve(t, passes // 2, cfr.CFR_PLUS, schedule=cfr.ALTERNATING)
    e_sim = br.exploitability(t, cfr.average_strategy(t, sim.S))["expl"]
    e_alt = br.exploitability(t, cfr.average_strategy(t, alt.S))["expl"]
    assert e_alt < e_sim / factor, (e_alt, e_sim)


# ---------------------------------------------------------------- path enumeration

def _paths(t):
    """(node, list of (acting player, edge prob)) via explicit parent walks."""
    out = {}
    for v in range(t.n):
        edges = []
        x = v
        while t.parent[x] >= 0:
            p = t.parent[x]
            a = t.children[p].index(x)
            edges.append((p, a))
            x = p
        out[v] = edges
    return out


@pytest.mark.parametrize("seed", range(4))
def test_reaches_and_values_match_path_products(seed):
    g = games.random_game(seed, deal="sequential")
    t = _tree(g)
    T, R, S = games.random_state(g, seed)
    st = cfr.State(T, [float(x) for x in R], [float(x) for x in S])
    _, info = cfr.iterate(t, st, record=True)
    sigma = info["sigma"]
    paths = _paths(t)
    for v in range(t.n):
        prods = {0: 1.0, 1: 1.0, 2: 1.0}
        for p, a in paths[v]:
            h = t.infoset[p]
            pl = t.player[h]
            prob = t.sigma0[h][a] if pl == 0 else sigma[t.qoff[h] + a]
            prods[pl] *= prob
        p1, p2, pc = info["node_reach"][v]
        assert (p1, p2, pc) == pytest.approx((prods[1], prods[2], prods[0]), abs=1e-15)
    # root value = sum over terminals of pi(t) u(t) (Section 2.2)
    total = 0.0
    for v in range(t.n):
        if t.is_terminal(v):
            p1, p2, pc = info["node_reach"][v]
            total += p1 * p2 * pc * t.u1[v]
    assert info["root_value"] == pytest.approx(total, abs=1e-13)


# ---------------------------------------------------------------- the paper's matrix form

@pytest.mark.parametrize("maker", [
    lambda: games.kuhn_like(3, "joint"),
    lambda: games.kuhn_like(3, "sequential"),
    lambda: games.random_game(1, deal="joint"),
    lambda: games.random_game(2, deal="sequential", n_types=(3, 2)),
    lambda: games.random_game(5, deal="none", depth=5),
])
def test_matrix_formulation_equals_recursion(maker):
    g = maker()
    t = _tree(g)
    L = literal.Literal(t)
    Q = t.Q
    sigma = L.sigma1.copy()
    rbar = np.zeros(Q)
    sigmabar = L.sigma1.copy()
    pisum = np.zeros(L.MHQ.shape[0])
    st = cfr.State.zeros(t)
    for T in range(1, 31):
        out = L.iterate(sigma, rbar, sigmabar, pisum, T)
        st_new, info = cfr.iterate(t, st, record=True)
        np.testing.assert_allclose(sigma, info["sigma"], atol=1e-12)
        np.testing.assert_allclose(out["rtilde"], info["rtilde"], atol=1e-12)
        np.testing.assert_allclose(out["U"][:, 0], info["node_u"], atol=1e-12)
        np.testing.assert_allclose(out["U"][:, 1], -np.asarray(info["node_u"]), atol=1e-12)
        pib = np.array([info["pibar"][h] for h in t.rational])
        np.testing.assert_allclose(out["pibar"], pib, atol=1e-12)
        np.testing.assert_allclose(out["rbar"], np.asarray(st_new.R) / T, atol=1e-12)
        np.testing.assert_allclose(out["sigmabar"],
                                   cfr.average_strategy(t, st_new.S), atol=1e-12)
        np.testing.assert_allclose(out["sigma_next"], info["next_sigma"], atol=1e-12)
        sigma, rbar, sigmabar, pisum = (out["sigma_next"], out["rbar"], out["sigmabar"],
                                        out["pibar_sum"])
        st = st_new


# ---------------------------------------------------------------- LP and best response

@pytest.mark.parametrize("seed", range(8))
def test_random_games_lp_and_cfr_agree(seed):
    deal = ["joint", "sequential", "none"][seed % 3]
    g = games.random_game(seed, deal=deal, depth=3)
    t = _tree(g)
    value, prof = lp.solve(t)
    e = br.exploitability(t, prof)
    assert e["expl"] < 1e-8
    assert e["value"] == pytest.approx(value, abs=1e-8)
    st = cfr.solve(t, 1500, cfr.CFR_PLUS)
    e2 = br.exploitability(t, cfr.average_strategy(t, st.S))
    assert e2["expl"] < 5e-3
    assert e2["value"] == pytest.approx(value, abs=1e-2)


@pytest.mark.parametrize("seed", range(6))
def test_best_response_equals_brute_force(seed):
    g = games.random_game(seed, deal="joint", depth=3, n_types=(2, 2))
    t = _tree(g)
    rng = np.random.default_rng(seed)
    prof = []
    for h in t.rational:
        w = rng.random(t.nact[h])
        prof.extend((w / w.sum()).tolist())
    for i in (1, 2):
        assert br.best_response_value(t, prof, i) == pytest.approx(
            br.brute_force_br(t, prof, i), abs=1e-13)


def test_kuhn_best_response_equals_brute_force():
    t = _tree(games.kuhn_like(3, "joint"))
    st = cfr.solve(t, 17)
    avg = cfr.average_strategy(t, st.S)
    for i in (1, 2):
        assert br.best_response_value(t, avg, i) == pytest.approx(
            br.brute_force_br(t, avg, i), abs=1e-13)


# ---------------------------------------------------------------- invariants and bounds

@pytest.mark.parametrize("maker,variant", [
    (lambda: games.kuhn_like(3, "joint"), cfr.VANILLA),
    (lambda: games.random_game(3, deal="joint", depth=4), cfr.VANILLA),
    (lambda: games.random_game(4, deal="sequential", depth=4), cfr.CFR_PLUS),
    (lambda: games.leduc_like(3, 2, deal="sequential"), cfr.CFR_PLUS),
])
def test_invariants(maker, variant):
    t = _tree(maker())
    st = cfr.State.zeros(t)
    for _ in range(12):
        st, info = cfr.iterate(t, st, variant)
        for h in t.rational:
            o, k = t.qoff[h], t.nact[h]
            s = info["next_sigma"][o:o + k]
            assert min(s) >= 0.0 and abs(sum(s) - 1.0) < 1e-12
        if variant == cfr.CFR_PLUS:
            assert min(st.R) >= 0.0
    e = br.exploitability(t, cfr.average_strategy(t, st.S))
    assert e["expl"] >= -1e-12


@pytest.mark.parametrize("maker", [
    lambda: games.kuhn_like(3, "joint"),
    lambda: games.random_game(6, deal="joint", depth=4),
    lambda: games.random_game(7, deal="sequential", depth=3, n_types=(3, 3)),
])
def test_vanilla_regret_bounds(maker):
    g = maker()
    t = _tree(g)
    u = [t.u1[v] for v in range(t.n) if t.is_terminal(v)]
    delta = max(u) - min(u)
    st = cfr.State.zeros(t)
    for T in range(1, 301):
        st, _ = cfr.iterate(t, st)
        if T in (1, 10, 100, 300):
            e = br.exploitability(t, cfr.average_strategy(t, st.S))
            imm = sum(max(max(st.R[t.qoff[h] + a] for a in range(t.nact[h])), 0.0)
                      for h in t.rational) / T
            assert e["nash_conv"] <= imm + 1e-12
            bound = 0.0
            for i in (1, 2):
                hs = [h for h in t.rational if t.player[h] == i]
                amax = max(t.nact[h] for h in hs)
                bound += delta * len(hs) * math.sqrt(amax) / math.sqrt(T)
            assert e["nash_conv"] <= bound


def test_exploitability_falls_at_least_like_inverse_sqrt():
    t = _tree(games.kuhn_like(3, "joint"))
    st = cfr.State.zeros(t)
    ex = {}
    for T in range(1, 1601):
        st, _ = cfr.iterate(t, st)
        if T in (100, 1600):
            ex[T] = br.exploitability(t, cfr.average_strategy(t, st.S))["expl"]
    slope = math.log(ex[1600] / ex[100]) / math.log(16)
    assert slope < -0.45


# ---------------------------------------------------------------- discounted CFR

@pytest.mark.parametrize("gamma", [1.0, 2.0])
@pytest.mark.parametrize("maker", [
    lambda: games.kuhn_like(3, "joint"),
    lambda: games.random_game(8, deal="sequential", depth=4),
    lambda: games.leduc_like(3, 2, deal="sequential"),
])
def test_dcfr_with_unit_exponents_is_linear_cfr(maker, gamma):
    """Linear CFR accumulates s * r~_s and s^gamma * pibar sigma_s with no discount; the
    discounted recursion with alpha = beta = 1 must equal it divided by (t+1) (regrets) and
    (t+1)^gamma (strategy sums) after every iteration t, with the same strategies."""
    t = _tree(maker())
    st = cfr.State.zeros(t)
    RL, SL = [0.0] * t.Q, [0.0] * t.Q
    for it in range(1, 41):
        st, info = cfr.iterate(t, st, cfr.DCFR, dcfr=(1.0, 1.0, gamma))
        # linear CFR's own step at its own regrets: a vanilla walk supplies sigma, r~ and pibar
        _, lin = cfr.iterate(t, cfr.State(it - 1, list(RL), list(SL)), cfr.VANILLA)
        np.testing.assert_allclose(info["sigma"], lin["sigma"], rtol=0, atol=1e-12)
        for h in t.rational:
            for a in range(t.nact[h]):
                q = t.qoff[h] + a
                RL[q] += it * lin["rtilde"][q]
                SL[q] += it ** gamma * lin["pibar"][h] * lin["sigma"][q]
        scale_r = max(max(abs(x) for x in RL), 1e-300)
        scale_s = max(max(abs(x) for x in SL), 1e-300)
        assert max(abs(st.R[q] * (it + 1) - RL[q]) for q in range(t.Q)) <= 1e-10 * scale_r
        assert max(abs(st.S[q] * (it + 1) ** gamma - SL[q]) for q in range(t.Q)) <= 1e-10 * scale_s


@pytest.mark.parametrize("maker", [
    lambda: games.random_game(9, deal="joint", depth=4),
    lambda: games.leduc_like(3, 2, deal="sequential"),
])
def test_dcfr_discounts_negative_regrets_by_their_own_factor(maker):
    """beta = -40 makes the factor on non-positive cumulative regrets 2^-40 or less from the
    second iteration on, alpha = 1 keeps positive ones: no regret may stay below
    -1e-9 of the largest, some must stay positive, and the strategy is still a distribution.
    Testing the sign before adding r~, or swapping the two factors, fails this."""
    t = _tree(maker())
    st = cfr.State.zeros(t)
    for it in range(1, 31):
        st, info = cfr.iterate(t, st, cfr.DCFR, dcfr=(1.0, -40.0, 2.0))
        top = max(abs(x) for x in st.R)
        if it >= 2:
            assert min(st.R) >= -1e-9 * top
        assert max(st.R) > 0.0
        for h in t.rational:
            s = info["next_sigma"][t.qoff[h]:t.qoff[h] + t.nact[h]]
            assert min(s) >= 0.0 and abs(sum(s) - 1.0) < 1e-12


def test_dcfr_converges_faster_than_vanilla_on_a_poker_game():
    """The weighting work's claim on poker-like games, at its recommended (1.5, 0, 2)."""
    t = _tree(games.leduc_like(3, 2, deal="sequential"))
    ex = {}
    for variant in (cfr.VANILLA, cfr.DCFR):
        st = cfr.State.zeros(t)
        for it in range(1, 201):
            st, _ = cfr.iterate(t, st, variant)
            if it in (20, 200):
                ex[variant, it] = br.exploitability(t, cfr.average_strategy(t, st.S))["expl"]
    assert ex[cfr.DCFR, 200] < ex[cfr.DCFR, 20] / 4
    assert ex[cfr.DCFR, 200] < ex[cfr.VANILLA, 200] / 2
