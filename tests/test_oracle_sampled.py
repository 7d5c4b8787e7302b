"""Pin for the one-infoset-at-a-time oracle: on games small enough for the full
recursive walk, its per-infoset update (path products for reach, subtree walks
for values) equals the recursive oracle's for every infoset."""
import numpy as np
import pytest

import games
from oracle import cfr
from oracle.sampled import InfosetSampler
from oracle.tree import Tree


@pytest.mark.parametrize("maker,variant", [
    (lambda: games.kuhn_like(3, "joint"), "vanilla"),
    (lambda: games.random_game(41, deal="sequential", depth=5), "cfr+"),
    (lambda: games.poker_game(5, 2, 2, 40, max_deals=6), "cfr+"),
    (lambda: games.subgame(102), "vanilla"),
    (lambda: games.random_game(42, deal="joint", depth=5), "dcfr"),
])
def test_sampler_equals_recursive_oracle(maker, variant):
    g = maker()
    T, R, S = games.random_state(g, seed=3, nonnegative=(variant == "cfr+"))
    t = Tree(g)
    new, info = cfr.iterate(t, cfr.State(T, [float(x) for x in R], [float(x) for x in S]), variant)
    samp = InfosetSampler(g)
    hs = t.rational if len(t.rational) <= 60 else \
        np.random.default_rng(0).choice(t.rational, 60, replace=False).tolist()
    for h in hs:
        out = samp.update(R, S, T, int(h), variant)
        o, k = t.qoff[h], t.nact[h]
        assert out["q"] == list(range(o, o + k))
        np.testing.assert_allclose(out["rtilde"], info["rtilde"][o:o + k], atol=1e-12)
        np.testing.assert_allclose(out["R"], new.R[o:o + k], atol=1e-12)
        np.testing.assert_allclose(out["S"], new.S[o:o + k], atol=1e-12)
        assert out["pibar"] == pytest.approx(info["pibar"][h], abs=1e-12)


@pytest.mark.parametrize("maker,seed", [
    (lambda: games.kuhn_like(3, "sequential"), 1),
    (lambda: games.random_game(45, deal="sequential", depth=6), 2),
    (lambda: games.poker_game(5, 2, 2, 40, max_deals=6), 3),
    (lambda: games.leduc_like(3, 2, deal="sequential"), 4),
])
def test_all_values_equal_the_recursive_walk(maker, seed):
    """The one-sweep values equal the recursive oracle's node values, and updates that take
    them equal updates that walk each member's subtree."""
    g = maker()
    T, R, S = games.random_state(g, seed=seed)
    t = Tree(g)
    _, info = cfr.iterate(t, cfr.State(T, [float(x) for x in R], [float(x) for x in S]),
                          record=True)
    samp = InfosetSampler(g)
    u = samp.all_values(R)
    np.testing.assert_allclose(u, info["node_u"], rtol=0, atol=1e-12)
    for h in t.rational[:20]:
        a = samp.update(R, S, T, int(h), values=u)
        b = samp.update(R, S, T, int(h))
        np.testing.assert_allclose(a["R"], b["R"], atol=1e-12)
        np.testing.assert_allclose(a["rtilde_scale"], b["rtilde_scale"], atol=1e-12)
