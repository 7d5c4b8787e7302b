"""GPU parity on the block-engine branches that the poker-shaped games never take.

* More than 4 actions at an infoset: the bottom-up and best-response kernels are instantiated
  for up to 16 action slots (the games below have 7, 8 and 9 actions).
* An infoset with more members than a bottom-up chunk holds: the infoset becomes a chunk of
  its own and its members are strided over the workgroup's threads (partial sums per thread,
  then summed in thread order), in the iteration and in the best response. The launch shape
  is set to chunks of 64 members so that infosets of 100-150 members take that branch.

Each game is checked as the other parity tests are: one iteration from a seeded state (R', S',
sigma', node values and reaches within 1e-6 of the FP64 oracle, norm-wise), the best response
against the GPU's own average strategy, and exploitability after T iterations within 1e-4. Each
test first asserts from the plan arrays that the branch it is about is taken.
"""
import numpy as np
import pytest

import games
from oracle import br, cfr
from oracle.tree import Tree

pytestmark = pytest.mark.gpu


def _wide_matrix():
    rng = np.random.default_rng(7)
    return games.matrix_game(rng.integers(-64, 65, size=(7, 9)) / 64.0, name="matrix7x9")


GAMES = {
    # (game, chunk members per workgroup or None for the tuned shapes, branch)
    "matrix7x9": (_wide_matrix, None, "wide"),
    "rand_wide": (lambda: games.random_game(41, n_types=(3, 2), depth=4, max_actions=8,
                                            deal="joint", allow_single_action=False), None, "wide"),
    "rand_big": (lambda: games.random_game(43, n_types=(150, 3), depth=4, deal="joint"), 64, "big"),
    "rand_big_wide": (lambda: games.random_game(44, n_types=(100, 2), depth=3, max_actions=6,
                                                deal="joint", allow_single_action=False), 64,
                      "big+wide"),
}


def _rel(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(float(np.abs(ref).max()) if ref.size else 0.0, 1e-30)
    return float(np.abs(gpu - ref).max()) / scale if ref.size else 0.0


def _solver(name, variant, engine="auto", keep_node_values=False):
    """engine 'auto' keeps every infoset in the per-level kernels, whose branches these tests
    are about; 'packs' lets the subtree packs take what fits them."""
    from paper_2408_14778_amd import Solver
    make, cap, branch = GAMES[name]
    g = make()
    s = Solver(g, variant, engine=engine, keep_node_values=keep_node_values)
    assert s.info["engine"] == 1, "expected the public-block engine"
    if cap is not None:
        s.set_launch_shape(up_threads=cap, up_members=1)
    # the branch is really taken: action slots past 4, or an infoset larger than a chunk
    if "wide" in branch:
        assert s.info["max_actions"] > 4
    if "big" in branch:
        from paper_2408_14778_amd.solver import host_layout
        mo = host_layout(g, ["x_member_offset"])["x_member_offset"]
        assert int(np.diff(mo).max()) > cap, "no infoset larger than a chunk"
    return g, s


@pytest.mark.parametrize("engine", ["auto", "packs"])
@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("name", sorted(GAMES))
def test_one_iteration_parity_on_wide_and_big_infosets(name, variant, engine):
    g, s = _solver(name, variant, engine, keep_node_values=True)
    T, R, S = games.random_state(g, seed=len(name) + 5, nonnegative=(variant == "cfr+"))
    s.set_state(T, R, S)
    s.iterate(1)
    T2, R2, S2 = s.get_state()
    sig2 = s.current_strategy()
    u1, reach = s.node_values()
    t = Tree(g)
    new, info = cfr.iterate(t, cfr.State(T, [float(x) for x in R], [float(x) for x in S]), variant,
                            record=True)
    assert T2 == T + 1
    assert _rel(R2, new.R) <= 1e-6 and _rel(S2, new.S) <= 1e-6
    nid = s.layout("node_id")
    assert _rel(u1, np.asarray(info["node_u"])[nid]) <= 1e-6
    ref_reach = np.asarray([info["node_reach"][v] for v in nid])
    dec = s.layout("node_player") >= 0
    for k in range(3):
        assert _rel(reach[dec, k], ref_reach[dec, k]) <= 1e-6
    ref_sig = np.asarray(info["next_sigma"])
    scale = max(float(np.abs(new.R).max()), 1e-30)
    for h in t.rational:
        o, k = t.qoff[h], t.nact[h]
        pos = sum(max(x, 0.0) for x in new.R[o:o + k])
        if 0.0 < pos < 1e-6 * scale:
            continue  # at regret matching's uniform-fallback discontinuity
        np.testing.assert_allclose(sig2[o:o + k], ref_sig[o:o + k], rtol=0, atol=2e-6)


@pytest.mark.parametrize("name", sorted(GAMES))
def test_best_response_on_wide_and_big_infosets(name):
    g, s = _solver(name, "cfr+")
    s.iterate(23)
    avg = s.average_strategy().astype(np.float64)
    e = s.exploitability()
    ref = br.exploitability(Tree(g), avg.tolist())
    scale = max(1.0, float(np.abs(g.payoff_u1).max()))
    assert abs(e["br1"] - ref["br1"]) <= 1e-5 * scale
    assert abs(e["br2"] - ref["br2"]) <= 1e-5 * scale


@pytest.mark.parametrize("name,variant,iters", [
    ("matrix7x9", "vanilla", 2000),
    ("matrix7x9", "cfr+", 1000),
    ("rand_wide", "cfr+", 400),
    ("rand_wide", "vanilla", 400),
    ("rand_big", "cfr+", 200),
    ("rand_big_wide", "cfr+", 200),
])
def test_exploitability_after_T_on_wide_and_big_infosets(name, variant, iters):
    g, s = _solver(name, variant)
    s.iterate(iters)
    e = s.exploitability()
    t = Tree(g)
    st = cfr.solve(t, iters, variant)
    ref = br.exploitability(t, cfr.average_strategy(t, st.S))
    assert abs(e["expl"] - ref["expl"]) <= 1e-4, (e, ref)
