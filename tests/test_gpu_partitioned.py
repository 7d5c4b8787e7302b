"""GPU parity of the subtree-partitioned, out-of-core iteration (cfr_build_partitioned) against
the FP64 oracle, at every cut level of small games and with windows of one subtree, of a few
subtrees and of the whole lower tree; the same tolerances as the in-core solvers (1e-6 norm-wise
for one iteration in FP32, 1e-12 in FP64; exploitability after T iterations within 1e-4, read by
moving the state into an in-core solver of the same game)."""
import numpy as np
import pytest

import games
from oracle import br, cfr
from oracle.tree import Tree

pytestmark = pytest.mark.gpu

GAMES = {
    "kuhn": lambda: games.kuhn_like(3, "joint"),
    "leduc3x2": lambda: games.leduc_like(3, 2, deal="sequential"),
    "rand_seq": lambda: games.random_game(22, deal="sequential", depth=6),
    "rand_joint": lambda: games.random_game(21, deal="joint", depth=5, n_types=(3, 3)),
    "subgame": lambda: games.subgame(102),
    "rps": lambda: games.rock_paper_scissors(),
    "deep": lambda: games.random_game(66, deal="sequential", depth=30, max_actions=2, p_terminal=0.3),
}


def _rel(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(float(np.abs(ref).max()) if ref.size else 0.0, 1e-300)
    return float(np.abs(gpu - ref).max()) / scale if ref.size else 0.0


def _cuts(g):
    from paper_2408_14778_amd import plan
    D = plan(g)["depth"]
    return sorted({1, max(1, D // 2), D - 1})


def _part(g, variant="vanilla", cut=1, window=1 << 30, **kw):
    from paper_2408_14778_amd import PartitionedSolver
    return PartitionedSolver(g, variant, cut_level=cut, max_window_nodes=window, **kw)


@pytest.mark.parametrize("window", [1, 97, 1 << 30])
@pytest.mark.parametrize("variant", ["vanilla", "cfr+", "dcfr"])
@pytest.mark.parametrize("name", sorted(GAMES))
def test_partitioned_one_iteration_parity(name, variant, window):
    g = GAMES[name]()
    T, R, S = games.random_state(g, seed=len(name) + 3, nonnegative=(variant == "cfr+"))
    t = Tree(g)
    new, info = cfr.iterate(t, cfr.State(T, [float(x) for x in R], [float(x) for x in S]),
                            variant, record=True)
    for cut in _cuts(g):
        s = _part(g, variant, cut, window)
        s.set_state(T, R, S)
        s.iterate(1)
        T2, R2, S2 = s.get_state()
        assert T2 == T + 1
        eR, eS = _rel(R2, new.R), _rel(S2, new.S)
        assert eR <= 1e-6 and eS <= 1e-6, (cut, s.n_partitions, eR, eS)
        s.close()


@pytest.mark.parametrize("variant", ["cfr+", "dcfr"])
@pytest.mark.parametrize("name", ["leduc3x2", "rand_seq", "deep"])
def test_partitioned_fp64_one_iteration_parity(name, variant):
    g = GAMES[name]()
    T, R, S = games.random_state(g, seed=7, nonnegative=(variant == "cfr+"))
    t = Tree(g)
    new, _ = cfr.iterate(t, cfr.State(T, [float(x) for x in R], [float(x) for x in S]), variant)
    for cut in _cuts(g):
        for window in (1, 50):
            s = _part(g, variant, cut, window, precision="f64")
            s.set_state(T, R.astype(np.float64), S.astype(np.float64))
            s.iterate(1)
            _, R2, S2 = s.get_state()
            assert R2.dtype == np.float64
            assert _rel(R2, new.R) <= 1e-12 and _rel(S2, new.S) <= 1e-12, (cut, window)
            s.close()


@pytest.mark.parametrize("variant", ["vanilla", "cfr+"])
@pytest.mark.parametrize("name", ["leduc3x2", "rand_joint"])
def test_partitioned_alternating_one_iteration_parity(name, variant):
    g = GAMES[name]()
    T, R, S = games.random_state(g, seed=5, nonnegative=(variant == "cfr+"))
    t = Tree(g)
    new, _ = cfr.iterate_alternating(t, cfr.State(T, [float(x) for x in R], [float(x) for x in S]),
                                     variant)
    for cut in _cuts(g):
        s = _part(g, variant, cut, 64, schedule="alternating")
        s.set_state(T, R, S)
        s.iterate(1)
        T2, R2, S2 = s.get_state()
        assert T2 == T + 1
        assert _rel(R2, new.R) <= 1e-6 and _rel(S2, new.S) <= 1e-6, cut


@pytest.mark.parametrize("name,variant,iters", [("kuhn", "cfr+", 1000), ("leduc3x2", "vanilla", 200),
                                                ("rand_seq", "cfr+", 400), ("deep", "cfr+", 200)])
def test_partitioned_exploitability_after_T_iterations(name, variant, iters):
    """T iterations partitioned, then the state moved into an in-core solver of the same game
    for the exploitability, against the oracle's run."""
    from paper_2408_14778_amd import Solver
    g = GAMES[name]()
    cut = _cuts(g)[len(_cuts(g)) // 2]
    s = _part(g, variant, cut, 16)
    assert s.n_partitions > 1
    s.iterate(iters)
    T, R, S = s.get_state()
    e = Solver(g, variant, engine="node")
    e.set_state(T, R, S)
    got = e.exploitability()["expl"]
    t = Tree(g)
    st = cfr.solve(t, iters, variant)
    ref = br.exploitability(t, cfr.average_strategy(t, st.S))
    assert abs(got - ref["expl"]) <= 1e-4, (got, ref)


def test_partitioned_refuses_whole_tree_calls():
    from paper_2408_14778_amd import CfrError
    g = GAMES["leduc3x2"]()
    s = _part(g, "cfr+", 3, 100)
    s.iterate(2)
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        s.exploitability()
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        s.node_values()
    with pytest.raises(KeyError):
        s.layout("parent")
    assert s.average_strategy().shape == (s.n_q,)


def test_partitioned_large_game_one_iteration(large_game):
    """The full large game (21,509,281 nodes) cut at level 8 with windows of at most 2^21 nodes,
    against the in-core block engine from the same seeded state: R' and S' agree to FP32
    reordering (the two sum the regrets in different orders), and the pass is timed."""
    import time

    import torch

    from paper_2408_14778_amd import Solver
    g = large_game
    T, R, S = games.random_state(g, seed=2, nonnegative=True)
    s = _part(g, "cfr+", 8, 1 << 21)
    print(f"partitions {s.n_partitions}, device workspace {s.info['workspace_bytes'] / 2**30:.2f} "
          f"GiB, pinned host {s.host_bytes / 2**30:.2f} GiB", flush=True)
    s.set_state(T, R, S)
    s.iterate(1)
    _, R2, S2 = s.get_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(5)
    torch.cuda.synchronize()
    print(f"partitioned iteration {(time.perf_counter() - t0) / 5 * 1e3:.2f} ms", flush=True)
    s.close()
    b = Solver(g, "cfr+")
    b.set_state(T, R, S)
    b.iterate(1)
    _, Rb, Sb = b.get_state()
    assert _rel(R2, Rb) <= 1e-5 and _rel(S2, Sb) <= 1e-5
