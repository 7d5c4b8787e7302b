"""Host checks of bench.py's bytes model: the two-sweep streaming model's per-iteration bytes
for the large game equal the 596.0 MB (27.7 B per node) that the model's derivation gives for
it (594.1 MB with the deepest decision level's reach taken in its bottom-up launch), and the
per-level counts it is built from add up to the plan's sizes."""
import numpy as np

import bench


def test_streaming_model_of_the_large_game(large_game):
    from paper_2408_14778_amd.solver import host_layout
    lay = host_layout(large_game, ["level_offset", "node_player", "parent", "q_offset",
                                   "child_begin", "member_offset", "members"])
    counts = bench.level_counts(lay)
    assert sum(c["nodes"] for c in counts) == large_game.n_nodes == 21509281
    assert sum(c["infosets"] for c in counts) == 793910
    assert sum(c["q"] for c in counts) == 2068430
    reach = bench.algorithmic_bytes("block_reach", counts)
    up = bench.algorithmic_bytes("block_up", counts)
    assert round((reach + up) / 1e6, 1) == 596.0
    assert round((reach + up) / large_game.n_nodes, 1) == 27.7
    # the deepest decision level (14) with its reach taken in its bottom-up launch: 24 B per
    # internal node leave the top-down pass, 12 B join the bottom-up one
    rl = np.full(16, 3, dtype=np.int32)
    rl[0] = 0
    rl[14] = 4
    assert counts[14]["decision"] == 154440
    assert bench.algorithmic_bytes("block_reach", counts, rl) == reach - 24 * 154440
    assert bench.algorithmic_bytes("block_up", counts, rl) == up + 12 * 154440
    assert round((bench.algorithmic_bytes("block_reach", counts, rl) +
                  bench.algorithmic_bytes("block_up", counts, rl)) / 1e6, 1) == 594.1
    # the node engine's split of the bottom-up terms adds up to the fused kernel's
    assert np.isclose(bench.algorithmic_bytes("value_level", counts) +
                      bench.algorithmic_bytes("infoset_update", counts), up)
    # FP64 values: the top-down term scales as 8 + 4r (24 -> 40 B per internal node), the pair
    # and infoset terms as r, the per-child term as 8 + r
    r64 = bench.algorithmic_bytes("block_reach", counts, rl, 8)
    assert r64 * 24 == bench.algorithmic_bytes("block_reach", counts, rl) * 40
    inf32 = bench.algorithmic_bytes("infoset_update", counts)
    assert np.isclose(bench.algorithmic_bytes("infoset_update", counts, None, 8), 2 * inf32)
    child = sum(c["nodes"] for c in counts[1:])
    dec = sum(c["decision"] for c in counts[:-1])
    assert np.isclose(bench.algorithmic_bytes("value_level", counts, None, 8),
                      16 * child + 16 * dec)


def test_forest_level_counts_add_up():
    """The batch roofline's per-level counts of a forest are the games' counts summed level by
    level (deeper games past the others' depth)."""
    import games
    gl = [games.subgame(s) for s in (101, 102, 103)]
    each = [bench.game_level_counts(g) for g in gl]
    forest = bench.forest_level_counts(gl)
    assert len(forest) == max(len(c) for c in each)
    for key in ("nodes", "decision", "infosets", "q", "player_children"):
        for l in range(len(forest)):
            assert forest[l][key] == sum(c[l][key] for c in each if l < len(c)), (key, l)
    assert sum(c["nodes"] for c in forest) == sum(g.n_nodes for g in gl)


def test_nplayer_model_hand_count():
    """The general-sum streaming model on a 2 x 3 x 2 three-player normal-form game, counted by
    hand: levels of 1, 2 and 6 decision nodes over 12 terminals, one infoset of 2, 3 and 2
    actions per level; fp32, 3 value columns, 4 reach planes."""
    import games
    from oracle.layout import canonical_layout
    g = games.normal_form_n(np.zeros((2, 3, 2, 3)))
    counts = bench.level_counts(canonical_layout(g))
    assert [c["decision"] for c in counts] == [1, 2, 6, 0]
    assert bench.algorithmic_bytes_n("reach_level", counts, 3) == (8 + 2 * 4 * 4) * (2 + 6)
    assert bench.algorithmic_bytes_n("value_level", counts, 3) == \
        (8 + 12) * (2 + 6 + 12) + 7 * 4 * (1 + 2 + 6)
    assert bench.algorithmic_bytes_n("infoset_update", counts, 3) == 36 * (2 + 3 + 2) + 8 * 3
