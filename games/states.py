"""Seeded synthetic CFR states (T, R, S) for one-iteration parity checks.

Values are drawn in fp32 so that promoting them to fp64 is exact: both sides
start from bit-identical numbers. R holds cumulative regrets, S cumulative
average-strategy weights, both indexed by the input's infoset-action order
(rational-player infosets in increasing id order, actions in index order).
"""
from __future__ import annotations

import numpy as np

from .tuple import Game


def n_player_q(game: Game) -> int:
    rational = game.infoset_player != 0
    return int(game.infoset_num_actions[rational].sum())


def random_state(game: Game, seed: int, T: int = 37, nonnegative: bool = False):
    """R: |N(0,1)| magnitudes, 20% exact zeros, 30% negated (none if ``nonnegative``);
    S: U(0,1). Returns (T, R, S) with R and S as float32 arrays."""
    rng = np.random.default_rng(seed)
    q = n_player_q(game)
    mag = np.abs(rng.standard_normal(q)).astype(np.float32)
    u = rng.random(q)
    r = np.where(u < 0.2, np.float32(0.0), np.where(u < 0.5, -mag, mag)).astype(np.float32)
    if nonnegative:
        r = np.maximum(r, np.float32(0.0))
    s = rng.random(q).astype(np.float32)
    return T, r, s
