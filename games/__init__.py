"""Seeded synthetic game generators: the inputs shared by the oracle and the GPU path.

Nothing here computes any part of CFR; it only emits game tuples
(Definition 1, Section 2.1) and seeded random solver states.
"""
from .tuple import Game, GameBuilder
from .small import matrix_game, rock_paper_scissors, kuhn_like, leduc_like, random_game
from .poker import poker_game, large_game, subgame, subgame_spec, template_size
from .states import random_state, n_player_q
from .nplayer import normal_form_n, kuhn3, random_game_n, with_silent_players

__all__ = [
    "Game", "GameBuilder", "matrix_game", "rock_paper_scissors", "kuhn_like", "leduc_like",
    "random_game", "poker_game", "large_game", "subgame", "subgame_spec", "template_size",
    "random_state", "n_player_q", "normal_form_n", "kuhn3", "random_game_n",
    "with_silent_players",
]
