"""The host planners (flattening, the public-block plan with its subtree packs, the batch
forest, the per-level tables the solver derives) built with the address and
undefined-behaviour sanitizers, in a plain g++ build of their sources (they make no HIP calls),
and run over the layout games (two-player ones and general-sum ones of 3 and 4 players) and a
batch of them. Any out-of-bounds access, use after free,
leak or undefined operation ends the run with a report."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import games

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_14778_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("flatten.cpp", "xplan.cpp", "host_layout.cpp",
                                            "partition_plan.cpp")]
DRIVER = os.path.join(ROOT, "tests", "host_check", "plan_driver.cpp")


def _games():
    out = [games.kuhn_like(3, "joint"), games.kuhn_like(3, "sequential").permuted(2),
           games.leduc_like(3, 2, deal="sequential"), games.leduc_like(6, 2, deal="joint"),
           games.rock_paper_scissors(), games.random_game(51, deal="sequential", depth=6,
                                                          n_types=(3, 2)),
           games.random_game(52, deal="none", depth=6),
           games.random_game(64, deal="sequential", depth=30, max_actions=2, p_terminal=0.3,
                             p_chance=0.05),
           games.random_game(43, n_types=(150, 3), depth=4, deal="joint")]
    out += [games.subgame(s) for s in (102, 103, 104, 109, 111, 113)]
    # general-sum games of 3 and 4 players (flattened with their player bound, partitioned)
    out += [games.kuhn3(), games.random_game_n(3, 3), games.random_game_n(7, 4, depth=5)]
    return out


def _write(path, game_list):
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(game_list)))
        for g in game_list:
            n = g.n_nodes
            f.write(struct.pack("<q", n))
            for a in (g.parent, g.node_infoset, g.node_action):
                f.write(np.ascontiguousarray(a, dtype="<i4").tobytes())
            f.write(struct.pack("<i", g.n_infosets))
            f.write(np.ascontiguousarray(g.infoset_player, dtype="i1").tobytes())
            f.write(np.ascontiguousarray(g.infoset_num_actions, dtype="<i4").tobytes())
            cp = np.ascontiguousarray(g.chance_prob, dtype="<f8")
            f.write(struct.pack("<q", cp.size))
            f.write(cp.tobytes())
            f.write(np.ascontiguousarray(g.payoff_u1, dtype="<f8").tobytes())


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planners_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread",
           "-I", os.path.join(ROOT, "include"), *SOURCES, DRIVER, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    data = str(tmp_path / "games.bin")
    _write(data, _games())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, data], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert r.stdout.strip().endswith("ok")
