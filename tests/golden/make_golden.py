"""Writes the stored expected values under tests/golden/ by calling only the oracle.

medium_game_expl.json: exploitability of the average strategy after 1,000 iterations of
vanilla CFR and of CFR+ on the medium two-round game (6 ranks x 2 suits, 100,981 nodes),
computed by the recursive FP64 oracle. Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import games  # noqa: E402
from oracle import br, cfr  # noqa: E402
from oracle.tree import Tree  # noqa: E402


def main():
    g = games.leduc_like(6, 2, deal="joint")
    t = Tree(g)
    out = {"game": "leduc_like(6, 2, deal='joint')", "nodes": g.n_nodes}
    for variant in ("vanilla", "cfr+"):
        t0 = time.time()
        st = cfr.solve(t, 1000, variant)
        e = br.exploitability(t, cfr.average_strategy(t, st.S))
        out[variant] = {"iterations": 1000, "expl": e["expl"], "br1": e["br1"], "br2": e["br2"],
                        "value": e["value"], "oracle_seconds": time.time() - t0}
        print(variant, out[variant], flush=True)
    path = os.path.join(ROOT, "tests", "golden", "medium_game_expl.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
