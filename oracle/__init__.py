"""Oracle: a plain, slow, obviously correct FP64 CPU implementation of CFR.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
link anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the GPU path: the
two meet only at the seeded game generators in ``games``.

Modules
-------
tree      the game tuple viewed as a tree with ordered child lists
cfr       recursive vanilla CFR and CFR+ iterations (Section 2.3 definitions)
literal   the paper's matrix formulation evaluated with dense matrices
          (Section 3: setup matrices, Tree Traversal, Average Strategy
          Profile, Next Strategy Profile)
br        best response, exploitability and a brute-force check
lp        sequence-form linear program for the game value
layout    an independent implementation of the canonical level-ordered layout
mlp       fp64 reference of the warm-start network (forward, backward, SGD)
"""
