"""MI355X-native CFR: one counterfactual-regret-minimisation iteration over a flattened,
level-ordered game tree, computed by hand-written gfx950 HIP kernels behind a C ABI
(include/cfr.h). This package holds the kernels' sources (csrc/), the build step and
the thin ctypes binding."""
from ._native import CfrError, load  # noqa: F401
from .solver import (BatchSolver, NPlayerSolver, PartitionedSolver, Solver,  # noqa: F401
                     host_layout, plan, plan_partitioned)

__all__ = ["Solver", "BatchSolver", "PartitionedSolver", "NPlayerSolver", "plan",
           "plan_partitioned", "host_layout", "CfrError", "load"]
