"""CPU FP64 oracle — TEST INFRASTRUCTURE ONLY.

Plain, slow, step-by-step NumPy/SciPy implementations of what the GPU path
computes, used by the tests, by the package's smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this package,
and this package imports nothing from the product path: the two share only
the seeded input generator in ``synth``.
"""
from .scocg import (  # noqa: F401
    CONVERGED, MAXITER, BREAKDOWN, NONFINITE, ScocgResult, initial_seed,
    inner_cg, scocg, scocg_projected, local_system, solve_rhs, solve_problem,
)
from .dense import dense_solve, green_eig, true_residual  # noqa: F401
from . import mlp, features, integrate  # noqa: F401
from .qmr import scocg_lanczos, sqmr  # noqa: F401
