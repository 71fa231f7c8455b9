"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package draws random numbers and lays out lattices, block-sparse
matrices, shift lists, right-hand-side indices and local clusters.  It holds
none of the solver's arithmetic: nothing here applies an operator, forms an
inner product or runs an iteration.
"""
from .tb import (  # noqa: F401
    Bsr, Problem, CONFIGS, make_config, make_problem, lattice_sc, lattice_fcc,
    cluster_offsets_fcc, cluster_offsets_sc, bsr_to_dense, bsr_to_scipy, rngs_for, mlp_init_weights,
)
