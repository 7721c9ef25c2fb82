"""Seeded synthetic inputs (matrices and right-hand sides).

This package only generates input data.  It contains none of the solver's
arithmetic, and both the GPU library's tests/benchmarks and the CPU oracle
receive their inputs from it.
"""
from .csr import CSR
from .rng import SplitMix64, mix64
from .grids import lap7, varcoef7, uniform_rhs, cell_coefficients
from .q1 import q1_stretched, q1_rhs, q1_rhs_sequence, node_z

__all__ = ["CSR", "SplitMix64", "mix64", "lap7", "varcoef7", "uniform_rhs",
           "cell_coefficients", "q1_stretched", "q1_rhs", "q1_rhs_sequence", "node_z"]
