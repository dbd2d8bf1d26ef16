"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only builds matrices and right-hand sides.  It contains none of
the factorization's arithmetic: no ordering, no elimination, no solves.
"""
from .matrices import (  # noqa: F401
    CSR,
    laplace2d,
    laplace3d,
    laplace1d,
    fv2d,
    fv3d,
    landice,
    batch_fv3d,
    rhs,
    dense_to_csr,
    random_spd_pattern,
    csr_block_diag,
    serving_requests,
    shifted,
    nonsymmetric,
)
