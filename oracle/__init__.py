"""ORACLE -- test infrastructure, not part of the product.

Plain FP64 CPU sparse Cholesky (C, single thread, no FMA contraction), a dense
restricted-pivoting LDL^T (``oracle.ldlt``, numpy), a dense LU with the same
restricted row pivoting (``oracle.lu``, numpy) and the checks built on
them.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library; the only thing both sides receive is the seeded input from
``gen`` and, as data, the library's final permutation.
"""
from .oracle import (  # noqa: F401
    NotSPD,
    OracleFactor,
    build,
    lib_path,
    symbolic,
    supernodes,
    relaxed_supernodes,
    factor,
    solve,
    factor_error,
    permuted_lower,
    rel_residual,
    logdet,
    flops_from_counts,
)
