"""ORACLE -- test infrastructure, not part of the product.

LU of a general matrix with a symmetric sparsity pattern, with pivoting
restricted to diagonal blocks (the paper's Tacho section lists LU of such
matrices among the factorization types and, for speed, looks for pivots only
within each diagonal block; its land-ice systems are nonsymmetric).

Plain dense definition, for inputs of up to a few thousand unknowns:

* C = P A P^T from every stored entry of A, P the analysis permutation
  (taken as data, like the Cholesky oracle).
* The columns are partitioned into diagonal blocks exactly as for the
  restricted LDL^T: the relaxed supernodes of C (this oracle's own symbolic
  routines), each cut into consecutive pieces of at most ``tile`` columns.
* Q C = L U with Q a row permutation that moves a row only within its
  diagonal block, L unit lower triangular, U upper triangular; the columns
  keep their order.
* Pivot of column k: the entry of largest magnitude among rows k .. b1 - 1
  (b1 the end of k's diagonal block) of the partially eliminated column,
  ties to the smallest row; rows below the block are never candidates.  A
  column whose candidates are all zero cannot be factored (``ZeroPivot``).

Right-looking elimination on a dense copy of C, one column at a time, in the
textbook order.  Shares nothing with the GPU library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import oracle as _chol
from .ldlt import ZeroPivot, diagonal_blocks  # noqa: F401  (same block rule, same error)


@dataclass
class LUFactor:
    n: int
    perm: np.ndarray    # analysis permutation P (new -> old)
    q: np.ndarray       # row order: row i of L U is row q[i] of C
    L: np.ndarray       # dense unit lower triangular n x n
    U: np.ndarray       # dense upper triangular n x n
    blocks: list        # diagonal blocks [(b0, b1)]


def permuted_full(A, perm) -> np.ndarray:
    """Dense C = P A P^T from all stored entries (C[pinv[i], pinv[j]] = A[i, j])."""
    perm = np.asarray(perm)
    pinv = np.empty_like(perm)
    pinv[perm] = np.arange(perm.size)
    C = np.zeros((A.n, A.n))
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    C[pinv[rows], pinv[A.colind]] = A.values
    return C


def factor_dense(C: np.ndarray, blocks: list, perm=None) -> LUFactor:
    """Row-pivoted LU of the dense C, pivots searched inside the diagonal blocks."""
    n = C.shape[0]
    S = np.array(C, dtype=np.float64, copy=True)
    L = np.eye(n)
    U = np.zeros((n, n))
    q = np.arange(n)
    block_end = np.zeros(n, dtype=np.int64)
    for b0, b1 in blocks:
        block_end[b0:b1] = b1
    for k in range(n):
        b1 = int(block_end[k])
        p = k + int(np.argmax(np.abs(S[k:b1, k])))   # first of equal maxima
        if S[p, k] == 0.0:
            raise ZeroPivot(k)
        if p != k:
            S[[k, p], :] = S[[p, k], :]
            L[[k, p], :k] = L[[p, k], :k]            # rows of the eliminated columns
            q[[k, p]] = q[[p, k]]
        U[k, k:] = S[k, k:]
        l = S[k + 1:, k] / S[k, k]
        L[k + 1:, k] = l
        S[k + 1:, k + 1:] -= np.outer(l, S[k, k + 1:])
    return LUFactor(n, None if perm is None else np.asarray(perm), q, L, U, list(blocks))


def factor(A, perm, tile: int = 64) -> LUFactor:
    """L U of Q P A P^T with row pivoting restricted to the diagonal blocks."""
    blocks = diagonal_blocks(A, perm, tile)
    F = factor_dense(permuted_full(A, perm), blocks)
    F.perm = np.asarray(perm)
    return F


def reconstruct(F: LUFactor) -> np.ndarray:
    """Q^T L U (which equals C up to rounding)."""
    M = F.L @ F.U
    out = np.empty_like(M)
    out[F.q] = M
    return out


def solve(F: LUFactor, b: np.ndarray) -> np.ndarray:
    """x = A^{-1} b: C (P x) = P b, so P x = U^{-1} L^{-1} Q P b."""
    vec = b.ndim == 1
    B = b.reshape(F.n, -1)
    y = np.linalg.solve(F.L, B[F.perm][F.q])
    z = np.linalg.solve(F.U, y)
    x = np.empty_like(z)
    x[F.perm] = z
    return x[:, 0] if vec else x


def growth(F: LUFactor) -> float:
    """max |U| / max |C|: the element growth that restricted pivoting allows."""
    return float(np.abs(F.U).max() / np.abs(reconstruct(F)).max())


__all__ = ["LUFactor", "ZeroPivot", "diagonal_blocks", "permuted_full", "factor_dense", "factor",
           "reconstruct", "solve", "growth", "_chol"]
