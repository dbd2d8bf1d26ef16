"""ORACLE -- test infrastructure, not part of the product.

Symmetric indefinite LDL^T with pivoting restricted to diagonal blocks (the
paper's Tacho section: besides the Cholesky factorization of an SPD matrix,
Tacho factors a symmetric indefinite matrix as L D L^T and looks for pivots
only within each diagonal block).

Plain dense definition, for inputs of up to a few thousand unknowns:

* C = P A P^T, P the analysis permutation (taken as data, like the Cholesky
  oracle).
* The columns are partitioned into diagonal blocks: the relaxed supernodes
  of C (computed by this oracle's own symbolic routines), each cut into
  consecutive pieces of at most ``tile`` columns.
* C = Q L D L^T Q^T with Q a permutation that moves a column only within its
  diagonal block, L unit lower triangular, D block diagonal with 1x1 and 2x2
  blocks, a 2x2 block never straddling two diagonal blocks.
* Pivots by Bunch-Kaufman partial pivoting (alpha = (1 + sqrt 17) / 8),
  with every candidate row and column limited to the columns of the current
  diagonal block that are not yet eliminated; rows below the block are never
  searched.  Ties go to the smallest index.  A block whose remaining
  candidates are all zero in the pivot column and on the diagonal cannot be
  factored (``ZeroPivot``).

Right-looking elimination on a dense copy of C, one pivot (1x1 or 2x2) at a
time, in the textbook order.  Shares nothing with the GPU library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import oracle as _chol

ALPHA = (1.0 + np.sqrt(17.0)) / 8.0


class ZeroPivot(Exception):
    def __init__(self, index: int):
        super().__init__(f"no usable pivot in the diagonal block at permuted column {index}")
        self.index = index


@dataclass
class LDLFactor:
    n: int
    perm: np.ndarray    # analysis permutation P (new -> old)
    q: np.ndarray       # pivot order within blocks: row i of L is row q[i] of C
    L: np.ndarray       # dense unit lower triangular n x n
    d: np.ndarray       # diagonal of D
    e: np.ndarray       # subdiagonal of D (e[k] couples k and k + 1; 0 outside 2x2 blocks)
    two: np.ndarray     # bool[n]: True at the first column of each 2x2 block
    blocks: list        # diagonal blocks [(b0, b1)]

    def D(self) -> np.ndarray:
        return np.diag(self.d) + np.diag(self.e[:-1], -1) + np.diag(self.e[:-1], 1)


def diagonal_blocks(A, perm, tile: int = 64) -> list:
    """Relaxed supernodes of C = P A P^T, each cut into pieces of at most
    ``tile`` columns."""
    parent, counts = _chol.symbolic(A, perm)
    sptr, _ = _chol.relaxed_supernodes(parent, counts)
    out = []
    for s in range(len(sptr) - 1):
        for b0 in range(int(sptr[s]), int(sptr[s + 1]), tile):
            out.append((b0, min(b0 + tile, int(sptr[s + 1]))))
    return out


def permuted_dense(A, perm) -> np.ndarray:
    """Dense C = P A P^T from the original lower triangle's values."""
    lower = _chol.permuted_lower(A, perm).toarray()
    return lower + np.tril(lower, -1).T


def factor_dense(C: np.ndarray, blocks: list, perm=None) -> LDLFactor:
    """Restricted Bunch-Kaufman L D L^T of the dense symmetric C."""
    n = C.shape[0]
    S = np.array(C, dtype=np.float64, copy=True)
    L = np.eye(n)
    d = np.zeros(n)
    e = np.zeros(n)
    two = np.zeros(n, dtype=bool)
    q = np.arange(n)
    block_end = np.zeros(n, dtype=np.int64)
    for b0, b1 in blocks:
        block_end[b0:b1] = b1

    def swap(i, j):
        if i == j:
            return
        S[[i, j], :] = S[[j, i], :]
        S[:, [i, j]] = S[:, [j, i]]
        L[[i, j], :i] = L[[j, i], :i]   # rows of the columns already eliminated
        q[[i, j]] = q[[j, i]]

    k = 0
    while k < n:
        b1 = int(block_end[k])
        cand = np.arange(k + 1, b1)
        col = np.abs(S[cand, k])
        lam = float(col.max()) if cand.size else 0.0
        akk = abs(S[k, k])
        size = 1
        if lam == 0.0:
            if S[k, k] == 0.0:
                raise ZeroPivot(k)
        elif akk >= ALPHA * lam:
            pass
        else:
            r = int(cand[int(np.argmax(col))])
            others = [j for j in range(k, b1) if j != r]
            sigma = float(np.abs(S[r, others]).max())
            if akk * sigma >= ALPHA * lam * lam:
                pass
            elif abs(S[r, r]) >= ALPHA * sigma:
                swap(k, r)
            else:
                swap(k + 1, r)
                size = 2
        if size == 1:
            piv = S[k, k]
            d[k] = piv
            l = S[k + 1:, k] / piv
            L[k + 1:, k] = l
            S[k + 1:, k + 1:] -= np.outer(l, S[k + 1:, k])
            k += 1
        else:
            E = S[k:k + 2, k:k + 2].copy()
            d[k], d[k + 1], e[k] = E[0, 0], E[1, 1], E[1, 0]
            two[k] = True
            Cb = S[k + 2:, k:k + 2]
            Lb = Cb @ np.linalg.inv(E)
            L[k + 2:, k:k + 2] = Lb
            S[k + 2:, k + 2:] -= Lb @ Cb.T
            k += 2
    return LDLFactor(n, None if perm is None else np.asarray(perm), q, L, d, e, two, list(blocks))


def factor(A, perm, tile: int = 64) -> LDLFactor:
    """L D L^T of C = P A P^T with pivoting restricted to its diagonal blocks."""
    blocks = diagonal_blocks(A, perm, tile)
    F = factor_dense(permuted_dense(A, perm), blocks)
    F.perm = np.asarray(perm)
    return F


def reconstruct(F: LDLFactor) -> np.ndarray:
    """Q L D L^T Q^T (which equals C up to rounding)."""
    M = F.L @ F.D() @ F.L.T
    out = np.empty_like(M)
    out[np.ix_(F.q, F.q)] = M
    return out


def solve(F: LDLFactor, b: np.ndarray) -> np.ndarray:
    """x = A^{-1} b through x = P^T Q L^{-T} D^{-1} L^{-1} Q^T P b."""
    vec = b.ndim == 1
    B = b.reshape(F.n, -1)
    y = B[F.perm][F.q]                              # Q^T P b
    z = np.linalg.solve(F.L, y)                     # L^{-1}
    w = np.linalg.solve(F.D(), z)                   # D^{-1}
    v = np.linalg.solve(F.L.T, w)                   # L^{-T}
    x = np.empty_like(v)
    x[F.perm[F.q]] = v
    return x[:, 0] if vec else x


def inertia(F: LDLFactor) -> tuple:
    """(positive, negative, zero) eigenvalue counts of D."""
    ev = []
    k = 0
    while k < F.n:
        if F.two[k]:
            ev.extend(np.linalg.eigvalsh(F.D()[k:k + 2, k:k + 2]))
            k += 2
        else:
            ev.append(F.d[k])
            k += 1
    ev = np.asarray(ev)
    return int((ev > 0).sum()), int((ev < 0).sum()), int((ev == 0).sum())
