"""ORACLE -- test infrastructure, not part of the product.

ctypes wrapper around ``oracle.c`` plus the reports of the plain definition
C = P A P^T = L L^T, x = P^T L^{-T} L^{-1} P b (Tacho section of the paper;
the three phases of the Trilinos section):

* ``factor_error``  ||C - L L^T||_F / ||C||_F over pattern(L) u pattern(C)
* ``rel_residual``  ||b - A x||_2 / ||b||_2 per right-hand side
* ``logdet``        2 sum_j log L_jj
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_symbolic.argtypes = [ctypes.c_int64, _i64p, _i32p, _i32p, _i32p, _i64p]
        lib.oracle_supernodes.argtypes = [ctypes.c_int64, _i32p, _i64p, _i32p, _i32p, _i64p]
        lib.oracle_relaxed_supernodes.argtypes = [ctypes.c_int64, _i32p, _i64p, _i32p, _i32p,
                                                  _i64p]
        lib.oracle_relaxed_supernodes.restype = ctypes.c_int
        lib.oracle_factor.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _i32p, _i32p, _i64p,
                                      _i32p, _f64p, _i64p]
        lib.oracle_solve.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _i32p, ctypes.c_int64,
                                     _f64p, ctypes.c_int64, _f64p, ctypes.c_int64]
        for f in (lib.oracle_symbolic, lib.oracle_supernodes, lib.oracle_factor, lib.oracle_solve):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


class NotSPD(Exception):
    def __init__(self, index: int):
        super().__init__(f"matrix is not SPD: first non-positive pivot at original index {index}")
        self.index = index


@dataclass
class OracleFactor:
    n: int
    perm: np.ndarray     # int32[n], new -> old
    parent: np.ndarray   # int32[n]
    colcount: np.ndarray  # int64[n]
    Lp: np.ndarray       # int64[n+1]
    Li: np.ndarray       # int32[nnz(L)]
    Lx: np.ndarray       # float64[nnz(L)]

    def L(self) -> sp.csc_matrix:
        return sp.csc_matrix((self.Lx, self.Li, self.Lp), shape=(self.n, self.n))

    @property
    def nnz(self) -> int:
        return int(self.Lp[-1])


def _perm(perm, n):
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    if perm.shape != (n,):
        raise ValueError("permutation has the wrong length")
    return perm


def symbolic(A, perm):
    """(parent int32[n], colcount int64[n]) of C = P A P^T."""
    lib = _load()
    n = A.n
    perm = _perm(perm, n)
    parent = np.empty(n, np.int32)
    cc = np.empty(n, np.int64)
    rc = lib.oracle_symbolic(n, _p(A.rowptr, _i64p), _p(A.colind, _i32p), _p(perm, _i32p),
                             _p(parent, _i32p), _p(cc, _i64p))
    if rc != 0:
        raise ValueError(f"oracle_symbolic failed ({rc})")
    return parent, cc


def supernodes(parent, colcount):
    """(super_ptr int32[ns+1], super_parent int32[ns]) -- fundamental supernodes."""
    lib = _load()
    n = len(parent)
    parent = np.ascontiguousarray(parent, np.int32)
    colcount = np.ascontiguousarray(colcount, np.int64)
    sptr = np.empty(n + 1, np.int32)
    spar = np.empty(max(n, 1), np.int32)
    ns = ctypes.c_int64(0)
    rc = lib.oracle_supernodes(n, _p(parent, _i32p), _p(colcount, _i64p), _p(sptr, _i32p),
                               _p(spar, _i32p), ctypes.byref(ns))
    if rc != 0:
        raise ValueError(f"oracle_supernodes failed ({rc})")
    k = ns.value
    return sptr[:k + 1].copy(), spar[:k].copy()


def relaxed_supernodes(parent, colcount):
    """(super_ptr, super_parent) of the relaxed supernodes (chains merged while the
    explicit zeros of the merged dense block stay small)."""
    lib = _load()
    n = len(parent)
    parent = np.ascontiguousarray(parent, np.int32)
    colcount = np.ascontiguousarray(colcount, np.int64)
    sptr = np.empty(n + 1, np.int32)
    spar = np.empty(max(n, 1), np.int32)
    ns = ctypes.c_int64(0)
    rc = lib.oracle_relaxed_supernodes(n, _p(parent, _i32p), _p(colcount, _i64p), _p(sptr, _i32p),
                                       _p(spar, _i32p), ctypes.byref(ns))
    if rc != 0:
        raise ValueError(f"oracle_relaxed_supernodes failed ({rc})")
    k = ns.value
    return sptr[:k + 1].copy(), spar[:k].copy()


def factor(A, perm) -> OracleFactor:
    lib = _load()
    n = A.n
    perm = _perm(perm, n)
    parent, cc = symbolic(A, perm)
    Lp = np.zeros(n + 1, np.int64)
    np.cumsum(cc, out=Lp[1:])
    nnz = int(Lp[-1])
    Li = np.empty(max(nnz, 1), np.int32)
    Lx = np.empty(max(nnz, 1), np.float64)
    fail = ctypes.c_int64(-1)
    vals = np.ascontiguousarray(A.values, np.float64)
    rc = lib.oracle_factor(n, _p(A.rowptr, _i64p), _p(A.colind, _i32p), _p(vals, _f64p),
                           _p(perm, _i32p), _p(parent, _i32p), _p(Lp, _i64p), _p(Li, _i32p),
                           _p(Lx, _f64p), ctypes.byref(fail))
    if rc == -3:
        raise NotSPD(int(fail.value))
    if rc != 0:
        raise ValueError(f"oracle_factor failed ({rc})")
    return OracleFactor(n, perm, parent, cc, Lp, Li[:nnz], Lx[:nnz])


def solve(F: OracleFactor, b: np.ndarray) -> np.ndarray:
    """x = P^T L^{-T} L^{-1} P b; b is n or n x nrhs."""
    lib = _load()
    vec = b.ndim == 1
    B = np.asfortranarray(b.reshape(F.n, -1), dtype=np.float64)
    X = np.empty_like(B, order="F")
    rc = lib.oracle_solve(F.n, _p(F.Lp, _i64p), _p(F.Li, _i32p), _p(F.Lx, _f64p),
                          _p(F.perm, _i32p), B.shape[1], _p(B, _f64p), F.n, _p(X, _f64p), F.n)
    if rc != 0:
        raise ValueError(f"oracle_solve failed ({rc})")
    return X[:, 0] if vec else X


def permuted_lower(A, perm) -> sp.csc_matrix:
    """Lower triangle of C = P A P^T built from the original lower triangle's values."""
    perm = np.asarray(perm)
    pinv = np.empty_like(perm)
    pinv[perm] = np.arange(len(perm))
    M = A.to_scipy().tocoo()
    keep = M.row >= M.col
    r = pinv[M.row[keep]]
    c = pinv[M.col[keep]]
    rr = np.maximum(r, c)
    cc = np.minimum(r, c)
    return sp.csc_matrix((M.data[keep], (rr, cc)), shape=A.to_scipy().shape)


def factor_error(A, perm, L: sp.spmatrix) -> float:
    """||C - L L^T||_F / ||C||_F on the lower triangle, counting off-diagonal terms twice."""
    C = permuted_lower(A, perm)
    LLt = sp.tril(sp.csc_matrix(L) @ sp.csc_matrix(L).T).tocsc()
    D = (C - LLt).tocoo()
    w = np.where(D.row == D.col, 1.0, 2.0)
    Cc = C.tocoo()
    wc = np.where(Cc.row == Cc.col, 1.0, 2.0)
    return float(np.sqrt(np.sum(w * D.data ** 2)) / np.sqrt(np.sum(wc * Cc.data ** 2)))


def rel_residual(A, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """||b - A x||_2 / ||b||_2 per column (FP64)."""
    M = A.to_scipy()
    X = x.reshape(A.n, -1)
    B = b.reshape(A.n, -1)
    R = B - M @ X
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)


def logdet(F: OracleFactor) -> float:
    return float(2.0 * np.sum(np.log(F.Lx[F.Lp[:-1]])))


def flops_from_counts(colcount) -> int:
    """Algorithmic flop count sum_j eta_j^2."""
    c = np.asarray(colcount, dtype=np.int64)
    return int(np.sum(c * c))
