"""Seeded synthetic SPD matrices and right-hand sides.

Every matrix is returned as a full (both triangles) symmetric CSR with sorted
column indices: ``rowptr`` int64[n+1], ``colind`` int32[nnz], ``values``
float64[nnz].  Random numbers come from ``numpy.random.default_rng(seed)``
(PCG64) so that every consumer sees the same bits for the same seed.

The shapes follow the workloads of the paper's Tacho section: 2D/3D model
problems and an extruded, anisotropic, two-DOF-per-node land-ice-like mesh
(the Albany Antarctica meshes themselves are not available; these stand in
for them), plus batches of small 3D subdomain problems (the analogue of many
MPI ranks sharing one GPU).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int64[n+1]
    colind: np.ndarray  # int32[nnz]
    values: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.values, self.colind, self.rowptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def _from_scipy(M) -> CSR:
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.eliminate_zeros()  # structural pattern = stored nonzeros only
    M.sort_indices()
    return CSR(
        n=M.shape[0],
        rowptr=np.ascontiguousarray(M.indptr, dtype=np.int64),
        colind=np.ascontiguousarray(M.indices, dtype=np.int32),
        values=np.ascontiguousarray(M.data, dtype=np.float64),
    )


def dense_to_csr(A: np.ndarray, keep_zeros_mask: np.ndarray | None = None) -> CSR:
    """CSR of a dense matrix; ``keep_zeros_mask`` marks explicit zeros to keep."""
    A = np.asarray(A, dtype=np.float64)
    mask = A != 0 if keep_zeros_mask is None else (A != 0) | keep_zeros_mask
    r, c = np.nonzero(mask)
    M = sp.csr_matrix((A[r, c], (r, c)), shape=A.shape)
    M.sort_indices()
    return CSR(A.shape[0], M.indptr.astype(np.int64), M.indices.astype(np.int32),
               M.data.astype(np.float64))


def laplace1d(n: int) -> CSR:
    """tridiag(-1, 2, -1), natural order."""
    main = 2.0 * np.ones(n)
    off = -np.ones(n - 1)
    return _from_scipy(sp.diags([off, main, off], [-1, 0, 1], format="csr"))


def laplace2d(m: int) -> CSR:
    """5-point Dirichlet Laplacian on an m x m grid, stencil 4 / -1, natural order."""
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    I = sp.identity(m)
    return _from_scipy(sp.kron(I, T) + sp.kron(T, I))


def _fv_operator(shape: tuple[int, ...], k: np.ndarray) -> CSR:
    """Cell-centred finite-volume operator with Dirichlet walls.

    Interior face weight: harmonic mean 2 k_c k_d / (k_c + k_d).  A boundary
    face adds 2 k_c to the diagonal.  A_cc = sum of face weights, A_cd = -t_cd.
    Cell index is x + nx*(y + ny*z) (first axis fastest).
    """
    dims = len(shape)
    n = int(np.prod(shape))
    kk = k.reshape(shape[::-1])  # C-order array indexed [z, y, x]
    idx = np.arange(n, dtype=np.int64).reshape(shape[::-1])
    diag = np.zeros(shape[::-1])
    rows, cols, vals = [], [], []
    for ax in range(dims):
        a = dims - 1 - ax  # numpy axis for grid axis `ax`
        lo = [slice(None)] * dims
        hi = [slice(None)] * dims
        lo[a] = slice(0, -1)
        hi[a] = slice(1, None)
        kc, kd = kk[tuple(lo)], kk[tuple(hi)]
        t = 2.0 * kc * kd / (kc + kd)
        diag[tuple(lo)] += t
        diag[tuple(hi)] += t
        ic, id_ = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        rows += [ic, id_]
        cols += [id_, ic]
        vals += [-t.ravel(), -t.ravel()]
        # Dirichlet walls at both ends of this axis
        first = [slice(None)] * dims
        last = [slice(None)] * dims
        first[a] = slice(0, 1)
        last[a] = slice(-1, None)
        diag[tuple(first)] += 2.0 * kk[tuple(first)]
        diag[tuple(last)] += 2.0 * kk[tuple(last)]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return _from_scipy(M.tocsr())


def fv3d(nx: int, ny: int | None = None, nz: int | None = None, seed: int = 1,
         lognormal: bool = True, rng: np.random.Generator | None = None) -> CSR:
    """3D 7-point cell-centred operator on nx*ny*nz cells, k_c = exp(N(0,1))."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    if lognormal:
        rng = np.random.default_rng(seed) if rng is None else rng
        k = np.exp(rng.standard_normal(n))
    else:
        k = np.full(n, 0.5)  # 2 k_c k_d/(k_c+k_d) = 0.5, wall 2k = 1
    return _fv_operator((nx, ny, nz), k)


def fv2d(nx: int, ny: int | None = None, seed: int = 1, lognormal: bool = True,
         rng: np.random.Generator | None = None) -> CSR:
    """2D 5-point cell-centred operator, lognormal cell coefficients."""
    ny = nx if ny is None else ny
    n = nx * ny
    if lognormal:
        rng = np.random.default_rng(seed) if rng is None else rng
        k = np.exp(rng.standard_normal(n))
    else:
        k = np.full(n, 0.5)
    return _fv_operator((nx, ny), k)


def _half_offsets_27():
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dz, dy, dx) > (0, 0, 0):
                    out.append((dx, dy, dz))
    return out


def landice(nx: int = 200, ny: int = 200, nl: int = 11, seed: int = 3,
            sigma_rel: float = 1e-4, vertical_weight: float = 1e3) -> CSR:
    """Extruded land-ice-shaped SPD system, 2 DOF per node.

    Nodes (ix, iy, il) on an nx x ny x nl grid, node id ix + nx*(iy + ny*il),
    DOF 2*node + d.  Every pair of 27-point neighbours is an edge e with a
    random SPD block S_e = G G^T + 0.1 I (G ~ N(0,1)^{2x2}) and weight w_e
    (``vertical_weight`` for pure-vertical pairs, 1 otherwise).
    A = sum_e (e_i - e_j)(e_i - e_j)^T (x) w_e S_e + sigma I with
    sigma = sigma_rel * mean(diag), SPD by construction.
    """
    rng = np.random.default_rng(seed)
    nn = nx * ny * nl
    node = np.arange(nn, dtype=np.int64).reshape(nl, ny, nx)
    dblk = np.zeros((nn, 2, 2))
    rows, cols, vals = [], [], []
    for (dx, dy, dz) in _half_offsets_27():
        sl_a = (slice(max(0, -dz), nl - max(0, dz)), slice(max(0, -dy), ny - max(0, dy)),
                slice(max(0, -dx), nx - max(0, dx)))
        sl_b = (slice(max(0, dz), nl - max(0, -dz)), slice(max(0, dy), ny - max(0, -dy)),
                slice(max(0, dx), nx - max(0, -dx)))
        ia = node[sl_a].ravel()
        ib = node[sl_b].ravel()
        ne = ia.size
        G = rng.standard_normal((ne, 2, 2))
        S = G @ np.transpose(G, (0, 2, 1)) + 0.1 * np.eye(2)
        w = vertical_weight if (dx, dy, dz) == (0, 0, 1) else 1.0
        S *= w
        np.add.at(dblk, ia, S)
        np.add.at(dblk, ib, S)
        for a in range(2):
            for b in range(2):
                rows += [2 * ia + a, 2 * ib + a]
                cols += [2 * ib + b, 2 * ia + b]
                vals += [-S[:, a, b], -S[:, b, a]]
    diag_mean = np.mean(np.concatenate([dblk[:, 0, 0], dblk[:, 1, 1]]))
    sigma = sigma_rel * diag_mean
    dblk[:, 0, 0] += sigma
    dblk[:, 1, 1] += sigma
    ii = np.arange(nn, dtype=np.int64)
    for a in range(2):
        for b in range(2):
            rows.append(2 * ii + a)
            cols.append(2 * ii + b)
            vals.append(dblk[:, a, b])
    n = 2 * nn
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return _from_scipy(M.tocsr())


def batch_fv3d(count: int = 256, seed: int = 4, lo: int = 8, hi: int = 32) -> list[CSR]:
    """``count`` independent 3D lognormal subdomain problems, sides uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=(count, 3))
    return [fv3d(int(s[0]), int(s[1]), int(s[2]), rng=rng) for s in sides]


def csr_block_diag(mats: list[CSR]) -> CSR:
    """Block-diagonal union of independent systems."""
    return _from_scipy(sp.block_diag([m.to_scipy() for m in mats], format="csr"))


def rhs(n: int, nrhs: int = 1, seed: int = 2) -> np.ndarray:
    """n x nrhs column-major N(0,1) right-hand sides; column k is the k-th draw of n values."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((nrhs, n)).T)


def random_spd_pattern(n: int, density: float, seed: int, shift: float = 1.0) -> CSR:
    """Random symmetric pattern with SPD values (diagonally dominant)."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="coo")
    M = sp.triu(M, 1)
    vals = rng.uniform(-1.0, 1.0, size=M.nnz)
    M = sp.coo_matrix((vals, (M.row, M.col)), shape=(n, n))
    S = (M + M.T).tocsr()
    d = np.asarray(abs(S).sum(axis=1)).ravel() + shift
    return _from_scipy(S + sp.diags(d))


def serving_requests(count: int = 2000, seed: int = 5, rate: float = 100.0,
                     repeat_frac: float = 0.3, n2d=(1000, 250000), n3d=(4000, 300000),
                     max_rhs: int = 16):
    """Request stream: Poisson arrivals of factor+solve or repeat-RHS solve requests.

    Returns a list of dicts with keys ``t`` (arrival time, s), ``kind``
    ('factor' or 'repeat'), ``dim`` (2 or 3), ``side`` (tuple), ``nrhs`` and
    ``seed`` (coefficients / RHS seed).  Repeat requests name ``target``, the
    index of an earlier factor request, chosen uniformly.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    factor_ids = []
    for i in range(count):
        nrhs = int(rng.integers(1, max_rhs + 1))
        if factor_ids and rng.random() < repeat_frac:
            tgt = factor_ids[int(rng.integers(0, len(factor_ids)))]
            out.append(dict(t=float(t[i]), kind="repeat", target=tgt, nrhs=nrhs,
                            seed=int(rng.integers(1 << 30))))
            continue
        if rng.random() < 0.5:
            n = float(np.exp(rng.uniform(np.log(n2d[0]), np.log(n2d[1]))))
            s = max(2, int(round(np.sqrt(n))))
            side = (s, s)
            dim = 2
        else:
            n = float(np.exp(rng.uniform(np.log(n3d[0]), np.log(n3d[1]))))
            s = max(2, int(round(n ** (1.0 / 3.0))))
            side = (s, s, s)
            dim = 3
        out.append(dict(t=float(t[i]), kind="factor", dim=dim, side=side, nrhs=nrhs,
                        seed=int(rng.integers(1 << 30))))
        factor_ids.append(i)
    return out


def shifted(A: CSR, frac: float) -> CSR:
    """Symmetric indefinite A - sigma I with sigma = frac * mean(diag(A)) (a
    Helmholtz-like shift into the spectrum of an SPD operator); same pattern."""
    M = A.to_scipy().tocsr()
    sigma = frac * float(M.diagonal().mean())
    return _from_scipy((M - sigma * sp.identity(A.n, format="csr")).tocsr())


def nonsymmetric(A: CSR, skew: float, seed: int) -> CSR:
    """Same pattern, nonsymmetric values: every off-diagonal pair (i, j), (j, i)
    becomes a_ij (1 + skew u), a_ji (1 - skew u) with u uniform in [-1, 1]
    drawn per pair (a convection-like perturbation of a symmetric operator)."""
    M = A.to_scipy().tocoo()
    rng = np.random.default_rng(seed)
    lo, hi = np.minimum(M.row, M.col), np.maximum(M.row, M.col)
    key = lo.astype(np.int64) * A.n + hi
    uniq, inv = np.unique(key, return_inverse=True)
    u = rng.uniform(-1.0, 1.0, uniq.size)[inv]
    sign = np.where(M.row < M.col, 1.0, np.where(M.row > M.col, -1.0, 0.0))
    data = M.data * (1.0 + skew * sign * u)
    return _from_scipy(sp.csr_matrix((data, (M.row, M.col)), shape=M.shape))


def laplace3d(m: int) -> CSR:
    """7-point Dirichlet Laplacian on an m^3 grid, stencil 6 / -1, natural order."""
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    I = sp.identity(m)
    return _from_scipy(sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I)
                       + sp.kron(sp.kron(T, I), I))
