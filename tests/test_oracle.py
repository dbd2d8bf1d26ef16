"""Pins of the oracle against what mathematics fixes independently of it.

* brute-force dense boolean elimination (pattern of L, etree, column counts,
  fundamental supernodes) on tiny inputs;
* LAPACK's dense Cholesky (numpy.linalg.cholesky) of the permuted matrix;
* closed forms: the tridiagonal factor and Green's function, nnz(L) of the
  2D grid in natural order, dense / diagonal / arrowhead patterns, and the
  determinant of constant-coefficient Dirichlet Laplacians;
* the first non-positive pivot of a plain dense elimination.
"""
import numpy as np
import pytest

import gen


def brute_pattern(A, perm):
    """Boolean pattern of L by dense elimination of the pattern of C = P A P^T."""
    M = np.zeros((A.n, A.n), dtype=bool)
    M[np.repeat(np.arange(A.n), np.diff(A.rowptr)), A.colind] = True  # stored pattern
    C = M[np.ix_(perm, perm)] | np.eye(A.n, dtype=bool)
    G = np.tril(C)
    n = A.n
    for j in range(n):
        rows = np.nonzero(G[j + 1:, j])[0] + j + 1
        if rows.size:
            G[np.ix_(rows, rows)] |= np.tril(np.ones((rows.size, rows.size), dtype=bool))
    return np.tril(G)


def brute_symbolic(G):
    n = G.shape[0]
    parent = np.full(n, -1, np.int32)
    for j in range(n):
        below = np.nonzero(G[j + 1:, j])[0]
        if below.size:
            parent[j] = j + 1 + below[0]
    counts = G.sum(axis=0).astype(np.int64)
    nchild = np.bincount(parent[parent >= 0], minlength=n)
    starts = [0]
    for j in range(1, n):
        same = (parent[j - 1] == j and nchild[j] == 1
                and set(np.nonzero(G[:, j - 1])[0]) == {j - 1} | set(np.nonzero(G[:, j])[0]))
        if not same:
            starts.append(j)
    starts.append(n)
    return parent, counts, np.array(starts, np.int32)


def brute_relaxed(G, starts, parent):
    """Relaxed supernodes computed from the dense pattern: merged row sets are
    unions of the columns' patterns, zeros counted entry by entry."""
    n = G.shape[0]
    groups = []
    for p in range(len(starts) - 1):
        f, l = int(starts[p]), int(starts[p + 1])
        if groups and groups[-1][1] == f and parent[f - 1] == f:
            cols = range(groups[-1][0], l)
            rowset = np.zeros(n, dtype=bool)
            for j in cols:
                rowset |= G[:, j]
            rows = np.nonzero(rowset)[0]
            padded = sum(int(np.sum(rows >= j)) for j in cols)
            true = int(sum(G[:, j].sum() for j in cols))
            m = rows.size
            div = 2 if m <= 16 else (5 if m <= 64 else 20)
            if (padded - true) * div <= padded:
                groups[-1][1] = l
                continue
        groups.append([f, l])
    return np.array([g[0] for g in groups] + [n], np.int32)


def random_perm(n, seed):
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


TINY = [
    ("random", lambda: gen.random_spd_pattern(40, 0.08, seed=11)),
    ("random_dense", lambda: gen.random_spd_pattern(30, 0.3, seed=12)),
    ("random_sparse", lambda: gen.random_spd_pattern(60, 0.02, seed=13)),
    ("grid2d", lambda: gen.laplace2d(7)),
    ("grid3d", lambda: gen.fv3d(4, 3, 3, seed=5)),
    ("landice", lambda: gen.landice(3, 3, 3, seed=6)),
]


@pytest.mark.parametrize("name,make", TINY, ids=[t[0] for t in TINY])
@pytest.mark.parametrize("pseed", [None, 1, 2])
def test_symbolic_vs_brute_force(oracle_lib, name, make, pseed):
    A = make()
    perm = np.arange(A.n, dtype=np.int32) if pseed is None else random_perm(A.n, pseed)
    G = brute_pattern(A, perm)
    bparent, bcounts, bstarts = brute_symbolic(G)
    parent, counts = oracle_lib.symbolic(A, perm)
    np.testing.assert_array_equal(parent, bparent)
    np.testing.assert_array_equal(counts, bcounts)
    sptr, spar = oracle_lib.supernodes(parent, counts)
    np.testing.assert_array_equal(sptr, bstarts)
    rptr, rpar = oracle_lib.relaxed_supernodes(parent, counts)
    np.testing.assert_array_equal(rptr, brute_relaxed(G, bstarts, bparent))
    # supernodal parent: supernode that holds parent(last column)
    for ptr, par in ((sptr, spar), (rptr, rpar)):
        col2s = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
        for s in range(len(ptr) - 1):
            last = ptr[s + 1] - 1
            want = -1 if bparent[last] < 0 else col2s[bparent[last]]
            assert par[s] == want
    # the numeric factor has exactly the brute-force pattern
    F = oracle_lib.factor(A, perm)
    Ld = F.L().toarray()
    rows, cols = np.nonzero(G)
    assert F.nnz == G.sum()
    assert set(zip(*np.nonzero(F.L().toarray() != 0))) <= set(zip(rows, cols))
    assert np.all(np.diff(F.Li[F.Lp[0]:F.Lp[1]]) > 0) if F.Lp[1] - F.Lp[0] > 1 else True
    del Ld


@pytest.mark.parametrize("name,make", TINY, ids=[t[0] for t in TINY])
@pytest.mark.parametrize("pseed", [None, 3])
def test_factor_vs_lapack(oracle_lib, name, make, pseed):
    A = make()
    perm = np.arange(A.n, dtype=np.int32) if pseed is None else random_perm(A.n, pseed)
    C = A.dense()[np.ix_(perm, perm)]
    Lref = np.linalg.cholesky(C)
    F = oracle_lib.factor(A, perm)
    L = F.L().toarray()
    colmax = np.abs(Lref).max(axis=0)
    err = np.abs(L - Lref).max(axis=0) / colmax
    # Cholesky perturbation bound: relative factor error of order cond(C) * u
    tol = max(1e-13, 4.0 * np.linalg.cond(C) * np.finfo(float).eps)
    assert err.max() < tol
    # solves against dense LAPACK-based solve
    b = gen.rhs(A.n, 3, seed=7)
    x = oracle_lib.solve(F, b)
    Ad = A.dense()
    xref = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    assert np.abs(x - xref).max() / np.abs(xref).max() < max(1e-13, 8 * kappa * 2.2e-16)
    # normwise backward error of a backward-stable Cholesky solve is O(u)
    r = b - Ad @ x
    berr = np.linalg.norm(r, axis=0) / (np.linalg.norm(Ad, 2) * np.linalg.norm(x, axis=0)
                                         + np.linalg.norm(b, axis=0))
    assert berr.max() < 1e-15
    assert oracle_lib.factor_error(A, perm, F.L()) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 17, 200])
def test_tridiagonal_closed_form(oracle_lib, n):
    A = gen.laplace1d(n)
    perm = np.arange(n, dtype=np.int32)
    F = oracle_lib.factor(A, perm)
    L = F.L().toarray()
    j = np.arange(1, n + 1, dtype=np.float64)  # 1-based
    np.testing.assert_allclose(np.diag(L), np.sqrt((j + 1) / j), rtol=1e-14)
    if n > 1:
        np.testing.assert_allclose(np.diag(L, -1), -np.sqrt(j[:-1] / (j[:-1] + 1)), rtol=1e-14)
    assert F.nnz == 2 * n - 1
    parent, _ = oracle_lib.symbolic(A, perm)
    np.testing.assert_array_equal(parent[:-1], np.arange(1, n))
    assert parent[-1] == -1
    # Green's function: (A^{-1})_{ik} = min(i,k) (n+1-max(i,k)) / (n+1), 1-based
    I = np.eye(n)
    X = oracle_lib.solve(F, I)
    ii, kk = np.meshgrid(j, j, indexing="ij")
    G = np.minimum(ii, kk) * (n + 1 - np.maximum(ii, kk)) / (n + 1)
    assert np.abs(X - G).max() / np.abs(G).max() < 1e-12


@pytest.mark.parametrize("m", [2, 3, 5, 32])
def test_grid2d_natural_nnz(oracle_lib, m):
    A = gen.laplace2d(m)
    n = m * m
    parent, counts = oracle_lib.symbolic(A, np.arange(n, dtype=np.int32))
    assert counts.sum() == (n - m) * (m + 1) + 2 * m - 1
    np.testing.assert_array_equal(parent[:-1], np.arange(1, n))


def test_dense_pattern_one_supernode(oracle_lib):
    n = 23
    rng = np.random.default_rng(3)
    B = rng.standard_normal((n, n))
    A = gen.dense_to_csr(B @ B.T + n * np.eye(n))
    perm = random_perm(n, 4)
    parent, counts = oracle_lib.symbolic(A, perm)
    assert counts.sum() == n * (n + 1) // 2
    assert oracle_lib.flops_from_counts(counts) == n * (n + 1) * (2 * n + 1) // 6
    sptr, spar = oracle_lib.supernodes(parent, counts)
    np.testing.assert_array_equal(sptr, [0, n])
    np.testing.assert_array_equal(spar, [-1])
    np.testing.assert_array_equal(oracle_lib.relaxed_supernodes(parent, counts)[0], [0, n])


def test_diagonal_forest(oracle_lib):
    n = 9
    A = gen.dense_to_csr(np.diag(np.arange(1.0, n + 1)))
    parent, counts = oracle_lib.symbolic(A, np.arange(n, dtype=np.int32))
    assert (parent == -1).all() and (counts == 1).all()
    sptr, spar = oracle_lib.supernodes(parent, counts)
    np.testing.assert_array_equal(sptr, np.arange(n + 1))
    assert (spar == -1).all()
    F = oracle_lib.factor(A, np.arange(n, dtype=np.int32))
    np.testing.assert_allclose(F.Lx, np.sqrt(np.arange(1.0, n + 1)), rtol=1e-15)


def test_arrowhead_star(oracle_lib):
    n = 12
    D = np.diag(np.full(n, float(n)))
    D[-1, :] = 1.0
    D[:, -1] = 1.0
    D[-1, -1] = float(n)
    A = gen.dense_to_csr(D)
    parent, counts = oracle_lib.symbolic(A, np.arange(n, dtype=np.int32))
    assert (parent[:-1] == n - 1).all() and parent[-1] == -1
    assert counts.sum() == (n - 1) * 2 + 1  # no fill
    # dense-last-row-first order fills everything
    perm = np.r_[n - 1, np.arange(n - 1)].astype(np.int32)
    _, c2 = oracle_lib.symbolic(A, perm)
    assert c2.sum() == n * (n + 1) // 2


def _logdet_laplace(m, dims):
    k = np.arange(1, m + 1)
    lam = 4 * np.sin(np.pi * k / (2 * (m + 1))) ** 2
    grids = np.meshgrid(*([lam] * dims), indexing="ij")
    return float(np.sum(np.log(sum(grids))))


def test_logdet_closed_form_2d(oracle_lib):
    A = gen.laplace2d(32)
    want = _logdet_laplace(32, 2)
    assert abs(want - 1210.72312053205) < 1e-9
    for perm in (np.arange(A.n, dtype=np.int32), random_perm(A.n, 9)):
        F = oracle_lib.factor(A, perm)
        assert abs(oracle_lib.logdet(F) - want) / want < 1e-12


def test_logdet_closed_form_3d(oracle_lib):
    A = gen.laplace3d(9)
    want = _logdet_laplace(9, 3)
    F = oracle_lib.factor(A, random_perm(A.n, 10))
    assert abs(oracle_lib.logdet(F) - want) / want < 1e-12


def dense_first_bad_pivot(C):
    C = C.copy()
    n = C.shape[0]
    for j in range(n):
        if not C[j, j] > 0:
            return j
        C[j + 1:, j] /= np.sqrt(C[j, j])
        C[j + 1:, j + 1:] -= np.outer(C[j + 1:, j], C[j + 1:, j]) / 1.0
        C[j + 1:, j + 1:] = C[j + 1:, j + 1:]  # keep full symmetric trailing block
        C[j, j + 1:] = C[j + 1:, j]
    return -1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_not_spd_first_pivot(oracle_lib, seed):
    A = gen.random_spd_pattern(40, 0.1, seed=20 + seed, shift=1.0)
    M = A.to_scipy().tolil()
    rng = np.random.default_rng(seed)
    bad = int(rng.integers(0, 40))
    M[bad, bad] = -5.0
    B = gen.matrices._from_scipy(M.tocsr())
    perm = random_perm(40, 30 + seed)
    j = dense_first_bad_pivot(B.dense()[np.ix_(perm, perm)])
    assert j >= 0
    with pytest.raises(oracle_lib.NotSPD) as e:
        oracle_lib.factor(B, perm)
    assert e.value.index == perm[j]


def test_missing_diagonal_added(oracle_lib):
    # zero diagonal entry absent from the pattern -> structural diagonal, not SPD
    D = np.array([[2.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 2.0]])
    A = gen.dense_to_csr(D)
    parent, counts = oracle_lib.symbolic(A, np.arange(3, dtype=np.int32))
    assert counts.tolist() == [2, 2, 1]
    # pivot of column 1 is 0 - 1/2 < 0
    with pytest.raises(oracle_lib.NotSPD) as e:
        oracle_lib.factor(A, np.arange(3, dtype=np.int32))
    assert e.value.index == 1


def test_manufactured_solution(oracle_lib):
    A = gen.fv3d(6, 5, 4, seed=3)
    x_true = gen.rhs(A.n, 2, seed=4)
    b = A.to_scipy() @ x_true
    F = oracle_lib.factor(A, random_perm(A.n, 5))
    x = oracle_lib.solve(F, b)
    cond = np.linalg.cond(A.dense())
    assert np.abs(x - x_true).max() / np.abs(x_true).max() < cond * 1e-15


def test_explicit_zeros_count_in_pattern(oracle_lib):
    """An explicitly stored zero is structural: it creates fill like any entry."""
    n = 8
    D = np.diag(np.full(n, 4.0))
    keep = np.zeros((n, n), dtype=bool)
    keep[0, 5] = keep[5, 0] = True  # stored zero
    D[1, 6] = D[6, 1] = -1.0
    A = gen.dense_to_csr(D, keep_zeros_mask=keep)
    assert A.nnz == n + 4
    perm = np.arange(n, dtype=np.int32)
    G = brute_pattern(A, perm)
    parent, counts = oracle_lib.symbolic(A, perm)
    bparent, bcounts, _ = brute_symbolic(G)
    np.testing.assert_array_equal(parent, bparent)
    np.testing.assert_array_equal(counts, bcounts)
    assert parent[0] == 5 and counts[0] == 2


@pytest.mark.parametrize("m,pseed", [(6, None), (9, 4), (12, None)])
def test_relaxed_supernodes_on_grids(oracle_lib, m, pseed):
    """Grids with crossing separators: relaxed groups vs brute force, and the
    merge never adds more than the allowed share of zeros per group."""
    A = gen.fv3d(m, m, max(2, m // 2), seed=1)
    perm = np.arange(A.n, dtype=np.int32) if pseed is None else random_perm(A.n, pseed)
    G = brute_pattern(A, perm)
    bparent, bcounts, bstarts = brute_symbolic(G)
    rptr, _ = oracle_lib.relaxed_supernodes(bparent, bcounts)
    np.testing.assert_array_equal(rptr, brute_relaxed(G, bstarts, bparent))
    assert len(rptr) <= len(bstarts)


# ---------------------------------------------------------------------------
# Pins of the oracle's report functions.  Every GPU solve and factor check is
# judged through them, so each is tied to a value fixed by hand arithmetic on
# integer data (exact in floating point), chosen so that a wrong axis, a
# wrong triangle, a transposed operand, a dropped factor of two or a zero
# result changes the number.


def test_rel_residual_closed_form(oracle_lib):
    """tridiag(-1,2,-1) times the all-ones vector is e_1 + e_n exactly, so
    ||b||_2 = sqrt(2); perturbing x_k by d gives r = -d A e_k, whose norm is
    |d| sqrt(6) inside and |d| sqrt(5) at either end."""
    n = 9
    A = gen.laplace1d(n)
    x = np.ones((n, 4))
    b = np.zeros((n, 4))
    b[0, :] = b[-1, :] = 1.0
    np.testing.assert_array_equal(oracle_lib.rel_residual(A, x, b), np.zeros(4))
    xp = x.copy()
    xp[4, 0] += 0.5       # interior
    xp[0, 1] -= 0.25      # first row: (2, -1)
    xp[8, 2] += 2.0       # last row: (-1, 2)
    # column 3 untouched
    rho = oracle_lib.rel_residual(A, xp, b)
    assert rho.shape == (4,)
    want = np.array([0.5 * np.sqrt(6), 0.25 * np.sqrt(5), 2.0 * np.sqrt(5), 0.0]) / np.sqrt(2)
    np.testing.assert_allclose(rho, want, rtol=1e-15, atol=0)
    # one column given as a vector
    assert oracle_lib.rel_residual(A, xp[:, 0], b[:, 0]).shape == (1,)


def test_rel_residual_uses_both_triangles(oracle_lib):
    """A nonsymmetric CSR whose upper triangle differs from the lower one: the
    residual is the plain b - A x of the stored matrix (both triangles)."""
    M = np.array([[3.0, 1.0, 0.0], [0.0, 5.0, 2.0], [4.0, 0.0, 7.0]])
    A = gen.dense_to_csr(M)
    x = np.array([[1.0], [2.0], [-1.0]])
    b = M @ x  # [5, 8, -3] exactly
    assert oracle_lib.rel_residual(A, x, b)[0] == 0.0
    b2 = b + np.array([[0.0], [3.0], [4.0]])
    assert oracle_lib.rel_residual(A, x, b2)[0] == 5.0 / np.linalg.norm(b2)


def _integer_factor_problem(perm):
    """An integer lower-triangular L (positive diagonal, with fill), C = L L^T
    exactly, and A = P^T C P so that C = P A P^T."""
    L = np.array([[2, 0, 0, 0, 0],
                  [1, 1, 0, 0, 0],
                  [0, 3, 2, 0, 0],
                  [1, 0, 1, 1, 0],
                  [0, 2, 0, 1, 3]], dtype=np.float64)
    C = L @ L.T
    A = np.empty_like(C)
    A[np.ix_(perm, perm)] = C
    return L, C, gen.dense_to_csr(A)


@pytest.mark.parametrize("perm", [np.arange(5), np.array([3, 0, 4, 1, 2])])
def test_factor_error_closed_form(oracle_lib, perm):
    """||C - L'L'^T||_F / ||C||_F for L' = L + d e_i e_j^T: with v = L[:, j],
    C - L'L'^T = -d (e_i v^T + v e_i^T) - d^2 e_i e_i^T, whose squared
    Frobenius norm is (2 d v_i + d^2)^2 + 2 d^2 sum_{b != i} v_b^2."""
    import scipy.sparse as sp
    perm = perm.astype(np.int32)
    L, C, A = _integer_factor_problem(perm)
    assert oracle_lib.factor_error(A, perm, sp.csc_matrix(L)) == 0.0
    cn = np.sqrt(np.sum(C * C))
    for (i, j, d) in ((2, 1, 0.5), (4, 4, -1.0), (3, 0, 2.0)):
        Lp = L.copy()
        Lp[i, j] += d
        v = L[:, j].copy()
        rest = np.sum(v * v) - v[i] ** 2
        want = np.sqrt((2 * d * v[i] + d * d) ** 2 + 2 * d * d * rest) / cn
        got = oracle_lib.factor_error(A, perm, sp.csc_matrix(Lp))
        assert abs(got - want) <= 1e-15 * want, (i, j, got, want)
    # a transposed factor is not a factor of C
    assert oracle_lib.factor_error(A, perm, sp.csc_matrix(L.T)) > 0.1


def test_permuted_lower_definition(oracle_lib):
    """Lower triangle of C[i][j] = S[p[i]][p[j]], where S is the symmetric
    matrix defined by the stored lower triangle (the upper triangle's values
    are not read)."""
    rng = np.random.default_rng(17)
    n = 11
    M = rng.standard_normal((n, n))
    M[np.abs(M) < 0.6] = 0.0
    M += np.diag(np.full(n, 10.0))
    # same pattern in both triangles, different values above the diagonal
    pat = (M != 0) | (M.T != 0)
    low = np.tril(np.where(pat, M, 0.0))
    upper = np.triu(np.where(pat, 1000.0 + rng.standard_normal((n, n)), 0.0), 1)
    A = gen.dense_to_csr(low + upper, keep_zeros_mask=pat)
    S = low + np.tril(low, -1).T
    perm = rng.permutation(n).astype(np.int32)
    got = oracle_lib.permuted_lower(A, perm).toarray()
    want = np.tril(S[np.ix_(perm, perm)])
    np.testing.assert_array_equal(got, want)
