"""Pins of the LU oracle (row pivoting restricted to diagonal blocks) against
what the mathematics fixes: hand-worked pivot decisions on tiny matrices
(largest entry of the column, ties to the first row, a block boundary that
hides the unrestricted choice, a column without a usable pivot), LAPACK's
partial-pivoting LU when one block spans the matrix, the Cholesky oracle's
factor for a symmetric diagonally dominant matrix (no interchange can occur
there: U = D L^T), Q C = L U, and solutions against a dense LAPACK solve."""
import numpy as np
import pytest
import scipy.linalg

import gen
import oracle
from oracle import lu


def F_of(C, blocks):
    return lu.factor_dense(np.asarray(C, dtype=float), blocks)


def test_largest_entry_becomes_pivot():
    F = F_of([[1.0, 2.0], [4.0, 3.0]], [(0, 2)])
    assert list(F.q) == [1, 0]
    np.testing.assert_array_equal(F.L, [[1.0, 0.0], [0.25, 1.0]])
    np.testing.assert_array_equal(F.U, [[4.0, 3.0], [0.0, 1.25]])


def test_tie_goes_to_first_row():
    F = F_of([[-2.0, 1.0], [2.0, 5.0]], [(0, 2)])
    assert list(F.q) == [0, 1]
    np.testing.assert_array_equal(F.L, [[1.0, 0.0], [-1.0, 1.0]])
    np.testing.assert_array_equal(F.U, [[-2.0, 1.0], [0.0, 6.0]])


def test_block_boundary_hides_larger_entry():
    # column 0's largest entry (100) lies in row 2, outside block [0, 2):
    # the pivot is row 1 (3 > 1), and row 2 keeps its place
    C = [[1.0, 1.0, 0.0], [3.0, 2.0, 0.0], [100.0, 0.0, 1.0]]
    F = F_of(C, [(0, 2), (2, 3)])
    assert list(F.q) == [1, 0, 2]
    np.testing.assert_allclose(F.L[:, 0], [1.0, 1.0 / 3.0, 100.0 / 3.0], rtol=1e-15)
    np.testing.assert_allclose(F.U[0], [3.0, 2.0, 0.0], rtol=0)
    np.testing.assert_allclose(F.U[1, 1], 1.0 - 2.0 / 3.0, rtol=1e-15)
    np.testing.assert_allclose(lu.reconstruct(F), C, rtol=0, atol=1e-13)
    # unrestricted, row 2 would have been chosen
    assert list(F_of(C, [(0, 3)]).q)[0] == 2


def test_zero_column_in_block_is_reported():
    C = [[0.0, 1.0, 1.0], [0.0, 2.0, 0.0], [5.0, 0.0, 1.0]]
    with pytest.raises(lu.ZeroPivot) as e:
        F_of(C, [(0, 2), (2, 3)])
    assert e.value.index == 0
    # with one block the 5 is a valid pivot
    F = F_of(C, [(0, 3)])
    assert F.q[0] == 2


def test_one_block_equals_lapack_partial_pivoting():
    rng = np.random.default_rng(3)
    C = rng.standard_normal((40, 40))
    F = F_of(C, [(0, 40)])
    P, L, U = scipy.linalg.lu(C)
    np.testing.assert_array_equal(F.q, np.argmax(P, axis=0))
    np.testing.assert_allclose(F.L, L, rtol=0, atol=1e-12)
    np.testing.assert_allclose(F.U, U, rtol=0, atol=1e-12 * np.abs(U).max())


def test_restricted_factor_properties():
    rng = np.random.default_rng(4)
    C = rng.standard_normal((150, 150))
    blocks = [(0, 64), (64, 128), (128, 150)]
    F = F_of(C, blocks)
    assert np.array_equal(F.L, np.tril(F.L)) and np.all(np.diag(F.L) == 1.0)
    assert np.array_equal(F.U, np.triu(F.U))
    for b0, b1 in blocks:   # rows move only inside their block
        assert sorted(F.q[b0:b1]) == list(range(b0, b1))
        blk = np.abs(F.L[b0:b1, b0:b1])
        assert blk.max() <= 1.0
    np.testing.assert_allclose(lu.reconstruct(F), C, rtol=0, atol=1e-12 * np.abs(C).max())


def test_symmetric_dominant_is_cholesky():
    """A symmetric, strictly diagonally dominant matrix: every column's
    largest candidate stays its diagonal, so no interchange occurs and
    U = D L^T, L sqrt(D) = the Cholesky factor (C oracle)."""
    A = gen.fv3d(6, 5, 4, seed=3)
    perm = np.arange(A.n)
    F = lu.factor(A, perm)
    assert np.array_equal(F.q, np.arange(A.n))
    d = np.diag(F.U)
    np.testing.assert_allclose(F.U, d[:, None] * F.L.T, rtol=0, atol=1e-12 * d.max())
    Fc = oracle.factor(A, perm)
    Lc = Fc.L().toarray()
    np.testing.assert_allclose(F.L * np.sqrt(d), Lc, rtol=0, atol=1e-12 * np.abs(Lc).max())


def test_solve_matches_dense_solve():
    A = gen.nonsymmetric(gen.shifted(gen.fv3d(7, 6, 5, seed=2), 0.6), 0.5, seed=8)
    rng = np.random.default_rng(9)
    perm = rng.permutation(A.n)
    F = lu.factor(A, perm)
    M = A.to_scipy().toarray()
    assert not np.allclose(M, M.T)
    b = gen.rhs(A.n, 3, seed=1)
    np.testing.assert_allclose(lu.solve(F, b), np.linalg.solve(M, b), rtol=1e-9, atol=1e-12)
    C = lu.permuted_full(A, perm)
    np.testing.assert_allclose(C, M[np.ix_(perm, perm)], rtol=0, atol=0)
    np.testing.assert_allclose(lu.reconstruct(F), C, rtol=0, atol=1e-12 * np.abs(C).max())


def test_nonsymmetric_generator_keeps_pattern():
    A = gen.fv3d(5, 4, 3, seed=1)
    B = gen.nonsymmetric(A, 0.5, seed=2)
    np.testing.assert_array_equal(A.rowptr, B.rowptr)
    np.testing.assert_array_equal(A.colind, B.colind)
    MA, MB = A.to_scipy().toarray(), B.to_scipy().toarray()
    np.testing.assert_array_equal(np.diag(MA), np.diag(MB))
    # a_ij + a_ji is kept, a_ij / a_ji moves by at most the skew
    np.testing.assert_allclose(MB + MB.T, MA + MA.T, rtol=1e-14, atol=1e-14)
