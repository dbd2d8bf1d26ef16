"""Pins of the LDL^T oracle (pivoting restricted to diagonal blocks) against
what the mathematics fixes: hand-worked pivot decisions of Bunch-Kaufman on
tiny matrices (1x1 without and with interchange, 2x2, a block boundary that
hides the unrestricted choice, a block without a usable pivot), the
Cholesky factor of a diagonally dominant SPD matrix (no interchange can
occur there), Sylvester's law of inertia against the eigenvalues of C,
C = Q L D L^T Q^T, and solutions against a dense LAPACK solve."""
import numpy as np
import pytest

import gen
from oracle import ldlt

pytestmark = []


def F_of(C, blocks):
    return ldlt.factor_dense(np.asarray(C, dtype=float), blocks)


def test_two_by_two_pivot_on_zero_diagonal():
    F = F_of([[0.0, 1.0], [1.0, 0.0]], [(0, 2)])
    assert F.two[0] and list(F.q) == [0, 1]
    np.testing.assert_array_equal(F.D(), [[0.0, 1.0], [1.0, 0.0]])
    np.testing.assert_array_equal(F.L, np.eye(2))


def test_one_by_one_without_interchange():
    F = F_of([[2.0, 1.0], [1.0, 3.0]], [(0, 2)])
    assert not F.two.any() and list(F.q) == [0, 1]
    np.testing.assert_allclose(F.d, [2.0, 2.5], rtol=0, atol=1e-15)
    assert F.L[1, 0] == 0.5


def test_one_by_one_with_interchange():
    # |a11| = 1e-3 < alpha * 1, |a11| sigma = 1e-3 < alpha, |a22| = 1 >= alpha sigma:
    # the second row becomes the pivot
    F = F_of([[1e-3, 1.0], [1.0, 1.0]], [(0, 2)])
    assert not F.two.any() and list(F.q) == [1, 0]
    assert F.d[0] == 1.0 and F.L[1, 0] == 1.0
    assert F.d[1] == 1e-3 - 1.0


def test_block_boundary_hides_the_larger_entry():
    C = np.array([[1e-3, 1e-4, 1.0], [1e-4, 1.0, 0.0], [1.0, 0.0, 1.0]])
    # restricted to the block {0, 1}: lambda = 1e-4 and |a11| >= alpha lambda
    F = F_of(C, [(0, 2), (2, 3)])
    assert list(F.q) == [0, 1, 2] and not F.two.any()
    s11 = 1.0 - 1e-8 / 1e-3
    s21 = -1e-4 / 1e-3
    assert F.d[0] == 1e-3
    np.testing.assert_allclose(F.d[1], s11, rtol=1e-15)
    np.testing.assert_allclose(F.L[2, 1], s21 / s11, rtol=1e-15)
    np.testing.assert_allclose(F.d[2], (1.0 - 1.0 / 1e-3) - s21 * s21 / s11, rtol=1e-14)
    # one block over all three columns: row 2 (lambda = 1) takes the first pivot
    G = F_of(C, [(0, 3)])
    assert G.q[0] == 2


def test_block_without_usable_pivot():
    with pytest.raises(ldlt.ZeroPivot) as e:
        F_of([[0.0, 1.0], [1.0, 0.0]], [(0, 1), (1, 2)])
    assert e.value.index == 0


def _random_indefinite(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return (M + M.T) / 2


def _random_blocks(n, seed):
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.choice(np.arange(1, n), size=n // 6, replace=False))
    b = [0, *cuts.tolist(), n]
    return [(b[i], b[i + 1]) for i in range(len(b) - 1)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_indefinite_invariants(seed):
    n = 48
    C = _random_indefinite(n, seed)
    blocks = _random_blocks(n, seed)
    F = F_of(C, blocks)
    # Q moves columns only within their block; 2x2 pivots do not straddle
    for b0, b1 in blocks:
        assert sorted(F.q[b0:b1]) == list(range(b0, b1))
        assert not F.two[b1 - 1]
    assert np.allclose(np.triu(F.L, 1), 0) and np.all(np.diag(F.L) == 1)
    R = ldlt.reconstruct(F)
    growth = np.abs(F.L).max() ** 2 * np.abs(F.D()).max()
    assert np.abs(R - C).max() <= 64 * n * np.finfo(float).eps * max(growth, np.abs(C).max())
    ev = np.linalg.eigvalsh(C)
    pos, neg, zero = ldlt.inertia(F)
    assert (pos, neg, zero) == (int((ev > 0).sum()), int((ev < 0).sum()), 0)
    assert F.two.any()  # these matrices need 2x2 pivots


def test_spd_diagonally_dominant_is_cholesky():
    """No interchange happens when |c_kk| >= sum_i |c_ik| (so >= alpha lambda)
    at every step, which diagonal dominance keeps through elimination: then
    L sqrt(D) is the Cholesky factor."""
    A = gen.random_spd_pattern(60, 0.2, seed=3)
    perm = np.arange(A.n, dtype=np.int32)
    F = ldlt.factor(A, perm)
    assert list(F.q) == list(range(A.n)) and not F.two.any() and np.all(F.d > 0)
    C = ldlt.permuted_dense(A, perm)
    Lc = np.linalg.cholesky(C)
    np.testing.assert_allclose(F.L * np.sqrt(F.d), Lc, rtol=1e-12, atol=1e-14)


def test_solve_matches_dense_solve():
    A = gen.shifted(gen.fv3d(6, 5, 4, seed=1), 0.9)
    rng = np.random.default_rng(0)
    perm = rng.permutation(A.n).astype(np.int32)
    F = ldlt.factor(A, perm, tile=8)
    b = gen.rhs(A.n, 3, seed=4)
    x = ldlt.solve(F, b)
    xd = np.linalg.solve(A.to_scipy().toarray(), b)
    np.testing.assert_allclose(x, xd, rtol=1e-10, atol=1e-12 * np.abs(xd).max())
    ev = np.linalg.eigvalsh(A.to_scipy().toarray())
    assert (ev < 0).any() and (ev > 0).any()   # the shifted operator is indefinite
    pos, neg, _ = ldlt.inertia(F)
    assert (pos, neg) == (int((ev > 0).sum()), int((ev < 0).sum()))
