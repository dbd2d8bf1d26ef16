"""Synthetic inputs: sizes, symmetry and positive definiteness."""
import numpy as np
import pytest

import gen


def test_sizes():
    A = gen.laplace2d(32)
    assert (A.n, A.nnz) == (1024, 4992)
    B = gen.fv3d(64)
    assert (B.n, B.nnz) == (262144, 1810432)
    off = gen.matrices._half_offsets_27()
    edges = sum((200 - abs(dx)) * (200 - abs(dy)) * (11 - abs(dz)) for dx, dy, dz in off)
    assert edges == 5322862
    assert 4 * (200 * 200 * 11 + 2 * edges) == 44342896


@pytest.mark.parametrize("make", [
    lambda: gen.fv3d(5, 4, 3, seed=1),
    lambda: gen.fv2d(7, 5, seed=2),
    lambda: gen.landice(4, 3, 3, seed=3),
    lambda: gen.landice(3, 3, 2, seed=3, sigma_rel=1e-7),
    lambda: gen.random_spd_pattern(30, 0.2, seed=4),
    lambda: gen.csr_block_diag(gen.batch_fv3d(3, seed=4, lo=2, hi=4)),
])
def test_spd(make):
    A = make()
    D = A.dense()
    assert np.array_equal(D, D.T)
    assert np.linalg.eigvalsh(D).min() > 0
    assert np.all(np.diff(A.rowptr) > 0)
    for r in range(A.n):
        cols = A.colind[A.rowptr[r]:A.rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0)


def test_seeds_reproducible():
    a = gen.fv3d(6, seed=1)
    b = gen.fv3d(6, seed=1)
    assert np.array_equal(a.values, b.values)
    r1 = gen.rhs(100, 1, seed=2)
    r16 = gen.rhs(100, 16, seed=2)
    assert np.array_equal(r1[:, 0], r16[:, 0])
    assert r16.flags.f_contiguous


def test_batch_sides_in_range():
    mats = gen.batch_fv3d(20, seed=4)
    for m in mats:
        assert 8 ** 3 <= m.n <= 32 ** 3
