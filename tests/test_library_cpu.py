"""Host-side checks of the library: exported C ABI, symbolic analysis bit-exact
against the oracle, input validation.  No GPU work is queued by these calls."""
import ctypes
import os
import re

import numpy as np
import pytest

import gen
import paper_2506_05793_amd as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not os.path.exists(T.LIB_PATH):
        T_build = __import__("paper_2506_05793_amd.build", fromlist=["build"])
        T_build.build()


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tacho.h")).read()
    return sorted(set(re.findall(r"\b(tacho_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(T.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name


def symbolic_matches_oracle(A, opts=None):
    import oracle
    s = T.tacho_analyze(A.n, A.rowptr, A.colind, opts)
    a = T.tacho_get_symbolic(s)
    q = T.tacho_query_symbolic(s)
    assert np.array_equal(np.sort(a.perm), np.arange(A.n))
    parent, counts = oracle.symbolic(A, a.perm)
    np.testing.assert_array_equal(a.parent, parent)
    np.testing.assert_array_equal(a.colcount, counts)
    sptr, spar = oracle.relaxed_supernodes(parent, counts)
    np.testing.assert_array_equal(a.super_ptr, sptr)
    np.testing.assert_array_equal(a.super_parent, spar)
    assert q["nnz_l"] == int(counts.sum())
    assert q["flops"] == oracle.flops_from_counts(counts)
    # levels: leaves 0, parent strictly higher
    lev = a.level
    for s_, p in enumerate(a.super_parent):
        if p >= 0:
            assert lev[p] > lev[s_]
    return s, a, q


CASES = [
    ("lap2d_32", lambda: gen.laplace2d(32)),
    ("fv3d_12", lambda: gen.fv3d(12, seed=1)),
    ("fv3d_9x7x5", lambda: gen.fv3d(9, 7, 5, seed=2)),
    ("fv2d_40x30", lambda: gen.fv2d(40, 30, seed=3)),
    ("landice_8x7x4", lambda: gen.landice(8, 7, 4, seed=3)),
    ("random", lambda: gen.random_spd_pattern(400, 0.01, seed=5)),
    ("tridiag", lambda: gen.laplace1d(300)),
    ("dense", lambda: gen.dense_to_csr(np.ones((40, 40)) + 40 * np.eye(40))),
    ("diagonal", lambda: gen.dense_to_csr(np.eye(17) * 3.0)),
    ("single", lambda: gen.dense_to_csr(np.array([[2.0]]))),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_symbolic_bit_exact(name, make):
    symbolic_matches_oracle(make())


@pytest.mark.parametrize("leaf", [1, 4, 64])
def test_symbolic_leaf_sizes(leaf):
    symbolic_matches_oracle(gen.fv3d(10, 9, 8, seed=4), T.tacho_default_options(nd_leaf_size=leaf))


@pytest.mark.slow
def test_symbolic_full_size_3d():
    """The 64^3 workload: symbolic parity at full size (oracle is O(nnz(L)))."""
    _, _, q = symbolic_matches_oracle(gen.fv3d(64, seed=1))
    assert q["n"] == 262144


def test_unsorted_rows_accepted():
    A = gen.fv3d(5, 4, 3, seed=1)
    rng = np.random.default_rng(0)
    ci = A.colind.copy()
    for i in range(A.n):
        seg = ci[A.rowptr[i]:A.rowptr[i + 1]]
        rng.shuffle(seg)
    s = T.tacho_analyze(A.n, A.rowptr, ci)
    s2 = T.tacho_analyze(A.n, A.rowptr, A.colind)
    assert np.array_equal(T.tacho_get_symbolic(s).perm, T.tacho_get_symbolic(s2).perm)


def test_missing_diagonal_added():
    D = np.array([[2.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 2.0]])
    A = gen.dense_to_csr(D)
    assert A.nnz == 6
    s = T.tacho_analyze(A.n, A.rowptr, A.colind)
    assert T.tacho_query_symbolic(s)["nnz_a"] == 7


def test_rejects_unsymmetric_pattern():
    rowptr = np.array([0, 2, 3], np.int64)
    colind = np.array([0, 1, 1], np.int32)  # (0,1) without (1,0)
    with pytest.raises(T.TachoError) as e:
        T.tacho_analyze(2, rowptr, colind)
    assert e.value.code == T.TACHO_ERR_PATTERN


def test_rejects_duplicates_and_bad_indices():
    with pytest.raises(T.TachoError) as e:
        T.tacho_analyze(2, np.array([0, 2, 3], np.int64), np.array([0, 0, 1], np.int32))
    assert e.value.code == T.TACHO_ERR_INVALID
    with pytest.raises(T.TachoError) as e:
        T.tacho_analyze(2, np.array([0, 1, 2], np.int64), np.array([0, 5], np.int32))
    assert e.value.code == T.TACHO_ERR_INVALID
    with pytest.raises(T.TachoError) as e:
        T.tacho_analyze(2, np.array([1, 1, 2], np.int64), np.array([0, 1], np.int32))
    assert e.value.code == T.TACHO_ERR_INVALID


def test_empty_matrix():
    s = T.tacho_analyze(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    q = T.tacho_query_symbolic(s)
    assert q["n"] == 0 and q["nsuper"] == 0


def test_batch_is_block_diagonal_union():
    import oracle
    mats = gen.batch_fv3d(5, seed=4, lo=3, hi=7)
    s = T.tacho_analyze_batch([(m.n, m.rowptr, m.colind) for m in mats])
    q = T.tacho_query_symbolic(s)
    assert q["nsystems"] == 5 and q["n"] == sum(m.n for m in mats)
    U = gen.csr_block_diag(mats)
    a = T.tacho_get_symbolic(s)
    parent, counts = oracle.symbolic(U, a.perm)
    np.testing.assert_array_equal(a.parent, parent)
    np.testing.assert_array_equal(a.colcount, counts)
    # each system alone has the same column counts (ordering is shift-invariant)
    alone = np.concatenate([T.tacho_get_symbolic(T.tacho_analyze(m.n, m.rowptr, m.colind)).colcount
                            for m in mats])
    assert sorted(alone.tolist()) == sorted(a.colcount.tolist())


@pytest.mark.parametrize("ordering", [0, 1, 2])
def test_indistinguishable_dofs_stay_consecutive(ordering):
    """Both DOFs of a mesh node have equal pattern rows; the ordering works on
    the node graph and keeps each node's DOFs next to each other."""
    A = gen.landice(9, 8, 4, seed=3)
    s, a, q = symbolic_matches_oracle(A, T.tacho_default_options(ordering=ordering))
    pinv = np.empty(A.n, np.int64)
    pinv[a.perm] = np.arange(A.n)
    assert np.all(pinv[1::2] == pinv[0::2] + 1)



def test_plan_parameters_accepted_and_reserved_rejected():
    """The plan's batching parameters only regroup work: any setting analyses
    to the same symbolic result; the reserved fields must stay 0."""
    A = gen.fv3d(12, 11, 10, seed=7)
    base = T.tacho_get_symbolic(T.tacho_analyze(A.n, A.rowptr, A.colind))
    for params in ({"u_range": 4, "chain_min": 2, "solve_level_fronts": 16, "asm_cols": 4,
                    "solo_m": 2000, "chain_inplace": -1},
                   {"u_range": 16, "chain_min": -1, "solve_level_fronts": 4096, "asm_cols": 32,
                    "solo_m": -1, "chain_inplace": 1}):
        s = T.tacho_analyze(A.n, A.rowptr, A.colind, T.tacho_default_options(**params))
        a = T.tacho_get_symbolic(s)
        assert np.array_equal(a.perm, base.perm) and np.array_equal(a.super_ptr, base.super_ptr)
    for bad in ({"small_front": 32}, {"block_size": 32}):
        with pytest.raises(T.TachoError):
            T.tacho_analyze(A.n, A.rowptr, A.colind, T.tacho_default_options(**bad))


def test_tuning_table_roundtrip(tmp_path):
    from paper_2506_05793_amd import autotune
    key = autotune.workload_key(262144, 1810432)
    assert key == autotune.workload_key(262144, 1810432, 1, T.TACHO_FP64)
    assert key != autotune.workload_key(262144, 1810432, 1, T.TACHO_FP32)
    path = str(tmp_path / "t.json")
    tab = autotune.TuningTable(path)
    assert tab.get(key) is None
    tab.put(key, {"u_range": 16, "chain_min": 4}, {"factor_ms": 1.0})
    tab.save()
    assert autotune.TuningTable(path).get(key) == {"u_range": 16, "chain_min": 4}
    opt = autotune.options_for(262144, 1810432, table=path, asm_cols=4)
    assert (opt.u_range, opt.chain_min, opt.asm_cols) == (16, 4, 4)
    assert autotune.options_for(1000, 5000, table=path).u_range == 0  # library default


def test_binding_rejects_bad_arguments():
    """The binding checks dtype, length and layout before any pointer reaches
    the library (a wrong buffer would be read or written out of bounds)."""
    import torch
    A = gen.fv3d(5, 4, 3, seed=1)
    s = T.tacho_analyze(A.n, A.rowptr, A.colind)
    assert s.n == A.n and s.nnz == A.nnz and s.nsys == 1
    num = T.NumericHandle(None, s, T.TACHO_FP64)  # no library handle: calls must fail first
    with pytest.raises(ValueError):
        T._values_arg(s, A.values[:-1])
    with pytest.raises(TypeError):
        T._values_arg(s, torch.from_numpy(A.values).float())
    with pytest.raises(ValueError):
        T._values_arg(s, torch.from_numpy(np.concatenate([A.values, A.values]))[::2])
    with pytest.raises(TypeError):
        T._values_arg(s, list(A.values))
    addr, on_dev, keep = T._values_arg(s, A.values.astype(np.float32))  # host arrays are converted
    assert on_dev == 0 and keep.dtype == np.float64
    b = gen.rhs(A.n, 3, seed=1)
    with pytest.raises(ValueError):
        T._solve_args(num, b[:-1], None)
    with pytest.raises(ValueError):
        T._solve_args(num, b, np.empty((A.n, 2)))
    with pytest.raises(ValueError):
        T._solve_args(num, b, np.empty((A.n, 3), order="C"))
    with pytest.raises(TypeError):
        T._solve_args(num, b, torch.empty(A.n, 3, dtype=torch.float64))
    with pytest.raises(TypeError):
        T._solve_args(num, torch.from_numpy(b).float(), None)
    with pytest.raises(TypeError):  # host torch tensors are not device tensors
        T._solve_args(num, torch.from_numpy(b), None)
    bb, xx, nrhs, ld, on_dev = T._solve_args(num, b, None)
    assert nrhs == 3 and ld == A.n and on_dev == 0 and xx.flags.f_contiguous


def test_batch_csr_validation():
    A = gen.fv3d(4, 4, 3, seed=1)
    rp = A.rowptr.copy()
    rp_bad = rp + 5  # rowptr[0] != 0
    with pytest.raises(T.TachoError) as e:
        T.tacho_analyze_batch([(A.n, A.rowptr, A.colind), (A.n, rp_bad, A.colind)])
    assert e.value.code == T.TACHO_ERR_INVALID and "rowptr[0]" in str(e.value)
    rp_dec = rp.copy()
    rp_dec[3] = rp_dec[4] + 1
    with pytest.raises(T.TachoError) as e:
        T.tacho_analyze_batch([(A.n, rp_dec, A.colind)])
    assert e.value.code == T.TACHO_ERR_INVALID
