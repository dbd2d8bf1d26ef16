"""GPU path vs the oracle, through the C ABI (HIP kernels on gfx950).

Bars: symbolic arrays bit-exact; FP64 factor column-max-normalized error
<= 1e-10 with the oracle's exact pattern; FP64 relative residual <= 1e-12;
FP32 factor + FP64 refinement relative residual <= 1e-10; the first
non-positive pivot reported at the oracle's index; results bitwise equal
run to run and alone vs in a batch.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2506_05793_amd as T

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]

FP64_FACTOR_TOL = 1e-10
FP64_RESID_TOL = 1e-12
MIXED_RESID_TOL = 1e-10
# ||x - x_oracle|| / ||x_oracle|| per column for the FP64 path: both solutions
# carry a forward error of order kappa(A) u, and the factor's own bar
# (1e-10, column-normalized) bounds what the solves may add on top
FP64_SOLUTION_TOL = 1e-10


def analyze(A, **opt):
    s = T.tacho_analyze(A.n, A.rowptr, A.colind, T.tacho_default_options(**opt) if opt else None)
    return s, T.tacho_get_symbolic(s)


def colnorm_error(factor, F):
    """max_j max_i |dL_ij| / max_i |L_ij| over the oracle's columns."""
    e = colnorm_errors(factor, F)
    return float(e.max()) if e.size else 0.0


def colnorm_errors(factor, F):
    """Per column j of the oracle's factor: max_i |dL_ij| / max_i |L_ij|.

    The library stores relaxed supernodes: its columns hold every row of the
    oracle's column plus rows that are structurally zero, which must be exact
    zeros."""
    Lp, Li, Lx = factor
    n = F.n
    if n == 0:
        return np.zeros(0)
    assert np.all(np.diff(Lp) >= np.diff(F.Lp))
    gcol = np.repeat(np.arange(n, dtype=np.int64), np.diff(Lp))
    ocol = np.repeat(np.arange(n, dtype=np.int64), np.diff(F.Lp))
    gkey = gcol * n + Li
    okey = ocol * n + F.Li
    pos = np.searchsorted(gkey, okey)
    assert np.all(pos < gkey.size) and np.array_equal(gkey[pos], okey), "oracle row missing"
    extra = np.ones(gkey.size, dtype=bool)
    extra[pos] = False
    assert np.all(Lx[extra] == 0.0), "structural zero stored as nonzero"
    d = np.abs(Lx[pos] - F.Lx)
    cm = np.maximum.reduceat(np.abs(F.Lx), F.Lp[:-1])
    dm = np.maximum.reduceat(d, F.Lp[:-1])
    return dm / cm


def solution_error(x, xo):
    """Per column ||x - x_oracle||_2 / ||x_oracle||_2."""
    x = x.reshape(xo.shape)
    return np.linalg.norm(x - xo, axis=0) / np.linalg.norm(xo, axis=0)


CASES = [
    ("lap2d_32", lambda: gen.laplace2d(32)),
    ("fv3d_12", lambda: gen.fv3d(12, seed=1)),
    ("fv3d_17x13x11", lambda: gen.fv3d(17, 13, 11, seed=7)),
    ("fv3d_24", lambda: gen.fv3d(24, seed=8)),
    ("fv3d_36", lambda: gen.fv3d(36, seed=8)),  # fronts wider than 512 with update matrices
    ("fv2d_45x37", lambda: gen.fv2d(45, 37, seed=3)),
    ("landice_9x8x4", lambda: gen.landice(9, 8, 4, seed=3)),
    ("random_500", lambda: gen.random_spd_pattern(500, 0.01, seed=5)),
    ("tridiag_300", lambda: gen.laplace1d(300)),
    ("dense_300", lambda: gen.random_spd_pattern(300, 1.0, seed=9)),
    ("dense_130", lambda: gen.random_spd_pattern(130, 1.0, seed=10)),
    ("single", lambda: gen.dense_to_csr(np.array([[4.0]]))),
]


@pytest.mark.parametrize("front", [0, 1], ids=["dataflow", "stepwise"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fp64_factor_and_solve_parity(name, make, front):
    A = make()
    s, a = analyze(A, front_kernel=front)
    F = oracle.factor(A, a.perm)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    err = colnorm_error(T.tacho_get_factor(num), F)
    print(f"{name}: column-normalized factor error {err:.3e}")
    assert err <= FP64_FACTOR_TOL
    for nrhs in (1, 16, 19):
        b = gen.rhs(A.n, nrhs, seed=2)
        x = T.tacho_solve(num, b)
        xo = oracle.solve(F, b)
        rho = oracle.rel_residual(A, x, b)
        rel = solution_error(x, xo)
        print(f"  nrhs={nrhs} rho={rho.max():.2e} |x-x_oracle|/|x_oracle|={rel.max():.2e}")
        assert rho.max() <= FP64_RESID_TOL, (nrhs, rho.max())
        assert rel.max() <= FP64_SOLUTION_TOL, (nrhs, rel.max())


PLAN_SETTINGS = [
    {"u_range": 4, "chain_min": 2, "solve_level_fronts": 16, "asm_cols": 4, "solo_m": 2000,
     "chain_inplace": -1},
    {"u_range": 16, "chain_min": -1, "solve_level_fronts": 4096, "asm_cols": 16, "solo_m": -1},
    {"chain_min": 2, "chain_inplace": 1},
]


@pytest.mark.parametrize("plan", PLAN_SETTINGS, ids=["fine", "coarse", "inplace"])
@pytest.mark.parametrize("name", ["fv3d_36", "landice_9x8x4", "dense_300"])
def test_plan_parameters_keep_parity(name, plan):
    """The autotuner's plan parameters regroup tasks and launches: every
    setting must still match the oracle (factor and 1/16-RHS solves)."""
    A = dict(CASES)[name]()
    s, a = analyze(A, **plan)
    F = oracle.factor(A, a.perm)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    err = colnorm_error(T.tacho_get_factor(num), F)
    print(f"{name} {plan}: column-normalized factor error {err:.3e}")
    assert err <= FP64_FACTOR_TOL
    for nrhs in (1, 16):
        b = gen.rhs(A.n, nrhs, seed=2)
        x = T.tacho_solve(num, b)
        assert oracle.rel_residual(A, x, b).max() <= FP64_RESID_TOL
        assert solution_error(x, oracle.solve(F, b)).max() <= FP64_SOLUTION_TOL


# Plan parameters that only regroup work must not change a single bit.
NEUTRAL_SETTINGS = [
    {"asm_cols": 4}, {"asm_cols": 16}, {"solo_m": -1}, {"solo_m": 2000},
    {"solve_level_fronts": 16}, {"solve_level_fronts": 4096},
]


@pytest.mark.parametrize("prec", [T.TACHO_FP64, T.TACHO_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("name", ["fv3d_36", "landice_9x8x4", "dense_300"])
def test_order_neutral_parameters_are_bitwise(name, prec):
    A = dict(CASES)[name]()
    b = gen.rhs(A.n, 3, seed=5)
    s0, _ = analyze(A)
    n0 = T.tacho_factorize(s0, A.values, prec)
    L0, x0 = T.tacho_get_factor(n0)[2], T.tacho_solve(n0, b)
    for opt in NEUTRAL_SETTINGS:
        s, _ = analyze(A, **opt)
        num = T.tacho_factorize(s, A.values, prec)
        assert np.array_equal(T.tacho_get_factor(num)[2], L0), opt
        assert np.array_equal(T.tacho_solve(num, b), x0), opt


def test_logdet_closed_form_c1():
    A = gen.laplace2d(32)
    s, a = analyze(A)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    Lp, Li, Lx = T.tacho_get_factor(num)
    logdet = 2 * np.sum(np.log(Lx[Lp[:-1]]))
    assert abs(logdet - 1210.72312053205) / 1210.72312053205 < 1e-12


def test_device_pointers_and_in_place():
    A = gen.fv3d(10, 9, 8, seed=3)
    s, a = analyze(A)
    vals = torch.from_numpy(A.values).cuda()
    num = T.tacho_factorize(s, vals, T.TACHO_FP64)
    b = gen.rhs(A.n, 5, seed=4)
    x_host = T.tacho_solve(num, b)
    bd = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()  # column-major view
    xd = T.tacho_solve(num, bd)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(xd.cpu().numpy(), x_host)
    bd2 = bd.clone()
    T.tacho_solve(num, bd2, bd2)  # x aliases b
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bd2.cpu().numpy(), x_host)


def test_multi_rhs_equals_column_by_column():
    A = gen.fv3d(11, 10, 9, seed=5)
    s, _ = analyze(A)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    b = gen.rhs(A.n, 16, seed=6)
    X = T.tacho_solve(num, b)
    for c in (0, 7, 15):
        xc = T.tacho_solve(num, np.asfortranarray(b[:, c:c + 1]))
        assert np.max(np.abs(xc[:, 0] - X[:, c])) <= 1e-13 * np.max(np.abs(X[:, c]))


def test_run_to_run_bitwise():
    A = gen.fv3d(14, 12, 10, seed=8)
    s, _ = analyze(A)
    n1 = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    n2 = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    assert np.array_equal(T.tacho_get_factor(n1)[2], T.tacho_get_factor(n2)[2])
    b = gen.rhs(A.n, 3, seed=1)
    assert np.array_equal(T.tacho_solve(n1, b), T.tacho_solve(n2, b))


def test_refactorize_new_values():
    A = gen.fv3d(9, 9, 9, seed=1)
    B = gen.fv3d(9, 9, 9, seed=11)  # same pattern, other coefficients
    assert np.array_equal(A.colind, B.colind)
    s, a = analyze(A)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    T.tacho_refactorize(num, B.values)
    F = oracle.factor(B, a.perm)
    assert colnorm_error(T.tacho_get_factor(num), F) <= FP64_FACTOR_TOL


@pytest.mark.parametrize("seed", [0, 1])
def test_not_spd_reports_first_pivot(seed):
    A = gen.fv3d(8, 7, 6, seed=seed)
    M = A.to_scipy().tolil()
    bad = int(np.random.default_rng(seed).integers(0, A.n))
    M[bad, bad] = -1.0
    B = gen.matrices._from_scipy(M.tocsr())
    s, a = analyze(B)
    with pytest.raises(oracle.NotSPD) as eo:
        oracle.factor(B, a.perm)
    with pytest.raises(T.TachoError) as eg:
        T.tacho_factorize(s, B.values, T.TACHO_FP64)
    assert eg.value.code == T.TACHO_ERR_NOT_SPD
    assert eg.value.fail_index == eo.value.index


@pytest.mark.parametrize("name,make", [
    ("fv3d_16", lambda: gen.fv3d(16, seed=2)),
    ("landice_10x9x5", lambda: gen.landice(10, 9, 5, seed=3)),
    ("dense_200", lambda: gen.random_spd_pattern(200, 1.0, seed=3)),
])
@pytest.mark.parametrize("front", [0, 1], ids=["dataflow", "stepwise"])
def test_fp32_refinement(name, make, front):
    A = make()
    s, a = analyze(A, front_kernel=front)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP32)
    b = gen.rhs(A.n, 4, seed=2)
    x, info = T.tacho_solve(num, b, with_info=True)
    rho = oracle.rel_residual(A, x, b)
    xo = oracle.solve(oracle.factor(A, a.perm), b)
    fwd = np.linalg.norm(x - xo, axis=0) / np.linalg.norm(xo, axis=0)
    print(f"{name}: iters={info['iters']} fell_back={info['fell_back']} rho={rho.max():.2e} "
          f"err_vs_oracle={fwd.max():.2e}")
    assert rho.max() <= MIXED_RESID_TOL
    assert info["relres_max"] <= MIXED_RESID_TOL


def test_batch_alone_equals_batched():
    """FP64 batch: the factor of the block-diagonal union and every system's
    solution match the oracle, and each system alone gives the same bits."""
    mats = gen.batch_fv3d(6, seed=4, lo=4, hi=9)
    sb, ab = analyze_batch(mats)
    vals = np.concatenate([m.values for m in mats])
    nb = T.tacho_factorize(sb, vals, T.TACHO_FP64)
    U = gen.csr_block_diag(mats)
    F = oracle.factor(U, ab.perm)
    assert colnorm_error(T.tacho_get_factor(nb), F) <= FP64_FACTOR_TOL
    rhs = [gen.rhs(m.n, 2, seed=10 + k) for k, m in enumerate(mats)]
    bb = np.asfortranarray(np.concatenate(rhs, axis=0))
    xb = T.tacho_solve(nb, bb)
    xo = oracle.solve(F, bb)
    off = 0
    for k, m in enumerate(mats):
        assert solution_error(xb[off:off + m.n], xo[off:off + m.n]).max() <= FP64_SOLUTION_TOL, k
        s, _ = analyze(m)
        num = T.tacho_factorize(s, m.values, T.TACHO_FP64)
        x = T.tacho_solve(num, rhs[k])
        assert np.array_equal(x, xb[off:off + m.n]), k
        off += m.n


def analyze_batch(mats, opt=None):
    s = T.tacho_analyze_batch([(m.n, m.rowptr, m.colind) for m in mats], opt)
    return s, T.tacho_get_symbolic(s)


@pytest.mark.slow
def sampled_llt_error(num, A, perm, count=2000, seed=0):
    """max over sampled pattern entries (i, j) of C = P A P^T of
    |(L L^T)_ij - C_ij| / sqrt(C_ii C_jj); Cholesky's backward error is
    bounded entrywise by (|L||L^T|)_ij <= sqrt(C_ii C_jj)."""
    import scipy.sparse as sp
    Lp, Li, Lx = T.tacho_get_factor(num)
    Lr = sp.csc_matrix((Lx, Li, Lp), shape=(A.n, A.n)).tocsr()
    C = oracle.oracle.permuted_lower(A, perm).tocoo()
    pick = np.random.default_rng(seed).choice(C.nnz, size=min(count, C.nnz), replace=False)
    diag = C.tocsr().diagonal()
    worst = 0.0
    for k in pick:
        i, j = C.row[k], C.col[k]
        v = Lr.getrow(i).multiply(Lr.getrow(j)).sum()
        worst = max(worst, abs(v - C.data[k]) / np.sqrt(diag[i] * diag[j]))
    return worst


def bench_plan(A, precision):
    """Plan options the bench times for this workload (tuning table)."""
    from paper_2506_05793_amd import autotune
    return autotune.options_for(A.n, A.nnz, precision)


def test_full_size_3d_64_mixed():
    """64^3 lognormal workload, FP32 factor + FP64 refinement in the bench's
    plan: residual within the metric's bound for 1 and 16 right-hand sides,
    forward error against the FP64 path printed."""
    A = gen.fv3d(64, seed=1)
    s = T.tacho_analyze(A.n, A.rowptr, A.colind, bench_plan(A, T.TACHO_FP32))
    num = T.tacho_factorize(s, A.values, T.TACHO_FP32)
    s64 = T.tacho_analyze(A.n, A.rowptr, A.colind, bench_plan(A, T.TACHO_FP64))
    num64 = T.tacho_factorize(s64, A.values, T.TACHO_FP64)
    for nrhs in (1, 16):
        b = gen.rhs(A.n, nrhs, seed=2)
        x, info = T.tacho_solve(num, b, with_info=True)
        x64 = T.tacho_solve(num64, b)
        rho = oracle.rel_residual(A, x, b)
        err = np.linalg.norm(x - x64, axis=0) / np.linalg.norm(x64, axis=0)
        print(f"64^3 mixed nrhs={nrhs}: iters={info['iters']} fell_back={info['fell_back']} "
              f"rho={rho.max():.2e} |x-x_fp64|/|x_fp64|={err.max():.2e}")
        assert rho.max() <= MIXED_RESID_TOL
        assert info["fell_back"] == 0


def test_full_size_landice():
    """Land-ice-shaped workload at full size (880,000 unknowns) in the bench's
    plans: FP64 residual and sampled (L L^T)_ij = C_ij; FP32 + refinement
    residual within the metric's bound."""
    A = gen.landice(seed=3)
    assert A.n == 880000
    s = T.tacho_analyze(A.n, A.rowptr, A.colind, bench_plan(A, T.TACHO_FP64))
    a = T.tacho_get_symbolic(s)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    b = gen.rhs(A.n, 1, seed=2)
    x = T.tacho_solve(num, b)
    rho = oracle.rel_residual(A, x, b)
    worst = sampled_llt_error(num, A, a.perm, count=500)
    print(f"land-ice FP64: rho={rho.max():.2e} sampled LL^T error {worst:.2e}")
    assert rho.max() <= FP64_RESID_TOL
    assert worst <= 1e-12
    del num
    s32 = T.tacho_analyze(A.n, A.rowptr, A.colind, bench_plan(A, T.TACHO_FP32))
    num32 = T.tacho_factorize(s32, A.values, T.TACHO_FP32)
    x32, info = T.tacho_solve(num32, b, with_info=True)
    rho32 = oracle.rel_residual(A, x32, b)
    print(f"land-ice mixed: iters={info['iters']} fell_back={info['fell_back']} "
          f"rho={rho32.max():.2e} |x-x_fp64|/|x_fp64|="
          f"{np.linalg.norm(x32 - x) / np.linalg.norm(x):.2e}")
    assert rho32.max() <= MIXED_RESID_TOL


def test_full_size_3d_64():
    """64^3 lognormal workload in the bench's plan: FP64 factor column by
    column and solutions (1 and 16 right-hand sides) against the oracle,
    repeated solves bitwise equal."""
    A = gen.fv3d(64, seed=1)
    s = T.tacho_analyze(A.n, A.rowptr, A.colind, bench_plan(A, T.TACHO_FP64))
    a = T.tacho_get_symbolic(s)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    F = oracle.factor(A, a.perm)
    err = colnorm_error(T.tacho_get_factor(num), F)
    print(f"64^3 FP64: column-normalized factor error {err:.2e}")
    assert err <= FP64_FACTOR_TOL
    for nrhs in (1, 16):
        b = gen.rhs(A.n, nrhs, seed=2)
        x = T.tacho_solve(num, b)
        rho = oracle.rel_residual(A, x, b)
        ex = solution_error(x, oracle.solve(F, b))
        print(f"64^3 nrhs={nrhs}: rho={rho.max():.2e} |x-x_oracle|/|x_oracle|={ex.max():.2e}")
        assert rho.max() <= FP64_RESID_TOL
        assert ex.max() <= FP64_SOLUTION_TOL
        # the dataflow solves run thousands of concurrent tasks: repeat them
        # and require the same bits every time
        for _ in range(4):
            assert np.array_equal(T.tacho_solve(num, b), x)


def test_graph_replays_match_eager():
    """The captured factorization graph, replayed several times with other
    values and eager work in between, gives the eager result bitwise."""
    A = gen.fv3d(13, 12, 11, seed=21)
    B = gen.fv3d(13, 12, 11, seed=22)
    s_e = T.tacho_analyze(A.n, A.rowptr, A.colind, T.tacho_default_options(graphs=0))
    s_g = T.tacho_analyze(A.n, A.rowptr, A.colind, T.tacho_default_options(graphs=1))
    want = {}
    for name, M in (("A", A), ("B", B)):
        ne = T.tacho_factorize(s_e, M.values, T.TACHO_FP64)
        want[name] = T.tacho_get_factor(ne)[2]
    ng = T.tacho_factorize(s_g, A.values, T.TACHO_FP64)
    b = gen.rhs(A.n, 2, seed=3)
    for name in ("A", "B", "A", "B"):
        M = A if name == "A" else B
        T.tacho_refactorize(ng, M.values)
        x = T.tacho_solve(ng, b)  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(T.tacho_get_factor(ng)[2], want[name]), name
        assert oracle.rel_residual(M, x, b).max() <= FP64_RESID_TOL


def test_batch_fp32_refinement_alone_equals_batched():
    """Refinement converges per system, so a batched FP32+IR result equals the
    system's result alone, bitwise."""
    mats = gen.batch_fv3d(5, seed=7, lo=5, hi=10)
    sb = T.tacho_analyze_batch([(m.n, m.rowptr, m.colind) for m in mats])
    nb = T.tacho_factorize(sb, np.concatenate([m.values for m in mats]), T.TACHO_FP32)
    rhs = [gen.rhs(m.n, 3, seed=30 + k) for k, m in enumerate(mats)]
    xb, info = T.tacho_solve(nb, np.asfortranarray(np.concatenate(rhs, axis=0)), with_info=True)
    assert info["relres_max"] <= MIXED_RESID_TOL
    off = 0
    for k, m in enumerate(mats):
        s, _ = analyze(m)
        num = T.tacho_factorize(s, m.values, T.TACHO_FP32)
        x = T.tacho_solve(num, rhs[k])
        assert np.array_equal(x, xb[off:off + m.n]), k
        assert oracle.rel_residual(m, x, rhs[k]).max() <= MIXED_RESID_TOL
        off += m.n


def _ill_conditioned_dense(n, cond, seed):
    """Q diag(lambda) Q^T with lambda log-spaced over [1/cond, 1] (SPD)."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.logspace(0, -np.log10(cond), n)
    M = (Q * lam) @ Q.T
    return gen.dense_to_csr((M + M.T) / 2)


def _shifted_tridiagonal(n, gap):
    """1D Laplacian shifted so that its smallest eigenvalue is `gap`."""
    lam_min = 4 * np.sin(np.pi / (2 * (n + 1))) ** 2
    M = (np.diag(np.full(n, 2.0 - lam_min + gap)) - np.diag(np.ones(n - 1), 1)
         - np.diag(np.ones(n - 1), -1))
    return gen.dense_to_csr(M)


@pytest.mark.parametrize("name,make", [
    ("dense_150_cond1e12", lambda: _ill_conditioned_dense(150, 1e12, seed=1)),
    ("tridiag_200_gap1e-10", lambda: _shifted_tridiagonal(200, 1e-10)),
])
@pytest.mark.parametrize("front", [0, 1], ids=["dataflow", "stepwise"])
def test_fp32_breakdown_or_stall_falls_back_to_fp64(name, make, front):
    """FP32 cannot resolve these (kappa * u_fp32 >> 1): the FP32 path must end
    in the FP64 factorization of the same values, bitwise equal to a direct
    FP64 factorization and solve."""
    A = make()
    s, a = analyze(A, front_kernel=front)
    b = gen.rhs(A.n, 3, seed=4)
    num32 = T.tacho_factorize(s, A.values, T.TACHO_FP32)
    x32, info = T.tacho_solve(num32, b, with_info=True)
    num64 = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    x64 = T.tacho_solve(num64, b)
    print(f"{name}: iters={info['iters']} fell_back={info['fell_back']} "
          f"relres={info['relres_max']:.2e}")
    assert info["fell_back"] == 1
    assert np.array_equal(x32, x64)
    rho = oracle.rel_residual(A, x64, b).max()
    # both residuals are FP64 sums with cancellation: they agree to within the
    # rounding bound of b - A x, n u (|A| |x| + |b|) relative to |b|
    M = abs(A.to_scipy())
    bound = max(np.linalg.norm(M @ abs(x64[:, c]) + abs(b[:, c])) / np.linalg.norm(b[:, c])
                for c in range(b.shape[1]))
    assert abs(info["relres_max"] - rho) <= 4 * A.n * np.finfo(float).eps * bound


def test_solve_give_up_is_reported_and_cleared():
    """With the test hook that raises the solve's hang flag before its launches,
    every dependency wait gives up at once (the kernels still finish) and the
    queued device solve must be reported by tacho_check_factor; the report
    clears the flag, so a solve on a handle without the hook is normal."""
    A = gen.fv3d(20, 18, 16, seed=4)
    s_bad = T.tacho_analyze(A.n, A.rowptr, A.colind,
                            T.tacho_default_options(debug_flags=T.TACHO_DEBUG_SOLVE_GIVE_UP))
    num = T.tacho_factorize(s_bad, A.values, T.TACHO_FP64)
    b = torch.from_numpy(np.ascontiguousarray(gen.rhs(A.n, 2, seed=1).T)).cuda().t()
    x = T.tacho_solve(num, b)  # queued only
    with pytest.raises(T.TachoError) as e:
        T.tacho_check_factor(num)
    assert e.value.code == T.TACHO_ERR_HIP and "timed out" in str(e.value)
    T.tacho_check_factor(num)  # reported once, then cleared
    with pytest.raises(T.TachoError):  # host path checks before returning
        T.tacho_solve(num, gen.rhs(A.n, 1, seed=3))
    del x
    s = T.tacho_analyze(A.n, A.rowptr, A.colind)
    good = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    bh = gen.rhs(A.n, 2, seed=1)
    xg = T.tacho_solve(good, bh)
    T.tacho_check_factor(good)
    assert oracle.rel_residual(A, xg, bh).max() <= FP64_RESID_TOL


def test_batch_fallback_is_per_system():
    """One system that FP32 cannot resolve (cond 1e12) batched with
    well-conditioned ones: only its columns take the FP64 solution; the others
    keep their refined FP32 results, bitwise equal to the systems alone."""
    good = gen.batch_fv3d(3, seed=12, lo=5, hi=9)
    bad = _ill_conditioned_dense(120, 1e12, seed=2)
    mats = [good[0], bad, good[1], good[2]]
    sb = T.tacho_analyze_batch([(m.n, m.rowptr, m.colind) for m in mats])
    nb = T.tacho_factorize(sb, np.concatenate([m.values for m in mats]), T.TACHO_FP32)
    rhs = [gen.rhs(m.n, 2, seed=40 + k) for k, m in enumerate(mats)]
    xb, info = T.tacho_solve(nb, np.asfortranarray(np.concatenate(rhs, axis=0)), with_info=True)
    print("fell back per unit (system x column):", info["fell_back_units"].tolist())
    assert info["fell_back"] == 1
    assert info["fell_back_units"].shape == (4, 2)
    assert info["fell_back_units"][1].tolist() == [1, 1]
    assert info["fell_back_units"][[0, 2, 3]].sum() == 0
    off = 0
    for k, m in enumerate(mats):
        s, _ = analyze(m)
        if k == 1:
            x = T.tacho_solve(T.tacho_factorize(s, m.values, T.TACHO_FP64), rhs[k])
        else:
            x = T.tacho_solve(T.tacho_factorize(s, m.values, T.TACHO_FP32), rhs[k])
        assert np.array_equal(x, xb[off:off + m.n]), k
        if k != 1:  # the cond 1e12 system carries its FP64 solution (residual ~ kappa u)
            assert oracle.rel_residual(m, xb[off:off + m.n], rhs[k]).max() <= MIXED_RESID_TOL
        off += m.n
