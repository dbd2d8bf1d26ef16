"""Partitioned-inverse solves against the oracle, through the C ABI, in both
forms (TACHO_SOLVE_PARTITIONED_INVERSE: merged products per supernode;
TACHO_SOLVE_LEVEL_CSR: one CSR product per level): FP64 solutions per column
within the FP64 bars, FP32 factor + FP64 refinement within the mixed bar, the
inverse rebuilt by every refactorization, switching back to the default
variant, a batch of independent systems equal to each system alone, and the
variants refused for LDL^T."""
import numpy as np
import pytest

import gen
import oracle
import paper_2506_05793_amd as T
from test_gpu_parity import (CASES, FP64_RESID_TOL, FP64_SOLUTION_TOL, MIXED_RESID_TOL, analyze,
                             solution_error)

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]

PINV = T.TACHO_SOLVE_PARTITIONED_INVERSE
VARIANTS = [T.TACHO_SOLVE_PARTITIONED_INVERSE, T.TACHO_SOLVE_LEVEL_CSR]
VIDS = ["pinv", "csr"]


@pytest.mark.parametrize("variant", VARIANTS, ids=VIDS)
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_pinv_fp64_solve_parity(name, make, variant):
    A = make()
    s, a = analyze(A)
    F = oracle.factor(A, a.perm)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    T.tacho_set_solve_variant(num, variant)
    for nrhs in (1, 16, 19):
        b = gen.rhs(A.n, nrhs, seed=2)
        x = T.tacho_solve(num, b)
        rho = oracle.rel_residual(A, x, b)
        rel = solution_error(x, oracle.solve(F, b))
        print(f"{name}: nrhs={nrhs} rho={rho.max():.2e} |x-x_oracle|/|x_oracle|={rel.max():.2e}")
        assert rho.max() <= FP64_RESID_TOL, (nrhs, rho.max())
        assert rel.max() <= FP64_SOLUTION_TOL, (nrhs, rel.max())


@pytest.mark.parametrize("name,make", [
    ("fv3d_16", lambda: gen.fv3d(16, seed=2)),
    ("landice_10x9x5", lambda: gen.landice(10, 9, 5, seed=3)),
    ("dense_200", lambda: gen.random_spd_pattern(200, 1.0, seed=3)),
])
@pytest.mark.parametrize("variant", VARIANTS, ids=VIDS)
def test_pinv_fp32_refinement(name, make, variant):
    A = make()
    s, a = analyze(A)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP32)
    T.tacho_set_solve_variant(num, variant)
    b = gen.rhs(A.n, 4, seed=2)
    x, info = T.tacho_solve(num, b, with_info=True)
    rho = oracle.rel_residual(A, x, b)
    err = solution_error(x, oracle.solve(oracle.factor(A, a.perm), b))
    print(f"{name}: iters={info['iters']} fell_back={info['fell_back']} rho={rho.max():.2e} "
          f"err_vs_oracle={err.max():.2e}")
    assert info["fell_back"] == 0
    assert rho.max() <= MIXED_RESID_TOL
    assert info["relres_max"] <= MIXED_RESID_TOL


@pytest.mark.parametrize("variant", VARIANTS, ids=VIDS)
def test_pinv_rebuilt_by_refactorization_and_switch_back(variant):
    """New values through tacho_refactorize rebuild the inverse panels; the
    default variant works again afterwards and agrees to rounding."""
    A = gen.fv3d(20, 18, 16, seed=11)
    s, a = analyze(A)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
    T.tacho_set_solve_variant(num, variant)
    b = gen.rhs(A.n, 3, seed=4)
    x0 = T.tacho_solve(num, b)
    assert oracle.rel_residual(A, x0, b).max() <= FP64_RESID_TOL
    A2 = gen.shifted(A, -0.5)  # A + 0.5 mean(diag) I, same pattern
    T.tacho_refactorize(num, A2.values)
    x1 = T.tacho_solve(num, b)
    rel = solution_error(x1, oracle.solve(oracle.factor(A2, a.perm), b))
    assert oracle.rel_residual(A2, x1, b).max() <= FP64_RESID_TOL
    assert rel.max() <= FP64_SOLUTION_TOL
    T.tacho_set_solve_variant(num, T.TACHO_SOLVE_BLOCK_INVERSE)
    x2 = T.tacho_solve(num, b)
    assert oracle.rel_residual(A2, x2, b).max() <= FP64_RESID_TOL
    assert solution_error(x2, x1).max() <= FP64_SOLUTION_TOL


@pytest.mark.parametrize("variant", VARIANTS, ids=VIDS)
def test_pinv_batch_equals_alone(variant):
    """Fronts of independent systems never mix: a batched solve equals each
    system's solve alone, bitwise."""
    mats = gen.batch_fv3d(6, seed=5, lo=6, hi=14)
    sb = T.tacho_analyze_batch([(m.n, m.rowptr, m.colind) for m in mats])
    nb = T.tacho_factorize(sb, np.concatenate([m.values for m in mats]), T.TACHO_FP64)
    T.tacho_set_solve_variant(nb, variant)
    rhs = [gen.rhs(m.n, 2, seed=40 + k) for k, m in enumerate(mats)]
    xb = T.tacho_solve(nb, np.asfortranarray(np.concatenate(rhs, axis=0)))
    off = 0
    for k, m in enumerate(mats):
        s, _ = analyze(m)
        num = T.tacho_factorize(s, m.values, T.TACHO_FP64)
        T.tacho_set_solve_variant(num, variant)
        x = T.tacho_solve(num, rhs[k])
        assert np.array_equal(x, xb[off:off + m.n]), k
        assert oracle.rel_residual(m, x, rhs[k]).max() <= FP64_RESID_TOL
        off += m.n


def test_pinv_refused_for_ldlt():
    A = gen.shifted(gen.fv3d(6, 5, 4, seed=3), 0.9)
    s, _ = analyze(A)
    num = T.tacho_factorize(s, A.values, T.TACHO_LDLT)
    for variant in VARIANTS:
        with pytest.raises(T.TachoError) as e:
            T.tacho_set_solve_variant(num, variant)
        assert e.value.code == T.TACHO_ERR_INVALID
    with pytest.raises(T.TachoError):
        T.tacho_set_solve_variant(num, 7)
