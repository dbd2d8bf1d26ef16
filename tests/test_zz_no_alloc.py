"""tacho_solve_noalloc (the solve for callers that cannot allocate device
memory) against tacho_solve, through the C ABI: the same kernels, so the
same bits, on two calls in a row (the second with a smaller system and fewer
right-hand sides, which reuses the shared device scratch); its argument
limits are errors, not allocations."""
import numpy as np
import pytest

import gen
import paper_2506_05793_amd as T

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()  # column-major


@pytest.mark.parametrize("prec", [T.TACHO_FP32, T.TACHO_FP64], ids=["fp32", "fp64"])
def test_noalloc_equals_solve(prec):
    cases = [(gen.fv3d(20, 18, 16, seed=4), 4), (gen.fv3d(10, 9, 8, seed=5), 2)]
    for A, nrhs in cases:  # second call: smaller input
        s = T.tacho_analyze(A.n, A.rowptr, A.colind)
        num = T.tacho_factorize(s, A.values, prec)
        b = _dev(gen.rhs(A.n, nrhs, seed=7))
        x_ref, info_ref = T.tacho_solve(num, b, torch.empty_like(b), with_info=True)
        x = torch.full_like(b, float("nan"))
        _, info = T.tacho_solve_noalloc(num, b, x, with_info=True)
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref), (A.n, nrhs)
        assert info["iters"] == info_ref["iters"] and info["fell_back"] == 0
        assert info["relres_max"] == info_ref["relres_max"]
        r = b.cpu().numpy() - A.to_scipy() @ x.cpu().numpy()
        rho = np.linalg.norm(r, axis=0) / np.linalg.norm(b.cpu().numpy(), axis=0)
        assert rho.max() <= (1e-12 if prec == T.TACHO_FP64 else 1e-10)


def test_noalloc_limits_are_errors():
    A = gen.fv3d(10, 9, 8, seed=5)
    s = T.tacho_analyze(A.n, A.rowptr, A.colind)
    num = T.tacho_factorize(s, A.values, T.TACHO_FP32)
    b = _dev(gen.rhs(A.n, 17, seed=1))
    with pytest.raises(T.TachoError) as e:  # more than 16 right-hand sides
        T.tacho_solve_noalloc(num, b, torch.empty_like(b))
    assert e.value.code == T.TACHO_ERR_INVALID
    b2 = _dev(gen.rhs(A.n, 2, seed=1))
    with pytest.raises(T.TachoError):  # in place with an FP32 factor
        T.tacho_solve_noalloc(num, b2, b2)
    # refinement scratch beyond the 64 MiB array: n * nrhs * 8 > 64 MiB
    B = gen.fv3d(82, seed=2)
    sb = T.tacho_analyze(B.n, B.rowptr, B.colind)
    nb = T.tacho_factorize(sb, B.values, T.TACHO_FP32)
    bb = _dev(gen.rhs(B.n, 16, seed=1))
    assert B.n * 16 * 8 > 64 << 20
    with pytest.raises(T.TachoError) as e:
        T.tacho_solve_noalloc(nb, bb, torch.empty_like(bb))
    assert e.value.code == T.TACHO_ERR_INVALID and "exceeds" in str(e.value)
