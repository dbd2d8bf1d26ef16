"""Serving loop: continuous batching of factor / repeat-solve requests.

Each result must be the same alone and in the mix (bitwise: the kernels do
not depend on what else runs), requests must overlap on the device, and the
HBM budget must be respected (with eviction of idle resident factors).
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2506_05793_amd as T

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a ROCm GPU")]


def build_requests(count, seed, rate, mixed_frac=0.0):
    from paper_2506_05793_amd.serve import Request
    specs = gen.serving_requests(count, seed=seed, rate=rate, n2d=(100, 4000), n3d=(125, 6000),
                                 max_rhs=4)
    pick = np.random.default_rng(seed + 100)
    reqs, mats = [], {}
    for i, sp in enumerate(specs):
        if sp["kind"] == "factor":
            A = gen.fv2d(*sp["side"], seed=sp["seed"]) if sp["dim"] == 2 else \
                gen.fv3d(*sp["side"], seed=sp["seed"])
            mats[i] = A
            prec = T.TACHO_FP32 if pick.random() < mixed_frac else T.TACHO_FP64
            reqs.append(Request(i, sp["t"], "factor", gen.rhs(A.n, sp["nrhs"], seed=sp["seed"] + 1),
                                matrix=A, precision=prec))
        else:
            A = mats[sp["target"]]
            reqs.append(Request(i, sp["t"], "repeat", gen.rhs(A.n, sp["nrhs"], seed=sp["seed"]),
                                target=sp["target"]))
    return reqs, mats


def test_serving_mix_equals_alone():
    """FP64 and FP32 + refinement requests mixed: every result equals the
    request's result alone, bitwise; repeated patterns reuse the analysis."""
    from paper_2506_05793_amd.serve import Server, summarize
    reqs, mats = build_requests(40, seed=5, rate=2000.0, mixed_frac=0.5)
    budget = 64 << 20  # small: forces queueing and eviction
    srv = Server(budget, slots=4)
    t0 = __import__("time").perf_counter()
    res = srv.run(reqs)
    wall = __import__("time").perf_counter() - t0
    srv.close()
    summ = summarize(res, wall)
    print(summ, "admitted while busy:", srv.admitted_while_busy, "peak bytes:", srv.peak_used,
          "analyses:", srv.analyses, "symbolic reuses:", srv.symbolic_hits)
    assert len(res) == len(reqs) and summ["errors"] == 0
    assert srv.admitted_while_busy > 0
    assert srv.peak_used <= budget
    assert srv.analyses + srv.symbolic_hits >= sum(r.kind == "factor" for r in reqs)
    by_id = {r.rid: r for r in reqs}
    prec_of = {r.rid: r.precision for r in reqs if r.kind == "factor"}
    assert {o.precision for o in res} == {T.TACHO_FP64, T.TACHO_FP32}
    for out in res:
        r = by_id[out.rid]
        A = r.matrix if r.kind == "factor" else mats[r.target]
        prec = prec_of[r.rid if r.kind == "factor" else r.target]
        assert out.precision == prec
        s = T.tacho_analyze(A.n, A.rowptr, A.colind, srv.options)
        num = T.tacho_factorize(s, A.values, prec)
        alone = T.tacho_solve(num, r.rhs)
        assert np.array_equal(alone, out.x), out.rid
        tol = 1e-12 if prec == T.TACHO_FP64 else 1e-10
        assert oracle.rel_residual(A, out.x, r.rhs).max() <= tol


def test_serving_reports_solve_errors():
    """Every retired job is checked, repeats included: with the solve test hook
    (every dependency wait gives up at once) each result carries the error."""
    from paper_2506_05793_amd.serve import Server
    reqs, _ = build_requests(8, seed=9, rate=2000.0)
    opts = T.tacho_default_options(ordering=2, debug_flags=T.TACHO_DEBUG_SOLVE_GIVE_UP)
    srv = Server(1 << 30, slots=2, options=opts)
    res = srv.run(reqs)
    srv.close()
    assert len(res) == len(reqs)
    kinds = {r.kind for r in res}
    assert "repeat" in kinds
    for out in res:
        assert out.error is not None and "timed out" in out.error, (out.rid, out.kind)
