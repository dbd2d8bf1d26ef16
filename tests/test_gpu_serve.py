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


def build_requests(count, seed, rate):
    from paper_2506_05793_amd.serve import Request
    specs = gen.serving_requests(count, seed=seed, rate=rate, n2d=(100, 4000), n3d=(125, 6000),
                                 max_rhs=4)
    reqs, mats = [], {}
    for i, sp in enumerate(specs):
        if sp["kind"] == "factor":
            A = gen.fv2d(*sp["side"], seed=sp["seed"]) if sp["dim"] == 2 else \
                gen.fv3d(*sp["side"], seed=sp["seed"])
            mats[i] = A
            reqs.append(Request(i, sp["t"], "factor", gen.rhs(A.n, sp["nrhs"], seed=sp["seed"] + 1),
                                matrix=A))
        else:
            A = mats[sp["target"]]
            reqs.append(Request(i, sp["t"], "repeat", gen.rhs(A.n, sp["nrhs"], seed=sp["seed"]),
                                target=sp["target"]))
    return reqs, mats


def test_serving_mix_equals_alone():
    from paper_2506_05793_amd.serve import Server, summarize
    reqs, mats = build_requests(30, seed=5, rate=2000.0)
    budget = 64 << 20  # small: forces queueing and eviction
    srv = Server(budget, slots=4)
    t0 = __import__("time").perf_counter()
    res = srv.run(reqs)
    wall = __import__("time").perf_counter() - t0
    srv.close()
    summ = summarize(res, wall)
    print(summ, "admitted while busy:", srv.admitted_while_busy, "peak bytes:", srv.peak_used)
    assert len(res) == len(reqs)
    assert srv.admitted_while_busy > 0
    assert srv.peak_used <= budget
    by_id = {r.rid: r for r in reqs}
    for out in res:
        r = by_id[out.rid]
        A = r.matrix if r.kind == "factor" else mats[r.target]
        s = T.tacho_analyze(A.n, A.rowptr, A.colind, srv.options)
        num = T.tacho_factorize(s, A.values, T.TACHO_FP64)
        alone = T.tacho_solve(num, r.rhs)
        assert np.array_equal(alone, out.x), out.rid
        assert oracle.rel_residual(A, out.x, r.rhs).max() <= 1e-12


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
