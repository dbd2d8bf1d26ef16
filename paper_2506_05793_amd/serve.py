"""Request server for factor/solve requests of uneven size on one GPU.

The paper's Trilinos section motivates the handles this loop is built on: the
symbolic analysis is amortized across value changes and a numerical factor
is reused for many right-hand sides.  The loop adds continuous batching:

* arrivals enter an admission queue; the host-side symbolic analysis of a
  factor request starts at arrival in a worker thread, and requests whose
  sparsity pattern was seen before reuse that symbolic handle (an analysis
  depends on the pattern only);
* a request is admitted as soon as a device slot (a stream) is free and its
  numeric handle fits the HBM budget; idle resident factors are evicted
  least-recently-used to make room;
* an admitted FP64 factor request queues its values upload, factorization and
  first solve on its slot's stream without waiting, so the work of requests
  admitted while others run overlaps on the device; an FP32 + refinement
  request (whose solve reads residual norms on the host between corrections)
  runs the same steps in a worker thread bound to its slot's stream;
* factors stay resident after completion, so repeat requests (new
  right-hand sides on an earlier matrix) only queue a solve;
* completion is detected with events (or the worker's future); latency is
  completion minus arrival.

All device work runs in the HIP library; this module only schedules it.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import time
from dataclasses import dataclass, field

import numpy as np

from . import (TACHO_FP32, TACHO_FP64, TachoError, tacho_analyze, tacho_check_factor,
               tacho_default_options, tacho_numeric_bytes, tacho_numeric_create,
               tacho_refactorize, tacho_solve)


@dataclass
class Request:
    rid: int
    t_arrival: float            # seconds after the start of the run
    kind: str                   # "factor" or "repeat"
    rhs: np.ndarray             # n x nrhs (column-major)
    matrix: object = None       # CSR (gen.CSR-like: n, rowptr, colind, values) for "factor"
    target: int = -1            # rid of the factor request whose factor a "repeat" reuses
    precision: int = TACHO_FP64  # factor requests: TACHO_FP64 or TACHO_FP32 (+ refinement)


@dataclass
class Result:
    rid: int
    kind: str
    n: int
    nrhs: int
    t_arrival: float
    t_admit: float
    t_done: float
    x: np.ndarray
    error: str | None = None    # library error of the request's factorization or solve
    precision: int = TACHO_FP64
    info: dict | None = None    # refinement report (FP32 requests)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class _Resident:
    num: object
    sym: object
    matrix: object
    nbytes: int
    precision: int
    busy: bool = False


@dataclass
class _Job:
    req: Request
    slot: int
    event: object
    x_host: object
    t_admit: float
    num: object = None
    precision: int = TACHO_FP64
    future: object = None       # FP32 jobs: worker future returning (x, error, info)
    keep: list = field(default_factory=list)


class Server:
    """Continuous-batching request loop (one host thread + analysis workers +
    one worker per slot for refined solves)."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 4, analysis_workers: int = 4,
                 options=None, reuse_symbolic: bool = True, symbolic_cache: int = 512):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        # Level-structure dissection only: on the grid operators of the request
        # mix it gives fewer flops than the multilevel one and analyses several
        # times faster, and analysis time is part of a factor request's latency.
        # Eager launches: a request's handle is factored once, so capturing its
        # launch sequence into a graph would only add host time.
        self.options = options if options is not None else tacho_default_options(ordering=2,
                                                                                graphs=0)
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.pool = cf.ThreadPoolExecutor(max_workers=analysis_workers)
        self.slot_workers = cf.ThreadPoolExecutor(max_workers=slots)
        self.resident: "collections.OrderedDict[int, _Resident]" = collections.OrderedDict()
        self.used = 0
        self.peak_used = 0
        self.admitted_while_busy = 0
        self.reuse_symbolic = reuse_symbolic
        self.symbolic_cache = symbolic_cache
        self._sym: "collections.OrderedDict[tuple, tuple]" = collections.OrderedDict()
        self.analyses = 0
        self.symbolic_hits = 0

    # -- helpers -------------------------------------------------------------
    def _analyze(self, A):
        return tacho_analyze(A.n, A.rowptr, A.colind, self.options)

    def _symbolic_future(self, A):
        """Future of A's symbolic handle: shared by every request with the
        same pattern (checked entry by entry), analysed once."""
        if not self.reuse_symbolic:
            self.analyses += 1
            return self.pool.submit(self._analyze, A)
        rp = np.ascontiguousarray(A.rowptr)
        ci = np.ascontiguousarray(A.colind)
        key = (int(A.n), int(rp[-1]) if rp.size else 0, hash(rp.tobytes()), hash(ci.tobytes()))
        hit = self._sym.get(key)
        if hit is not None and np.array_equal(hit[1], rp) and np.array_equal(hit[2], ci):
            self._sym.move_to_end(key)
            self.symbolic_hits += 1
            return hit[0]
        fut = self.pool.submit(self._analyze, A)
        self.analyses += 1
        self._sym[key] = (fut, rp, ci)
        while len(self._sym) > self.symbolic_cache:
            self._sym.popitem(last=False)
        return fut

    def _evict_for(self, need: int) -> bool:
        """Free idle resident factors (LRU first) until `need` more bytes fit."""
        while self.used + need > self.budget:
            victim = next((k for k, r in self.resident.items() if not r.busy), None)
            if victim is None:
                return False
            r = self.resident.pop(victim)
            self.used -= r.nbytes
            del r
        return True

    def _launch_solve(self, job: _Job, num, rhs: np.ndarray, stream):
        torch = self.torch
        b = torch.from_numpy(np.ascontiguousarray(rhs.T)).pin_memory()
        with torch.cuda.stream(stream):
            bd = b.to("cuda", non_blocking=True).t()  # column-major view
            xd = torch.empty_like(bd)
            tacho_solve(num, bd, xd, stream=stream.cuda_stream)
            xh = torch.empty(xd.shape[::-1], dtype=torch.float64).pin_memory().t()
            xh.copy_(xd, non_blocking=True)
        job.keep += [b, bd, xd]
        job.x_host = xh

    def _refined(self, num, values, rhs: np.ndarray, stream):
        """Worker thread of an FP32 job: (factorization when `values` is
        given) + refined solve on the slot's stream; returns (x, error, info)."""
        torch = self.torch
        try:
            with torch.cuda.stream(stream):
                if values is not None:
                    vd = torch.from_numpy(np.ascontiguousarray(values)).to("cuda")
                    tacho_refactorize(num, vd, stream=stream.cuda_stream, sync=False)
                bd = torch.from_numpy(np.ascontiguousarray(rhs.T)).to("cuda").t()
                xd = torch.empty_like(bd)
                _, info = tacho_solve(num, bd, xd, stream=stream.cuda_stream, with_info=True)
                x = xd.cpu().numpy().copy(order="F")
            stream.synchronize()
            tacho_check_factor(num)
            return x, None, {"iters": info["iters"], "fell_back": info["fell_back"],
                             "relres_max": info["relres_max"]}
        except TachoError as e:
            stream.synchronize()
            return np.full(rhs.shape, np.nan, order="F"), str(e), None

    # -- main loop -----------------------------------------------------------
    def run(self, requests: list[Request]) -> list[Result]:
        torch = self.torch
        reqs = sorted(requests, key=lambda r: (r.t_arrival, r.rid))
        pending = collections.deque(reqs)
        queue: list[Request] = []
        futures = {}
        free = list(range(len(self.streams)))
        inflight: list[_Job] = []
        results: list[Result] = []
        matrices = {r.rid: r for r in reqs if r.kind == "factor"}
        t0 = time.perf_counter()
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].t_arrival <= now:
                r = pending.popleft()
                queue.append(r)
                if r.kind == "factor":
                    futures[r.rid] = self._symbolic_future(r.matrix)
            # retire finished jobs
            still = []
            for job in inflight:
                done = job.future.done() if job.future is not None else job.event.query()
                if not done:
                    still.append(job)
                    continue
                t_done = time.perf_counter() - t0
                r = job.req
                info = None
                if job.future is not None:
                    x, err, info = job.future.result()
                else:
                    # every retired job: the factorization's failure flag (factor
                    # requests) and the solve's timed-out-wait flag
                    err = None
                    try:
                        tacho_check_factor(job.num)
                    except TachoError as e:
                        err = str(e)
                    x = job.x_host.numpy().copy(order="F")
                key = r.rid if r.kind == "factor" else r.target
                self.resident[key].busy = False
                self.resident.move_to_end(key)
                results.append(Result(r.rid, r.kind, x.shape[0], x.shape[1], r.t_arrival,
                                      job.t_admit, t_done, x, err, job.precision, info))
                free.append(job.slot)
            inflight = still
            # admit what fits, in arrival order, skipping requests that must wait
            i = 0
            while free and i < len(queue):
                r = queue[i]
                if r.kind == "factor":
                    fut = futures[r.rid]
                    if not fut.done():
                        i += 1
                        continue
                    sym = fut.result()
                    need = tacho_numeric_bytes(sym, r.precision)
                    if need > self.budget:
                        raise RuntimeError(f"request {r.rid} needs {need} bytes, over the budget")
                    if not self._evict_for(need):
                        i += 1
                        continue
                    slot = free.pop()
                    st = self.streams[slot]
                    if inflight:
                        self.admitted_while_busy += 1
                    job = _Job(r, slot, None, None, time.perf_counter() - t0,
                               precision=r.precision)
                    num = tacho_numeric_create(sym, r.precision)
                    self.used += need
                    self.peak_used = max(self.peak_used, self.used)
                    self.resident[r.rid] = _Resident(num, sym, r.matrix, need, r.precision,
                                                     busy=True)
                    job.num = num
                    if r.precision == TACHO_FP32:
                        job.future = self.slot_workers.submit(self._refined, num, r.matrix.values,
                                                              r.rhs, st)
                    else:
                        vals = torch.from_numpy(np.ascontiguousarray(r.matrix.values)).pin_memory()
                        with torch.cuda.stream(st):
                            vd = vals.to("cuda", non_blocking=True)
                            tacho_refactorize(num, vd, stream=st.cuda_stream, sync=False)
                        job.keep += [vals, vd]
                        self._launch_solve(job, num, r.rhs, st)
                else:
                    res = self.resident.get(r.target)
                    if res is None:
                        if r.target not in matrices:
                            raise RuntimeError("repeat target unknown")
                        # target evicted: run as a new factor request of the same matrix
                        tgt = matrices[r.target]
                        if not any(q.rid == r.target for q in queue) and all(
                                j.req.rid != r.target for j in inflight):
                            nr = Request(r.rid, r.t_arrival, "factor", r.rhs, tgt.matrix,
                                         precision=tgt.precision)
                            queue[i] = nr
                            futures[nr.rid] = self._symbolic_future(nr.matrix)
                            matrices[nr.rid] = nr
                        i += 1
                        continue
                    if res.busy:
                        i += 1
                        continue
                    slot = free.pop()
                    st = self.streams[slot]
                    if inflight:
                        self.admitted_while_busy += 1
                    res.busy = True
                    job = _Job(r, slot, None, None, time.perf_counter() - t0, num=res.num,
                               precision=res.precision)
                    if res.precision == TACHO_FP32:
                        job.future = self.slot_workers.submit(self._refined, res.num, None, r.rhs, st)
                    else:
                        self._launch_solve(job, res.num, r.rhs, st)
                if job.future is None:
                    ev = torch.cuda.Event()
                    ev.record(self.streams[job.slot])
                    job.event = ev
                inflight.append(job)
                queue.pop(i)
            if not free or (not queue and not pending) or (queue and i >= len(queue)):
                time.sleep(20e-6)
        return sorted(results, key=lambda r: r.rid)

    def close(self):
        self.pool.shutdown(wait=True)
        self.slot_workers.shutdown(wait=True)
        self.resident.clear()
        self._sym.clear()


def summarize(results: list[Result], wall_s: float) -> dict:
    """p50/p99 latency per request kind and precision, and solve throughput."""
    out = {"requests": len(results), "wall_s": wall_s,
           "rhs_solves_per_s": sum(r.nrhs for r in results) / wall_s if wall_s > 0 else None,
           "errors": sum(r.error is not None for r in results)}
    for kind in ("factor", "repeat"):
        for prec, pname in ((None, "all"), (TACHO_FP64, "fp64"), (TACHO_FP32, "mixed")):
            lat = [r.latency for r in results
                   if r.kind == kind and (prec is None or r.precision == prec)]
            if lat:
                out[f"{kind}_{pname}"] = {"count": len(lat),
                                          "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                          "p99_ms": float(np.percentile(lat, 99) * 1e3)}
    return out
