"""Request server for factor/solve requests of uneven size on one GPU.

The paper's Trilinos section motivates the handles this loop is built on: the
symbolic analysis is amortized across value changes and a numerical factor
is reused for many right-hand sides.  The loop adds continuous batching:

* arrivals enter an admission queue; the host-side symbolic analysis of a
  factor request starts at arrival in a worker thread;
* a request is admitted as soon as a device slot (a stream) is free and its
  numeric handle fits the HBM budget; idle resident factors are evicted
  least-recently-used to make room;
* an admitted factor request queues its values upload, factorization and
  first solve on its slot's stream without waiting, so the work of requests
  admitted while others run overlaps on the device;
* factors stay resident after completion, so repeat requests (new
  right-hand sides on an earlier matrix) only queue a solve;
* completion is detected with events; latency is completion minus arrival.

All device work runs in the HIP library; this module only schedules it.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import time
from dataclasses import dataclass, field

import numpy as np

from . import (TACHO_FP64, TachoError, tacho_analyze, tacho_check_factor, tacho_default_options,
               tacho_numeric_bytes, tacho_numeric_create, tacho_refactorize, tacho_solve)


@dataclass
class Request:
    rid: int
    t_arrival: float            # seconds after the start of the run
    kind: str                   # "factor" or "repeat"
    rhs: np.ndarray             # n x nrhs (column-major)
    matrix: object = None       # CSR (gen.CSR-like: n, rowptr, colind, values) for "factor"
    target: int = -1            # rid of the factor request whose factor a "repeat" reuses


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

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class _Resident:
    num: object
    sym: object
    matrix: object
    nbytes: int
    busy: bool = False


@dataclass
class _Job:
    req: Request
    slot: int
    event: object
    x_host: object
    t_admit: float
    num: object = None
    keep: list = field(default_factory=list)


class Server:
    """Continuous-batching request loop (one host thread + analysis workers)."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 4, precision: int = TACHO_FP64,
                 analysis_workers: int = 4, options=None):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.precision = precision
        # Level-structure dissection only: on the grid operators of the request
        # mix it gives fewer flops than the multilevel one and analyses several
        # times faster, and analysis time is part of a factor request's latency.
        self.options = options if options is not None else tacho_default_options(ordering=2)
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.pool = cf.ThreadPoolExecutor(max_workers=analysis_workers)
        self.resident: "collections.OrderedDict[int, _Resident]" = collections.OrderedDict()
        self.used = 0
        self.peak_used = 0
        self.admitted_while_busy = 0

    # -- helpers -------------------------------------------------------------
    def _analyze(self, A):
        return tacho_analyze(A.n, A.rowptr, A.colind, self.options)

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
        matrices = {r.rid: r.matrix for r in reqs if r.kind == "factor"}
        t0 = time.perf_counter()
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].t_arrival <= now:
                r = pending.popleft()
                queue.append(r)
                if r.kind == "factor":
                    futures[r.rid] = self.pool.submit(self._analyze, r.matrix)
            # retire finished jobs
            still = []
            for job in inflight:
                if job.event.query():
                    t_done = time.perf_counter() - t0
                    r = job.req
                    # every retired job: the factorization's failure flag (factor
                    # requests) and the solve's timed-out-wait flag
                    err = None
                    try:
                        tacho_check_factor(job.num)
                    except TachoError as e:
                        err = str(e)
                    if r.kind == "factor":
                        self.resident[r.rid].busy = False
                        self.resident.move_to_end(r.rid)
                    else:
                        self.resident[r.target].busy = False
                        self.resident.move_to_end(r.target)
                    x = job.x_host.numpy().copy(order="F")
                    results.append(Result(r.rid, r.kind, x.shape[0], x.shape[1], r.t_arrival,
                                          job.t_admit, t_done, x, err))
                    free.append(job.slot)
                else:
                    still.append(job)
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
                    need = tacho_numeric_bytes(sym, self.precision)
                    if need > self.budget:
                        raise RuntimeError(f"request {r.rid} needs {need} bytes, over the budget")
                    if not self._evict_for(need):
                        i += 1
                        continue
                    slot = free.pop()
                    st = self.streams[slot]
                    if inflight:
                        self.admitted_while_busy += 1
                    job = _Job(r, slot, None, None, time.perf_counter() - t0)
                    num = tacho_numeric_create(sym, self.precision)
                    self.used += need
                    self.peak_used = max(self.peak_used, self.used)
                    self.resident[r.rid] = _Resident(num, sym, r.matrix, need, busy=True)
                    vals = torch.from_numpy(np.ascontiguousarray(r.matrix.values)).pin_memory()
                    with torch.cuda.stream(st):
                        vd = vals.to("cuda", non_blocking=True)
                        tacho_refactorize(num, vd, stream=st.cuda_stream, sync=False)
                    job.keep += [vals, vd]
                    job.num = num
                    self._launch_solve(job, num, r.rhs, st)
                else:
                    res = self.resident.get(r.target)
                    if res is None:
                        if r.target in futures and r.target not in matrices:
                            raise RuntimeError("repeat target unknown")
                        # target evicted: run as a new factor request of the same matrix
                        if r.target in matrices and not any(
                                q.rid == r.target for q in queue) and all(
                                j.req.rid != r.target for j in inflight):
                            nr = Request(r.rid, r.t_arrival, "factor", r.rhs, matrices[r.target])
                            queue[i] = nr
                            futures[nr.rid] = self.pool.submit(self._analyze, nr.matrix)
                            matrices[nr.rid] = nr.matrix
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
                    job = _Job(r, slot, None, None, time.perf_counter() - t0, num=res.num)
                    self._launch_solve(job, res.num, r.rhs, st)
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
        self.resident.clear()


def summarize(results: list[Result], wall_s: float) -> dict:
    """p50/p99 latency per request kind and solve throughput."""
    out = {"requests": len(results), "wall_s": wall_s,
           "rhs_solves_per_s": sum(r.nrhs for r in results) / wall_s if wall_s > 0 else None}
    for kind in ("factor", "repeat"):
        lat = [r.latency for r in results if r.kind == kind]
        if lat:
            out[kind] = {"count": len(lat), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                         "p99_ms": float(np.percentile(lat, 99) * 1e3)}
    return out
