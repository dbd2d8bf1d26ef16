"""Autotuner of the launch plan's batching parameters.

The numeric kernels have fixed tile shapes (64-column pivot blocks on the
matrix cores, fronts of order <= 64 in LDS).  What the plan can vary is how
work is grouped into tasks and launches (the paper's Tacho section batches
the many small fronts of the low levels and gives the few large ones at the
top their own kernels; where the boundary between the two regimes lies
depends on the matrix and the device):

* ``u_range`` - pivot blocks per update-matrix range task of the dataflow
  front kernel (the current plan forms update matrices in a launch of their
  own, over all pivot blocks, so it is kept in the table but not searched);
* ``chain_min`` - fronts with at least this many pivot blocks run their
  diagonal blocks as one chain task (negative: never);
* ``solve_level_fronts`` - solve levels below the last level with more than
  this many fronts run level by level, the rest as one dataflow launch;
* ``asm_cols`` - front columns per assembly work item of a front taller than
  the assembly tile;
* ``solo_m`` - fronts with one pivot block and at most this many rows run as
  one task each (negative: never);
* ``chain_inplace`` - chain fronts: the product for the next diagonal block's
  row tile is subtracted in place (>= 0) or left in a slot (< 0).

``asm_cols``, ``solo_m`` and ``solve_level_fronts`` only regroup work: every
setting gives bitwise the same factor and solution.  ``u_range``,
``chain_min`` and ``chain_inplace`` change the order in which a front's
contributions are summed (results agree to rounding).  The table therefore
keeps the order-neutral parameters per workload class and the order-changing
ones per precision only ("order/fp64", "order/fp32"), tuned on one workload
and used for all: a system then gets the same arithmetic alone, in a batch,
or in a larger problem of another class.

``tune`` times candidates on the device by coordinate descent from the
defaults (each candidate must reach the residual bound) and returns the
best setting; ``TuningTable`` keeps settings in a JSON file, which the
library reads itself (``tacho_options.autotune_path``); ``options_for``
returns options that point the library at the table.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import (TACHO_FP64, tacho_analyze, tacho_default_options, tacho_factorize,
               tacho_query_symbolic, tacho_refactorize, tacho_solve)

DEFAULTS = {"u_range": 8, "chain_min": 3, "solve_level_fronts": 256, "asm_cols": 8,
            "solo_m": 192, "chain_inplace": 0}
CANDIDATES = {
    "u_range": (8,),
    "chain_min": (2, 3, 4, 6, -1),
    "solve_level_fronts": (64, 256, 1024),
    "asm_cols": (4, 8, 16),
    "solo_m": (-1, 128, 192, 256, 320),
    "chain_inplace": (0, -1),
}


ORDER_NEUTRAL = ("asm_cols", "solo_m", "solve_level_fronts")
ORDER_CHANGING = ("u_range", "chain_min", "chain_inplace")


def _prec(precision: int) -> str:
    return "fp64" if precision == TACHO_FP64 else "fp32"


def workload_key(n: int, nnz: int, precision: int = TACHO_FP64) -> str:
    """Workload class of the order-neutral parameters: lg = the integer
    nearest log2(n) (2^lg <= n < 2^(lg+1), plus one when n^2 >= 2^(2 lg + 1)),
    mean row degree nnz / n rounded half up, precision.  The library computes
    the same key from the same integers."""
    nn = max(int(n), 1)
    lg = nn.bit_length() - 1
    if nn * nn >= 1 << (2 * lg + 1):
        lg += 1
    deg = (2 * int(nnz) + nn) // (2 * nn)
    return f"n~2^{lg}/deg{deg}/{_prec(precision)}"


def order_key(precision: int = TACHO_FP64) -> str:
    """Entry of the order-changing parameters (one per precision)."""
    return f"order/{_prec(precision)}"


def _residual(rowptr, colind, values, x, b):
    """Max over columns of ||b - A x||_2 / ||b||_2 (full symmetric CSR)."""
    import scipy.sparse as sp
    n = len(rowptr) - 1
    A = sp.csr_matrix((values, colind, rowptr), shape=(n, n))
    r = b - A @ x
    return float(np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)))


def measure(n, rowptr, colind, values, params, precision=TACHO_FP64, reps=7, ordering=0,
            tol=None):
    """Median device times (ms) of a refactorization and of a 1-RHS solve with
    the given plan parameters; ``None`` if the residual bound is missed."""
    import torch
    opts = tacho_default_options(ordering=ordering, **params)
    sym = tacho_analyze(n, rowptr, colind, opts)
    vals = torch.from_numpy(np.ascontiguousarray(values)).cuda()
    num = tacho_factorize(sym, vals, precision)
    b = np.random.default_rng(0).standard_normal((n, 1))
    bd = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()
    xd = torch.empty_like(bd)
    for _ in range(2):
        tacho_refactorize(num, vals, sync=True)
        tacho_solve(num, bd, xd)
    torch.cuda.synchronize()
    tf, ts = [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        tacho_refactorize(num, vals, sync=False)
        e[1].record()
        tacho_solve(num, bd, xd)
        e[2].record()
        torch.cuda.synchronize()
        tf.append(e[0].elapsed_time(e[1]))
        ts.append(e[1].elapsed_time(e[2]))
    tacho_refactorize(num, vals, sync=True)
    rho = _residual(rowptr, colind, values, xd.cpu().numpy(), b)
    bound = tol if tol is not None else (1e-12 if precision == TACHO_FP64 else 1e-10)
    if not rho <= bound:
        return None
    return {"factor_ms": float(np.median(tf)), "solve_ms": float(np.median(ts)), "rho": rho}


def tune(n, rowptr, colind, values, precision=TACHO_FP64, reps=7, passes=1,
         objective="request", log=print, candidates=None, start=None):
    """Coordinate descent over ``candidates`` (default CANDIDATES) from DEFAULTS
    updated with ``start`` (e.g. the precision's order-changing parameters,
    held fixed when they are not among the candidates).

    objective "request": factor + 1-RHS solve time; "factor": factor time.
    Returns (best parameters, best measurement, history)."""
    sym = tacho_analyze(n, rowptr, colind)
    ordering = int(tacho_query_symbolic(sym)["ordering"])
    del sym

    def score(m):
        return m["factor_ms"] + (m["solve_ms"] if objective == "request" else 0.0)

    best = dict(DEFAULTS)
    best.update(start or {})
    best_m = measure(n, rowptr, colind, values, best, precision, reps, ordering)
    if best_m is None:
        raise RuntimeError("the default plan misses the residual bound")
    history = [(dict(best), best_m)]
    log(f"[autotune] defaults {best}: {best_m}")
    for _ in range(passes):
        for name, values_ in (candidates or CANDIDATES).items():
            for v in values_:
                if v == best[name]:
                    continue
                cand = dict(best)
                cand[name] = v
                t0 = time.perf_counter()
                m = measure(n, rowptr, colind, values, cand, precision, reps, ordering)
                history.append((cand, m))
                log(f"[autotune] {name}={v}: {m} ({time.perf_counter() - t0:.1f} s)")
                if m is not None and score(m) < score(best_m):
                    best, best_m = cand, m
    log(f"[autotune] best {best}: {best_m}")
    return best, best_m, history


class TuningTable:
    """Tuned parameters per workload class, stored as JSON."""

    def __init__(self, path: str):
        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as fh:
                self.entries = json.load(fh)

    def get(self, key: str):
        e = self.entries.get(key)
        return dict(e["params"]) if e else None

    def put(self, key: str, params: dict, info: dict | None = None):
        self.entries[key] = {"params": dict(params), "info": info or {}}

    def save(self):
        with open(self.path, "w") as fh:
            json.dump(self.entries, fh, indent=1, sort_keys=True)


DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def tuned_params(n: int, nnz: int, precision: int = TACHO_FP64, table: str | None = None) -> dict:
    """Parameters the library takes from the table for this workload class and
    precision ({} when the table has neither entry)."""
    tab = TuningTable(table or DEFAULT_TABLE)
    out = {}
    w = tab.get(workload_key(n, nnz, precision)) or {}
    o = tab.get(order_key(precision)) or {}
    out.update({k: v for k, v in w.items() if k in ORDER_NEUTRAL})
    out.update({k: v for k, v in o.items() if k in ORDER_CHANGING})
    return out


def options_for(n: int, nnz: int, precision: int = TACHO_FP64, table: str | None = None,
                **overrides):
    """tacho_options that let the library read the tuning table (parameters
    left at 0 take the table's values for this workload class and precision),
    then ``overrides``."""
    return tacho_default_options(autotune_path=table or DEFAULT_TABLE,
                                 autotune_precision=precision, **overrides)


def store(tab: "TuningTable", n: int, nnz: int, precision: int, best: dict, info: dict,
          order_too: bool):
    """Put a tuned setting into the table: the order-neutral parameters under
    the workload class, the order-changing ones (when ``order_too``) under the
    precision's entry."""
    tab.put(workload_key(n, nnz, precision), {k: best[k] for k in ORDER_NEUTRAL if k in best}, info)
    if order_too:
        tab.put(order_key(precision), {k: best[k] for k in ORDER_CHANGING if k in best}, info)
