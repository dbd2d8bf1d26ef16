#!/usr/bin/env python3
"""Benchmark of the supernodal multifrontal Cholesky on one MI355X.

Workload (default): the land-ice-shaped SPD system, 200 x 200 x 11 nodes x
2 DOF (n = 880,000), 27-point node coupling with random SPD 2x2 blocks and
vertical anisotropy 1e3, nested-dissection ordering; FP64 multifrontal
factorization against FP32 factorization + FP64 iterative refinement, with
solves of 1 and 16 right-hand sides ~ N(0,1).  Inputs are synthetic, seeded,
and resident in HBM before timing starts.

One step = FP64 refactorization of the values (assembly, extend-add, dense
partial factorizations of every front, level by level) + a 1-RHS solve + a
16-RHS solve.  W untimed warmup steps, then K timed steps bracketed by
device synchronization.  `value` is the FP64 factorization rate
sum_j eta_j^2 / (median device factorization time) in TFLOP/s; the same
number of mixed steps (FP32 factor, refined solves) is timed after it.
Solves/s, p50/p99 latencies, the mixed result's error against the FP64
result and the solves' fraction of the HBM peak are reported beside it,
every rate with the residual it was obtained at.  The 3D 64^3 lognormal
workload is measured too (key "fv3d64").

Also reported: the roofline of the dominant kernel (per-launch hipEvent
timing inside this run on the library's stream, algorithmic flops or bytes
from the launch plan) for both precisions, and a CPU baseline (the oracle on
the 50 x 50 x 11 x 2 land-ice sample), whose solution also gives the
error of both GPU paths against the oracle.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "factor TFLOP/s + solves/s at rel. residual <=1e-10 (mixed vs FP64); p50/p99"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
COPY_PROBE_ELEMS = 1 << 27  # FP64 elements: 1 GiB read + 1 GiB written

# Measured HBM traffic per launch (rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# runs, calibrated on a copy kernel of known size), written by
# --traffic-summary and read back by the roofline.  Each summary records a
# hash of the kernel and launch-plan sources and of the tuned plan of its
# workload; when they change, the figures no longer describe the kernels and
# the roofline reports traffic null.
TRAFFIC_SOURCES = ("paper_2506_05793_amd/csrc/kernels.hip", "paper_2506_05793_amd/csrc/plan.cpp",
                   "paper_2506_05793_amd/csrc/plan.hpp")


def traffic_file(tag):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{tag}.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, p):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), p))


def residual(A, x, b):
    import numpy as np
    M = A.to_scipy()
    X = x.reshape(A.n, -1)
    B = b.reshape(A.n, -1)
    return np.linalg.norm(B - M @ X, axis=0) / np.linalg.norm(B, axis=0)


def rel_err(x, ref):
    import numpy as np
    x = x.reshape(ref.shape)
    return float(np.max(np.linalg.norm(x - ref, axis=0) / np.linalg.norm(ref, axis=0)))


def dev_colmajor(torch, a):
    """Column-major device copy of a host n x k array."""
    return torch.from_numpy(a.T.copy()).cuda().t()


def cpu_model():
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return model


# ---------------------------------------------------------------------------
# timed runs


def run_steps(T, torch, num, vals, B1, B16, X1, X16, steps, warmup):
    """FP64 or mixed steps: refactorization + 1-RHS + 16-RHS solve.  The FP64
    path queues everything on the stream (events between the calls); the
    mixed path's solves synchronize (refinement reads residual norms), so
    their times are host wall times around the calls."""
    mixed = num.precision == T.TACHO_FP32
    infos = []

    def one(record):
        if not mixed:
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
            T.tacho_refactorize(num, vals, sync=False)
            ev[1].record()
            T.tacho_solve(num, B1, X1)
            ev[2].record()
            T.tacho_solve(num, B16, X16)
            ev[3].record()
            return ev
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        T.tacho_refactorize(num, vals, sync=False)
        e1.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, i1 = T.tacho_solve(num, B1, X1, with_info=True)
        t2 = time.perf_counter()
        _, i16 = T.tacho_solve(num, B16, X16, with_info=True)
        t3 = time.perf_counter()
        if record:
            infos.append((i1, i16))
        return (e0, e1, (t2 - t1) * 1e3, (t3 - t2) * 1e3)

    for _ in range(warmup):
        one(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [one(True) for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tacho_check_factor(num)
    if not mixed:
        out = dict(factor_ms=[e[0].elapsed_time(e[1]) for e in recs],
                   solve1_ms=[e[1].elapsed_time(e[2]) for e in recs],
                   solve16_ms=[e[2].elapsed_time(e[3]) for e in recs])
    else:
        out = dict(factor_ms=[r[0].elapsed_time(r[1]) for r in recs],
                   solve1_ms=[r[2] for r in recs], solve16_ms=[r[3] for r in recs],
                   iters1=[i[0]["iters"] for i in infos], iters16=[i[1]["iters"] for i in infos],
                   fell_back=int(any(i[0]["fell_back"] or i[1]["fell_back"] for i in infos)))
    out["wall_s"] = wall
    return out


def summarize(r, flops, tol, rho1, rho16, solve_bytes1, solve_bytes16):
    import numpy as np
    f = float(np.median(r["factor_ms"]))
    s1 = float(np.median(r["solve1_ms"]))
    s16 = float(np.median(r["solve16_ms"]))
    ok = rho1 <= tol and rho16 <= tol
    req = [a + b for a, b in zip(r["factor_ms"], r["solve1_ms"])]
    out = {
        "factor_ms_p50": f, "factor_ms_p99": pct(r["factor_ms"], 99),
        "factor_tflops": flops / (f * 1e-3) / 1e12,
        "solve_nrhs1_ms_p50": s1, "solve_nrhs1_ms_p99": pct(r["solve1_ms"], 99),
        "solve_nrhs16_ms_p50": s16, "solve_nrhs16_ms_p99": pct(r["solve16_ms"], 99),
        "request_factor_solve_ms_p50": pct(req, 50), "request_factor_solve_ms_p99": pct(req, 99),
        "fresh_factor_solves_per_s": 1e3 / pct(req, 50) if ok else None,
        "resident_rhs_solves_per_s_nrhs1": 1e3 / s1 if ok else None,
        "resident_rhs_solves_per_s_nrhs16": 16e3 / s16 if ok else None,
        # algorithmic solve bytes (every factor entry read twice, four vector
        # passes of n x nrhs FP64) over the whole solve call
        "solve_nrhs1_hbm_frac": solve_bytes1 / (s1 * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "solve_nrhs16_hbm_frac": solve_bytes16 / (s16 * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "rel_residual_nrhs1": rho1, "rel_residual_nrhs16": rho16,
        "residual_tol": tol, "meets_tol": bool(ok),
    }
    for k in ("iters1", "iters16"):
        if k in r:
            out["refine_" + k] = int(max(r[k])) if r[k] else 0
    if "fell_back" in r:
        out["fell_back"] = r["fell_back"]
    return out


def pinv_resident(T, torch, num, A, B1, B16, X1, X16, b1, b16, solve_bytes1, solve_bytes16, tol,
                  reps=10, variant=None):
    """Partitioned-inverse solves on the resident factor of ``num`` (merged
    products, or with ``variant`` the level CSR form): the setup (inverse
    panels) once, then 1- and 16-RHS solves; the handle goes back to the
    default variant afterwards."""
    import numpy as np
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T.tacho_set_solve_variant(num, variant or T.TACHO_SOLVE_PARTITIONED_INVERSE)
    out = {"setup_ms": (time.perf_counter() - t0) * 1e3}
    for k, B, X, b, sb in ((1, B1, X1, b1, solve_bytes1), (16, B16, X16, b16, solve_bytes16)):
        ts, iters = [], 0
        for it in range(reps + 2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = T.tacho_solve(num, B, X, with_info=True)
            torch.cuda.synchronize()
            if it >= 2:
                ts.append((time.perf_counter() - t) * 1e3)
                iters = max(iters, info["iters"])
        rho = float(residual(A, X.cpu().numpy(), b).max())
        ms = float(np.median(ts))
        out[f"solve_nrhs{k}_ms_p50"] = ms
        out[f"solve_nrhs{k}_ms_p99"] = pct(ts, 99)
        out[f"resident_rhs_solves_per_s_nrhs{k}"] = k * 1e3 / ms if rho <= tol else None
        out[f"solve_nrhs{k}_hbm_frac"] = sb / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS
        out[f"rel_residual_nrhs{k}"] = rho
        if num.precision == T.TACHO_FP32:
            out[f"refine_iters{k}"] = iters
    T.tacho_set_solve_variant(num, T.TACHO_SOLVE_BLOCK_INVERSE)
    return out


FACTOR_KERNELS = ("k_small", "k_assemble", "k_diag", "k_panel", "k_gemm", "k_gather", "k_front")
SOLVE_KERNELS = ("k_fwd", "k_bwd", "k_permute")


def kernel_profile(T, torch, num, vals, B1, B16, X1, X16):
    """One profiled step: per-kernel launches, device ms, algorithmic work."""
    torch.cuda.synchronize()
    T.tacho_profile(num, True)
    T.tacho_refactorize(num, vals, sync=False)
    T.tacho_solve(num, B1, X1)
    T.tacho_solve(num, B16, X16)
    torch.cuda.synchronize()
    prof = T.tacho_profile_read(num)
    T.tacho_profile(num, False)
    return prof


def roofline(prof, fp32, traffic):
    """Roofline object of the factorization kernel with the most device time."""
    factor = {k: v for k, v in prof.items() if k in FACTOR_KERNELS and v["launches"] > 0}
    name = max(factor, key=lambda k: factor[k]["ms"])
    p = factor[name]
    avg_ms = p["ms"] / p["launches"]
    tname = f"{name}<{'float' if fp32 else 'double'}>"
    if name in ("k_gemm", "k_front"):
        achieved = p["flops"] / (p["ms"] * 1e-3) / 1e12
        out = {"bound": "mfma", "peak": PEAK_FP32_MFMA_TFLOPS if fp32 else PEAK_FP64_MFMA_TFLOPS,
               "unit": "TFLOP/s"}
    elif name in ("k_small", "k_diag", "k_panel"):
        achieved = p["flops"] / (p["ms"] * 1e-3) / 1e12
        out = {"bound": "alu", "peak": PEAK_FP32_VECTOR_TFLOPS if fp32 else PEAK_FP64_VECTOR_TFLOPS,
               "unit": "TFLOP/s"}
    else:
        achieved = p["bytes"] / (p["ms"] * 1e-3) / 1e9
        out = {"bound": "hbm", "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    out.update({"kernel": tname, "achieved": achieved, "frac": achieved / out["peak"],
                "traffic": (traffic or {}).get(tname),
                "algorithmic_flops_per_launch": p["flops"] / p["launches"],
                "algorithmic_bytes_per_launch": p["bytes"] / p["launches"],
                "launches": p["launches"], "avg_launch_ms": avg_ms,
                "share_of_factor_time": p["ms"] / sum(v["ms"] for v in factor.values())})
    return out


def solve_kernels(prof):
    """Forward and backward sweeps: algorithmic bytes over their device time."""
    out = {}
    for k in SOLVE_KERNELS:
        p = prof.get(k)
        if p and p["launches"] > 0 and p["ms"] > 0:
            gbs = p["bytes"] / (p["ms"] * 1e-3) / 1e9
            out[k] = {"launches": p["launches"], "ms": p["ms"], "bytes": p["bytes"],
                      "gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
    return out


# ---------------------------------------------------------------------------
# recorded HBM traffic (rocprofv3 counters)


def sources_hash(tag):
    """Hash of the kernel and plan sources and of the tuned plans of the
    workload the summary covers (what its launches depend on)."""
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    from paper_2506_05793_amd import autotune
    n, nnz = WORKLOAD_SHAPES[tag]
    for prec in (0, 1):
        h.update(json.dumps(autotune.tuned_params(n, nnz, prec), sort_keys=True).encode())
    return h.hexdigest()[:16]


# n, nnz(A) of the workloads a traffic summary may cover
WORKLOAD_SHAPES = {"landice200": (880000, 44342896), "fv3d64": (262144, 1810432)}


def recorded_traffic(tag):
    """{kernel<type>: HBM bytes per launch} from the workload's traffic
    summary, if it matches the current sources."""
    try:
        text = open(traffic_file(tag)).read()
    except OSError:
        return {}
    m = re.search(r"sources hash: `([0-9a-f]+)`", text)
    if not m or m.group(1) != sources_hash(tag):
        return {}
    out = {}
    for row in re.finditer(r"^\| (k_\w+<[^|]*>) \| (\d+) \| [^|]+\| [^|]+\| ([0-9.e+]+) \|", text, re.M):
        out[row.group(1)] = float(row.group(3))
    return out


def short_kernel(name):
    """k_name<template args> of a rocprofv3 kernel name."""
    m = re.search(r"::(k_[a-z0-9_]+)", name)
    if not m:
        return None
    t = re.search(r"::k_[a-z0-9_]+<([^<>]*)>", name)
    return m.group(1) + (f"<{t.group(1).replace(' ', '')}>" if t else "")


def read_counters(path, counter):
    """{dispatch id: (kernel name, value)} from a rocprofv3 counter_collection csv."""
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            name, v = out.get(d, (r["Kernel_Name"], 0.0))
            out[d] = (name, v + float(r["Counter_Value"]))
    return out


def traffic_summary(tag, fetch_csv, write_csv, command):
    """Write the per-kernel HBM traffic summary from the two counter runs."""
    fetch = read_counters(fetch_csv, "FETCH_SIZE")
    write = read_counters(write_csv, "WRITE_SIZE")
    probe_kib = COPY_PROBE_ELEMS * 8 / 1024

    def per_kernel(counts):
        agg, probe = {}, []
        for name, v in counts.values():
            if "neg_kernel" in name:
                probe.append(v)
                continue
            k = short_kernel(name)
            if k:
                agg.setdefault(k, []).append(v)
        return agg, max(probe)

    fa, fprobe = per_kernel(fetch)
    wa, wprobe = per_kernel(write)
    ff, fw = probe_kib / fprobe, probe_kib / wprobe
    lines = [
        f"# HBM traffic per launch, {WORKLOAD_TITLES[tag]}, FP64 and FP32 handles",
        "",
        "Two `rocprofv3 --pmc` runs of the same command (one counter each), eager launches.",
        f"Calibration: a plain FP64 negation kernel over {COPY_PROBE_ELEMS} elements "
        f"({probe_kib:.0f} KiB read, {probe_kib:.0f} KiB written) read FETCH_SIZE {fprobe:.0f} KiB "
        f"and WRITE_SIZE {wprobe:.0f} KiB; factors {ff:.4f} (fetch) and {fw:.4f} (write) are "
        "applied below.",
        "",
        f"sources hash: `{sources_hash(tag)}`",
        "",
        "Commands:",
        "",
        "```",
        command,
        "```",
        "",
        "| kernel | dispatches | fetch KiB/launch | write KiB/launch | HBM bytes/launch (scaled) |",
        "|---|---|---|---|---|",
    ]
    for k in sorted(fa, key=lambda k: -sum(fa[k])):
        f = sum(fa[k]) / len(fa[k])
        w = sum(wa.get(k, [0.0])) / max(1, len(wa.get(k, [])))
        lines.append(f"| {k} | {len(fa[k])} | {f:.1f} | {w:.1f} | {(f * ff + w * fw) * 1024:.4e} |")
    text = "\n".join(lines) + "\n"
    with open(traffic_file(tag), "w") as fh:
        fh.write(text)
    print(text)


def kernel_stats_summary(stats_csv, out_md, title, command, top=20):
    """Short markdown table from a rocprofv3 --stats kernel_stats.csv."""
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# {title}", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = short_kernel(r["Name"]) or r["Name"][:60]
        lines.append(f"| {name} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def overlap_summary(trace_csv, out_md, title, command):
    """Device concurrency of a kernel trace: the time during which kernels of
    two or more queues run at once, and per queue its busy time."""
    import csv
    ev = []
    busy = {}
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            q = r.get("Queue_Id") or r.get("Stream_Id")
            a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            if b <= a:
                continue
            ev.append((a, 1, q))
            ev.append((b, -1, q))
            busy[q] = busy.get(q, 0) + (b - a)
    ev.sort(key=lambda e: (e[0], e[1]))
    active = {}
    t_prev, any_ns, multi_ns, depth_ns = None, 0, 0, 0
    for t, d, q in ev:
        if t_prev is not None:
            nq = sum(1 for v in active.values() if v > 0)
            if nq >= 1:
                any_ns += t - t_prev
            if nq >= 2:
                multi_ns += t - t_prev
            depth_ns += nq * (t - t_prev)
        active[q] = active.get(q, 0) + d
        t_prev = t
    span = (ev[-1][0] - ev[0][0]) if ev else 0
    lines = [f"# {title}", "", "Command:", "", "```", command, "```", "",
             f"Trace span {span / 1e6:.1f} ms; a kernel running {any_ns / 1e6:.1f} ms; kernels of "
             f"two or more queues at once {multi_ns / 1e6:.1f} ms "
             f"({100.0 * multi_ns / max(any_ns, 1):.1f}% of the busy time); average queues "
             f"busy while any is {depth_ns / max(any_ns, 1):.2f}.", "",
             "| queue | kernel busy ms |", "|---|---|"]
    for q, v in sorted(busy.items(), key=lambda kv: -kv[1]):
        lines.append(f"| {q} | {v / 1e6:.1f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {out_md}")


def mfma_summary(csv_path, out_md, title, command):
    """MFMA busy fraction and executed MFMA flops per kernel from one
    rocprofv3 --pmc run of SQ_VALU_MFMA_BUSY_CYCLES, SQ_INSTS_VALU_MFMA_MOPS_F64,
    SQ_INSTS_VALU_MFMA_MOPS_F32, GRBM_GUI_ACTIVE.  GRBM_GUI_ACTIVE is counted
    once per XCD (8) and the chip has 1024 SIMDs; one MOPS unit is 512 flops."""
    per = {}
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            k = short_kernel(r["Kernel_Name"])
            if not k:
                continue
            d = per.setdefault(k, {}).setdefault(int(r["Dispatch_Id"]), {})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    lines = [f"# {title}", "", "One `rocprofv3 --pmc` run (eager launches).",
             "Busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 1024 SIMDs); executed "
             "MFMA flops = (SQ_INSTS_VALU_MFMA_MOPS_F64 + _F32) x 512.", "", "Command:", "", "```",
             command, "```", "",
             "| kernel | dispatches | MFMA busy (% of SIMD cycles) | executed MFMA flops per dispatch |",
             "|---|---|---|---|"]
    rows = []
    for k, ds in per.items():
        busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in ds.values())
        act = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in ds.values()) / 8 * 1024
        mops = sum(d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) + d.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)
                   for d in ds.values())
        if mops > 0:
            rows.append((k, len(ds), 100.0 * busy / max(act, 1.0), mops * 512 / len(ds)))
    for k, nd, b, f in sorted(rows, key=lambda r: -r[3] * r[1]):
        lines.append(f"| {k} | {nd} | {b:.1f} | {f:.4e} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# ---------------------------------------------------------------------------
# CPU baseline


def cpu_baseline(kind):
    """The oracle (plain left-looking FP64 Cholesky, 1 thread) on a bounded
    sample of the workload: factor + 1-RHS solve.  Returns the baseline and
    the sample (matrix, permutation, rhs, oracle solution)."""
    import gen
    import oracle
    import paper_2506_05793_amd as T
    if kind == "landice200":
        A = gen.landice(50, 50, 11, seed=3)
        desc = "land-ice 50x50x11 nodes x 2 DOF (n=55000), the stated down-scaled instance"
    else:
        A = gen.fv3d(46, seed=1)
        desc = "3D 7-point lognormal 46^3 (n=97336)"
    sym = T.tacho_analyze(A.n, A.rowptr, A.colind)
    perm = T.tacho_get_symbolic(sym).perm
    flops = T.tacho_query_symbolic(sym)["flops"]
    oracle.build(force=False)
    t0 = time.perf_counter()
    F = oracle.factor(A, perm)
    t1 = time.perf_counter()
    b = gen.rhs(A.n, 1, seed=2)
    xo = oracle.solve(F, b)
    t2 = time.perf_counter()
    base = {"value": flops / (t1 - t0) / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{desc}, library ordering, FP64 factor {t1 - t0:.2f} s ({flops:.3e} "
                      f"flops) + 1-RHS solve {t2 - t1:.2f} s, 1 thread of {os.cpu_count()} "
                      f"({cpu_model()})"}
    return base, (A, b, xo)


def sample_errors(T, torch, sample):
    """Both GPU paths on the CPU baseline's sample: relative error of the
    solution against the oracle's FP64 solution."""
    from paper_2506_05793_amd import autotune
    A, b, xo = sample
    out = {"sample_n": A.n}
    for name, prec in (("fp64", T.TACHO_FP64), ("mixed", T.TACHO_FP32)):
        s = T.tacho_analyze(A.n, A.rowptr, A.colind, autotune.options_for(A.n, A.nnz, prec))
        num = T.tacho_factorize(s, A.values, prec)
        x = T.tacho_solve(num, b)
        out[name] = {"rel_error_vs_oracle": rel_err(x, xo),
                     "rel_residual": float(residual(A, x, b).max())}
    return out


# ---------------------------------------------------------------------------
# single-system workloads


WORKLOAD_TITLES = {
    "landice200": "land-ice 200x200x11 nodes x 2 DOF (n=880000)",
    "fv3d64": "3D 7-point FV lognormal 64^3 (n=262144)",
}


def single_system(T, torch, A, tag, args, profile=True, steps=None, warmup=None):
    """FP64 and mixed steps on one system; returns the record of the run."""
    import numpy as np
    from paper_2506_05793_amd import autotune
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    extra = {"graphs": 0} if args.eager else {}

    def opts(prec):
        if args.no_tuning:
            return T.tacho_default_options(**extra)
        return autotune.options_for(A.n, A.nnz, prec, **extra)

    t0 = time.perf_counter()
    sym64 = T.tacho_analyze(A.n, A.rowptr, A.colind, opts(T.TACHO_FP64))
    analyze_s = time.perf_counter() - t0
    q = T.tacho_query_symbolic(sym64)
    sym32 = T.tacho_analyze(A.n, A.rowptr, A.colind, opts(T.TACHO_FP32))
    q32 = T.tacho_query_symbolic(sym32)
    plan = lambda qq: {k[5:]: qq[k] for k in qq if k.startswith("plan_")}  # noqa: E731
    log(f"[bench] {tag}: analyze {analyze_s:.2f}s n={A.n} nnz(L)={q['nnz_l']:.3e} "
        f"flops={q['flops']:.3e} supernodes={q['nsuper']} levels={q['nlevels']}")
    b1 = gen_rhs(A.n, 1)
    b16 = gen_rhs(A.n, 16)
    vals = torch.from_numpy(A.values).cuda()
    B1, B16 = dev_colmajor(torch, b1), dev_colmajor(torch, b16)
    X1, X16 = torch.empty_like(B1), torch.empty_like(B16)
    Y1, Y16 = torch.empty_like(B1), torch.empty_like(B16)
    nnz_l = q["nnz_l"]
    sbytes = lambda es, k: 2.0 * nnz_l * es + 4.0 * A.n * k * 8  # noqa: E731
    rec = {"n": A.n, "nnz_a": int(A.nnz), "nnz_l": nnz_l, "flops": q["flops"],
           "supernodes": q["nsuper"], "levels": q["nlevels"], "max_front": q["max_front"],
           "analyze_s_host": analyze_s, "plan_fp64": plan(q), "plan_fp32": plan(q32)}

    log(f"[bench] {tag} FP64: {warmup} warmup + {steps} timed steps")
    num64 = T.tacho_factorize(sym64, vals, T.TACHO_FP64)
    r64 = run_steps(T, torch, num64, vals, B1, B16, X1, X16, steps, warmup)
    x1, x16 = X1.cpu().numpy(), X16.cpu().numpy()
    s64 = summarize(r64, q["flops"], 1e-12, float(residual(A, x1, b1).max()),
                    float(residual(A, x16, b16).max()), sbytes(8, 1), sbytes(8, 16))
    rec["fp64"] = s64
    rec["wall_s_fp64"] = r64["wall_s"]
    log(f"[bench] {tag} FP64 factor {s64['factor_ms_p50']:.2f} ms ({s64['factor_tflops']:.2f} "
        f"TFLOP/s), solve1 {s64['solve_nrhs1_ms_p50']:.2f} ms, solve16 "
        f"{s64['solve_nrhs16_ms_p50']:.2f} ms, rho {s64['rel_residual_nrhs1']:.1e}/"
        f"{s64['rel_residual_nrhs16']:.1e}")
    prof64 = kernel_profile(T, torch, num64, vals, B1, B16, X1, X16) if profile else None
    if not args.no_pinv:
        s64["partitioned_inverse"] = pinv_resident(T, torch, num64, A, B1, B16, X1, X16, b1, b16,
                                                   sbytes(8, 1), sbytes(8, 16), 1e-12)
        pv = s64["partitioned_inverse"]
        log(f"[bench] {tag} FP64 partitioned inverse: setup {pv['setup_ms']:.1f} ms, solve1 "
            f"{pv['solve_nrhs1_ms_p50']:.2f} ms, solve16 {pv['solve_nrhs16_ms_p50']:.2f} ms, rho "
            f"{pv['rel_residual_nrhs1']:.1e}")
        s64["level_csr"] = pinv_resident(T, torch, num64, A, B1, B16, X1, X16, b1, b16,
                                         sbytes(8, 1), sbytes(8, 16), 1e-12, reps=5,
                                         variant=T.TACHO_SOLVE_LEVEL_CSR)
        pv = s64["level_csr"]
        log(f"[bench] {tag} FP64 level CSR: setup {pv['setup_ms']:.1f} ms, solve1 "
            f"{pv['solve_nrhs1_ms_p50']:.2f} ms, solve16 {pv['solve_nrhs16_ms_p50']:.2f} ms, rho "
            f"{pv['rel_residual_nrhs1']:.1e}")
    if not args.no_mixed:
        log(f"[bench] {tag} mixed: FP32 factor + FP64 refinement")
        num32 = T.tacho_factorize(sym32, vals, T.TACHO_FP32)
        r32 = run_steps(T, torch, num32, vals, B1, B16, Y1, Y16, steps, min(warmup, 2))
        y1, y16 = Y1.cpu().numpy(), Y16.cpu().numpy()
        mixed = summarize(r32, q["flops"], 1e-10, float(residual(A, y1, b1).max()),
                          float(residual(A, y16, b16).max()), sbytes(4, 1), sbytes(4, 16))
        mixed["rel_error_vs_fp64_nrhs1"] = rel_err(y1, x1)
        mixed["rel_error_vs_fp64_nrhs16"] = rel_err(y16, x16)
        mixed["factor_speedup_vs_fp64"] = s64["factor_ms_p50"] / mixed["factor_ms_p50"]
        mixed["fresh_request_speedup_vs_fp64"] = (s64["request_factor_solve_ms_p50"] /
                                                  mixed["request_factor_solve_ms_p50"])
        rec["mixed"] = mixed
        log(f"[bench] {tag} mixed factor {mixed['factor_ms_p50']:.2f} ms, solve1 "
            f"{mixed['solve_nrhs1_ms_p50']:.2f} ms, rho {mixed['rel_residual_nrhs1']:.1e}, "
            f"error vs FP64 {mixed['rel_error_vs_fp64_nrhs1']:.1e}")
        prof32 = kernel_profile(T, torch, num32, vals, B1, B16, Y1, Y16) if profile else None
        if not args.no_pinv:
            mixed["partitioned_inverse"] = pinv_resident(T, torch, num32, A, B1, B16, Y1, Y16, b1,
                                                         b16, sbytes(4, 1), sbytes(4, 16), 1e-10)
            pv = mixed["partitioned_inverse"]
            log(f"[bench] {tag} mixed partitioned inverse: setup {pv['setup_ms']:.1f} ms, solve1 "
                f"{pv['solve_nrhs1_ms_p50']:.2f} ms, solve16 {pv['solve_nrhs16_ms_p50']:.2f} ms, "
                f"rho {pv['rel_residual_nrhs1']:.1e}")
        del num32
    else:
        prof32 = None
    if profile:
        traffic = recorded_traffic(tag) if tag in WORKLOAD_SHAPES else {}
        rec["roofline"] = roofline(prof64, False, traffic)
        rec["solve_kernels_fp64"] = solve_kernels(prof64)
        rec["kernels_fp64"] = prof64
        if prof32:
            rec["roofline_mixed"] = roofline(prof32, True, traffic)
            rec["solve_kernels_mixed"] = solve_kernels(prof32)
            rec["kernels_mixed"] = prof32
        roof = rec["roofline"]
        log(f"[bench] {tag} dominant {roof['kernel']}: {roof['achieved']:.2f} {roof['unit']} "
            f"({100 * roof['frac']:.1f}% of peak)")
    if not args.no_lu and tag == "landice200":
        lu = lu_leg(T, torch, A, sym64, B1, B16, X1, X16, b1, b16, max(3, steps // 4), 1, sbytes)
        rec["lu"] = lu
        log(f"[bench] {tag} LU factor {lu['factor_ms_p50']:.2f} ms ({lu['factor_tflops']:.2f} "
            f"TFLOP/s), solve1 {lu['solve_nrhs1_ms_p50']:.2f} ms, solve16 "
            f"{lu['solve_nrhs16_ms_p50']:.2f} ms, rho {lu['rel_residual_nrhs1']:.1e}, "
            f"interchanges {lu['row_interchanges']}, dominant {lu['roofline']['kernel']} "
            f"{100 * lu['roofline']['frac']:.1f}% of peak")
    del num64
    return rec


def lu_leg(T, torch, A, sym, B1, B16, X1, X16, b1, b16, steps, warmup, sbytes):
    """LU (restricted row pivoting) of the same pattern with nonsymmetric
    values (each off-diagonal pair skewed by up to 30%), on the FP64 analysis:
    refactorization + 1-RHS + 16-RHS solve steps, flops counted as
    2 sum eta_j^2 (the update runs on both halves), and its kernel profile."""
    import numpy as np
    import gen
    An = gen.nonsymmetric(A, 0.3, seed=11)
    assert np.array_equal(An.rowptr, A.rowptr) and np.array_equal(An.colind, A.colind)
    vals = torch.from_numpy(An.values).cuda()
    q = T.tacho_query_symbolic(sym)
    t0 = time.perf_counter()
    num = T.tacho_factorize(sym, vals, T.TACHO_LU)
    first_s = time.perf_counter() - t0
    r = run_steps(T, torch, num, vals, B1, B16, X1, X16, steps, warmup)
    x1, x16 = X1.cpu().numpy(), X16.cpu().numpy()
    out = summarize(r, 2 * q["flops"], 1e-10, float(residual(An, x1, b1).max()),
                    float(residual(An, x16, b16).max()), 2 * sbytes(8, 1), 2 * sbytes(8, 16))
    _, _, _, order = T.tacho_get_lu(num)
    out["row_interchanges"] = int((order != np.arange(A.n)).sum())
    out["first_factorization_s_host"] = first_s
    prof = kernel_profile(T, torch, num, vals, B1, B16, X1, X16)
    out["roofline"] = roofline(prof, False, {})
    out["kernels"] = prof
    del num
    return out


def gen_rhs(n, k):
    import gen
    return gen.rhs(n, k, seed=2)


def make_workload(tag, args):
    import gen
    if tag == "landice200":
        s = args.li_side
        log(f"[bench] building land-ice {s}x{s}x11x2")
        return gen.landice(s, s, 11, seed=3)
    log(f"[bench] building 3D lognormal {args.side}^3")
    return gen.fv3d(args.side, seed=1)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="landice",
                    choices=["landice", "3d", "2d", "batch", "serve"],
                    help="landice: extruded 2-DOF mesh (default, the metric's workload; "
                         "--li-side); 3d: 64^3 lognormal (--side); 2d: 32x32 Laplacian; "
                         "batch: 256 subdomain systems; serve: request stream")
    ap.add_argument("--li-side", type=int, default=200, help="land-ice base grid side")
    ap.add_argument("--side", type=int, default=64, help="grid side of the 3D workload")
    ap.add_argument("--no-fv3d", action="store_true",
                    help="landice: skip the extra 64^3 measurement")
    ap.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serve: mean arrival rate (requests/s; 0: all at once, i.e. capacity)")
    ap.add_argument("--load", type=str, default="",
                    help="serve: comma-separated fractions of the measured capacity to offer "
                         "after the capacity run (e.g. 0.5,0.8,0.95)")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="serve: HBM budget in GB (0: 0.8 x free device memory)")
    ap.add_argument("--workers", type=int, default=8, help="serve: host analysis workers")
    ap.add_argument("--mixed-frac", type=float, default=0.5,
                    help="serve: fraction of factor requests in FP32 + refinement")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-lu", action="store_true",
                    help="skip the LU measurement (land-ice pattern, nonsymmetric values)")
    ap.add_argument("--no-pinv", action="store_true",
                    help="skip the partitioned-inverse resident-solve measurement")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the plan parameters of the workload (FP64 and FP32) on the "
                         "device and store them in the package's tuning table")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the tuning table")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="launch the factorization kernels one by one instead of a graph")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB FP64 negation kernel first (counter calibration)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("TAG", "FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="write the HBM traffic summary of a workload (landice200 or fv3d64) "
                         "from two counter runs and exit")
    ap.add_argument("--kernel-summary", nargs=4, metavar=("STATS_CSV", "OUT_MD", "TITLE", "COMMAND"),
                    help="write a markdown kernel summary from rocprofv3 stats and exit")
    ap.add_argument("--overlap-summary", nargs=4, metavar=("TRACE_CSV", "OUT_MD", "TITLE", "COMMAND"),
                    help="write the device-concurrency summary of a kernel trace and exit")
    ap.add_argument("--mfma-summary", nargs=4, metavar=("CSV", "OUT_MD", "TITLE", "COMMAND"),
                    help="write the MFMA utilization summary from one counter run and exit")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.kernel_summary:
        kernel_stats_summary(*args.kernel_summary)
        return
    if args.mfma_summary:
        mfma_summary(*args.mfma_summary)
        return
    if args.overlap_summary:
        overlap_summary(*args.overlap_summary)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: every workload is measured on one MI355X "
              "(sharding across GPUs is a design note only).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2506_05793_amd as T

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        x = torch.ones(COPY_PROBE_ELEMS, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
    if args.workload in ("2d", "batch", "serve"):
        other_workload(args, T, torch)
        return
    tag = "landice200" if args.workload == "landice" else "fv3d64"
    A = make_workload(tag, args)
    if args.autotune:
        autotune_workload(args, T, A, tag)
        return
    rec = single_system(T, torch, A, tag, args, profile=not args.no_profile)
    fv3d = None
    if tag == "landice200" and not args.no_fv3d:
        B = make_workload("fv3d64", args)
        fv3d = single_system(T, torch, B, "fv3d64", args, profile=False,
                             steps=max(5, args.steps // 2), warmup=min(args.warmup, 2))
    cpu = errs = None
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle, bounded sample)")
        cpu, sample = cpu_baseline(tag)
        log(f"[bench] oracle {cpu['value'] * 1e3:.3f} GFLOP/s")
        errs = sample_errors(T, torch, sample)
        log(f"[bench] errors against the oracle on the sample: {errs}")
    s64 = rec["fp64"]
    title = WORKLOAD_TITLES[tag]
    line = {
        "metric": METRIC,
        "value": s64["factor_tflops"] if s64["meets_tol"] else None,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["wall_s_fp64"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{title}, 27-point node coupling, random SPD 2x2 blocks, vertical "
                         f"anisotropy 1e3: FP64 multifrontal Cholesky vs FP32 factor + FP64 "
                         f"refinement, 1 and 16 RHS" if tag == "landice200" else
                         f"{title}: FP64 multifrontal Cholesky vs FP32 factor + FP64 "
                         f"refinement, 1 and 16 RHS"),
            "ordering": "own nested dissection + etree postorder",
            **{k: rec[k] for k in ("n", "nnz_a", "nnz_l", "flops", "supernodes", "levels",
                                   "max_front", "analyze_s_host", "plan_fp64", "plan_fp32")},
        },
        "fp64": s64,
        "mixed": rec.get("mixed"),
        "roofline": rec.get("roofline"),
        "roofline_mixed": rec.get("roofline_mixed"),
        "solve_kernels_fp64": rec.get("solve_kernels_fp64"),
        "solve_kernels_mixed": rec.get("solve_kernels_mixed"),
        "error_vs_oracle_on_sample": errs,
        "cpu_baseline": cpu,
        "fv3d64": fv3d,
        "kernels_fp64": rec.get("kernels_fp64"),
        "kernels_mixed": rec.get("kernels_mixed"),
    }
    if rec.get("lu"):
        line["lu"] = {k: v for k, v in rec["lu"].items() if k != "kernels"}
        line["kernels_lu"] = rec["lu"]["kernels"]
    print(json.dumps(line), flush=True)


def autotune_workload(args, T, A, tag):
    """Coordinate descent on the device; the land-ice workload also sets the
    order-changing parameters of each precision."""
    from paper_2506_05793_amd import autotune
    tab = autotune.TuningTable(autotune.DEFAULT_TABLE)
    out = {}
    landice = tag == "landice200"
    cands = dict(autotune.CANDIDATES)
    if landice:  # analysis takes seconds here: a reduced candidate set
        cands = {"chain_min": (2, 3, 4, 6, 8, -1), "chain_inplace": (0, -1),
                 "asm_cols": (4, 8, 16), "solo_m": (-1, 128, 192, 256, 384),
                 "solve_level_fronts": (64, 256, 1024)}
    for prec, name in ((T.TACHO_FP64, "fp64"), (T.TACHO_FP32, "fp32")):
        fixed = {} if landice else autotune.tuned_params(1, 1, prec)  # order entry only
        c = {k: v for k, v in cands.items() if landice or k in autotune.ORDER_NEUTRAL}
        best, m, hist = autotune.tune(A.n, A.rowptr, A.colind, A.values, prec,
                                      reps=5 if landice else 7, log=log, candidates=c, start=fixed)
        autotune.store(tab, A.n, A.nnz, prec, best,
                       {"workload": WORKLOAD_TITLES[tag], "device": "MI355X",
                        "factor_ms": m["factor_ms"], "solve_ms": m["solve_ms"],
                        "default_factor_ms": hist[0][1]["factor_ms"],
                        "default_solve_ms": hist[0][1]["solve_ms"], "candidates": len(hist)},
                       order_too=landice)
        out[name] = {"best": best, "measured": m, "default": hist[0][1]}
    tab.save()
    print(json.dumps({"autotune": out}), flush=True)


def line_for(args, metric_value, unit, dtype, config, extra):
    out = {"metric": METRIC, "value": metric_value, "unit": unit, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def other_workload(args, T, torch):
    """C1 (2d), C4 (batch) and C5 (serve) measurements."""
    import numpy as np

    import gen
    from paper_2506_05793_amd import autotune
    if args.workload == "serve":
        serve_workload(args, T, torch)
        return
    if args.workload == "batch":
        mats = gen.batch_fv3d(256, seed=4)
        log(f"[bench] batch of {len(mats)} systems, n total {sum(m.n for m in mats)}")
        A = gen.csr_block_diag(mats)
        t0 = time.perf_counter()
        syms = {p: T.tacho_analyze_batch([(m.n, m.rowptr, m.colind) for m in mats],
                                         autotune.options_for(A.n, A.nnz, p))
                for p in (T.TACHO_FP64, T.TACHO_FP32)}
        analyze_s = (time.perf_counter() - t0) / 2
        vals_np = np.concatenate([m.values for m in mats])
        n = A.n
        b = np.asfortranarray(np.concatenate([gen.rhs(m.n, 1, seed=10 + k)
                                              for k, m in enumerate(mats)], axis=0))
        precisions = [("mixed", T.TACHO_FP32, 1e-10), ("fp64", T.TACHO_FP64, 1e-12)]
    else:
        A = gen.laplace2d(32)
        t0 = time.perf_counter()
        s = T.tacho_analyze(A.n, A.rowptr, A.colind)
        analyze_s = time.perf_counter() - t0
        syms = {T.TACHO_FP64: s, T.TACHO_FP32: s}
        vals_np = A.values
        n = A.n
        b = gen.rhs(n, 1, seed=0)
        precisions = [("fp64", T.TACHO_FP64, 1e-12), ("mixed", T.TACHO_FP32, 1e-10)]
    q = T.tacho_query_symbolic(syms[T.TACHO_FP64])
    log(f"[bench] analyze {analyze_s:.2f}s n={n} nnz(L)={q['nnz_l']:.3e} flops={q['flops']:.3e} "
        f"levels={q['nlevels']}")
    vals = torch.from_numpy(vals_np).cuda()
    B = dev_colmajor(torch, np.asarray(b).reshape(n, -1))
    X = torch.empty_like(B)
    results = {}
    for name, prec, tol in precisions:
        num = T.tacho_factorize(syms[prec], vals, prec)
        fms, sms, rows = [], [], []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            T.tacho_refactorize(num, vals, sync=False)
            e1.record()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = T.tacho_solve(num, B, X, with_info=True)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if it >= args.warmup:
                fms.append(e0.elapsed_time(e1))
                sms.append((t2 - t1) * 1e3)
                rows.append(info)
        rho = float(residual(A, X.cpu().numpy(), np.asarray(b).reshape(n, -1)).max())
        f50 = float(np.median(fms))
        s50 = float(np.median(sms))
        results[name] = {
            "factor_ms_p50": f50, "factor_ms_p99": pct(fms, 99),
            "factor_tflops": q["flops"] / (f50 * 1e-3) / 1e12,
            "solve_ms_p50": s50, "solve_ms_p99": pct(sms, 99),
            "request_factor_solve_ms_p50": pct([a + c for a, c in zip(fms, sms)], 50),
            "request_factor_solve_ms_p99": pct([a + c for a, c in zip(fms, sms)], 99),
            "rel_residual": rho, "residual_tol": tol, "meets_tol": rho <= tol,
            "refine_iters": max(r["iters"] for r in rows), "fell_back": max(r["fell_back"] for r in rows),
        }
        if args.workload == "batch":
            results[name]["systems_per_s"] = 256 / ((f50 + s50) * 1e-3)
        log(f"[bench] {name}: {results[name]}")
        del num
    main_name = precisions[0][0]
    line_for(args, results[main_name]["factor_tflops"], "TFLOP/s",
             "f32+f64-refine" if main_name == "mixed" else "f64",
             {"workload": {"2d": "2D 5-point Laplacian 32x32",
                           "batch": "256 3D lognormal subdomain systems, sides in [8,32]"}[args.workload],
              "n": n, "nnz_l": q["nnz_l"], "flops": q["flops"], "levels": q["nlevels"],
              "analyze_s_host": analyze_s}, results)


def serve_workload(args, T, torch):
    """C5: Poisson request stream through the continuous-batching server."""
    import gen
    from paper_2506_05793_amd.serve import Request, Server, summarize as serve_summary
    specs = gen.serving_requests(args.requests, seed=5, rate=1.0, n2d=(1000, 250000),
                                 n3d=(4000, 300000))
    mats, reqs0 = {}, []
    pick = __import__("numpy").random.default_rng(6)
    log(f"[bench] building {len(specs)} requests")
    for i, sp in enumerate(specs):
        if sp["kind"] == "factor":
            A = gen.fv2d(*sp["side"], seed=sp["seed"]) if sp["dim"] == 2 else \
                gen.fv3d(*sp["side"], seed=sp["seed"])
            mats[i] = A
            prec = T.TACHO_FP32 if pick.random() < args.mixed_frac else T.TACHO_FP64
            reqs0.append(dict(rid=i, u=sp["t"], kind="factor", rhs=gen.rhs(A.n, sp["nrhs"],
                                                                          seed=sp["seed"] + 1),
                              matrix=A, precision=prec))
        else:
            A = mats[sp["target"]]
            reqs0.append(dict(rid=i, u=sp["t"], kind="repeat",
                              rhs=gen.rhs(A.n, sp["nrhs"], seed=sp["seed"]), target=sp["target"]))
    free, _ = torch.cuda.mem_get_info()
    budget = int(args.budget_gb * 1e9) if args.budget_gb > 0 else int(0.8 * free)

    def run(rate):
        reqs = [Request(r["rid"], r["u"] / rate if rate > 0 else 0.0, r["kind"], r["rhs"],
                        matrix=r.get("matrix"), target=r.get("target", -1),
                        precision=r.get("precision", T.TACHO_FP64)) for r in reqs0]
        srv = Server(budget, slots=4, analysis_workers=args.workers)
        t0 = time.perf_counter()
        res = srv.run(reqs)
        wall = time.perf_counter() - t0
        srv.close()
        summ = serve_summary(res, wall)
        worst = {"fp64": 0.0, "mixed": 0.0}
        for out in res[:: max(1, len(res) // 60)]:
            r = reqs[out.rid]
            A = r.matrix if r.kind == "factor" else mats[r.target]
            key = "mixed" if out.precision == T.TACHO_FP32 else "fp64"
            worst[key] = max(worst[key], float(residual(A, out.x, r.rhs).max()))
        summ.update({"offered_rate_per_s": rate if rate > 0 else None, "hbm_budget_bytes": budget,
                     "analysis_workers": args.workers,
                     "served_requests_per_s": len(res) / wall,
                     "admitted_while_busy": srv.admitted_while_busy, "peak_bytes": srv.peak_used,
                     "analyses": srv.analyses, "symbolic_reuses": srv.symbolic_hits,
                     "sampled_max_rel_residual": worst})
        log(f"[bench] serve rate={rate}: {summ}")
        return summ

    runs = {"capacity": run(args.rate)}
    cap = runs["capacity"]["served_requests_per_s"]
    for f in [float(x) for x in args.load.split(",") if x]:
        runs[f"load_{f:g}"] = run(f * cap)
    line_for(args, runs["capacity"]["rhs_solves_per_s"], "RHS solves/s", "f64+f32-refine",
             {"workload": f"Poisson request stream, {len(reqs0)} requests, 2D n 1k-250k and "
                          f"3D n 4k-300k lognormal, 1-16 RHS, 30% repeat, "
                          f"{args.mixed_frac:.0%} of factor requests FP32 + refinement"},
             {"serve": runs})


if __name__ == "__main__":
    main()
