#!/usr/bin/env python3
"""Benchmark of the supernodal multifrontal Cholesky on one MI355X.

Workload (default): the 3D 7-point cell-centred operator on a 64^3 grid
(n = 262,144) with lognormal(0,1) cell coefficients, nested-dissection
ordering, FP64 multifrontal factorization plus solves with 1 and 16
right-hand sides ~ N(0,1).  Inputs are synthetic, seeded, and resident in
HBM before timing starts.

One step = refactorization of the values (assembly, extend-add, dense
partial factorizations of every front, level by level) + a 1-RHS solve + a
16-RHS solve.  W untimed warmup steps, then K timed steps bracketed by
device synchronization.  `value` is the FP64 factorization rate
sum_j eta_j^2 / (median device factorization time) in TFLOP/s; solves/s,
p50/p99 latencies and the FP32-factor + FP64-refinement (mixed) numbers are
reported beside it.  Every rate is reported only with the residual it was
obtained at.

Also reported: the roofline of the dominant kernel (per-launch hipEvent
timing inside this run, algorithmic flops or bytes from the launch plan) and
a CPU baseline (the oracle on a bounded sample).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import re
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "factor TFLOP/s + solves/s at rel. residual <=1e-10 (mixed vs FP64); p50/p99"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Measured HBM traffic per launch of the factorization kernels (rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs, calibrated on a copy kernel of known size),
# written by --traffic-summary and read back by the roofline.  The file records
# a hash of the kernel and launch-plan sources; when they change the recorded
# figures no longer describe the kernel and the roofline reports traffic null.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "factor_kernels_fv3d64_hbm_traffic.md")
TRAFFIC_SOURCES = ("paper_2506_05793_amd/csrc/kernels.hip", "paper_2506_05793_amd/csrc/plan.cpp",
                   "paper_2506_05793_amd/csrc/plan.hpp")
COPY_PROBE_ELEMS = 1 << 27  # FP64 elements: 1 GiB read + 1 GiB written


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
    return (np.linalg.norm(B - M @ X, axis=0) / np.linalg.norm(B, axis=0))


def dev_colmajor(torch, a):
    """Column-major device copy of a host n x k array."""
    return torch.from_numpy(a.T.copy()).cuda().t()


def run_fp64(T, torch, A, sym, vals, b1, b16, steps, warmup):
    B1, B16 = dev_colmajor(torch, b1), dev_colmajor(torch, b16)
    X1, X16 = torch.empty_like(B1), torch.empty_like(B16)
    num = T.tacho_factorize(sym, vals, T.TACHO_FP64)

    def step():
        T.tacho_refactorize(num, vals, sync=False)
        T.tacho_solve(num, B1, X1)
        T.tacho_solve(num, B16, X16)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record()
        T.tacho_refactorize(num, vals, sync=False)
        ev[i][1].record()
        T.tacho_solve(num, B1, X1)
        ev[i][2].record()
        T.tacho_solve(num, B16, X16)
        ev[i][3].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tacho_check_factor(num)
    f_ms = [e[0].elapsed_time(e[1]) for e in ev]
    s1_ms = [e[1].elapsed_time(e[2]) for e in ev]
    s16_ms = [e[2].elapsed_time(e[3]) for e in ev]
    rho1 = residual(A, X1.cpu().numpy(), b1)
    rho16 = residual(A, X16.cpu().numpy(), b16)
    return num, dict(wall_s=wall, factor_ms=f_ms, solve1_ms=s1_ms, solve16_ms=s16_ms,
                     rho1=float(rho1.max()), rho16=float(rho16.max()))


def run_mixed(T, torch, A, sym, vals, b1, b16, steps, warmup):
    B1, B16 = dev_colmajor(torch, b1), dev_colmajor(torch, b16)
    X1, X16 = torch.empty_like(B1), torch.empty_like(B16)
    num = T.tacho_factorize(sym, vals, T.TACHO_FP32)
    infos = []

    def step(record):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        T.tacho_refactorize(num, vals, sync=False)
        e1.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, i1 = T.tacho_solve(num, B1, X1, with_info=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, i16 = T.tacho_solve(num, B16, X16, with_info=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if record:
            infos.append((e0.elapsed_time(e1), (t2 - t1) * 1e3, (t3 - t2) * 1e3, i1, i16))

    for _ in range(warmup):
        step(False)
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    wall = time.perf_counter() - t0
    rho1 = residual(A, X1.cpu().numpy(), b1)
    rho16 = residual(A, X16.cpu().numpy(), b16)
    return num, dict(wall_s=wall, factor_ms=[i[0] for i in infos], solve1_ms=[i[1] for i in infos],
                     solve16_ms=[i[2] for i in infos],
                     iters1=[i[3]["iters"] for i in infos], iters16=[i[4]["iters"] for i in infos],
                     fell_back=int(any(i[3]["fell_back"] or i[4]["fell_back"] for i in infos)),
                     rho1=float(rho1.max()), rho16=float(rho16.max()))


def summarize(r, flops, tol):
    import numpy as np
    f = float(np.median(r["factor_ms"]))
    s1 = float(np.median(r["solve1_ms"]))
    s16 = float(np.median(r["solve16_ms"]))
    ok = r["rho1"] <= tol and r["rho16"] <= tol
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
        "rel_residual_nrhs1": r["rho1"], "rel_residual_nrhs16": r["rho16"],
        "residual_tol": tol, "meets_tol": bool(ok),
    }
    for k in ("iters1", "iters16"):
        if k in r:
            out["refine_" + k] = int(max(r[k])) if r[k] else 0
    if "fell_back" in r:
        out["fell_back"] = r["fell_back"]
    return out


FACTOR_KERNELS = ("k_small", "k_assemble", "k_diag", "k_panel", "k_gemm", "k_gather", "k_front")


def kernel_profile(T, torch, num, vals, b1, b16):
    """One profiled step: per-kernel launches, device ms, algorithmic work."""
    B1, B16 = dev_colmajor(torch, b1), dev_colmajor(torch, b16)
    X1, X16 = torch.empty_like(B1), torch.empty_like(B16)
    torch.cuda.synchronize()
    T.tacho_profile(num, True)
    T.tacho_refactorize(num, vals, sync=False)
    T.tacho_solve(num, B1, X1)
    T.tacho_solve(num, B16, X16)
    torch.cuda.synchronize()
    prof = T.tacho_profile_read(num)
    T.tacho_profile(num, False)
    return prof


def roofline(prof):
    factor = {k: v for k, v in prof.items() if k in FACTOR_KERNELS and v["launches"] > 0}
    name = max(factor, key=lambda k: factor[k]["ms"])
    p = factor[name]
    avg_ms = p["ms"] / p["launches"]
    if name in ("k_gemm", "k_front"):
        achieved = p["flops"] / (p["ms"] * 1e-3) / 1e12
        out = {"bound": "mfma", "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s"}
    elif name in ("k_small", "k_diag", "k_panel"):
        achieved = p["flops"] / (p["ms"] * 1e-3) / 1e12
        out = {"bound": "alu", "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s"}
    else:
        achieved = p["bytes"] / (p["ms"] * 1e-3) / 1e9
        out = {"bound": "hbm", "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    traffic = recorded_traffic().get(name)
    out.update({"kernel": name, "achieved": achieved, "frac": achieved / out["peak"],
                "traffic": traffic, "algorithmic_bytes_per_launch": p["bytes"] / p["launches"],
                "launches": p["launches"], "avg_launch_ms": avg_ms,
                "share_of_factor_time": p["ms"] / sum(v["ms"] for v in factor.values())})
    return out


def sources_hash():
    """Hash of the kernel and plan sources and of the tuned FP64 plan of the 3D
    workload (what the traffic summary's launches depend on)."""
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    from paper_2506_05793_amd import autotune
    key = autotune.workload_key(262144, 1810432, 1, autotune.TACHO_FP64)  # 64^3: n, nnz(A)
    h.update(json.dumps(autotune.TuningTable(autotune.DEFAULT_TABLE).get(key),
                        sort_keys=True).encode())
    return h.hexdigest()[:16]


def recorded_traffic():
    """{kernel: HBM bytes per launch} from the traffic summary, if it matches the sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return {}
    m = re.search(r"sources hash: `([0-9a-f]+)`", text)
    if not m or m.group(1) != sources_hash():
        return {}
    out = {}
    for row in re.finditer(r"^\| (k_\w+) \| (\d+) \| [^|]+\| [^|]+\| ([0-9.e+]+) \|", text, re.M):
        out[row.group(1)] = float(row.group(3))
    return out


def short_kernel(name):
    m = re.search(r"::(k_[a-z0-9_]+)", name)
    return m.group(1) if m else None


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


def traffic_summary(fetch_csv, write_csv, command):
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
        "# HBM traffic per launch, factorization kernels, 3D 7-point lognormal 64^3, FP64",
        "",
        "Two `rocprofv3 --pmc` runs of the same command (one counter each), eager launches.",
        f"Calibration: a plain FP64 negation kernel over {COPY_PROBE_ELEMS} elements "
        f"({probe_kib:.0f} KiB read, {probe_kib:.0f} KiB written) read FETCH_SIZE {fprobe:.0f} KiB "
        f"and WRITE_SIZE {wprobe:.0f} KiB; factors {ff:.4f} (fetch) and {fw:.4f} (write) are "
        "applied below.",
        "",
        f"sources hash: `{sources_hash()}`",
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
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write(text)
    print(text)


def kernel_stats_summary(stats_csv, out_md, title, command, top=16):
    """Short markdown table from a rocprofv3 --stats kernel_stats.csv."""
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# {title}", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = short_kernel(r["Name"]) or r["Name"][:60]
        m = re.search(r"<([^<>]*)>\(", r["Name"])
        if m and short_kernel(r["Name"]):
            name += f"<{m.group(1)}>"
        lines.append(f"| {name} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cpu_baseline(side=46):
    """The oracle (plain left-looking FP64 Cholesky, 1 thread) on a bounded sample."""
    import gen
    import oracle
    import paper_2506_05793_amd as T
    A = gen.fv3d(side, seed=1)
    sym = T.tacho_analyze(A.n, A.rowptr, A.colind)
    perm = T.tacho_get_symbolic(sym).perm
    flops = T.tacho_query_symbolic(sym)["flops"]
    oracle.build(force=False)
    t0 = time.perf_counter()
    F = oracle.factor(A, perm)
    t1 = time.perf_counter()
    b = gen.rhs(A.n, 1, seed=2)
    oracle.solve(F, b)
    t2 = time.perf_counter()
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": flops / (t1 - t0) / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"3D 7-point lognormal {side}^3 (n={A.n}), same ordering method, FP64 "
                      f"factor {t1 - t0:.2f} s ({flops:.3e} flops) + 1-RHS solve {t2 - t1:.2f} s, "
                      f"1 thread of {os.cpu_count()} ({model})"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--side", type=int, default=64, help="grid side of the 3D workload")
    ap.add_argument("--workload", default="3d", choices=["3d", "2d", "landice", "batch", "serve"],
                    help="3d: 64^3 lognormal (default, the metric's workload); 2d: 32x32 "
                         "Laplacian; landice: extruded 2-DOF mesh (--li-side); batch: 256 "
                         "subdomain systems; serve: request stream")
    ap.add_argument("--li-side", type=int, default=200, help="land-ice base grid side")
    ap.add_argument("--requests", type=int, default=300, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=200.0,
                    help="serve: mean arrival rate (requests/s; 0: all at once, i.e. capacity)")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="serve: HBM budget in GB (0: 0.8 x free device memory)")
    ap.add_argument("--workers", type=int, default=8, help="serve: host analysis workers")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the plan parameters of the 3D workload (FP64 and FP32) on the "
                         "device and store them in the package's tuning table")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the tuning table")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="launch the factorization kernels one by one instead of a graph")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB FP64 negation kernel first (counter calibration)")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="write the HBM traffic summary from two counter runs and exit")
    ap.add_argument("--kernel-summary", nargs=4, metavar=("STATS_CSV", "OUT_MD", "TITLE", "COMMAND"),
                    help="write a markdown kernel summary from rocprofv3 stats and exit")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.kernel_summary:
        kernel_stats_summary(*args.kernel_summary)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the single-system workload is measured on one "
              "MI355X (multi-GPU sharding is a design note only).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
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
    if args.workload != "3d":
        other_workload(args, T, torch)
        return
    side = args.side
    log(f"[bench] building 3D lognormal {side}^3 workload")
    A = gen.fv3d(side, seed=1)
    b1 = gen.rhs(A.n, 1, seed=2)
    b16 = gen.rhs(A.n, 16, seed=2)
    from paper_2506_05793_amd import autotune
    if args.autotune:
        tab = autotune.TuningTable(autotune.DEFAULT_TABLE)
        out = {}
        for prec, name in ((T.TACHO_FP64, "fp64"), (T.TACHO_FP32, "fp32")):
            best, m, hist = autotune.tune(A.n, A.rowptr, A.colind, A.values, prec, log=log)
            key = autotune.workload_key(A.n, A.nnz, 1, prec)
            tab.put(key, best, {"workload": f"3D lognormal {side}^3", "device": "MI355X",
                                "factor_ms": m["factor_ms"], "solve_ms": m["solve_ms"],
                                "default_factor_ms": hist[0][1]["factor_ms"],
                                "default_solve_ms": hist[0][1]["solve_ms"],
                                "candidates": len(hist)})
            out[name] = {"key": key, "best": best, "measured": m, "default": hist[0][1]}
        tab.save()
        print(json.dumps({"autotune": out}), flush=True)
        return
    plan64 = {} if args.no_tuning else autotune.tuned_params(A.n, A.nnz, 1, T.TACHO_FP64)
    plan32 = {} if args.no_tuning else autotune.tuned_params(A.n, A.nnz, 1, T.TACHO_FP32)
    extra = {"graphs": 0} if args.eager else {}
    t0 = time.perf_counter()
    sym = T.tacho_analyze(A.n, A.rowptr, A.colind, T.tacho_default_options(**plan64, **extra))
    analyze_s = time.perf_counter() - t0
    sym32 = sym if plan32 == plan64 else T.tacho_analyze(
        A.n, A.rowptr, A.colind, T.tacho_default_options(**plan32, **extra))
    q = T.tacho_query_symbolic(sym)
    log(f"[bench] analyze {analyze_s:.2f}s nnz(L)={q['nnz_l']:.3e} flops={q['flops']:.3e} "
        f"supernodes={q['nsuper']} levels={q['nlevels']}")
    vals = torch.from_numpy(A.values).cuda()
    torch.cuda.synchronize()

    log(f"[bench] FP64: {args.warmup} warmup + {args.steps} timed steps")
    num64, r64 = run_fp64(T, torch, A, sym, vals, b1, b16, args.steps, args.warmup)
    s64 = summarize(r64, q["flops"], 1e-12)
    log(f"[bench] FP64 factor {s64['factor_ms_p50']:.2f} ms ({s64['factor_tflops']:.2f} TFLOP/s), "
        f"solve1 {s64['solve_nrhs1_ms_p50']:.2f} ms, solve16 {s64['solve_nrhs16_ms_p50']:.2f} ms, "
        f"rho {s64['rel_residual_nrhs1']:.1e}/{s64['rel_residual_nrhs16']:.1e}")
    mixed = None
    if not args.no_mixed:
        log("[bench] mixed FP32 factor + FP64 refinement")
        num32, r32 = run_mixed(T, torch, A, sym32, vals, b1, b16, max(3, args.steps // 2), 1)
        mixed = summarize(r32, q["flops"], 1e-10)
        log(f"[bench] mixed factor {mixed['factor_ms_p50']:.2f} ms, solve1 "
            f"{mixed['solve_nrhs1_ms_p50']:.2f} ms, rho {mixed['rel_residual_nrhs1']:.1e}")
        del num32
    prof = roof = None
    if not args.no_profile:
        log("[bench] kernel profile")
        prof = kernel_profile(T, torch, num64, vals, b1, b16)
        roof = roofline(prof)
        log(f"[bench] dominant {roof['kernel']}: {roof['achieved']:.2f} {roof['unit']} "
            f"({100 * roof['frac']:.1f}% of peak)")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle, bounded sample)")
        cpu = cpu_baseline()
        log(f"[bench] oracle {cpu['value'] * 1e3:.3f} GFLOP/s")

    ms_per_step = r64["wall_s"] * 1e3 / args.steps
    line = {
        "metric": METRIC,
        "value": s64["factor_tflops"] if s64["meets_tol"] else None,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D 7-point FV, lognormal(0,1) cells, {side}^3 grid, FP64 multifrontal "
                        f"Cholesky, 1 and 16 RHS",
            "n": A.n, "nnz_a": int(A.nnz), "nnz_l": q["nnz_l"], "flops": q["flops"],
            "supernodes": q["nsuper"], "levels": q["nlevels"], "max_front": q["max_front"],
            "ordering": "own nested dissection + etree postorder",
            "analyze_s_host": analyze_s,
            "plan_fp64": plan64 or "defaults", "plan_fp32": plan32 or "defaults",
        },
        "fp64": s64,
        "mixed": mixed,
        "roofline": roof,
        "kernels": prof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def line_for(args, metric_value, unit, dtype, config, extra):
    out = {"metric": METRIC, "value": metric_value, "unit": unit, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def other_workload(args, T, torch):
    """C1 (2d), C3 (landice), C4 (batch) and C5 (serve) measurements."""
    import numpy as np

    import gen
    if args.workload == "serve":
        from paper_2506_05793_amd.serve import Request, Server, summarize
        rate = args.rate if args.rate > 0 else 1e9
        specs = gen.serving_requests(args.requests, seed=5, rate=rate, n2d=(1000, 250000),
                                     n3d=(4000, 300000))
        reqs, mats = [], {}
        log(f"[bench] building {len(specs)} requests")
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
        free, _ = torch.cuda.mem_get_info()
        budget = int(args.budget_gb * 1e9) if args.budget_gb > 0 else int(0.8 * free)
        srv = Server(budget, slots=4, analysis_workers=args.workers)
        t0 = time.perf_counter()
        res = srv.run(reqs)
        wall = time.perf_counter() - t0
        srv.close()
        summ = summarize(res, wall)
        worst = 0.0
        for out in res[:: max(1, len(res) // 20)]:
            r = reqs[out.rid]
            A = r.matrix if r.kind == "factor" else mats[r.target]
            worst = max(worst, float(residual(A, out.x, r.rhs).max()))
        summ.update({"offered_rate_per_s": args.rate if args.rate > 0 else None,
                     "hbm_budget_bytes": budget, "analysis_workers": args.workers,
                     "served_requests_per_s": len(res) / wall,
                     "admitted_while_busy": srv.admitted_while_busy, "peak_bytes": srv.peak_used,
                     "sampled_max_rel_residual": worst})
        log(f"[bench] serve {summ}")
        line_for(args, summ["rhs_solves_per_s"], "RHS solves/s", "f64",
                 {"workload": f"Poisson request stream, {len(reqs)} requests, 2D n 1k-250k and "
                              f"3D n 4k-300k lognormal, 1-16 RHS, 30% repeat",
                  "offered_rate_per_s": args.rate if args.rate > 0 else "all at t=0"},
                 {"serve": summ})
        return
    plans = None
    if args.workload == "batch":
        mats = gen.batch_fv3d(256, seed=4)
        log(f"[bench] batch of {len(mats)} systems, n total {sum(m.n for m in mats)}")
        t0 = time.perf_counter()
        sym = T.tacho_analyze_batch([(m.n, m.rowptr, m.colind) for m in mats])
        analyze_s = time.perf_counter() - t0
        vals_np = np.concatenate([m.values for m in mats])
        n = sum(m.n for m in mats)
        b = np.asfortranarray(np.concatenate([gen.rhs(m.n, 1, seed=10 + k)
                                              for k, m in enumerate(mats)], axis=0))
        A = gen.csr_block_diag(mats)
        precisions = [("mixed", T.TACHO_FP32, 1e-10), ("fp64", T.TACHO_FP64, 1e-12)]
    elif args.workload == "2d":
        A = gen.laplace2d(32)
        t0 = time.perf_counter()
        sym = T.tacho_analyze(A.n, A.rowptr, A.colind)
        analyze_s = time.perf_counter() - t0
        vals_np = A.values
        n = A.n
        b = gen.rhs(n, 1, seed=0)
        precisions = [("fp64", T.TACHO_FP64, 1e-12), ("mixed", T.TACHO_FP32, 1e-10)]
    else:
        s = args.li_side
        log(f"[bench] building land-ice {s}x{s}x11x2")
        A = gen.landice(s, s, 11, seed=3)
        from paper_2506_05793_amd import autotune
        if args.autotune:
            # analysis takes seconds here: a reduced candidate set
            cands = {"asm_cols": (4, 8), "chain_min": (2, 3, 4), "solo_m": (-1, 128, 192),
                     "chain_inplace": (0, -1)}
            tab = autotune.TuningTable(autotune.DEFAULT_TABLE)
            out = {}
            for prec, name in ((T.TACHO_FP64, "fp64"), (T.TACHO_FP32, "fp32")):
                best, m, hist = autotune.tune(A.n, A.rowptr, A.colind, A.values, prec, reps=5,
                                              log=log, candidates=cands)
                key = autotune.workload_key(A.n, A.nnz, 1, prec)
                tab.put(key, best, {"workload": f"land-ice {s}x{s}x11 nodes x 2 DOF",
                                    "device": "MI355X", "factor_ms": m["factor_ms"],
                                    "solve_ms": m["solve_ms"],
                                    "default_factor_ms": hist[0][1]["factor_ms"],
                                    "default_solve_ms": hist[0][1]["solve_ms"],
                                    "candidates": len(hist)})
                out[name] = {"key": key, "best": best, "measured": m, "default": hist[0][1]}
            tab.save()
            print(json.dumps({"autotune": out}), flush=True)
            return
        plans = {p: ({} if args.no_tuning else autotune.tuned_params(A.n, A.nnz, 1, p))
                 for p in (T.TACHO_FP64, T.TACHO_FP32)}
        t0 = time.perf_counter()
        sym = T.tacho_analyze(A.n, A.rowptr, A.colind, T.tacho_default_options(**plans[T.TACHO_FP64]))
        analyze_s = time.perf_counter() - t0
        sym_by_prec = {T.TACHO_FP64: sym,
                       T.TACHO_FP32: sym if plans[T.TACHO_FP32] == plans[T.TACHO_FP64] else
                       T.tacho_analyze(A.n, A.rowptr, A.colind,
                                       T.tacho_default_options(**plans[T.TACHO_FP32]))}
        vals_np = A.values
        n = A.n
        b = gen.rhs(n, 1, seed=2)
        precisions = [("mixed", T.TACHO_FP32, 1e-10), ("fp64", T.TACHO_FP64, 1e-12)]
    q = T.tacho_query_symbolic(sym)
    log(f"[bench] analyze {analyze_s:.2f}s n={n} nnz(L)={q['nnz_l']:.3e} flops={q['flops']:.3e} "
        f"levels={q['nlevels']}")
    vals = torch.from_numpy(vals_np).cuda()
    B = dev_colmajor(torch, np.asarray(b).reshape(n, -1))
    X = torch.empty_like(B)
    results = {}
    for name, prec, tol in precisions:
        num = T.tacho_factorize(sym_by_prec.get(prec, sym) if args.workload == "landice" else sym,
                                vals, prec)
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
                           "landice": f"land-ice {args.li_side}x{args.li_side}x11 nodes x 2 DOF",
                           "batch": "256 3D lognormal subdomain systems, sides in [8,32]"}[args.workload],
              "n": n, "nnz_l": q["nnz_l"], "flops": q["flops"], "levels": q["nlevels"],
              "analyze_s_host": analyze_s,
              **({"plan_fp64": plans[T.TACHO_FP64] or "defaults",
                  "plan_fp32": plans[T.TACHO_FP32] or "defaults"} if plans else {})}, results)


if __name__ == "__main__":
    main()
