"""Python binding of the MI355X supernodal multifrontal Cholesky library.

Argument marshalling only: every step of the factorization and the solves
runs in the HIP library ``libtacho_mi355x.so`` (built by ``build.py``).  The
functions carry the names of the C ABI in ``include/tacho.h``.  Host arrays
are numpy arrays; device arrays are torch tensors on the current ROCm device,
used on torch's current stream.  There is no CPU fallback: if the library is
missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtacho_mi355x.so")

TACHO_OK = 0
TACHO_ERR_INVALID = -1
TACHO_ERR_PATTERN = -2
TACHO_ERR_NOT_SPD = -3
TACHO_ERR_NOMEM = -4
TACHO_ERR_HIP = -5
TACHO_ERR_SINGULAR = -6
TACHO_FP64 = 0
TACHO_FP32_IR = 1
TACHO_FP32 = TACHO_FP32_IR
TACHO_LDLT = 2
TACHO_LU = 3
TACHO_DEBUG_SOLVE_GIVE_UP = 1
TACHO_PROFILE_KINDS = 12
TACHO_SOLVE_BLOCK_INVERSE = 2
TACHO_SOLVE_PARTITIONED_INVERSE = 3
TACHO_SOLVE_LEVEL_CSR = 4

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class tacho_options(ctypes.Structure):
    _fields_ = [
        ("nd_leaf_size", ctypes.c_int32),
        ("small_front", ctypes.c_int32),
        ("scale_fp32", ctypes.c_int32),
        ("refine_max", ctypes.c_int32),
        ("refine_tol", ctypes.c_double),
        ("stall_ratio", ctypes.c_double),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("block_size", ctypes.c_int32),
        ("ordering", ctypes.c_int32),
        ("graphs", ctypes.c_int32),
        ("front_kernel", ctypes.c_int32),
        ("u_range", ctypes.c_int32),
        ("chain_min", ctypes.c_int32),
        ("solve_level_fronts", ctypes.c_int32),
        ("asm_cols", ctypes.c_int32),
        ("solo_m", ctypes.c_int32),
        ("chain_inplace", ctypes.c_int32),
        ("debug_flags", ctypes.c_int32),
        ("autotune_path", ctypes.c_char_p),
        ("autotune_precision", ctypes.c_int32),
        ("dof_block", ctypes.c_int32),
        ("dof_map", _i32p),
    ]


class tacho_sym_info(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "nnz_a", "nnz_l", "flops", "nsuper", "nlevels", "max_front", "max_width",
        "factor_bytes_fp64", "work_bytes_fp64", "device_bytes_fp64", "nsystems", "nnz_factor",
        "ordering", "t_order_us", "t_structure_us", "t_plan_us", "plan_u_range",
        "plan_chain_min", "plan_solve_level_fronts", "plan_asm_cols", "plan_solo_m",
        "plan_chain_inplace")]


class tacho_solve_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("fell_back", ctypes.c_int32),
        ("relres_max", ctypes.c_double),
        ("relres", _f64p),
        ("fell_back_units", _i32p),
    ]


class TachoError(RuntimeError):
    def __init__(self, code: int, message: str, fail_index: int = -1):
        super().__init__(f"{message} (code {code})")
        self.code = code
        self.fail_index = fail_index


_lib = None


def library_path() -> str:
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2506_05793_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "tacho_default_options": (None, [ctypes.POINTER(tacho_options)]),
        "tacho_analyze": (ctypes.c_int, [ctypes.c_int64, _i64p, _i32p,
                                         ctypes.POINTER(tacho_options), ctypes.POINTER(_vp)]),
        "tacho_analyze_batch": (ctypes.c_int, [ctypes.c_int64, _i64p, ctypes.POINTER(_i64p),
                                               ctypes.POINTER(_i32p),
                                               ctypes.POINTER(tacho_options),
                                               ctypes.POINTER(_vp)]),
        "tacho_query_symbolic": (ctypes.c_int, [_vp, ctypes.POINTER(tacho_sym_info)]),
        "tacho_get_symbolic": (ctypes.c_int, [_vp, _i32p, _i32p, _i64p, _i32p, _i32p, _i32p]),
        "tacho_factorize": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp,
                                           ctypes.POINTER(_vp), _i64p]),
        "tacho_refactorize": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, _i64p]),
        "tacho_numeric_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp)]),
        "tacho_numeric_bytes": (ctypes.c_int, [_vp, ctypes.c_int, _i64p]),
        "tacho_check_factor": (ctypes.c_int, [_vp, _i64p]),
        "tacho_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                       _vp, ctypes.POINTER(tacho_solve_info)]),
        "tacho_solve_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int64,
                                               _vp, ctypes.POINTER(tacho_solve_info)]),
        "tacho_set_solve_variant": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
        "tacho_get_factor": (ctypes.c_int, [_vp, _i64p, _i32p, _f64p]),
        "tacho_get_ldlt": (ctypes.c_int, [_vp, _f64p, _f64p, _i32p]),
        "tacho_get_lu": (ctypes.c_int, [_vp, _i64p, _i32p, _f64p, _i32p]),
        "tacho_last_times": (ctypes.c_int, [_vp, _f64p, _f64p]),
        "tacho_profile": (ctypes.c_int, [_vp, ctypes.c_int]),
        "tacho_profile_read": (ctypes.c_int, [_vp, ctypes.c_int, _i64p, _f64p, _f64p, _f64p]),
        "tacho_kernel_name": (ctypes.c_char_p, [ctypes.c_int]),
        "tacho_free_symbolic": (ctypes.c_int, [_vp]),
        "tacho_free_numeric": (ctypes.c_int, [_vp]),
        "tacho_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "tacho_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    """Names of the C ABI entry points this binding resolves."""
    _load()
    return [n for n in dir(_lib) if n.startswith("tacho_")]


def _check(rc: int, fail_index: int = -1):
    if rc != TACHO_OK:
        lib = _load()
        msg = lib.tacho_last_error().decode() or lib.tacho_strerror(rc).decode()
        raise TachoError(rc, msg, fail_index)


def tacho_default_options(**overrides) -> tacho_options:
    opt = tacho_options()
    _load().tacho_default_options(ctypes.byref(opt))
    for k, v in overrides.items():
        if k == "autotune_path" and isinstance(v, str):
            v = v.encode()
        if k == "dof_map" and v is not None:
            arr = np.ascontiguousarray(v, dtype=np.int32)
            opt._dof_map = arr  # kept alive with the options
            v = arr.ctypes.data_as(_i32p)
        setattr(opt, k, v)
    return opt


class SymbolicHandle:
    """Owner of a ``tacho_sym_t``; remembers the order and the number of
    values the caller's CSR holds (what factorizations and solves expect)."""

    def __init__(self, ptr: int, n: int = -1, nnz: int = -1, nsys: int = 1):
        self.ptr = ptr
        self.n = n
        self.nnz = nnz
        self.nsys = nsys
        self._lib = _load()

    def __del__(self):
        if getattr(self, "ptr", None):
            self._lib.tacho_free_symbolic(self.ptr)
            self.ptr = None


class NumericHandle:
    """Owner of a ``tacho_num_t``; keeps its symbolic handle alive."""

    def __init__(self, ptr: int, sym: SymbolicHandle, precision: int):
        self.ptr = ptr
        self.sym = sym
        self.precision = precision
        self._lib = _load()

    def __del__(self):
        if getattr(self, "ptr", None):
            self._lib.tacho_free_numeric(self.ptr)
            self.ptr = None


def tacho_analyze(n, rowptr, colind, options: tacho_options | None = None) -> SymbolicHandle:
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    dmap = getattr(options, "_dof_map", None)
    if options is not None and options.dof_map and (dmap is None or dmap.size != int(n)):
        raise ValueError(f"dof_map: expected {int(n)} entries")
    out = _vp()
    rc = lib.tacho_analyze(int(n), rowptr.ctypes.data_as(_i64p), colind.ctypes.data_as(_i32p),
                           ctypes.byref(options) if options is not None else None,
                           ctypes.byref(out))
    _check(rc)
    return SymbolicHandle(out.value, int(n), int(rowptr[-1]) if len(rowptr) else 0)


def tacho_analyze_batch(systems, options: tacho_options | None = None) -> SymbolicHandle:
    """``systems``: sequence of (n, rowptr, colind)."""
    lib = _load()
    k = len(systems)
    ns = np.array([int(s[0]) for s in systems], dtype=np.int64)
    rps = [np.ascontiguousarray(s[1], dtype=np.int64) for s in systems]
    cis = [np.ascontiguousarray(s[2], dtype=np.int32) for s in systems]
    rp_arr = (_i64p * k)(*[r.ctypes.data_as(_i64p) for r in rps])
    ci_arr = (_i32p * k)(*[c.ctypes.data_as(_i32p) for c in cis])
    out = _vp()
    rc = lib.tacho_analyze_batch(k, ns.ctypes.data_as(_i64p), rp_arr, ci_arr,
                                 ctypes.byref(options) if options is not None else None,
                                 ctypes.byref(out))
    _check(rc)
    return SymbolicHandle(out.value, int(ns.sum()), int(sum(int(r[-1]) for r in rps if len(r))), k)


def tacho_query_symbolic(sym: SymbolicHandle) -> dict:
    info = tacho_sym_info()
    _check(_load().tacho_query_symbolic(sym.ptr, ctypes.byref(info)))
    return {name: int(getattr(info, name)) for name, _ in tacho_sym_info._fields_}


@dataclass
class SymbolicArrays:
    perm: np.ndarray
    parent: np.ndarray
    colcount: np.ndarray
    super_ptr: np.ndarray
    super_parent: np.ndarray
    level: np.ndarray


def tacho_get_symbolic(sym: SymbolicHandle) -> SymbolicArrays:
    q = tacho_query_symbolic(sym)
    n, ns = q["n"], q["nsuper"]
    perm = np.empty(n, np.int32)
    parent = np.empty(n, np.int32)
    cc = np.empty(n, np.int64)
    sp = np.empty(ns + 1, np.int32)
    spar = np.empty(ns, np.int32)
    lev = np.empty(ns, np.int32)
    _check(_load().tacho_get_symbolic(sym.ptr, perm.ctypes.data_as(_i32p),
                                      parent.ctypes.data_as(_i32p), cc.ctypes.data_as(_i64p),
                                      sp.ctypes.data_as(_i32p), spar.ctypes.data_as(_i32p),
                                      lev.ctypes.data_as(_i32p)))
    return SymbolicArrays(perm, parent, cc, sp, spar, lev)


def _stream_ptr(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _is_torch(arr) -> bool:
    mod = type(arr).__module__
    return mod.startswith("torch")


def _check_device(t):
    """A device tensor must live on the current device (the library's stream)."""
    import torch
    if t.device.type != "cuda":
        raise TypeError("expected a numpy array or a device (ROCm) tensor")
    if t.device.index is not None and t.device.index != torch.cuda.current_device():
        raise ValueError(f"tensor on device {t.device.index}, current device is "
                         f"{torch.cuda.current_device()}")


def _values_arg(sym: SymbolicHandle, values):
    """(address, on_device, keep-alive) of the caller's values: float64, one per
    stored CSR entry, contiguous."""
    if isinstance(values, np.ndarray):
        v = np.ascontiguousarray(values, dtype=np.float64)
        if v.ndim != 1 or (sym.nnz >= 0 and v.size != sym.nnz):
            raise ValueError(f"values: expected {sym.nnz} entries, got shape {values.shape}")
        return v.ctypes.data, 0, v
    if _is_torch(values):
        import torch
        if values.dtype != torch.float64:
            raise TypeError(f"values: expected float64, got {values.dtype}")
        if values.dim() != 1 or not values.is_contiguous() or (
                sym.nnz >= 0 and values.numel() != sym.nnz):
            raise ValueError(f"values: expected a contiguous vector of {sym.nnz} entries")
        if values.device.type == "cpu":
            return values.data_ptr(), 0, values
        _check_device(values)
        return values.data_ptr(), 1, values
    raise TypeError("values: expected a numpy array or a torch tensor")


def tacho_factorize(sym: SymbolicHandle, values, precision: int = TACHO_FP64,
                    stream=None) -> NumericHandle:
    lib = _load()
    addr, on_dev, values = _values_arg(sym, values)
    out = _vp()
    fi = ctypes.c_int64(-1)
    rc = lib.tacho_factorize(sym.ptr, addr, on_dev, int(precision), _stream_ptr(stream),
                             ctypes.byref(out), ctypes.byref(fi))
    _check(rc, fi.value)
    return NumericHandle(out.value, sym, precision)


def tacho_numeric_create(sym: SymbolicHandle, precision: int = TACHO_FP64) -> NumericHandle:
    out = _vp()
    _check(_load().tacho_numeric_create(sym.ptr, int(precision), ctypes.byref(out)))
    return NumericHandle(out.value, sym, precision)


def tacho_numeric_bytes(sym: SymbolicHandle, precision: int = TACHO_FP64) -> int:
    b = ctypes.c_int64(0)
    _check(_load().tacho_numeric_bytes(sym.ptr, int(precision), ctypes.byref(b)))
    return b.value


def tacho_refactorize(num: NumericHandle, values, stream=None, sync: bool = True) -> None:
    lib = _load()
    addr, on_dev, values = _values_arg(num.sym, values)
    fi = ctypes.c_int64(-1)
    rc = lib.tacho_refactorize(num.ptr, addr, on_dev, _stream_ptr(stream), int(bool(sync)),
                               ctypes.byref(fi))
    _check(rc, fi.value)


def tacho_check_factor(num: NumericHandle) -> None:
    fi = ctypes.c_int64(-1)
    rc = _load().tacho_check_factor(num.ptr, ctypes.byref(fi))
    _check(rc, fi.value)


def _solve_args(num: NumericHandle, b, x):
    """Checked (b, x, nrhs, ld, on_device) of a solve: float64 column-major
    blocks of n rows, x of the same kind and layout as b (same leading
    dimension), device tensors on the current device."""
    n = num.sym.n
    if isinstance(b, np.ndarray):
        if b.ndim not in (1, 2) or (n >= 0 and b.shape[0] != n):
            raise ValueError(f"b: expected {n} rows, got shape {b.shape}")
        b = np.asfortranarray(b, dtype=np.float64)
        if x is None:
            x = np.empty_like(b, order="F")
        elif not isinstance(x, np.ndarray):
            raise TypeError("x: expected a numpy array like b")
        elif x.dtype != np.float64 or x.shape != b.shape or not x.flags.f_contiguous:
            raise ValueError("x: expected a column-major float64 array of b's shape")
        nrhs = 1 if b.ndim == 1 else b.shape[1]
        return b, x, nrhs, max(n, 1), 0
    if not _is_torch(b):
        raise TypeError("b: expected a numpy array or a device tensor")
    import torch
    if b.dtype != torch.float64:
        raise TypeError(f"b: expected float64, got {b.dtype}")
    _check_device(b)
    if b.dim() not in (1, 2) or (n >= 0 and b.shape[0] != n):
        raise ValueError(f"b: expected {n} rows, got shape {tuple(b.shape)}")
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    if b.dim() == 1:
        if b.stride(0) != 1:
            b = b.contiguous()
        ld = max(n, 1)
    else:
        if b.stride(0) != 1 or (nrhs > 1 and b.stride(1) < n):
            b = b.t().contiguous().t()
        ld = b.stride(1) if nrhs > 1 else max(n, 1)
    if x is None:
        x = torch.empty_strided(b.shape, b.stride(), dtype=torch.float64, device=b.device)
    else:
        if not _is_torch(x) or x.dtype != torch.float64:
            raise TypeError("x: expected a float64 device tensor like b")
        _check_device(x)
        if tuple(x.shape) != tuple(b.shape) or x.stride(0) != 1 or (
                nrhs > 1 and x.stride(1) != ld):
            raise ValueError("x: expected b's shape and column-major layout with b's leading "
                             f"dimension {ld}")
    return b, x, nrhs, ld, 1


def _solve_info(num: NumericHandle, nrhs: int):
    info = tacho_solve_info()
    rr = np.zeros(max(nrhs, 1), np.float64)
    fb = np.zeros(max(nrhs * max(num.sym.nsys, 1), 1), np.int32)
    info.relres = rr.ctypes.data_as(_f64p)
    info.fell_back_units = fb.ctypes.data_as(_i32p)
    return info, rr, fb


def _info_dict(num, info, rr, fb, nrhs):
    return {"iters": info.iters, "fell_back": info.fell_back, "relres_max": info.relres_max,
            "relres": rr[:nrhs].copy(),
            "fell_back_units": fb[:nrhs * max(num.sym.nsys, 1)].reshape(nrhs, -1).T.copy()}


def tacho_solve(num: NumericHandle, b, x=None, stream=None, with_info: bool = False):
    """Solve A X = B.  ``b`` (n or n x nrhs, column-major) is a numpy array or a
    device tensor; ``x`` defaults to a new array of the same kind."""
    lib = _load()
    b, x, nrhs, ld, on_dev = _solve_args(num, b, x)
    info, rr, fb = _solve_info(num, nrhs)
    addr = (lambda a: a.ctypes.data) if on_dev == 0 else (lambda a: a.data_ptr())
    rc = lib.tacho_solve(num.ptr, addr(b), addr(x), int(nrhs), int(ld), on_dev,
                         _stream_ptr(stream), ctypes.byref(info))
    _check(rc)
    if with_info:
        return x, _info_dict(num, info, rr, fb, nrhs)
    return x


def tacho_solve_noalloc(num: NumericHandle, b, x, stream=None, with_info: bool = False):
    """tacho_solve without device allocation: ``b`` and ``x`` are device tensors
    (column-major n x nrhs, float64) that the caller owns."""
    lib = _load()
    if not (_is_torch(b) and _is_torch(x)):
        raise TypeError("tacho_solve_noalloc takes device tensors b and x")
    n = num.sym.n
    if b.stride(0) != 1 or (b.dim() == 2 and b.shape[1] > 1 and b.stride(1) < n):
        raise ValueError("b: expected a column-major block (no copy is made)")
    b, x, nrhs, ld, on_dev = _solve_args(num, b, x)
    info, rr, fb = _solve_info(num, nrhs)
    rc = lib.tacho_solve_noalloc(num.ptr, b.data_ptr(), x.data_ptr(), int(nrhs), int(ld),
                                 _stream_ptr(stream), ctypes.byref(info))
    _check(rc)
    if with_info:
        return x, _info_dict(num, info, rr, fb, nrhs)
    return x


def tacho_set_solve_variant(num: NumericHandle, variant: int, stream=None) -> None:
    """Select the solve variant of later solves on ``num``
    (TACHO_SOLVE_BLOCK_INVERSE, TACHO_SOLVE_PARTITIONED_INVERSE or
    TACHO_SOLVE_LEVEL_CSR)."""
    _check(_load().tacho_set_solve_variant(num.ptr, int(variant), _stream_ptr(stream)))


def tacho_get_factor(num: NumericHandle):
    """Factor L of P A P^T as CSC arrays (Lp, Li, Lx) on the host."""
    q = tacho_query_symbolic(num.sym)
    n, nnz = q["n"], q["nnz_factor"]
    Lp = np.empty(n + 1, np.int64)
    Li = np.empty(max(nnz, 1), np.int32)
    Lx = np.empty(max(nnz, 1), np.float64)
    _check(_load().tacho_get_factor(num.ptr, Lp.ctypes.data_as(_i64p), Li.ctypes.data_as(_i32p),
                                    Lx.ctypes.data_as(_f64p)))
    return Lp, Li[:nnz], Lx[:nnz]


def tacho_get_ldlt(num: NumericHandle):
    """(d, e, q) of a TACHO_LDLT factorization: diagonal and subdiagonal of D
    (e nonzero at the first column of each 2x2 pivot) and the pivot order
    (row i of L is row q[i] of P A P^T)."""
    n = max(num.sym.n, 0)
    d = np.empty(max(n, 1), np.float64)
    e = np.empty(max(n, 1), np.float64)
    q = np.empty(max(n, 1), np.int32)
    _check(_load().tacho_get_ldlt(num.ptr, d.ctypes.data_as(_f64p), e.ctypes.data_as(_f64p),
                                  q.ctypes.data_as(_i32p)))
    return d[:n], e[:n], q[:n]


def tacho_get_lu(num: NumericHandle):
    """(Up, Ui, Ux, q) of a TACHO_LU factorization: U^T as CSC arrays (column c
    holds U's row c) and the row order (row i of L U is row q[i] of P A P^T)."""
    info = tacho_query_symbolic(num.sym)
    n, nnz = info["n"], info["nnz_factor"]
    Up = np.empty(n + 1, np.int64)
    Ui = np.empty(max(nnz, 1), np.int32)
    Ux = np.empty(max(nnz, 1), np.float64)
    q = np.empty(max(n, 1), np.int32)
    _check(_load().tacho_get_lu(num.ptr, Up.ctypes.data_as(_i64p), Ui.ctypes.data_as(_i32p),
                                Ux.ctypes.data_as(_f64p), q.ctypes.data_as(_i32p)))
    return Up, Ui[:nnz], Ux[:nnz], q[:n]


def tacho_last_times(num: NumericHandle):
    """(factor_ms, solve_ms) of the last factorization and solve, hipEvent timed."""
    a = ctypes.c_double(0)
    b = ctypes.c_double(0)
    _check(_load().tacho_last_times(num.ptr, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def tacho_factor_ms(num: NumericHandle) -> float:
    a = ctypes.c_double(0)
    _check(_load().tacho_last_times(num.ptr, ctypes.byref(a), None))
    return a.value


def tacho_profile(num: NumericHandle, enable: bool = True) -> None:
    _check(_load().tacho_profile(num.ptr, int(bool(enable))))


def tacho_profile_read(num: NumericHandle) -> dict:
    """Per kernel: launches, total ms, algorithmic flops and bytes since enabling."""
    lib = _load()
    out = {}
    for k in range(TACHO_PROFILE_KINDS):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0)
        fl = ctypes.c_double(0)
        by = ctypes.c_double(0)
        _check(lib.tacho_profile_read(num.ptr, k, ctypes.byref(n), ctypes.byref(ms),
                                      ctypes.byref(fl), ctypes.byref(by)))
        out[lib.tacho_kernel_name(k).decode()] = {
            "launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}
    return out
