"""Thin ctypes binding of the HIP library ``lib/libftgemm.so`` (C ABI in
``include/ftgemm.h``).  Functions keep the C names and argument order; this
module only marshals arguments (device pointers, sizes, host arrays for the
report and the fault sites).  Every step of the computation runs in the HIP
kernels: if the library is missing this module raises, there is no fallback.

Device memory and streams come from PyTorch: pass ``tensor.data_ptr()`` for
matrices and ``torch.cuda.current_stream().cuda_stream`` for the stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# FTGEMM_LIB selects another build of the same sources (the sanitizer tests
# load one whose host API is built with ASan/UBSan)
LIB_PATH = os.environ.get("FTGEMM_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib",
                                                         "libftgemm.so")

F32, BF16, F8E4M3, F64, C64 = 0, 1, 2, 3, 4
FT_OFF, FT_DETECT, FT_CORRECT = 0, 1, 2
FT_RECOMPUTE = 0x10   # OR-ed into FT_DETECT or FT_CORRECT: recompute the tiles that end possibly wrong
OK, UNCORRECTABLE, NONFINITE_INPUT = 0, 1, 2
INVALID, UNSUPPORTED, HIP_ERROR, NO_MEMORY, LOG_OVERFLOW = -1, -2, -3, -4, -5
EV_CORRECTED, EV_CHECKSUM_ROW, EV_CHECKSUM_COL, EV_UNCORRECTABLE, EV_DETECTED, EV_NONFINITE = 1, 2, 3, 4, 5, 6
FAULT_ADD, FAULT_XOR = 0, 1

EVENT_DTYPE = np.dtype([("problem", "<i4"), ("tile_m", "<i4"), ("tile_n", "<i4"), ("kstep", "<i4"),
                        ("row", "<i4"), ("col", "<i4"), ("kind", "<i4"), ("n_rows", "<i4"),
                        ("n_cols", "<i4"), ("pad_", "<i4"), ("value_before", "<f4"),
                        ("value_after", "<f4"), ("r_row", "<f4"), ("r_col", "<f4"),
                        ("tau_row", "<f4"), ("tau_col", "<f4")])
FAULT_DTYPE = np.dtype([("tile_m", "<i4"), ("tile_n", "<i4"), ("kstep", "<i4"), ("row", "<i4"),
                        ("col", "<i4"), ("kind", "<i4"), ("payload", "<f4"), ("problem", "<i4")])
FAULT_LOG_DTYPE = np.dtype([("problem", "<i4"), ("tile_m", "<i4"), ("tile_n", "<i4"), ("kstep", "<i4"),
                            ("row", "<i4"), ("col", "<i4"), ("kind", "<i4"), ("check_step", "<i4"),
                            ("old_v", "<f4"), ("new_v", "<f4"), ("r_row", "<f4"), ("r_col", "<f4"),
                            ("tau_row", "<f4"), ("tau_col", "<f4"), ("delta", "<f8")])


class Config(ctypes.Structure):
    """(m_tile, n_tile, k_step, check_interval, check_m, check_n); a 4-tuple
    leaves the check shape 0, i.e. the compute tile."""
    _fields_ = [("m_tile", ctypes.c_int32), ("n_tile", ctypes.c_int32), ("k_step", ctypes.c_int32),
                ("check_interval", ctypes.c_int32), ("check_m", ctypes.c_int32), ("check_n", ctypes.c_int32)]

    def as_tuple(self):
        return (self.m_tile, self.n_tile, self.k_step, self.check_interval, self.check_m, self.check_n)

    def check_shape(self):
        return (self.check_m or self.m_tile, self.check_n or self.n_tile)


class Report(ctypes.Structure):
    _fields_ = [("checks", ctypes.c_uint64), ("detected", ctypes.c_uint64), ("corrected", ctypes.c_uint64),
                ("uncorrectable", ctypes.c_uint64), ("checksum_only", ctypes.c_uint64),
                ("nonfinite_input", ctypes.c_uint64), ("n_events", ctypes.c_uint32), ("cap_events", ctypes.c_uint32),
                ("events", ctypes.c_void_p), ("config", Config), ("bad_arg", ctypes.c_int32),
                ("tol_used", ctypes.c_float), ("bad_problem", ctypes.c_int32), ("recomputed", ctypes.c_uint32),
                ("recompute_failed", ctypes.c_uint32), ("pad_", ctypes.c_int32)]


class Tuned(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64), ("ft_level", ctypes.c_int64),
                ("config", Config)]


# ftgemm_problem_t: one problem of a batched call (96 bytes)
PROBLEM_DTYPE = np.dtype([("dtype", "<i4"), ("reserved_", "<i4"), ("m", "<i8"), ("n", "<i8"), ("k", "<i8"),
                          ("lda", "<i8"), ("ldb", "<i8"), ("ldc", "<i8"), ("alpha", "<f4"), ("beta", "<f4"),
                          ("scale_a", "<f4"), ("scale_b", "<f4"), ("A", "<u8"), ("B", "<u8"), ("C", "<u8")])


class ReportBuffer:
    """A Report plus the caller-owned host array its events are copied into."""

    def __init__(self, cap: int = 4096):
        self.events_buf = np.zeros(cap, dtype=EVENT_DTYPE)
        self.report = Report()
        self.report.cap_events = cap
        self.report.events = self.events_buf.ctypes.data

    @property
    def events(self) -> np.ndarray:
        return self.events_buf[: self.report.n_events].copy()

    def ptr(self):
        return ctypes.byref(self.report)


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_01024_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
        L.ftgemm_create.argtypes = [ctypes.POINTER(vp), i32, i32]
        L.ftgemm_destroy.argtypes = [vp]
        L.ftgemm_set_scales.argtypes = [vp, f32, f32]
        L.ftgemm_set_config.argtypes = [vp, ctypes.POINTER(Config)]
        L.ftgemm_select_config.argtypes = [i32, i64, i64, i64, i32, ctypes.POINTER(Config)]
        L.ftgemm_validate.argtypes = [i64, i64, i64, i64, i64, i64, i32, f32, ctypes.POINTER(ctypes.c_int32)]
        L.ftgemm_run.argtypes = [vp, i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, i32, f32, vp,
                                 ctypes.POINTER(Report)]
        L.ftgemm_run_nonfused.argtypes = [vp, i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, i32, f32, vp,
                                          ctypes.POINTER(Report)]
        L.ftgemm_run_noalloc.argtypes = [i32, i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, i32, f32, vp,
                                         ctypes.POINTER(Report)]
        f64 = ctypes.c_double
        L.ftgemm_run_f64.argtypes = [vp, i64, i64, i64, f64, vp, i64, vp, i64, f64, vp, i64, i32, f64, vp,
                                     ctypes.POINTER(Report)]
        dp2 = ctypes.POINTER(ctypes.c_double)
        L.ftgemm_run_z64.argtypes = [vp, i64, i64, i64, dp2, vp, i64, vp, i64, dp2, vp, i64, i32, f64, vp,
                                     ctypes.POINTER(Report)]
        L.ftgemm_set_injection.argtypes = [vp, vp, i32]
        L.ftgemm_get_injection_log.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_int)]
        L.ftgemm_batched.argtypes = [vp, i32, vp, i32, f32, vp, ctypes.POINTER(Report)]
        L.ftgemm_batched_config.argtypes = [vp, i32, ctypes.POINTER(Config)]
        L.ftgemm_tune.argtypes = [vp, i64, i64, i64, i32, i32, vp, ctypes.POINTER(Config)]
        L.ftgemm_get_tuned.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_int)]
        L.ftgemm_add_tuned.argtypes = [vp, ctypes.POINTER(Tuned)]
        L.ftgemm_tune_batched.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.ftgemm_status_string.argtypes = [i32]
        L.ftgemm_status_string.restype = ctypes.c_char_p
        for name in ("ftgemm_create", "ftgemm_destroy", "ftgemm_set_scales", "ftgemm_set_config",
                     "ftgemm_select_config", "ftgemm_validate", "ftgemm_run", "ftgemm_set_injection",
                     "ftgemm_get_injection_log", "ftgemm_batched", "ftgemm_batched_config", "ftgemm_tune", "ftgemm_get_tuned",
                     "ftgemm_add_tuned", "ftgemm_tune_batched", "ftgemm_run_nonfused", "ftgemm_run_f64",
                     "ftgemm_run_noalloc", "ftgemm_run_z64"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


class FtgemmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status} ({ftgemm_status_string(status)})")
        self.status = status


def _check(status: int, where: str) -> int:
    if status < 0:
        raise FtgemmError(status, where)
    return status


def ftgemm_status_string(status: int) -> str:
    return lib().ftgemm_status_string(status).decode()


_handle_dtype: dict = {}   # operand type of each live handle, for the tensor entry point


def ftgemm_create(dtype: int = F32, device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().ftgemm_create(ctypes.byref(h), dtype, device), "ftgemm_create")
    _handle_dtype[h.value] = (dtype, device)
    return h.value


def ftgemm_destroy(handle: int) -> None:
    _check(lib().ftgemm_destroy(handle), "ftgemm_destroy")
    _handle_dtype.pop(handle, None)


def ftgemm_set_scales(handle: int, scale_a: float, scale_b: float) -> None:
    _check(lib().ftgemm_set_scales(handle, scale_a, scale_b), "ftgemm_set_scales")


def ftgemm_set_config(handle: int, config: Config | tuple | None) -> None:
    if config is None:
        _check(lib().ftgemm_set_config(handle, None), "ftgemm_set_config")
        return
    if not isinstance(config, Config):
        config = Config(*config)
    _check(lib().ftgemm_set_config(handle, ctypes.byref(config)), "ftgemm_set_config")


def ftgemm_select_config(dtype: int, m: int, n: int, k: int, ft_level: int = FT_CORRECT) -> Config:
    c = Config()
    _check(lib().ftgemm_select_config(dtype, m, n, k, ft_level, ctypes.byref(c)), "ftgemm_select_config")
    return c


def ftgemm_validate(m, n, k, lda, ldb, ldc, ft_level=FT_CORRECT, tol=0.0):
    """Returns (status, bad_arg)."""
    bad = ctypes.c_int32(0)
    st = lib().ftgemm_validate(m, n, k, lda, ldb, ldc, ft_level, tol, ctypes.byref(bad))
    return st, bad.value


def ftgemm_run(handle: int, m: int, n: int, k: int, alpha: float, A: int, lda: int, B: int, ldb: int,
               beta: float, C: int, ldc: int, ft_level: int = FT_CORRECT, tol: float = 0.0,
               stream: int = 0, report: ReportBuffer | None = None) -> int:
    """C = alpha A B + beta C on device pointers (column-major).  Returns the
    status (0, 1 or 2); raises FtgemmError on negative statuses."""
    st = lib().ftgemm_run(handle, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ft_level, tol, stream,
                          report.ptr() if report is not None else None)
    return _check(st, "ftgemm_run")


def _swap_report(report: ReportBuffer) -> None:
    """Events and configuration of a run on the transposed problem C^T, in
    the coordinates of C: rows and columns (and everything attached to them)
    trade places."""
    ev = report.events_buf[: report.report.n_events]
    for a, b in (("tile_m", "tile_n"), ("row", "col"), ("n_rows", "n_cols"), ("r_row", "r_col"),
                 ("tau_row", "tau_col")):
        x = ev[a].copy()
        ev[a] = ev[b]
        ev[b] = x
    c = report.report.config
    c.m_tile, c.n_tile = c.n_tile, c.m_tile
    c.check_m, c.check_n = c.check_n, c.check_m


def ftgemm_matmul(handle: int, A, B, C=None, alpha: float = 1.0, beta: float = 0.0, ft_level: int = FT_CORRECT,
                  tol: float = 0.0, report: ReportBuffer | None = None):
    """Row-major entry for PyTorch tensors: C = alpha A B + beta C with A (m x k),
    B (k x n) and C (m x n, float32) on the handle's device, in PyTorch's
    row-major layout (unit column stride; the row stride is the leading
    dimension).  A and B are float32 for an F32 handle, bfloat16 for BF16 and
    float8_e4m3fn (or uint8 codes) for F8E4M3.  C = None allocates a zeroed C.

    A row-major m x n matrix is the column-major storage of its transpose, so
    this runs ftgemm_run on C^T = B^T A^T: the operands trade places, so do m
    and n, and the leading dimensions are the row strides.  The checks are
    symmetric in rows and columns (the row check of C^T is the column check of
    C), and the report's events and configuration are swapped back to C's
    coordinates.  Fault sites set with ftgemm_set_injection address the
    problem the library sees, C^T (tile_m/tile_n and row/col swapped).
    Runs on torch's current stream.  Returns (C, status)."""
    import torch

    if handle not in _handle_dtype:
        raise ValueError("unknown handle (create it with ftgemm_create)")
    dtype, device = _handle_dtype[handle]
    want = {F32: (torch.float32,), BF16: (torch.bfloat16,),
            F8E4M3: tuple(t for t in (getattr(torch, "float8_e4m3fn", None), torch.uint8) if t is not None)}
    if dtype not in want:
        raise ValueError("ftgemm_matmul takes F32, BF16 and F8E4M3 handles")
    for name, t in (("A", A), ("B", B)):
        if t.dim() != 2 or t.dtype not in want[dtype] or not t.is_cuda or t.device.index != device:
            raise ValueError(f"{name}: a 2-D {want[dtype][0]} tensor on cuda:{device} is required")
        if t.stride(1) != 1 or t.stride(0) < max(1, t.shape[1]):
            raise ValueError(f"{name}: rows must be contiguous (column stride 1, row stride >= columns)")
    m, k = A.shape
    if B.shape[0] != k:
        raise ValueError(f"inner dimensions differ: A is {tuple(A.shape)}, B is {tuple(B.shape)}")
    n = B.shape[1]
    if C is None:
        C = torch.zeros((m, n), dtype=torch.float32, device=A.device)
    if (C.dim() != 2 or tuple(C.shape) != (m, n) or C.dtype != torch.float32 or C.device != A.device
            or C.stride(1) != 1 or C.stride(0) < max(1, n)):
        raise ValueError(f"C: a row-major ({m}, {n}) float32 tensor on A's device is required")
    stream = torch.cuda.current_stream(A.device).cuda_stream
    st = ftgemm_run(handle, n, m, k, alpha, B.data_ptr(), max(1, B.stride(0)), A.data_ptr(),
                    max(1, A.stride(0)), beta, C.data_ptr(), max(1, C.stride(0)), ft_level, tol, stream, report)
    if report is not None:
        _swap_report(report)
    return C, st


def ftgemm_run_noalloc(dtype: int, m: int, n: int, k: int, alpha: float, A: int, lda: int, B: int, ldb: int,
                       beta: float, C: int, ldc: int, ft_level: int = FT_CORRECT, tol: float = 0.0,
                       stream: int = 0, report: ReportBuffer | None = None) -> int:
    """ftgemm_run without a handle and without allocating (static device
    workspace; the current device; calls on one device must not overlap).
    Returns the status (0, 1 or 2); raises FtgemmError on negative statuses."""
    st = lib().ftgemm_run_noalloc(dtype, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ft_level, tol, stream,
                                  report.ptr() if report is not None else None)
    return _check(st, "ftgemm_run_noalloc")


def ftgemm_run_f64(handle: int, m: int, n: int, k: int, alpha: float, A: int, lda: int, B: int, ldb: int,
                   beta: float, C: int, ldc: int, ft_level: int = FT_CORRECT, tol: float = 0.0,
                   stream: int = 0, report: ReportBuffer | None = None) -> int:
    """FP64 C = alpha A B + beta C on device pointers to double (column-major),
    for a handle created with F64.  Returns the status (0, 1 or 2); raises
    FtgemmError on negative statuses."""
    st = lib().ftgemm_run_f64(handle, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ft_level, tol, stream,
                              report.ptr() if report is not None else None)
    return _check(st, "ftgemm_run_f64")


def ftgemm_run_z64(handle: int, m: int, n: int, k: int, alpha: complex, A: int, lda: int, B: int, ldb: int,
                   beta: complex, C: int, ldc: int, ft_level: int = FT_CORRECT, tol: float = 0.0,
                   stream: int = 0, report: ReportBuffer | None = None) -> int:
    """Double-complex C = alpha A B + beta C on device pointers to (re, im)
    binary64 pairs (column-major, leading dimensions in complex elements), for
    a handle created with C64.  Events carry the component in `problem` (0
    real, 1 imaginary).  Returns the status (0, 1 or 2); raises FtgemmError
    on negative statuses."""
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    st = lib().ftgemm_run_z64(handle, m, n, k, al, A, lda, B, ldb, be, C, ldc, ft_level, tol, stream,
                              report.ptr() if report is not None else None)
    return _check(st, "ftgemm_run_z64")


def ftgemm_run_nonfused(handle: int, m: int, n: int, k: int, A: int, lda: int, B: int, ldb: int, C: int,
                        ldc: int, check_k: int = 0, tol: float = 0.0, stream: int = 0,
                        report: ReportBuffer | None = None, alpha: float = 1.0, beta: float = 0.0) -> int:
    """The same ABFT as ftgemm_run, not fused (separate launches around the
    plain FP32 kernel on k-chunks of check_k).  Returns the status (0, 1 or 2);
    raises FtgemmError on negative statuses."""
    st = lib().ftgemm_run_nonfused(handle, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, check_k, tol, stream,
                                   report.ptr() if report is not None else None)
    return _check(st, "ftgemm_run_nonfused")


def ftgemm_set_injection(handle: int, faults: np.ndarray | None) -> None:
    if faults is None or len(faults) == 0:
        _check(lib().ftgemm_set_injection(handle, None, 0), "ftgemm_set_injection")
        return
    arr = np.ascontiguousarray(faults, dtype=FAULT_DTYPE)
    _check(lib().ftgemm_set_injection(handle, arr.ctypes.data, len(arr)), "ftgemm_set_injection")


def ftgemm_get_injection_log(handle: int, cap: int = 16384) -> np.ndarray:
    out = np.zeros(cap, dtype=FAULT_LOG_DTYPE)
    n = ctypes.c_int(0)
    _check(lib().ftgemm_get_injection_log(handle, out.ctypes.data, cap, ctypes.byref(n)),
           "ftgemm_get_injection_log")
    return out[: n.value].copy()


def make_problems(count: int) -> np.ndarray:
    """A zeroed array of `count` batched problem descriptors."""
    return np.zeros(count, dtype=PROBLEM_DTYPE)


def ftgemm_batched(handle: int, problems: np.ndarray, ft_level: int = FT_CORRECT, tol: float = 0.0,
                   stream: int = 0, report: ReportBuffer | None = None) -> int:
    """All problems of a PROBLEM_DTYPE array in one persistent launch.  Keep
    `problems` unchanged between calls to reuse the handle's plan (required
    under stream capture).  Returns the status (0, 1 or 2); raises on errors."""
    arr = np.ascontiguousarray(problems, dtype=PROBLEM_DTYPE)
    st = lib().ftgemm_batched(handle, len(arr), arr.ctypes.data if len(arr) else None, ft_level, tol, stream,
                              report.ptr() if report is not None else None)
    return _check(st, "ftgemm_batched")


def ftgemm_batched_config(handle: int, p: int) -> Config:
    """Configuration of problem p in the handle's current batched plan."""
    c = Config()
    _check(lib().ftgemm_batched_config(handle, p, ctypes.byref(c)), "ftgemm_batched_config")
    return c


def ftgemm_tune(handle: int, m: int, n: int, k: int, ft_level: int = FT_CORRECT, max_k_between_checks: int = 0,
                stream: int = 0) -> Config:
    """Time every tile variant and check interval on this shape; the fastest
    is kept in the handle for later ftgemm_run calls and returned."""
    c = Config()
    _check(lib().ftgemm_tune(handle, m, n, k, ft_level, max_k_between_checks, stream, ctypes.byref(c)),
           "ftgemm_tune")
    return c


def ftgemm_get_tuned(handle: int) -> list:
    """The handle's tuned configurations as [(m, n, k, ft_level, Config.as_tuple())]."""
    n = ctypes.c_int(0)
    _check(lib().ftgemm_get_tuned(handle, None, 0, ctypes.byref(n)), "ftgemm_get_tuned")
    buf = (Tuned * max(1, n.value))()
    _check(lib().ftgemm_get_tuned(handle, buf, n.value, ctypes.byref(n)), "ftgemm_get_tuned")
    return [(t.m, t.n, t.k, t.ft_level, t.config.as_tuple()) for t in buf[: n.value]]


def ftgemm_add_tuned(handle: int, m: int, n: int, k: int, ft_level: int, config) -> None:
    cfg = config if isinstance(config, Config) else Config(*config)
    t = Tuned(m, n, k, ft_level, cfg)
    _check(lib().ftgemm_add_tuned(handle, ctypes.byref(t)), "ftgemm_add_tuned")


def save_tuned(handle: int, path: str) -> None:
    """Persist the handle's tuned configurations as JSON."""
    import json
    with open(path, "w") as f:
        json.dump([{"m": m, "n": n, "k": k, "ft_level": lv, "config": list(c)}
                   for (m, n, k, lv, c) in ftgemm_get_tuned(handle)], f, indent=1)


def load_tuned(handle: int, path: str) -> int:
    """Load tuned configurations written by save_tuned; returns how many."""
    import json
    with open(path) as f:
        rows = json.load(f)
    for r in rows:
        ftgemm_add_tuned(handle, int(r["m"]), int(r["n"]), int(r["k"]), int(r["ft_level"]), tuple(r["config"]))
    return len(rows)


def ftgemm_tune_batched(handle: int, stream: int = 0) -> np.ndarray:
    """Measure the batched tile variants' rates (multiply-adds per second)."""
    rates = (ctypes.c_double * 4)()
    _check(lib().ftgemm_tune_batched(handle, stream, rates), "ftgemm_tune_batched")
    return np.array(list(rates))
