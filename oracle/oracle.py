"""Python access to the FP64 CPU oracle (``ftgemm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.  It
shares no code with the HIP library or its binding.

Matrices are numpy arrays in the BLAS column-major convention: ``A`` is a
(lda, k) Fortran-ordered view holding the m x k operand, and so on.  Values are
converted to float64 exactly (every FP32, BF16 and FP8 value is representable).
Low-precision operands arrive as raw codes plus a power-of-two per-tensor scale
and are decoded here by :func:`decode_bf16` / :func:`decode_e4m3`, written from
the formats' definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ftgemm_oracle.c")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libftgemm_oracle.so")

EV_CORRECTED, EV_CHECKSUM_ROW, EV_CHECKSUM_COL, EV_UNCORRECTABLE, EV_DETECTED = 1, 2, 3, 4, 5
EV_NONFINITE = 6      # operands of the tile hold Inf/NaN: reported once, no decision
CLS_BENIGN, CLS_GREY, CLS_MUST = 0, 1, 2

U_FP32 = 2.0 ** -24   # unit roundoff of IEEE binary32 (round to nearest)
U_FP64 = 2.0 ** -53   # unit roundoff of IEEE binary64 (round to nearest)


def build(extra_flags=(), out=None) -> str:
    """Compile the oracle with gcc + OpenMP.  ``extra_flags`` lets the tests
    build planted-mistake variants of it (``-DORACLE_MUTANT=n``)."""
    out = out or LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           *extra_flags, SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class _Cfg(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("mc", ctypes.c_int64), ("nc", ctypes.c_int64), ("ku", ctypes.c_int64),
                ("g", ctypes.c_int64), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("u", ctypes.c_double), ("c", ctypes.c_double), ("ft_level", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


# comp: complex replay only, the component (0 real, 1 imaginary) of a fault or decision
INJ_DTYPE = np.dtype([("tile_m", "<i8"), ("tile_n", "<i8"), ("kstep", "<i8"), ("row", "<i8"),
                      ("col", "<i8"), ("old_v", "<f8"), ("new_v", "<f8"), ("force", "<i4"),
                      ("comp", "<i4")])
EV_DTYPE = np.dtype([("tile_m", "<i8"), ("tile_n", "<i8"), ("kstep", "<i8"), ("row", "<i8"),
                     ("col", "<i8"), ("kind", "<i4"), ("n_rows", "<i4"), ("n_cols", "<i4"),
                     ("comp", "<i4"), ("value_before", "<f8"), ("value_after", "<f8"),
                     ("r_row", "<f8"), ("r_col", "<f8"), ("tau_row", "<f8"), ("tau_col", "<f8")])
CLS_DTYPE = np.dtype([("cls", "<i4"), ("pad_", "<i4"), ("check_step", "<i8"), ("delta", "<f8"),
                      ("tau_row", "<f8"), ("tau_col", "<f8"), ("beta_row", "<f8"),
                      ("beta_col", "<f8")])

_libs: dict = {}
# FTGEMM_ORACLE_LIB selects another build (the planted-mistake tests use it)
_active = [os.environ.get("FTGEMM_ORACLE_LIB", LIB)]


class use:
    """Context manager that routes this module's functions to another build of
    the oracle (the tests use it to run the pins against planted mistakes)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        _active.append(self.path)
        return self

    def __exit__(self, *exc):
        _active.pop()


def load(path: str | None = None):
    """Load (building first if absent) the oracle shared library."""
    path = path or _active[-1]
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        if path != LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_gemm.argtypes = [i64, i64, i64, ctypes.c_double, dp, i64, dp, i64, ctypes.c_double, dp, i64]
    lib.oracle_gemm.restype = ctypes.c_int
    lib.oracle_encode_col.argtypes = [i64, i64, dp, i64, dp]
    lib.oracle_encode_col.restype = None
    lib.oracle_encode_row.argtypes = [i64, i64, dp, i64, dp]
    lib.oracle_encode_row.restype = None
    lib.oracle_beta.argtypes = [ctypes.c_double, i64, i64, ctypes.c_double, ctypes.c_double]
    lib.oracle_beta.restype = ctypes.c_double
    vp = ctypes.c_void_p
    lib.oracle_ftgemm_replay.argtypes = [ctypes.POINTER(_Cfg), dp, i64, dp, i64, dp, i64, dp, i64,
                                         vp, i64, vp, i64, vp, vp, i64]
    lib.oracle_ftgemm_replay.restype = i64
    lib.oracle_zgemm.argtypes = [i64, i64, i64, ctypes.c_double, ctypes.c_double, dp, i64, dp, i64,
                                 ctypes.c_double, ctypes.c_double, dp, i64]
    lib.oracle_zgemm.restype = ctypes.c_int
    lib.oracle_zencode_col.argtypes = [i64, i64, dp, i64, dp]
    lib.oracle_zencode_col.restype = None
    lib.oracle_zencode_row.argtypes = [i64, i64, dp, i64, dp]
    lib.oracle_zencode_row.restype = None
    lib.oracle_zftgemm_replay.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_double, ctypes.c_double, dp, i64, dp, i64,
                                          dp, i64, dp, i64, vp, i64, vp, i64, vp, vp, i64]
    lib.oracle_zftgemm_replay.restype = i64
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_sizeof.argtypes = [ctypes.c_int]
    lib.oracle_sizeof.restype = i64
    for which, want in ((0, ctypes.sizeof(_Cfg)), (1, INJ_DTYPE.itemsize), (2, EV_DTYPE.itemsize),
                        (3, CLS_DTYPE.itemsize)):
        got = lib.oracle_sizeof(which)
        if got != want:
            raise RuntimeError(f"oracle struct {which}: C size {got} != Python size {want}")
    _libs[path] = lib
    return lib


def _f64(x) -> np.ndarray:
    """Column-major float64 copy (exact for FP32/FP16/BF16 inputs)."""
    return np.asfortranarray(np.asarray(x, dtype=np.float64))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# decoders of the low-precision operand formats, from their definitions
# ---------------------------------------------------------------------------
def decode_bf16(codes: np.ndarray) -> np.ndarray:
    """bfloat16: the upper 16 bits of an IEEE binary32 (1 sign, 8 exponent,
    7 fraction bits).  Value = the binary32 whose low 16 bits are zero."""
    c = np.asarray(codes).astype(np.uint32)
    return (c << np.uint32(16)).view(np.float32).astype(np.float64)


def decode_e4m3(codes: np.ndarray) -> np.ndarray:
    """OCP FP8 E4M3 (bias 7, no infinities; S.1111.111 is NaN):
    normal  (-1)^s 2^(e-7) (1 + f/8) for e in 1..15,
    subnormal (-1)^s 2^(-6) (f/8) for e == 0."""
    c = np.asarray(codes).astype(np.int64) & 0xFF
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    f = (c & 0x7).astype(np.float64)
    val = np.where(e == 0, np.ldexp(f / 8.0, -6), np.ldexp(1.0 + f / 8.0, (e - 7).astype(np.int64)))
    val = np.where((e == 0xF) & ((c & 0x7) == 0x7), np.nan, val)
    return s * val


# ---------------------------------------------------------------------------
# plain product and encodings
# ---------------------------------------------------------------------------
def gemm(A, B, C0=None, alpha=1.0, beta=0.0, m=None, n=None, k=None) -> np.ndarray:
    """C = alpha*A*B + beta*C0 in FP64 (section 3.1).  A is m x k, B is k x n."""
    lib = load()
    A = _f64(A)
    B = _f64(B)
    m = A.shape[0] if m is None else m
    k = A.shape[1] if k is None else k
    n = B.shape[1] if n is None else n
    if C0 is None:
        C = np.zeros((max(m, 1), n), dtype=np.float64, order="F")
        if beta != 0.0:
            raise ValueError("beta != 0 needs C0")
    else:
        C = _f64(C0).copy(order="F")
    rc = lib.oracle_gemm(m, n, k, float(alpha), _dp(A), max(A.shape[0], 1), _dp(B), max(B.shape[0], 1),
                         float(beta), _dp(C), max(C.shape[0], 1))
    if rc != 0:
        raise ValueError(f"oracle_gemm: invalid argument {-rc}")
    return C


def encode_col(A) -> np.ndarray:
    """e^T A for an m x k block (Eq. 1): the column sums, length k."""
    lib = load()
    A = _f64(A)
    w = np.zeros(A.shape[1], dtype=np.float64)
    lib.oracle_encode_col(A.shape[0], A.shape[1], _dp(A), max(A.shape[0], 1), _dp(w))
    return w


def encode_row(B) -> np.ndarray:
    """B e for a k x n block (Eq. 2): the row sums, length k."""
    lib = load()
    B = _f64(B)
    v = np.zeros(B.shape[0], dtype=np.float64)
    lib.oracle_encode_row(B.shape[0], B.shape[1], _dp(B), max(B.shape[0], 1), _dp(v))
    return v


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(load().oracle_threads())


def set_threads(n: int) -> None:
    """OpenMP threads for later oracle calls from this thread."""
    load().oracle_set_threads(int(n))


def beta_bound(u, kprime, count, own_norm, other_norm_sum) -> float:
    """Roundoff bound on one checksum residual (see the C file's header)."""
    return load().oracle_beta(float(u), int(kprime), int(count), float(own_norm), float(other_norm_sum))


# ---------------------------------------------------------------------------
# online ABFT replay
# ---------------------------------------------------------------------------
@dataclass
class ReplayConfig:
    mc: int
    nc: int
    ku: int
    g: int = 1
    u: float = U_FP32
    c: float = 2.0
    ft_level: int = 2


@dataclass
class ReplayResult:
    C: np.ndarray
    events: np.ndarray        # EV_DTYPE, (tile_m, tile_n, kstep) order
    classes: np.ndarray       # CLS_DTYPE, aligned with the injections passed in
    n_events: int


def make_injections(rows) -> np.ndarray:
    """rows: iterable of (tile_m, tile_n, kstep, row, col, old_v, new_v[, force[, comp]])."""
    rows = list(rows)
    out = np.zeros(len(rows), dtype=INJ_DTYPE)
    for q, r in enumerate(rows):
        out[q]["tile_m"], out[q]["tile_n"], out[q]["kstep"] = r[0], r[1], r[2]
        out[q]["row"], out[q]["col"] = r[3], r[4]
        out[q]["old_v"], out[q]["new_v"] = r[5], r[6]
        out[q]["force"] = r[7] if len(r) > 7 else -1
        out[q]["comp"] = r[8] if len(r) > 8 else 0
    return out


def replay(A, B, cfg: ReplayConfig, C0=None, alpha=1.0, beta=0.0, injections=None,
           tiles=None, ev_cap=1 << 16) -> ReplayResult:
    """Replay the online FT-GEMM on the CPU in FP64.

    ``injections`` is an INJ_DTYPE array of faults (the GPU's injection log),
    ``tiles`` an optional list of (tile_m, tile_n) to restrict the replay to.
    """
    lib = load()
    A = _f64(A)
    B = _f64(B)
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), dtype=np.float64, order="F")
    C0a = _f64(C0) if C0 is not None else np.zeros((1, 1), dtype=np.float64, order="F")
    if beta != 0.0 and C0 is None:
        raise ValueError("beta != 0 needs C0")
    c = _Cfg(m=m, n=n, k=k, mc=cfg.mc, nc=cfg.nc, ku=cfg.ku, g=cfg.g, alpha=float(alpha),
             beta=float(beta), u=cfg.u, c=cfg.c, ft_level=cfg.ft_level, pad_=0)
    inj = np.ascontiguousarray(injections if injections is not None else np.zeros(0, INJ_DTYPE),
                               dtype=INJ_DTYPE)
    cls = np.zeros(len(inj), dtype=CLS_DTYPE)
    sel = None
    if tiles is not None:
        # each tile once: tiles are replayed in parallel and write their own block of C
        sel = np.ascontiguousarray(np.unique(np.asarray(tiles, dtype=np.int64).reshape(-1, 2), axis=0))
    ev = np.zeros(ev_cap, dtype=EV_DTYPE)
    total = lib.oracle_ftgemm_replay(
        ctypes.byref(c), _dp(A), max(m, 1), _dp(B), max(k, 1), _dp(C0a), max(C0a.shape[0], 1),
        _dp(C), max(m, 1), inj.ctypes.data if len(inj) else None, len(inj),
        sel.ctypes.data if sel is not None else None, 0 if sel is None else len(sel),
        cls.ctypes.data if len(inj) else None, ev.ctypes.data, ev_cap)
    if total < 0:
        raise ValueError(f"oracle_ftgemm_replay: invalid argument ({total})")
    return ReplayResult(C=C, events=ev[:min(total, ev_cap)].copy(), classes=cls, n_events=int(total))


# ---------------------------------------------------------------------------
# complex binary64 (double-complex GEMM, the data type section 6 names as
# future work): operands are numpy complex128 arrays, column-major
# ---------------------------------------------------------------------------
def _z(x) -> np.ndarray:
    """Column-major complex128 copy."""
    return np.asfortranarray(np.asarray(x, dtype=np.complex128))


def _zp(a: np.ndarray):
    """Pointer to the interleaved (re, im) doubles of a complex128 array."""
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def zgemm(A, B, C0=None, alpha=1.0, beta=0.0) -> np.ndarray:
    """C = alpha*A*B + beta*C0 in complex binary64 (alpha, beta complex)."""
    lib = load()
    A = _z(A)
    B = _z(B)
    m, k = A.shape
    n = B.shape[1]
    if C0 is None:
        if beta != 0:
            raise ValueError("beta != 0 needs C0")
        C = np.zeros((max(m, 1), n), dtype=np.complex128, order="F")
    else:
        C = _z(C0).copy(order="F")
    al, be = complex(alpha), complex(beta)
    rc = lib.oracle_zgemm(m, n, k, al.real, al.imag, _zp(A), max(m, 1), _zp(B), max(k, 1), be.real, be.imag,
                          _zp(C), max(C.shape[0], 1))
    if rc != 0:
        raise ValueError(f"oracle_zgemm: invalid argument {-rc}")
    return C[:m] if m == 0 else C


def zencode_col(A) -> np.ndarray:
    """Complex e^T A (Eq. 1), length k."""
    lib = load()
    A = _z(A)
    w = np.zeros(A.shape[1], dtype=np.complex128)
    lib.oracle_zencode_col(A.shape[0], A.shape[1], _zp(A), max(A.shape[0], 1), _zp(w))
    return w


def zencode_row(B) -> np.ndarray:
    """Complex B e (Eq. 2), length k."""
    lib = load()
    B = _z(B)
    v = np.zeros(B.shape[0], dtype=np.complex128)
    lib.oracle_zencode_row(B.shape[0], B.shape[1], _zp(B), max(B.shape[0], 1), _zp(v))
    return v


def zreplay(A, B, cfg: ReplayConfig, C0=None, alpha=1.0, beta=0.0, injections=None, tiles=None,
            ev_cap=1 << 16) -> ReplayResult:
    """Replay the online complex FT-GEMM on the CPU in complex binary64: complex
    encodings, products and reference checksums; the real and the imaginary
    part of every residual are checked, located and corrected on their own
    (injections and events carry the component in ``comp``); the bound takes
    2K' products per component and complex 2-norms.  Default u: binary64."""
    lib = load()
    A = _z(A)
    B = _z(B)
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), dtype=np.complex128, order="F")
    al, be = complex(alpha), complex(beta)
    if be != 0 and C0 is None:
        raise ValueError("beta != 0 needs C0")
    C0a = _z(C0) if C0 is not None else np.zeros((1, 1), dtype=np.complex128, order="F")
    c = _Cfg(m=m, n=n, k=k, mc=cfg.mc, nc=cfg.nc, ku=cfg.ku, g=cfg.g, alpha=al.real, beta=be.real, u=cfg.u,
             c=cfg.c, ft_level=cfg.ft_level, pad_=0)
    inj = np.ascontiguousarray(injections if injections is not None else np.zeros(0, INJ_DTYPE), dtype=INJ_DTYPE)
    cls = np.zeros(len(inj), dtype=CLS_DTYPE)
    sel = None
    if tiles is not None:
        sel = np.ascontiguousarray(np.unique(np.asarray(tiles, dtype=np.int64).reshape(-1, 2), axis=0))
    ev = np.zeros(ev_cap, dtype=EV_DTYPE)
    total = lib.oracle_zftgemm_replay(
        ctypes.byref(c), al.imag, be.imag, _zp(A), max(m, 1), _zp(B), max(k, 1), _zp(C0a), max(C0a.shape[0], 1),
        _zp(C), max(m, 1), inj.ctypes.data if len(inj) else None, len(inj),
        sel.ctypes.data if sel is not None else None, 0 if sel is None else len(sel),
        cls.ctypes.data if len(inj) else None, ev.ctypes.data, ev_cap)
    if total < 0:
        raise ValueError(f"oracle_zftgemm_replay: invalid argument ({total})")
    return ReplayResult(C=C, events=ev[:min(total, ev_cap)].copy(), classes=cls, n_events=int(total))
