"""Seeded synthetic workloads: operand generators, shape sets and fault sites.

This module only draws random numbers and lays them out; it holds none of the
fault-tolerance arithmetic.  Tests, the smoke check and the benchmark use it
to feed the same inputs to the GPU library and to the CPU oracle.

Conventions: operands are numpy arrays in BLAS column-major order
(``np.asfortranarray``), FP32 unless stated.  Seeds are
``SEED_BASE + 100 * workload + stream`` with streams A=0, B=1, C=2, sites=3,
shapes=4, so every workload is reproducible from its number alone.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_BASE = 2305_01024
STREAM_A, STREAM_B, STREAM_C, STREAM_SITES, STREAM_SHAPES = 0, 1, 2, 3, 4

# fault kinds understood by the library's injection hook
KIND_ADD = 0   # accumulator += payload
KIND_XOR = 1   # accumulator bits ^= 1 << payload

SITE_DTYPE = np.dtype([("tile_m", "<i4"), ("tile_n", "<i4"), ("kstep", "<i4"), ("row", "<i4"),
                       ("col", "<i4"), ("kind", "<i4"), ("payload", "<f4"), ("problem", "<i4")])


def seed(workload: int, stream: int) -> int:
    return SEED_BASE + 100 * workload + stream


def rng(workload: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(seed(workload, stream))


def uniform(shape, workload: int, stream: int, lo=-1.0, hi=1.0) -> np.ndarray:
    """i.i.d. U[lo, hi) in FP32, column-major."""
    g = rng(workload, stream)
    return np.asfortranarray(g.uniform(lo, hi, size=shape).astype(np.float32))


def normal(shape, workload: int, stream: int) -> np.ndarray:
    """i.i.d. N(0, 1) in FP32, column-major."""
    g = rng(workload, stream)
    return np.asfortranarray(g.standard_normal(size=shape, dtype=np.float32))


def uniform64(shape, workload: int, stream: int, lo=-1.0, hi=1.0) -> np.ndarray:
    """i.i.d. U[lo, hi) in FP64 (full 53-bit mantissas), column-major."""
    g = rng(workload, stream)
    return np.asfortranarray(g.uniform(lo, hi, size=shape))


def normal64(shape, workload: int, stream: int) -> np.ndarray:
    """i.i.d. N(0, 1) in FP64 (full 53-bit mantissas), column-major."""
    g = rng(workload, stream)
    return np.asfortranarray(g.standard_normal(size=shape))


def heavy_tailed(shape, workload: int, stream: int, frac=0.01, scale=100.0) -> np.ndarray:
    """N(0, 1) with a Bernoulli(frac) mask of entries multiplied by ``scale``
    (mask drawn from the same stream, after the values)."""
    g = rng(workload, stream)
    x = g.standard_normal(size=shape, dtype=np.float32)
    mask = g.random(size=shape) < frac
    x[mask] *= np.float32(scale)
    return np.asfortranarray(x)


def integers(shape, workload: int, stream: int, lo=-4, hi=4) -> np.ndarray:
    """Small integers in [lo, hi] as FP32: every product and partial sum of a
    GEMM with K <= 2**16 is then exact in FP32 and FP64."""
    g = rng(workload, stream)
    return np.asfortranarray(g.integers(lo, hi + 1, size=shape).astype(np.float32))


# ---------------------------------------------------------------------------
# shapes of the measured workloads
# ---------------------------------------------------------------------------
SQUARE_SIZES = (2048, 4096, 8192)           # FP32 square FT-GEMM, N(0,1), beta = 1
IRREGULAR_SHAPES = ((65536, 256, 4096), (256, 65536, 4096), (16384, 16384, 64), (3001, 1999, 4097))


def irregular_shapes(workload: int = 3):
    """The irregular shape set in a seeded order."""
    g = rng(workload, STREAM_SHAPES)
    order = g.permutation(len(IRREGULAR_SHAPES))
    return [IRREGULAR_SHAPES[i] for i in order]


@dataclass
class BatchedProblem:
    m: int
    n: int
    k: int
    dtype: str   # "f32" or "bf16"


def batched_problems(count=1024, lo=32, hi=2048, workload: int = 5):
    """M, N, K each exp(U[ln lo, ln hi]) rounded; dtype by a fair coin."""
    g = rng(workload, STREAM_SHAPES)
    dims = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), size=(count, 3)))).astype(np.int64)
    coin = g.random(count) < 0.5
    return [BatchedProblem(int(d[0]), int(d[1]), int(d[2]), "bf16" if c else "f32")
            for d, c in zip(dims, coin)]


# ---------------------------------------------------------------------------
# fault sites
# ---------------------------------------------------------------------------
def tile_grid(m, n, mc, nc):
    return (m + mc - 1) // mc, (n + nc - 1) // nc


def fault_sites(g: np.random.Generator, m, n, k, mc, nc, ku, gint, count, kind=KIND_ADD,
                payload=1e3, bits=range(0, 31), per_tile=None) -> np.ndarray:
    """Draw ``count`` fault sites, at most one per (tile, check interval).

    A check interval is ``gint`` consecutive k-steps of ``ku``; the last one may
    be shorter.  Row/col are tile-relative and lie inside C for border tiles.
    ``kind`` KIND_ADD uses ``payload`` as the additive offset; KIND_XOR draws a
    bit position uniformly from ``bits``.  ``per_tile`` (optional) places
    exactly that many faults in every tile instead of ``count`` overall.
    """
    ntm, ntn = tile_grid(m, n, mc, nc)
    nk = max(1, (k + ku - 1) // ku)
    nint = (nk + gint - 1) // gint
    slots = ntm * ntn * nint
    if per_tile is not None:
        if per_tile > nint:
            raise ValueError("more faults per tile than check intervals")
        chosen = []
        for t in range(ntm * ntn):
            ints = g.choice(nint, size=per_tile, replace=False)
            chosen.extend(t * nint + int(i) for i in ints)
        chosen = np.asarray(chosen, dtype=np.int64)
    else:
        if count > slots:
            raise ValueError(f"{count} faults > {slots} (tile, interval) slots")
        chosen = g.choice(slots, size=count, replace=False) if count else np.zeros(0, np.int64)
    out = np.zeros(len(chosen), dtype=SITE_DTYPE)
    bits = list(bits)
    for q, s in enumerate(sorted(int(x) for x in chosen)):
        tile, interval = divmod(s, nint)
        tm, tn = divmod(tile, ntn)
        rows = min(mc, m - tm * mc)
        cols = min(nc, n - tn * nc)
        s0 = interval * gint
        s1 = min(nk, s0 + gint)
        out[q]["tile_m"], out[q]["tile_n"] = tm, tn
        out[q]["kstep"] = g.integers(s0, s1)
        out[q]["row"] = g.integers(0, rows)
        out[q]["col"] = g.integers(0, cols)
        out[q]["kind"] = kind
        out[q]["payload"] = payload if kind == KIND_ADD else float(bits[g.integers(0, len(bits))])
    return out


def rate_schedule(g: np.random.Generator, rate_per_s: float, t_launch_s: float, launches: int):
    """Split round(rate * t * launches) faults over ``launches`` launches
    (multinomial, uniform): returns the per-launch counts."""
    total = int(round(rate_per_s * t_launch_s * launches))
    if total == 0:
        return np.zeros(launches, dtype=np.int64), 0
    counts = np.bincount(g.integers(0, launches, size=total), minlength=launches)
    return counts, total


# ---------------------------------------------------------------------------
# low-precision operands (input preparation: rounding to the storage format)
# ---------------------------------------------------------------------------
def to_bf16_codes(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 (round to nearest, ties to even) and
    return the 16-bit codes (finite inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16).reshape(np.shape(x))


def quantize_bf16(x: np.ndarray):
    """bfloat16 codes of x (column-major kept) and the per-tensor scale.
    bfloat16 shares FP32's exponent range, so no rescaling is needed and the
    scale is 1."""
    codes = np.asfortranarray(to_bf16_codes(np.asarray(x, dtype=np.float32)))
    return codes, 1.0


E4M3_MAX = 448.0


def to_e4m3_codes(x: np.ndarray) -> np.ndarray:
    """Round finite values to OCP FP8 E4M3 (bias 7, 3 mantissa bits; round to
    nearest, ties to even; magnitudes above 448 saturate to 448) and return
    the 8-bit codes."""
    x = np.asarray(x, dtype=np.float64)
    sign = (np.signbit(x)).astype(np.uint8) << 7
    ax = np.minimum(np.abs(x), E4M3_MAX)
    code = np.zeros(ax.shape, dtype=np.int64)
    sub = ax < 2.0 ** -6
    # subnormals (and zero): multiples of 2^-9; q == 8 is the smallest normal
    code[sub] = np.rint(ax[sub] * 2.0 ** 9).astype(np.int64)
    nrm = ~sub
    e = np.floor(np.log2(ax[nrm])).astype(np.int64)
    q = np.rint(ax[nrm] / np.exp2(e - 3)).astype(np.int64)      # 8 .. 16
    e = np.where(q == 16, e + 1, e)
    q = np.where(q == 16, 8, q)
    code[nrm] = ((e + 7) << 3) | (q - 8)
    code = np.minimum(code, 0x7E)                                 # saturate at 448
    return (code.astype(np.uint8) | sign).reshape(x.shape)


def quantize_e4m3(x: np.ndarray):
    """Per-tensor power-of-two absmax scaling to E4M3: returns (codes, s) with
    x ~= s * decode(codes), s = 2^ceil(log2(absmax / 448))."""
    x = np.asarray(x, dtype=np.float32)
    amax = float(np.max(np.abs(x))) if x.size else 0.0
    s = 1.0 if amax == 0.0 else float(2.0 ** np.ceil(np.log2(amax / E4M3_MAX)))
    codes = np.asfortranarray(to_e4m3_codes(x.astype(np.float64) / s))
    return codes, s
