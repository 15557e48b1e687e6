"""Measured margin of the detection threshold on the GPU.

The paper leaves the threshold as a constant fixed in advance (section 2.2); the
library uses the analytic roundoff bound beta of the oracle (tau = c * beta,
c = 2 by default).  Two measurements per operand type, on clean 8192^3 runs
in the benchmarked configuration:

* max|r|/beta over every check of the launch: the largest c at which a check
  still flags, found by bisection on c.  It must be below 1 (no check of a
  clean run reaches beta), so the default c = 2 keeps a margin of at least 2.
* the element-wise accumulation error of the plain kernel against the exact
  product, as a fraction of the gamma_K model K u (|A||B|)_ij that the
  bound's derivation assumes for the matrix-core accumulation.

Two data sets: N(0,1) (heavy-tailed for BF16/FP8: 1% of entries x100) and
all-positive U[0.5, 1) operands, where the Cauchy-Schwarz step of the bound is
nearly tight and rounding errors do not cancel.  The figures are printed
(`pytest -s`)."""
import functools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

pytestmark = pytest.mark.gpu
N = 8192
U32 = 2.0 ** -24

DTYPES = {
    "f32": (F.F32, None, None, np.float32),
    "bf16": (F.BF16, W.quantize_bf16, O.decode_bf16, np.int16),
    "fp8": (F.F8E4M3, W.quantize_e4m3, O.decode_e4m3, np.uint8),
}


@functools.lru_cache(maxsize=1)
def _operands(dtype, data):
    """(device A, device B, decoded float64 A, decoded float64 B, scale) at 8192^3."""
    import torch
    wl = 7
    if data == "normal":
        gen = W.normal if dtype == "f32" else W.heavy_tailed
        A = gen((N, N), wl, W.STREAM_A)
        B = gen((N, N), wl, W.STREAM_B)
    else:
        A = W.uniform((N, N), wl, W.STREAM_A, 0.5, 1.0)
        B = W.uniform((N, N), wl, W.STREAM_B, 0.5, 1.0)
    dt = DTYPES[dtype]
    if dt[1] is None:
        dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
        dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
        return dA, dB, A, B, 1.0
    Ac, sa = dt[1](A)
    Bc, sb = dt[1](B)
    dA = torch.from_numpy(np.ascontiguousarray(Ac.T).view(dt[3])).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(Bc.T).view(dt[3])).cuda()
    # the checks run on the unscaled decoded codes; the scales only enter the epilogue
    return dA, dB, np.asfortranarray(dt[2](Ac)), np.asfortranarray(dt[2](Bc)), sa * sb


@pytest.fixture(scope="module", params=sorted(DTYPES))
def h(request):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(DTYPES[request.param][0], 0)
    yield handle, request.param
    F.ftgemm_destroy(handle)


def _detected(handle, dA, dB, dC, c):
    """Checks of a clean online run at threshold factor c that flagged."""
    import torch
    rep = F.ReportBuffer(1)
    try:
        F.ftgemm_run(handle, N, N, N, 1.0, dA.data_ptr(), N, dB.data_ptr(), N, 0.0, dC.data_ptr(), N,
                     F.FT_CORRECT, c, torch.cuda.current_stream().cuda_stream, rep)
    except F.FtgemmError as e:   # a tiny c flags every check: the one-entry event buffer overflows
        assert e.status == F.LOG_OVERFLOW
    return int(rep.report.detected), int(rep.report.checks)


@pytest.mark.parametrize("data", ["normal", "positive"])
def test_clean_residuals_stay_below_the_bound(h, data):
    import torch
    handle, dtype = h
    dA, dB, _, _, _ = _operands(dtype, data)
    dC = torch.zeros((N, N), device="cuda")
    det, checks = _detected(handle, dA, dB, dC, 1.0)
    assert checks == (N // 256) ** 2 * (N // 256), checks   # 1024 tiles x 32 checks (a check every 256 k)
    assert det == 0, f"{dtype}/{data}: a clean check reached beta"
    # bisection on log2(c): the largest c that still flags is max|r|/beta
    lo, hi = -40.0, 0.0            # flags at 2^lo (asserted), none at 2^hi
    assert _detected(handle, dA, dB, dC, 2.0 ** lo)[0] > 0
    for _ in range(14):
        mid = 0.5 * (lo + hi)
        if _detected(handle, dA, dB, dC, 2.0 ** mid)[0] > 0:
            lo = mid
        else:
            hi = mid
    ratio = 2.0 ** hi
    print(f"\n[threshold] {dtype} {data} 8192^3: max|r|/beta = {ratio:.3e} (margin {1 / ratio:.0f}x at c = 1)")
    assert ratio < 1.0


@pytest.mark.parametrize("data", ["normal", "positive"])
def test_accumulation_error_within_the_model(h, data):
    """Plain kernel (FT off) at 8192^3 on a sampled 256 x 256 block of C: the
    error against the exact FP64 product of the decoded operands, per element,
    over K u (|A||B|)_ij."""
    import torch
    handle, dtype = h
    dA, dB, A, B, _ = _operands(dtype, data)
    dC = torch.zeros((N, N), device="cuda")
    F.ftgemm_run(handle, N, N, N, 1.0, dA.data_ptr(), N, dB.data_ptr(), N, 0.0, dC.data_ptr(), N,
                 F.FT_OFF, 0.0, torch.cuda.current_stream().cuda_stream, None)
    torch.cuda.synchronize()
    g = np.random.default_rng(11)
    rows = np.sort(g.choice(N, 256, replace=False))
    cols = np.sort(g.choice(N, 256, replace=False))
    # column-major C lives in the (N, N) tensor as C^T: element (i, j) is dC[j, i]
    C = dC[torch.from_numpy(cols).cuda()][:, torch.from_numpy(rows).cuda()].cpu().numpy().T.astype(np.float64)
    Ar = A[rows].astype(np.float64)
    Bc = B[:, cols].astype(np.float64)
    exact = Ar @ Bc                          # scales 1 and alpha 1: C holds the product of the decoded codes
    model = N * U32 * (np.abs(Ar) @ np.abs(Bc))
    ratio = float(np.max(np.abs(C - exact) / model))
    print(f"\n[accumulation] {dtype} {data} 8192^3: max |C - AB| / (K u |A||B|) = {ratio:.3e}")
    assert ratio <= 1.0
