"""GPU parity of the low-precision-input online ABFT GEMMs (BF16 and FP8
E4M3 operands, FP32 accumulation, FP32 checksums on the exactly decoded
operands) against the FP64 oracle on the same quantised values.  Bar: relative
Frobenius error <= 2e-2 against the oracle on the quantised operands (the
stated bound for BF16/FP8; the products are exact, so the measured error is
the FP32 accumulation's, checked at 1e-5 too); event logs equal to the
oracle replay's exactly."""
import functools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import U_FP8_ACC, elementwise_ratio, event_keys, rel_fro, replay_against_gpu

pytestmark = pytest.mark.gpu
TOL_LOWP = 2e-2
# Accumulation check on top of the stated bound: bf16 products are exact and
# the MFMA accumulates them in FP32 (1e-5, as FP32).  The FP8 MFMA sums its 16
# products per instruction at less than FP32 precision (measured 1.5e-5 at
# K = 64), so its accumulation check is 1e-4.
TOL_ACC = {"bf16": 1e-5, "fp8": 1e-4}
# Element-wise bound (k + 2) u (|A||B|)_ij of gpu_util.elementwise_ratio: u =
# 2^-24 for BF16 (exact products, binary32 accumulation); for FP8 the model
# of its instruction's accumulation (gpu_util.U_FP8_ACC).
ACC_U = {"bf16": 2.0 ** -24, "fp8": U_FP8_ACC}

DTYPES = {
    "bf16": (F.BF16, W.quantize_bf16, O.decode_bf16, np.int16, "bf16"),
    "fp8": (F.F8E4M3, W.quantize_e4m3, O.decode_e4m3, np.uint8, "fp8"),
}


@pytest.fixture(scope="module", params=sorted(DTYPES))
def h(request):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dt = DTYPES[request.param]
    handle = F.ftgemm_create(dt[0], 0)
    yield handle, dt
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


@pytest.fixture(autouse=True)
def _reset(h):
    F.ftgemm_set_config(h[0], None)
    F.ftgemm_set_injection(h[0], None)
    F.ftgemm_set_scales(h[0], 1.0, 1.0)
    yield


def _quant(dt, x):
    codes, s = dt[1](x)
    return codes, s


def _dev_codes(dt, codes):
    import torch
    return torch.from_numpy(np.ascontiguousarray(codes.T).view(dt[3])).cuda()


def _run(h, Ac, Bc, sa=1.0, sb=1.0, C0=None, alpha=1.0, beta=0.0, level=F.FT_CORRECT, cap=16384):
    import torch
    handle, dt = h
    m, k = Ac.shape
    n = Bc.shape[1]
    F.ftgemm_set_scales(handle, sa, sb)
    dA, dB = _dev_codes(dt, Ac), _dev_codes(dt, Bc)
    dC = (torch.from_numpy(np.ascontiguousarray(np.asarray(C0, np.float32).T)).cuda() if C0 is not None
          else torch.zeros((n, m), device="cuda"))
    rep = F.ReportBuffer(cap)
    st = F.ftgemm_run(handle, m, n, k, alpha, dA.data_ptr(), m, dB.data_ptr(), k, beta, dC.data_ptr(), m,
                      level, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    return st, np.asfortranarray(dC.cpu().numpy().T), rep


def _decoded(h, Ac, Bc):
    dec = h[1][2]
    return np.asfortranarray(dec(Ac)), np.asfortranarray(dec(Bc))


@pytest.mark.parametrize("shape", [(256, 256, 64), (512, 768, 640), (300, 520, 200), (1000, 37, 999), (1, 1, 1)])
def test_clean_matches_oracle(h, shape):
    m, n, k = shape
    Ac, sa = _quant(h[1], W.normal((m, k), 300, 0))
    Bc, sb = _quant(h[1], W.normal((k, n), 300, 1))
    A, B = _decoded(h, Ac, Bc)
    st, C, rep = _run(h, Ac, Bc, sa, sb)
    ref = O.gemm(A, B, alpha=sa * sb)
    assert st == F.OK and rep.report.n_events == 0
    err = rel_fro(C, ref)
    assert err <= TOL_LOWP
    assert err <= TOL_ACC[h[1][4]], err
    assert elementwise_ratio(C, ref, A, B, alpha=sa * sb, acc_u=ACC_U[h[1][4]]) <= 1.0


@pytest.mark.parametrize("shape", [(512, 768, 640), (300, 520, 200), (1000, 37, 999), (200, 136, 100),
                                   (136, 200, 190), (64, 64, 1)])
def test_plain_level_matches_oracle(h, shape):
    """ft_level 0 (the plain kernel, FT compiled out): same bar on the product,
    no event, including ragged tiles and a partial last k-step; 1, 2 and 3
    k-steps cover the ends of the FP8 plain kernel's two-step-ahead loads."""
    m, n, k = shape
    Ac, sa = _quant(h[1], W.normal((m, k), 301, 0))
    Bc, sb = _quant(h[1], W.normal((k, n), 301, 1))
    A, B = _decoded(h, Ac, Bc)
    C0 = W.normal((m, n), 301, 2)
    st, C, rep = _run(h, Ac, Bc, sa, sb, C0=C0, alpha=0.5, beta=2.0, level=F.FT_OFF)
    ref = O.gemm(A, B, C0, alpha=0.5 * sa * sb, beta=2.0)
    assert st == F.OK and rep.report.n_events == 0 and rep.report.checks == 0
    assert rel_fro(C, ref) <= TOL_ACC[h[1][4]]


def test_integer_operands_exact(h):
    Ac, sa = _quant(h[1], W.integers((320, 448), 301, 0))
    Bc, sb = _quant(h[1], W.integers((448, 288), 301, 1))
    A, B = _decoded(h, Ac, Bc)
    st, C, rep = _run(h, Ac, Bc, sa, sb)
    assert st == F.OK and rep.report.n_events == 0
    assert np.array_equal(C.astype(np.float64), O.gemm(A, B, alpha=sa * sb))


def test_scales_alpha_beta_ragged(h):
    m, n, k = 300, 520, 200
    Ac, _ = _quant(h[1], W.normal((m, k), 302, 0))
    Bc, _ = _quant(h[1], W.normal((k, n), 302, 1))
    C0 = W.normal((m, n), 302, 2)
    A, B = _decoded(h, Ac, Bc)
    st, C, rep = _run(h, Ac, Bc, 2.0, 0.25, C0, alpha=1.5, beta=-0.5)
    assert st == F.OK and rep.report.n_events == 0
    assert rel_fro(C, O.gemm(A, B, C0, alpha=1.5 * 2.0 * 0.25, beta=-0.5)) <= TOL_ACC[h[1][4]]


def test_unaligned_leading_dimensions(h):
    """lda, ldb not multiples of the vector width take the element-wise load path."""
    import torch
    handle, dt = h
    m, n, k = 200, 136, 190
    lda, ldb = m + 3, k + 5
    Ac, _ = _quant(dt, W.normal((m, k), 303, 0))
    Bc, _ = _quant(dt, W.normal((k, n), 303, 1))
    A, B = _decoded(h, Ac, Bc)
    pa = np.zeros((lda, k), dtype=Ac.dtype, order="F")
    pa[:m] = Ac
    pb = np.zeros((ldb, n), dtype=Bc.dtype, order="F")
    pb[:k] = Bc
    dA, dB = _dev_codes(dt, pa), _dev_codes(dt, pb)
    dC = torch.zeros((n, m), device="cuda")
    rep = F.ReportBuffer(64)
    st = F.ftgemm_run(handle, m, n, k, 1.0, dA.data_ptr(), lda, dB.data_ptr(), ldb, 0.0, dC.data_ptr(), m,
                      F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    C = np.asfortranarray(dC.cpu().numpy().T)
    assert st == F.OK and rep.report.n_events == 0
    assert rel_fro(C, O.gemm(A, B)) <= TOL_ACC[h[1][4]]


def test_heavy_tailed_clean_no_false_positive(h):
    m = n = k = 1024
    Ac, sa = _quant(h[1], W.heavy_tailed((m, k), 4, W.STREAM_A))
    Bc, sb = _quant(h[1], W.heavy_tailed((k, n), 4, W.STREAM_B))
    A, B = _decoded(h, Ac, Bc)
    st, C, rep = _run(h, Ac, Bc, sa, sb)
    assert st == F.OK and rep.report.n_events == 0
    assert rel_fro(C, O.gemm(A, B, alpha=sa * sb)) <= TOL_ACC[h[1][4]]


@pytest.mark.parametrize("kind", [W.KIND_ADD, W.KIND_XOR])
def test_fault_injection_exact_site_log(h, kind):
    m, n, k = 768, 512, 1024
    Ac, sa = _quant(h[1], W.normal((m, k), 304, 0))
    Bc, sb = _quant(h[1], W.normal((k, n), 304, 1))
    A, B = _decoded(h, Ac, Bc)
    cfg = (256, 256, 64, 4)
    # the checks see the unscaled codes: a fault of 1e3 in the scaled result
    # is 1e3 / (s_a s_b) in the accumulator
    sites = W.fault_sites(W.rng(304, 3), m, n, k, 256, 256, 64, 4, 20, kind=kind, payload=1e3 / (sa * sb),
                          bits=range(23, 31))
    F.ftgemm_set_config(h[0], cfg)
    F.ftgemm_set_injection(h[0], sites)
    st, C, rep = _run(h, Ac, Bc)
    log = F.ftgemm_get_injection_log(h[0])
    F.ftgemm_set_injection(h[0], None)
    assert len(log) == 20
    res, cls, n_grey, bad = replay_against_gpu(A, B, cfg, rep, log)
    assert bad == 0
    must = int(np.sum(cls["cls"] == O.CLS_MUST))
    assert rep.report.corrected >= must and (kind == W.KIND_XOR or must == 20)
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, res.C) <= TOL_ACC[h[1][4]]
    assert elementwise_ratio(C, res.C, A, B, cfg, events=rep.events, oracle_events=res.events, log=log,
                             acc_u=ACC_U[h[1][4]]) <= 1.0


@functools.lru_cache(maxsize=1)
def _full_operands(name):
    """8192 x 8192 heavy-tailed N(0,1) operands (1% x100) quantised to the
    dtype, shared by the full-size tests of that dtype."""
    dt = DTYPES[name]
    Ac, sa = _quant(dt, W.heavy_tailed((8192, 8192), 4, W.STREAM_A))
    Bc, sb = _quant(dt, W.heavy_tailed((8192, 8192), 4, W.STREAM_B))
    return Ac, sa, Bc, sb


def test_full_size_8192_sampled_tiles(h):
    """8192^3 with heavy-tailed N(0,1) operands (1% x100), per-tensor
    power-of-two scaling: no event in a clean run, and sampled tiles match the
    oracle replay on the decoded operands."""
    m = n = k = 8192
    Ac, sa, Bc, sb = _full_operands(h[1][4])
    st, C, rep = _run(h, Ac, Bc, sa, sb)
    cfg = rep.report.config.as_tuple()
    assert st == F.OK and rep.report.n_events == 0
    tiles = [(0, 0), (m // cfg[0] - 1, n // cfg[1] - 1), (5, 17)]
    A, B = _decoded(h, Ac, Bc)
    res = O.replay(A, B, O.ReplayConfig(mc=cfg[0], nc=cfg[1], ku=cfg[2], g=cfg[3]), alpha=sa * sb, tiles=tiles)
    assert res.n_events == 0
    for (tm, tn) in tiles:
        sl = (slice(tm * cfg[0], (tm + 1) * cfg[0]), slice(tn * cfg[1], (tn + 1) * cfg[1]))
        assert rel_fro(C[sl], res.C[sl]) <= TOL_ACC[h[1][4]], (tm, tn)
        assert elementwise_ratio(C, res.C, A, B, cfg, alpha=sa * sb, tile=(tm, tn), acc_u=ACC_U[h[1][4]]) <= 1.0


def test_full_size_8192_one_fault_per_tile(h):
    """The full-size operands, automatic configuration, one +1e7 fault in
    every tile at a seeded k-step, row and column, checked on the unscaled
    codes (scales 1): the oracle replays every tile with the GPU's applied
    faults, classes every fault must-detect, its event log equals the GPU's
    and C equals the replay element by element (corrected elements within
    their check's beta_row).  The bound at full K is about 4e5 here
    (heavy-tailed rows: |a_i| ~ 900), so 1e7 is must-detect at every k-step."""
    m = n = k = 8192
    Ac, _, Bc, _ = _full_operands(h[1][4])
    cfg = F.ftgemm_select_config(h[1][0], m, n, k).as_tuple()
    ntiles = (m // cfg[0]) * (n // cfg[1])
    sites = W.fault_sites(W.rng(8192, W.STREAM_SITES), m, n, k, *cfg[:4], 0, payload=1e7, per_tile=1)
    F.ftgemm_set_injection(h[0], sites)
    st, C, rep = _run(h, Ac, Bc)
    log = F.ftgemm_get_injection_log(h[0])
    F.ftgemm_set_injection(h[0], None)
    assert st == F.OK and rep.report.config.as_tuple()[:4] == cfg[:4]
    assert len(log) == len(sites) == ntiles
    assert rep.report.corrected == ntiles and rep.report.uncorrectable == 0
    A, B = _decoded(h, Ac, Bc)
    res, cls, _, bad = replay_against_gpu(A, B, cfg, rep, log)
    assert bad == 0 and np.all(cls["cls"] == O.CLS_MUST)
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, res.C) <= TOL_ACC[h[1][4]]
    assert elementwise_ratio(C, res.C, A, B, cfg, events=rep.events, oracle_events=res.events, log=log,
                             acc_u=ACC_U[h[1][4]]) <= 1.0
