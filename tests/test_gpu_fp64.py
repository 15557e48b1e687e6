"""GPU tests of the FP64 path (ftgemm_run_f64: binary64 operands, products,
accumulation, checksums and check, threshold with u = 2^-53), against the
FP64 oracle replayed at the same roundoff.  Bar: relative Frobenius error
<= 1e-12 against the oracle product (binary64 accumulations in a different
order), event logs equal."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import event_keys, rel_fro, replay_against_gpu

pytestmark = pytest.mark.gpu
TOL_F64 = 1e-12
CFG = (128, 128, 16, 16)   # the compiled FP64 configuration: a check every 256 k


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.F64, 0)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64).T)).cuda()


def _host(d, rows, cols):
    return np.asfortranarray(d.cpu().numpy().reshape(cols, rows).T)


def _run(h, A, B, C0=None, alpha=1.0, beta=0.0, level=F.FT_CORRECT, sites=None, cap=4096):
    import torch
    m, k = A.shape
    n = B.shape[1]
    dA, dB = _dev(A), _dev(B)
    dC = _dev(C0) if C0 is not None else torch.full((n, m), 7.0, dtype=torch.float64, device="cuda")
    F.ftgemm_set_injection(h, sites)
    try:
        rep = F.ReportBuffer(cap)
        st = F.ftgemm_run_f64(h, m, n, k, alpha, dA.data_ptr(), m, dB.data_ptr(), k, beta, dC.data_ptr(), m, level,
                              0.0, torch.cuda.current_stream().cuda_stream, rep)
        log = F.ftgemm_get_injection_log(h) if sites is not None else None
    finally:
        F.ftgemm_set_injection(h, None)
    return st, _host(dC, m, n), rep, log


def _checks(m, n, k, level=F.FT_CORRECT):
    nk = -(-k // CFG[2])
    per = -(-nk // CFG[3]) if level == F.FT_CORRECT else 1
    return -(-m // CFG[0]) * -(-n // CFG[1]) * per


@pytest.mark.parametrize("shape", [(512, 512, 512), (300, 520, 200), (1000, 37, 999), (129, 257, 17), (1, 1, 1)])
def test_clean_matches_oracle(h, shape):
    m, n, k = shape
    A = W.normal64((m, k), 701, 0)
    B = W.normal64((k, n), 701, 1)
    st, C, rep, _ = _run(h, A, B)
    assert st == F.OK and rep.report.n_events == 0 and rep.report.detected == 0
    assert rep.report.checks == _checks(m, n, k)
    assert rep.report.config.as_tuple() == CFG + CFG[:2]
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F64


def test_alpha_beta_and_level_off(h):
    m, n, k = 333, 222, 111
    A = W.uniform64((m, k), 702, 0)
    B = W.uniform64((k, n), 702, 1)
    C0 = W.uniform64((m, n), 702, 2)
    ref = O.gemm(A, B, C0, alpha=0.75, beta=-1.25)
    for level in (F.FT_OFF, F.FT_DETECT, F.FT_CORRECT):
        st, C, rep, _ = _run(h, A, B, C0, alpha=0.75, beta=-1.25, level=level)
        assert st == F.OK and rep.report.n_events == 0
        assert rel_fro(C, ref) <= TOL_F64


def test_k_zero_scales_c(h):
    import torch
    m, n = 70, 50
    C0 = W.uniform64((m, n), 703, 0)
    dC = _dev(C0)
    dummy = torch.zeros(1, dtype=torch.float64, device="cuda")
    rep = F.ReportBuffer(4)
    st = F.ftgemm_run_f64(h, m, n, 0, 1.0, dummy.data_ptr(), m, dummy.data_ptr(), 1, 0.5, dC.data_ptr(), m,
                          F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    assert st == F.OK
    assert np.array_equal(_host(dC, m, n), 0.5 * C0)


def test_one_fault_per_tile_corrected_at_its_site(h):
    """768 x 640 x 1024 N(0,1): one +1e3 fault per tile at a seeded k-step,
    row and column; every one is corrected and the event log equals the
    binary64 oracle replay's."""
    m, n, k = 768, 640, 1024
    A = W.normal64((m, k), 704, 0)
    B = W.normal64((k, n), 704, 1)
    sites = W.fault_sites(W.rng(704, W.STREAM_SITES), m, n, k, *CFG, 0, payload=1e3, per_tile=1)
    st, C, rep, log = _inject_and_replay(h, A, B, sites)
    assert st == F.OK and rep.report.corrected == len(sites) == (m // 128) * (n // 128)
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F64


def _inject_and_replay(h, A, B, sites, level=F.FT_CORRECT):
    st, C, rep, log = _run(h, A, B, level=level, sites=sites)
    assert len(log) == len(sites)
    res, cls, n_grey, bad = replay_against_gpu(A, B, CFG, rep, log, ft_level=level, u=O.U_FP64)
    assert bad == 0
    assert event_keys(rep.events) == event_keys(res.events)
    return st, C, rep, log


def test_small_fault_invisible_to_fp32_checks_is_corrected(h):
    """A +1e-6 fault: below what a binary32 check could see at this size,
    well above the binary64 threshold; corrected at its site."""
    m = n = k = 256
    A = W.normal64((m, k), 705, 0)
    B = W.normal64((k, n), 705, 1)
    sites = np.zeros(1, dtype=F.FAULT_DTYPE)
    sites[0] = (1, 0, 5, 17, 99, W.KIND_ADD, 1e-6, 0)
    st, C, rep, log = _inject_and_replay(h, A, B, sites)
    assert st == F.OK and rep.report.corrected == 1
    e = rep.events[0]
    assert (int(e["tile_m"]), int(e["tile_n"]), int(e["row"]), int(e["col"])) == (1, 0, 17, 99)
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F64


def test_two_faults_in_one_interval_are_uncorrectable(h):
    m = n = k = 512
    A = W.uniform64((m, k), 706, 0)
    B = W.uniform64((k, n), 706, 1)
    sites = np.zeros(2, dtype=F.FAULT_DTYPE)
    sites[0] = (1, 2, 3, 5, 7, W.KIND_ADD, 1e3, 0)
    sites[1] = (1, 2, 9, 40, 100, W.KIND_ADD, 1e3, 0)
    st, C, rep, log = _inject_and_replay(h, A, B, sites)
    assert st == F.UNCORRECTABLE and rep.report.uncorrectable == 1
    e = rep.events[0]
    assert e["kind"] == F.EV_UNCORRECTABLE and e["n_rows"] == 2 and e["n_cols"] == 2


def test_exponent_bit_flips_ragged(h):
    """600 x 500 x 700 N(0,1): 40 flips of exponent bits 52..58 (x or / 2^1 ..
    2^64) at seeded sites, at most one per (tile, interval)."""
    m, n, k = 600, 500, 700
    A = W.normal64((m, k), 707, 0)
    B = W.normal64((k, n), 707, 1)
    sites = W.fault_sites(W.rng(707, W.STREAM_SITES), m, n, k, *CFG, 40, kind=W.KIND_XOR, bits=range(52, 59))
    st, C, rep, log = _inject_and_replay(h, A, B, sites)
    assert rep.report.uncorrectable == 0


def test_detect_only_level(h):
    m, n, k = 384, 256, 512
    A = W.uniform64((m, k), 708, 0)
    B = W.uniform64((k, n), 708, 1)
    sites = np.zeros(2, dtype=F.FAULT_DTYPE)
    sites[0] = (0, 1, 2, 17, 3, W.KIND_ADD, 1e3, 0)
    sites[1] = (2, 0, 20, 100, 120, W.KIND_ADD, -5e2, 0)
    st, C, rep, log = _inject_and_replay(h, A, B, sites, level=F.FT_DETECT)
    assert rep.report.detected == 2 and all(int(e["kind"]) == F.EV_DETECTED for e in rep.events)
    assert rep.report.checks == _checks(m, n, k, F.FT_DETECT)


def test_unsupported_combinations(h):
    import torch
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    with pytest.raises(F.FtgemmError):     # an FP64 handle through the float entry point
        F.ftgemm_run(h, 8, 8, 8, 1.0, d.data_ptr(), 8, d.data_ptr(), 8, 0.0, d.data_ptr(), 8, F.FT_CORRECT, 0.0, s)
    with pytest.raises(F.FtgemmError):     # recompute is not offered for FP64
        F.ftgemm_run_f64(h, 8, 8, 8, 1.0, d.data_ptr(), 8, d.data_ptr(), 8, 0.0, d.data_ptr(), 8,
                         F.FT_CORRECT | F.FT_RECOMPUTE, 0.0, s)
    h32 = F.ftgemm_create(F.F32, 0)
    try:
        with pytest.raises(F.FtgemmError):
            F.ftgemm_run_f64(h32, 8, 8, 8, 1.0, d.data_ptr(), 8, d.data_ptr(), 8, 0.0, d.data_ptr(), 8,
                             F.FT_CORRECT, 0.0, s)
        flip40 = np.zeros(1, dtype=F.FAULT_DTYPE)
        flip40[0] = (0, 0, 0, 0, 0, W.KIND_XOR, 40.0, 0)
        with pytest.raises(F.FtgemmError):  # bit 40 exists only in a 64-bit element
            F.ftgemm_set_injection(h32, flip40)
        F.ftgemm_set_injection(h, flip40)
        F.ftgemm_set_injection(h, None)
    finally:
        F.ftgemm_destroy(h32)


def test_leading_dimensions_and_padding_untouched(h):
    """lda > m, ldb > k, ldc > m: the product lands in C's m x n block, the
    padding rows of C keep their values."""
    import torch
    m, n, k = 200, 150, 100
    lda, ldb, ldc = 256, 128, 240
    A = W.normal64((m, k), 709, 0)
    B = W.normal64((k, n), 709, 1)
    C0 = W.normal64((ldc, n), 709, 2)
    Ap = np.zeros((lda, k)); Ap[:m] = A
    Bp = np.zeros((ldb, n)); Bp[:k] = B
    dA = torch.from_numpy(np.ascontiguousarray(Ap.T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(Bp.T)).cuda()
    dC = torch.from_numpy(np.ascontiguousarray(C0.T)).cuda()
    rep = F.ReportBuffer(16)
    st = F.ftgemm_run_f64(h, m, n, k, 1.0, dA.data_ptr(), lda, dB.data_ptr(), ldb, 0.5, dC.data_ptr(), ldc,
                          F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    C = dC.cpu().numpy().T
    assert st == F.OK and rep.report.n_events == 0
    assert rel_fro(C[:m], O.gemm(A, B, C0[:m], beta=0.5)) <= TOL_F64
    assert np.array_equal(C[m:], C0[m:])


@pytest.mark.parametrize("off_a,off_b,pad", [(1, 0, 0), (0, 1, 0), (1, 1, 2), (0, 0, 1)])
def test_interior_loads_unaligned_operands(h, off_a, off_b, pad):
    """Whole tiles and whole k-steps with A or B starting 8 bytes past a
    16-byte boundary (off_* doubles), or an odd leading dimension (pad = 1):
    the interior panels then take the per-element loads instead of the
    16-byte ones; the product, clean and with one fault per tile, is the
    oracle's either way."""
    import torch
    m, n, k = 256, 256, 96
    lda, ldb, ldc = m + pad, k + pad, m
    A = W.normal64((m, k), 733, 0)
    B = W.normal64((k, n), 733, 1)
    Ap = np.zeros((lda, k)); Ap[:m] = A
    Bp = np.zeros((ldb, n)); Bp[:k] = B
    # device buffers with the operand `off` doubles past the (256-byte aligned) allocation start
    bufA = torch.zeros(off_a + lda * k, dtype=torch.float64, device="cuda")
    bufB = torch.zeros(off_b + ldb * n, dtype=torch.float64, device="cuda")
    bufA[off_a:] = torch.from_numpy(np.ascontiguousarray(Ap.T).reshape(-1)).cuda()
    bufB[off_b:] = torch.from_numpy(np.ascontiguousarray(Bp.T).reshape(-1)).cuda()
    pA = bufA.data_ptr() + 8 * off_a
    pB = bufB.data_ptr() + 8 * off_b
    assert (pA % 16 == 8) == (off_a == 1) and (pB % 16 == 8) == (off_b == 1)
    sites = W.fault_sites(W.rng(733, W.STREAM_SITES), m, n, k, *CFG, 0, payload=1e3, per_tile=1)
    for inj in (None, sites):
        dC = torch.zeros((n, ldc), dtype=torch.float64, device="cuda")
        F.ftgemm_set_injection(h, inj)
        try:
            rep = F.ReportBuffer(64)
            st = F.ftgemm_run_f64(h, m, n, k, 1.0, pA, lda, pB, ldb, 0.0, dC.data_ptr(), ldc, F.FT_CORRECT, 0.0,
                                  torch.cuda.current_stream().cuda_stream, rep)
            log = F.ftgemm_get_injection_log(h) if inj is not None else None
        finally:
            F.ftgemm_set_injection(h, None)
        C = _host(dC, m, n)
        assert st == F.OK
        assert rel_fro(C, O.gemm(A, B)) <= TOL_F64
        if inj is None:
            assert rep.report.n_events == 0
        else:
            assert len(log) == len(sites) == 4
            res, cls, _, bad = replay_against_gpu(A, B, CFG, rep, log, u=O.U_FP64)
            assert bad == 0
            assert event_keys(rep.events) == event_keys(res.events)
            assert rep.report.corrected == 4


def test_full_size_8192_sampled_tiles(h):
    """8192^3 N(0,1) A, B, C, alpha = beta = 1, as benchmarked: a clean run
    raises no event and three sampled tiles (two corners, one inside) match
    the binary64 oracle replay of those tiles; a run with one +1e3 fault per
    tile corrects all 4096 of them, and on the sampled tiles the event log
    equals the replay's and C matches it."""
    m = n = k = 8192
    A = W.normal64((m, k), 64, 0)
    B = W.normal64((k, n), 64, 1)
    C0 = W.normal64((m, n), 64, 2)
    tiles = [(0, 0), (m // CFG[0] - 1, n // CFG[1] - 1), (37, 11)]
    in_sample = lambda e: (int(e["tile_m"]), int(e["tile_n"])) in tiles

    def sample(C):
        return np.concatenate([C[tm * CFG[0]:(tm + 1) * CFG[0], tn * CFG[1]:(tn + 1) * CFG[1]].ravel()
                               for tm, tn in tiles])

    st, C, rep, _ = _run(h, A, B, C0, alpha=1.0, beta=1.0)
    assert st == F.OK and rep.report.n_events == 0 and rep.report.checks == _checks(m, n, k)
    rc = O.ReplayConfig(mc=CFG[0], nc=CFG[1], ku=CFG[2], g=CFG[3], c=float(rep.report.tol_used), u=O.U_FP64)
    clean = O.replay(A, B, rc, C0=C0, alpha=1.0, beta=1.0, tiles=tiles)
    assert clean.n_events == 0
    assert rel_fro(sample(C), sample(clean.C)) <= TOL_F64

    sites = W.fault_sites(W.rng(64, W.STREAM_SITES), m, n, k, *CFG, 0, payload=1e3, per_tile=1)
    st, C, rep, log = _run(h, A, B, C0, alpha=1.0, beta=1.0, sites=sites, cap=8192)
    assert st == F.OK and len(log) == len(sites) == (m // CFG[0]) * (n // CFG[1])
    assert rep.report.corrected == len(sites) and rep.report.uncorrectable == 0
    part = log[np.array([in_sample(l) for l in log], dtype=bool)]
    res, _, _, bad = replay_against_gpu(A, B, CFG, rep, part, C0=C0, alpha=1.0, beta=1.0, tiles=tiles,
                                        u=O.U_FP64)
    assert bad == 0 and len(part) == len(tiles)
    ev = rep.events[np.array([in_sample(e) for e in rep.events], dtype=bool)]
    assert event_keys(ev) == event_keys(res.events)
    assert rel_fro(sample(C), sample(res.C)) <= TOL_F64
