"""GPU parity of the FP32 online ABFT GEMM against the FP64 oracle, through the
C ABI.  Bar: relative Frobenius error <= 1e-5 for FP32 results; event logs
(tile, k-step, row, col, kind) equal to the oracle's replay exactly, with
must-detect faults always corrected, benign ones never flagged, and no event
anywhere else."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import corrected_value_errors, elementwise_ratio, event_keys, replay_against_gpu, rel_fro, run

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-5
VARIANTS = [(256, 256, 32), (256, 128, 32), (128, 256, 32), (128, 128, 32), (64, 64, 32)]


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.F32, 0)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


@pytest.fixture(autouse=True)
def _reset(h):
    F.ftgemm_set_config(h, None)
    F.ftgemm_set_injection(h, None)
    yield


# ---------------------------------------------------------------------------
# clean runs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(256, 256, 256), (300, 200, 130), (513, 769, 257), (64, 64, 32),
                                   (1, 1, 1), (1000, 37, 999), (33, 1500, 70), (2048, 2048, 512)])
@pytest.mark.parametrize("level", [F.FT_OFF, F.FT_DETECT, F.FT_CORRECT])
def test_clean_matches_oracle(h, shape, level):
    m, n, k = shape
    A = W.uniform((m, k), 200, 0)
    B = W.uniform((k, n), 200, 1)
    st, C, rep = run(h, A, B, ft_level=level)
    ref = O.gemm(A, B)
    assert st == F.OK
    assert rel_fro(C, ref) <= TOL_F32
    assert elementwise_ratio(C, ref, A, B) <= 1.0
    assert rep.report.n_events == 0 and rep.report.detected == 0


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("g", [1, 3])
def test_every_variant_ragged_alpha_beta(h, variant, g):
    m, n, k = 300, 520, 200   # ragged in m, n and the last k-step
    A = W.normal((m, k), 201, 0)
    B = W.normal((k, n), 201, 1)
    C0 = W.normal((m, n), 201, 2)
    F.ftgemm_set_config(h, (*variant, g))
    st, C, rep = run(h, A, B, C0, alpha=0.5, beta=-1.5)
    assert st == F.OK and rep.report.config.as_tuple()[:4] == (*variant, g)
    assert rep.report.config.check_shape() == tuple(variant[:2])
    ref = O.gemm(A, B, C0, alpha=0.5, beta=-1.5)
    assert rel_fro(C, ref) <= TOL_F32
    assert elementwise_ratio(C, ref, A, B, alpha=0.5, beta=-1.5, C0=C0) <= 1.0
    assert rep.report.n_events == 0
    nt = -(-m // variant[0]) * -(-n // variant[1])
    assert rep.report.checks == nt * -(-(-(-k // variant[2])) // g)   # counted on the device


def test_integer_operands_are_exact(h):
    """Small-integer operands make every partial sum exact: bitwise equality."""
    A = W.integers((333, 777), 202, 0)
    B = W.integers((777, 555), 202, 1)
    st, C, rep = run(h, A, B)
    assert st == F.OK and rep.report.n_events == 0
    assert np.array_equal(C.astype(np.float64), O.gemm(A, B))


def test_unaligned_leading_dimensions(h):
    """lda, ldb, ldc not multiples of 4 take the element-wise load path."""
    import torch
    m, n, k = 301, 203, 157
    A = W.normal((m, k), 203, 0)
    B = W.normal((k, n), 203, 1)
    lda, ldb, ldc = m + 3, k + 1, m + 5
    Ab = np.zeros((lda, k), np.float32, order="F"); Ab[:m] = A
    Bb = np.zeros((ldb, n), np.float32, order="F"); Bb[:k] = B
    dA = torch.from_numpy(np.ascontiguousarray(Ab.T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(Bb.T)).cuda()
    dC = torch.full((n, ldc), 7.0, device="cuda")
    rep = F.ReportBuffer(16)
    st = F.ftgemm_run(h, m, n, k, 1.0, dA.data_ptr(), lda, dB.data_ptr(), ldb, 0.0, dC.data_ptr(), ldc,
                      F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    Cb = dC.cpu().numpy().T
    assert st == F.OK and rep.report.n_events == 0
    assert rel_fro(Cb[:m], O.gemm(A, B)) <= TOL_F32
    assert np.all(Cb[m:] == 7.0)   # padding rows untouched


def test_blas_quick_returns(h):
    A = W.normal((40, 30), 204, 0)
    B = W.normal((30, 50), 204, 1)
    C0 = W.normal((40, 50), 204, 2)
    st, C, _ = run(h, A[:, :0], B[:0, :], C0, alpha=1.0, beta=2.0)           # k = 0
    assert st == F.OK and np.array_equal(C, 2.0 * C0)
    st, C, _ = run(h, A, B, C0, alpha=0.0, beta=-1.0)                       # alpha = 0
    assert st == F.OK and np.array_equal(C, -C0)
    st, C, _ = run(h, A, B, np.full((40, 50), np.nan, np.float32), beta=0.0)  # C not read
    assert st == F.OK and np.isfinite(C).all()
    st, C, _ = run(h, A[:0], B)                                             # m = 0
    assert st == F.OK and C.shape == (0, 50)


def test_bad_arguments_report_position(h):
    rep = F.ReportBuffer(4)
    st = F.lib().ftgemm_run(h, 8, 8, 8, 1.0, None, 4, None, 8, 0.0, None, 8, 2, 0.0, None, rep.ptr())
    assert st == F.INVALID and rep.report.bad_arg == 7


def test_repeat_runs_are_bitwise_identical(h):
    A = W.normal((1024, 1024), 205, 0)
    B = W.normal((1024, 1024), 205, 1)
    outs = [run(h, A, B)[1] for _ in range(4)]
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_determinism_canary_8192(h):
    """Twenty clean online runs of the benchmarked 8192^3 configuration give
    bitwise the same C (compared on the device)."""
    import torch
    m = n = k = 8192
    A = torch.from_numpy(np.ascontiguousarray(W.normal((m, k), 2, W.STREAM_A).T)).cuda()
    B = torch.from_numpy(np.ascontiguousarray(W.normal((k, n), 2, W.STREAM_B).T)).cuda()
    C0 = torch.from_numpy(np.ascontiguousarray(W.normal((m, n), 2, W.STREAM_C).T)).cuda()
    s = torch.cuda.current_stream().cuda_stream
    first = None
    for r in range(20):
        C = C0.clone()
        st = F.ftgemm_run(h, m, n, k, 1.0, A.data_ptr(), m, B.data_ptr(), k, 1.0, C.data_ptr(), m,
                          F.FT_CORRECT, 0.0, s, None)
        assert st == F.OK
        if first is None:
            first = C
        else:
            assert torch.equal(first, C), r


def test_repeat_runs_with_corrections(h):
    """Ten runs with the same faults: the event log and every element no
    correction touched are bitwise the same; a corrected element is rebuilt
    from a row checksum whose cross-wave sum of B e may add in a different
    order, so it is compared within beta_row of the oracle's."""
    m, n, k = 1024, 1024, 1024
    A = W.normal((m, k), 213, 0)
    B = W.normal((k, n), 213, 1)
    cfg = (256, 256, 32, 8)
    sites = W.fault_sites(W.rng(213, 3), m, n, k, 256, 256, 32, 8, 0, payload=1e4, per_tile=1)
    F.ftgemm_set_config(h, cfg)
    F.ftgemm_set_injection(h, sites)
    runs = [run(h, A, B) for _ in range(10)]
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    keys = [event_keys(r[2].events) for r in runs]
    assert all(kk == keys[0] for kk in keys) and len(keys[0]) == 16
    mask = np.ones((m, n), dtype=bool)
    for e in runs[0][2].events:
        mask[int(e["tile_m"]) * 256 + int(e["row"]), int(e["tile_n"]) * 256 + int(e["col"])] = False
    for r in runs[1:]:
        assert np.array_equal(r[1][mask], runs[0][1][mask])
    res, cls, _, bad = replay_against_gpu(A, B, cfg, runs[0][2], log)
    for st, C, rep in runs:
        assert corrected_value_errors(rep.events, res.events, rep.report.tol_used)[0] <= 1.0


# ---------------------------------------------------------------------------
# fault injection
# ---------------------------------------------------------------------------
def _inject(h, A, B, cfg, sites, C0=None, alpha=1.0, beta=0.0, level=F.FT_CORRECT, tiles=None):
    F.ftgemm_set_config(h, cfg)
    F.ftgemm_set_injection(h, sites)
    st, C, rep = run(h, A, B, C0, alpha=alpha, beta=beta, ft_level=level)
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    res, cls, n_grey, bad = replay_against_gpu(A, B, cfg, rep, log, C0=C0, alpha=alpha, beta=beta,
                                              ft_level=level, tiles=tiles)
    return st, C, rep, log, res, cls, n_grey, bad


def test_one_additive_fault_per_tile_256(h):
    """256^3, U[-1,1], 128 x 128 check tiles, a check after every k-step,
    one +1e3 fault per tile at a seeded (k-step, row, col)."""
    m = n = k = 256
    A = W.uniform((m, k), 1, W.STREAM_A)
    B = W.uniform((k, n), 1, W.STREAM_B)
    cfg = (128, 128, 32, 1)
    sites = W.fault_sites(W.rng(1, W.STREAM_SITES), m, n, k, 128, 128, 32, 1, 0, payload=1e3, per_tile=1)
    st, C, rep, log, res, cls, n_grey, bad = _inject(h, A, B, cfg, sites)
    assert len(log) == 4 and np.all(cls["cls"] == O.CLS_MUST)
    assert st == F.OK and rep.report.corrected == 4 and rep.report.detected == 4
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, res.C) <= TOL_F32
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32     # all corrected: the clean product
    assert elementwise_ratio(C, res.C, A, B, cfg, events=rep.events, oracle_events=res.events, log=log) <= 1.0
    worst, ncmp = corrected_value_errors(rep.events, res.events, rep.report.tol_used)
    assert ncmp == 4 and worst <= 1.0
    assert rep.report.checks == 4 * 8


@pytest.mark.parametrize("cfg", [(128, 128, 32, 1), (256, 256, 32, 4), (64, 64, 32, 2)])
def test_many_faults_across_tiles_and_intervals(h, cfg):
    m, n, k = 700, 600, 900
    A = W.normal((m, k), 206, 0)
    B = W.normal((k, n), 206, 1)
    nk = -(-k // cfg[2])
    nint = -(-nk // cfg[3])
    ntiles = -(-m // cfg[0]) * -(-n // cfg[1])
    count = min(ntiles * nint, 120)
    sites = W.fault_sites(W.rng(206, 3), m, n, k, cfg[0], cfg[1], cfg[2], cfg[3], count, payload=-5e2)
    st, C, rep, log, res, cls, n_grey, bad = _inject(h, A, B, cfg, sites)
    assert len(log) == count and np.all(cls["cls"] == O.CLS_MUST)
    assert st == F.OK and rep.report.corrected == count
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32
    assert elementwise_ratio(C, res.C, A, B, cfg, events=rep.events, oracle_events=res.events, log=log) <= 1.0
    worst, ncmp = corrected_value_errors(rep.events, res.events, rep.report.tol_used)
    assert ncmp == count and worst <= 1.0


@pytest.mark.parametrize("bits", [range(23, 31), range(0, 31)])
def test_bit_flips_exact_site_log(h, bits):
    """Bit flips in accumulator lanes: must-detect flips are corrected at
    their site, benign flips never flagged, grey flips take either outcome
    (the oracle then follows the GPU), and no event appears elsewhere."""
    m, n, k = 1024, 768, 1024
    A = W.normal((m, k), 207, 0)
    B = W.normal((k, n), 207, 1)
    cfg = (128, 128, 32, 8)
    sites = W.fault_sites(W.rng(207, 3), m, n, k, 128, 128, 32, 8, 150, kind=W.KIND_XOR, bits=bits)
    st, C, rep, log, res, cls, n_grey, bad = _inject(h, A, B, cfg, sites)
    assert len(log) == 150 and bad == 0
    must = int(np.sum(cls["cls"] == O.CLS_MUST))
    assert rep.report.corrected >= must
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, res.C) <= TOL_F32
    assert elementwise_ratio(C, res.C, A, B, cfg, events=rep.events, oracle_events=res.events, log=log) <= 1.0
    assert corrected_value_errors(rep.events, res.events, rep.report.tol_used)[0] <= 1.0
    if bits == range(23, 31):
        assert must > 0


def test_two_faults_in_one_interval_are_uncorrectable(h):
    m = n = k = 256
    A = W.uniform((m, k), 208, 0)
    B = W.uniform((k, n), 208, 1)
    sites = np.zeros(2, dtype=F.FAULT_DTYPE)
    sites[0] = (0, 1, 3, 5, 7, W.KIND_ADD, 1e3, 0)
    sites[1] = (0, 1, 3, 9, 2, W.KIND_ADD, 1e3, 0)
    st, C, rep, log, res, cls, n_grey, bad = _inject(h, A, B, (128, 128, 32, 1), sites)
    assert st == F.UNCORRECTABLE and rep.report.uncorrectable == 1
    assert event_keys(rep.events) == event_keys(res.events)
    assert rep.events[0]["n_rows"] == 2 and rep.events[0]["n_cols"] == 2
    assert rel_fro(C, res.C) <= TOL_F32


def test_detect_only_level(h):
    m = n = k = 256
    A = W.uniform((m, k), 209, 0)
    B = W.uniform((k, n), 209, 1)
    sites = W.fault_sites(W.rng(209, 3), m, n, k, 128, 128, 32, 8, 0, payload=1e3, per_tile=1)
    st, C, rep, log, res, cls, n_grey, bad = _inject(h, A, B, (128, 128, 32, 1), sites, level=F.FT_DETECT)
    assert rep.report.detected == 4 and rep.report.corrected == 0
    assert all(e["kind"] == F.EV_DETECTED and e["kstep"] == 7 for e in rep.events)
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, res.C) <= TOL_F32


def test_level_off_leaves_faults_in_C(h):
    m = n = k = 256
    A = W.uniform((m, k), 210, 0)
    B = W.uniform((k, n), 210, 1)
    sites = W.fault_sites(W.rng(210, 3), m, n, k, 128, 128, 32, 1, 0, payload=1e3, per_tile=1)
    st, C, rep, log, res, cls, n_grey, bad = _inject(h, A, B, (128, 128, 32, 1), sites, level=F.FT_OFF)
    assert rep.report.n_events == 0 and len(log) == 4
    assert rel_fro(C, res.C) <= TOL_F32
    assert rel_fro(C, O.gemm(A, B)) > 1e-3


# ---------------------------------------------------------------------------
# full size, launch configuration of the benchmark, sampled tiles
# ---------------------------------------------------------------------------
def test_full_size_8192_sampled_tiles(h):
    """8192^3, N(0,1), beta = 1, automatic configuration (as benchmarked):
    no event in a clean run, and three sampled tiles (corners and one inside)
    match the oracle replay of those tiles."""
    m = n = k = 8192
    A = W.normal((m, k), 2, W.STREAM_A)
    B = W.normal((k, n), 2, W.STREAM_B)
    C0 = W.normal((m, n), 2, W.STREAM_C)
    st, C, rep = run(h, A, B, C0, alpha=1.0, beta=1.0)
    cfg = rep.report.config.as_tuple()
    assert st == F.OK and rep.report.n_events == 0 and cfg[:2] == (256, 256)
    tiles = [(0, 0), (m // cfg[0] - 1, n // cfg[1] - 1), (13, 21)]
    rc = O.ReplayConfig(mc=cfg[0], nc=cfg[1], ku=cfg[2], g=cfg[3])
    res = O.replay(A, B, rc, C0=C0, alpha=1.0, beta=1.0, tiles=tiles)
    assert res.n_events == 0
    for (tm, tn) in tiles:
        sl = (slice(tm * cfg[0], (tm + 1) * cfg[0]), slice(tn * cfg[1], (tn + 1) * cfg[1]))
        assert rel_fro(C[sl], res.C[sl]) <= TOL_F32, (tm, tn)
        assert elementwise_ratio(C, res.C, A, B, cfg, alpha=1.0, beta=1.0, C0=C0, tile=(tm, tn)) <= 1.0
    assert rep.report.checks == 1024 * 32


def test_full_size_8192_one_fault_per_tile(h):
    """8192^3 N(0,1), beta = 1, automatic configuration, one +1e5 fault in
    every one of the 1024 tiles at a seeded k-step, row and column: the oracle
    replays every tile with the same faults and threshold constant, classes
    every fault must-detect, and its event log equals the GPU's; C equals the
    replay element by element within the accumulation bound (corrected
    elements within beta_row), and every corrected value is within beta_row
    of the replay's.  At this size the bound passes 1e3 about half way
    through K (c 2u (K'+n+1) |a_i| sum_j |b_j| ~ 4e3 at K' = 8192 with c = 2
    and 256 N(0,1) columns), so a +1e3 fault in the second half lies inside
    the rounding bound and is left alone by design (465 of 1024 were
    corrected in a run with that payload)."""
    m = n = k = 8192
    A = W.normal((m, k), 2, W.STREAM_A)
    B = W.normal((k, n), 2, W.STREAM_B)
    C0 = W.normal((m, n), 2, W.STREAM_C)
    cfg = F.ftgemm_select_config(F.F32, m, n, k).as_tuple()
    assert cfg[:2] == (256, 256)
    sites = W.fault_sites(W.rng(8192, W.STREAM_SITES), m, n, k, *cfg[:4], 0, payload=1e5, per_tile=1)
    F.ftgemm_set_injection(h, sites)
    st, C, rep = run(h, A, B, C0, alpha=1.0, beta=1.0)
    log = F.ftgemm_get_injection_log(h)
    assert st == F.OK and rep.report.config.as_tuple()[:4] == cfg[:4]
    assert len(log) == len(sites) == 1024
    assert rep.report.corrected == 1024 and rep.report.uncorrectable == 0
    assert rep.report.checks == 1024 * 32
    res, cls, _, bad = replay_against_gpu(A, B, cfg, rep, log, C0=C0, alpha=1.0, beta=1.0)
    assert bad == 0 and np.all(cls["cls"] == O.CLS_MUST)
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, res.C) <= TOL_F32
    ratio = elementwise_ratio(C, res.C, A, B, cfg, alpha=1.0, beta=1.0, C0=C0, events=rep.events,
                              oracle_events=res.events, log=log)
    worst, ncmp = corrected_value_errors(rep.events, res.events, rep.report.tol_used)
    print(f"\n[8192 fault per tile] element-wise ratio {ratio:.3e}, corrected values {worst:.3e} of beta_row")
    assert ratio <= 1.0 and ncmp == 1024 and worst <= 1.0


def test_full_size_8192_bit_flips_exact_site_log(h):
    """8192^3 N(0,1), beta = 1, automatic configuration, 64 bit flips in
    bits 0..30 (the benchmark's injection model): the oracle replays every
    tile that holds a fault, classifying each (must-detect, benign, grey);
    the GPU's event log equals the replay's, no other tile raises an event,
    and C on the replayed tiles matches."""
    m = n = k = 8192
    A = W.normal((m, k), 2, W.STREAM_A)
    B = W.normal((k, n), 2, W.STREAM_B)
    C0 = W.normal((m, n), 2, W.STREAM_C)
    cfg = F.ftgemm_select_config(F.F32, m, n, k).as_tuple()
    sites = W.fault_sites(W.rng(8193, W.STREAM_SITES), m, n, k, *cfg[:4], 64, kind=W.KIND_XOR)
    F.ftgemm_set_injection(h, sites)
    st, C, rep = run(h, A, B, C0, alpha=1.0, beta=1.0)
    log = F.ftgemm_get_injection_log(h)
    assert st == F.OK and len(log) == len(sites) == 64
    tiles = sorted({(int(s["tile_m"]), int(s["tile_n"])) for s in sites})
    res, cls, _, bad = replay_against_gpu(A, B, cfg, rep, log, C0=C0, alpha=1.0, beta=1.0, tiles=tiles)
    assert bad == 0
    assert event_keys(rep.events) == event_keys(res.events)
    assert all((int(e["tile_m"]), int(e["tile_n"])) in tiles for e in rep.events)
    assert rep.report.corrected >= int(np.sum(cls["cls"] == O.CLS_MUST))
    assert corrected_value_errors(rep.events, res.events, rep.report.tol_used)[0] <= 1.0
    for (tm, tn) in tiles:
        sl = (slice(tm * cfg[0], (tm + 1) * cfg[0]), slice(tn * cfg[1], (tn + 1) * cfg[1]))
        assert rel_fro(C[sl], res.C[sl]) <= TOL_F32, (tm, tn)
        assert elementwise_ratio(C, res.C, A, B, cfg, alpha=1.0, beta=1.0, C0=C0, events=rep.events,
                                 oracle_events=res.events, log=log, tile=(tm, tn)) <= 1.0, (tm, tn)
