"""GPU tests of the wavefront-tile check (warp-level ABFT, section 4.2.2): the
FP32 128x128 tile computed by 2x2 wavefronts checks each wavefront's 64x64
sub-tile against its own encodings and reference checksums.  Events and
fault sites address check
tiles, so the FP64 oracle replays the run with (mc, nc) = the check tile and
the event log, the counts and C are compared exactly as for compute-tile
checks.  Bar: relative Frobenius error <= 1e-5 against the oracle, event
logs equal."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import check_cfg, event_keys, rel_fro, replay_against_gpu, run

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-5
# (m_tile, n_tile, k_step, check_interval, check_m, check_n)
WAVE_CFGS = [(128, 128, 32, 8, 64, 64)]
WAVES = {(128, 128): (2, 2)}


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.F32, 0)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_set_config(handle, None)
    F.ftgemm_destroy(handle)


@pytest.fixture(autouse=True)
def _reset(h):
    yield
    F.ftgemm_set_config(h, None)
    F.ftgemm_set_injection(h, None)


def _inject(h, A, B, cfg, sites, level=F.FT_CORRECT, C0=None, beta=0.0):
    F.ftgemm_set_config(h, cfg)
    F.ftgemm_set_injection(h, sites)
    try:
        st, C, rep = run(h, A, B, C0, beta=beta, ft_level=level)
        log = F.ftgemm_get_injection_log(h)
    finally:
        F.ftgemm_set_injection(h, None)
    res, cls, n_grey, bad = replay_against_gpu(A, B, cfg, rep, log, C0=C0, beta=beta,
                                              ft_level=level & ~F.FT_RECOMPUTE)
    assert bad == 0
    return st, C, rep, log, res, cls


def _n_checks(m, n, k, cfg, level=F.FT_CORRECT):
    cm, cn, ku, g = check_cfg(cfg)
    nk = -(-k // ku)
    per = -(-nk // g) if level == F.FT_CORRECT else 1
    return -(-m // cm) * -(-n // cn) * per


@pytest.mark.parametrize("cfg", WAVE_CFGS)
def test_config_is_reported_with_its_check_shape(h, cfg):
    m = n = k = 256
    A = W.uniform((m, k), 601, 0)
    B = W.uniform((k, n), 601, 1)
    F.ftgemm_set_config(h, cfg)
    st, C, rep = run(h, A, B)
    assert st == F.OK and rep.report.config.as_tuple() == cfg
    assert rep.report.config.check_shape() == cfg[4:]


@pytest.mark.parametrize("cfg", WAVE_CFGS)
@pytest.mark.parametrize("shape", [(512, 512, 512), (300, 520, 200), (1000, 37, 999), (130, 70, 33), (1, 1, 1)])
def test_clean_matches_oracle(h, cfg, shape):
    """No event, one check per (check tile holding part of C, check
    interval), C equal to the FP64 product; ragged edges leave wavefront
    tiles partly or wholly outside C."""
    m, n, k = shape
    A = W.uniform((m, k), 602, 0)
    B = W.uniform((k, n), 602, 1)
    F.ftgemm_set_config(h, cfg)
    st, C, rep = run(h, A, B)
    assert st == F.OK and rep.report.n_events == 0 and rep.report.detected == 0
    assert rep.report.checks == _n_checks(m, n, k, cfg)
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32


@pytest.mark.parametrize("cfg", WAVE_CFGS)
def test_one_fault_per_wave_tile_corrected(h, cfg):
    """1024^3 N(0,1): one +1e3 fault in every wavefront tile at a seeded
    check interval, row and column; each is corrected at its site and the
    event log equals the oracle's at the wavefront tile."""
    m = n = k = 1024
    A = W.normal((m, k), 603, 0)
    B = W.normal((k, n), 603, 1)
    cm, cn, ku, g = check_cfg(cfg)
    sites = W.fault_sites(W.rng(603, W.STREAM_SITES), m, n, k, cm, cn, ku, g, 0, payload=1e3, per_tile=1)
    st, C, rep, log, res, cls = _inject(h, A, B, cfg, sites)
    assert len(log) == len(sites) == (m // cm) * (n // cn)
    assert np.all(cls["cls"] == O.CLS_MUST)
    assert st == F.OK and rep.report.corrected == len(sites) and rep.report.uncorrectable == 0
    assert event_keys(rep.events) == event_keys(res.events)
    assert rep.report.checks == _n_checks(m, n, k, cfg)
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32


def _same_interval_sites(cfg, tiles_m, tiles_n, kstep, g):
    """One +1e3 fault in every wavefront tile of the given compute tiles, all
    at k-step `kstep` (so all in one check interval), at seeded rows/cols."""
    wm, wn = WAVES[cfg[:2]]
    cm, cn = cfg[4], cfg[5]
    rows = []
    for tm in tiles_m:
        for tn in tiles_n:
            for a in range(wm):
                for b in range(wn):
                    rows.append((tm * wm + a, tn * wn + b, kstep, int(g.integers(0, cm)), int(g.integers(0, cn)),
                                 W.KIND_ADD, 1e3, 0))
    sites = np.zeros(len(rows), dtype=F.FAULT_DTYPE)
    for q, r in enumerate(rows):
        sites[q] = r
    return sites


def _to_compute_tile(sites, cfg):
    """The same fault sites in compute-tile coordinates."""
    wm, wn = WAVES[cfg[:2]]
    out = sites.copy()
    out["tile_m"] = sites["tile_m"] // wm
    out["tile_n"] = sites["tile_n"] // wn
    out["row"] = sites["row"] + (sites["tile_m"] % wm) * cfg[4]
    out["col"] = sites["col"] + (sites["tile_n"] % wn) * cfg[5]
    order = np.lexsort((out["kstep"], out["tile_n"], out["tile_m"]))
    return out[order]


@pytest.mark.parametrize("cfg", WAVE_CFGS)
def test_granularity_corrects_what_the_compute_tile_cannot(h, cfg):
    """Every wavefront tile of two compute tiles gets a fault in the same
    check interval.  Wavefront-tile checks correct all of them; the same
    faults under compute-tile checks are several per tile and interval, which
    the oracle and the GPU both classify uncorrectable."""
    m = n = k = 512
    A = W.normal((m, k), 604, 0)
    B = W.normal((k, n), 604, 1)
    sites = _same_interval_sites(cfg, [0, 1], [1], 3, W.rng(604, W.STREAM_SITES))
    st, C, rep, log, res, cls = _inject(h, A, B, cfg, sites)
    assert st == F.OK and rep.report.corrected == len(sites) and rep.report.uncorrectable == 0
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32

    tile_cfg = cfg[:4]
    st, C, rep, log, res, cls = _inject(h, A, B, tile_cfg, _to_compute_tile(sites, cfg))
    assert st == F.UNCORRECTABLE and rep.report.uncorrectable == 2 and rep.report.corrected == 0
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, O.gemm(A, B)) > 1e-3


@pytest.mark.parametrize("cfg", WAVE_CFGS)
def test_uncorrectable_wave_tile_beside_corrected_ones(h, cfg):
    """Two faults in one wavefront tile within one interval (uncorrectable
    there) and one fault in each of two other wavefront tiles of the same
    compute tile in that interval (corrected): the outcome is per check
    tile."""
    m = n = k = 512
    A = W.uniform((m, k), 605, 0)
    B = W.uniform((k, n), 605, 1)
    rows = [(1, 2, 4, 5, 7, W.KIND_ADD, 1e3, 0), (1, 2, 4, 40, 30, W.KIND_ADD, 1e3, 0),
            (0, 2, 4, 17, 3, W.KIND_ADD, -1e3, 0), (1, 3, 5, 60, 11, W.KIND_ADD, 1e3, 0)]
    sites = np.zeros(len(rows), dtype=F.FAULT_DTYPE)
    for q, r in enumerate(rows):
        sites[q] = r
    st, C, rep, log, res, cls = _inject(h, A, B, cfg, sites)
    assert st == F.UNCORRECTABLE
    assert rep.report.uncorrectable == 1 and rep.report.corrected == 2
    assert event_keys(rep.events) == event_keys(res.events)
    bad = [e for e in rep.events if e["kind"] == F.EV_UNCORRECTABLE][0]
    assert (int(bad["tile_m"]), int(bad["tile_n"]), int(bad["n_rows"]), int(bad["n_cols"])) == (1, 2, 2, 2)
    assert rel_fro(C, res.C) <= TOL_F32


@pytest.mark.parametrize("cfg", WAVE_CFGS)
def test_detect_only_with_recompute(h, cfg):
    """Detect-only level on wavefront tiles: one DETECTED event per flagged
    wavefront tile (after the last k-step); every compute tile holding one is
    recomputed and C is the clean product."""
    m, n, k = 768, 512, 640
    A = W.uniform((m, k), 606, 0)
    B = W.uniform((k, n), 606, 1)
    rows = [(0, 1, 2, 17, 3, W.KIND_ADD, 1e3, 0), (0, 2, 9, 5, 5, W.KIND_ADD, 1e3, 0),
            (3, 0, 15, 60, 20, W.KIND_ADD, -5e2, 0)]
    sites = np.zeros(len(rows), dtype=F.FAULT_DTYPE)
    for q, r in enumerate(rows):
        sites[q] = r
    wm, wn = WAVES[cfg[:2]]
    tiles = {(r[0] // wm, r[1] // wn) for r in rows}
    st, C, rep, log, res, cls = _inject(h, A, B, cfg, sites, level=F.FT_DETECT | F.FT_RECOMPUTE)
    assert event_keys(rep.events) == event_keys(res.events)
    assert all(int(e["kind"]) == F.EV_DETECTED for e in rep.events) and rep.report.detected == 3
    # counted on the device, the recompute launch's checks included (each recomputed compute
    # tile checks its wave tiles once more)
    wm, wn = WAVES[cfg[:2]]
    assert rep.report.checks == _n_checks(m, n, k, cfg, F.FT_DETECT) + rep.report.recomputed * wm * wn
    assert rep.report.recomputed == len(tiles) and rep.report.recompute_failed == 0
    assert st == F.OK and rel_fro(C, O.gemm(A, B)) <= TOL_F32


@pytest.mark.parametrize("cfg", WAVE_CFGS)
def test_many_bit_flips_ragged(h, cfg):
    """700 x 600 x 900 N(0,1): 120 bit flips (bits 20..30) at seeded sites, at
    most one per (wavefront tile, interval); flips whose effect lies near the
    threshold take the GPU's decision if it is a valid one, the rest must
    match the oracle exactly."""
    m, n, k = 700, 600, 900
    A = W.normal((m, k), 607, 0)
    B = W.normal((k, n), 607, 1)
    cm, cn, ku, g = check_cfg(cfg)
    sites = W.fault_sites(W.rng(607, W.STREAM_SITES), m, n, k, cm, cn, ku, g, 120, kind=W.KIND_XOR,
                          bits=range(20, 31))
    st, C, rep, log, res, cls = _inject(h, A, B, cfg, sites)
    assert len(log) == 120
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, res.C) <= TOL_F32


@pytest.mark.parametrize("cfg", WAVE_CFGS)
def test_alpha_beta_with_faults(h, cfg):
    """alpha = 0.5, beta = -1.25 with C0: one fault in each of three
    wavefront tiles; the oracle replay with the same alpha, beta and C0 gives
    the same events and C."""
    m, n, k = 384, 320, 416
    A = W.uniform((m, k), 610, 0)
    B = W.uniform((k, n), 610, 1)
    C0 = W.uniform((m, n), 610, 2)
    rows = [(0, 0, 2, 3, 4, W.KIND_ADD, 1e3, 0), (3, 2, 7, 60, 1, W.KIND_ADD, -1e3, 0),
            (5, 4, 12, 10, 63, W.KIND_ADD, 1e3, 0)]
    sites = np.zeros(len(rows), dtype=F.FAULT_DTYPE)
    for q, r in enumerate(rows):
        sites[q] = r
    F.ftgemm_set_config(h, cfg)
    F.ftgemm_set_injection(h, sites)
    try:
        st, C, rep = run(h, A, B, C0, alpha=0.5, beta=-1.25)
        log = F.ftgemm_get_injection_log(h)
    finally:
        F.ftgemm_set_injection(h, None)
    res, cls, n_grey, bad = replay_against_gpu(A, B, cfg, rep, log, C0=C0, alpha=0.5, beta=-1.25)
    assert bad == 0 and st == F.OK and rep.report.corrected == 3
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, O.gemm(A, B, C0, alpha=0.5, beta=-1.25)) <= TOL_F32


def test_sites_outside_their_check_tile_are_not_applied(h):
    """A site whose row or column lies beyond its wavefront tile addresses no
    element of it: nothing is applied, nothing is flagged."""
    cfg = WAVE_CFGS[0]
    m = n = k = 512
    A = W.uniform((m, k), 608, 0)
    B = W.uniform((k, n), 608, 1)
    sites = np.zeros(2, dtype=F.FAULT_DTYPE)
    sites[0] = (0, 0, 1, cfg[4], 0, W.KIND_ADD, 1e3, 0)
    sites[1] = (1, 1, 1, 0, cfg[5], W.KIND_ADD, 1e3, 0)
    F.ftgemm_set_config(h, cfg)
    F.ftgemm_set_injection(h, sites)
    st, C, rep = run(h, A, B)
    log = F.ftgemm_get_injection_log(h)
    assert st == F.OK and len(log) == 0 and rep.report.n_events == 0
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32


def test_graph_replays_match_eager(h):
    """The wavefront-check variant without report captured into a HIP graph:
    several replays, with eager work between them, reproduce the eager C."""
    import torch
    from gpu_util import dev, host
    cfg = WAVE_CFGS[0]
    m = n = k = 512
    A = W.uniform((m, k), 609, 0)
    B = W.uniform((k, n), 609, 1)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((n, m), device="cuda")
    F.ftgemm_set_config(h, cfg)

    def call():
        return F.ftgemm_run(h, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                            F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, None)
    assert call() == F.OK
    torch.cuda.synchronize()
    eager = host(dC, m, n).copy()
    assert rel_fro(eager, O.gemm(A, B)) <= TOL_F32
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    for r in range(3):
        dC.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(dC, m, n), eager), r
        x = torch.randn(1024, 1024, device="cuda")
        (x @ x).sum().item()
    del graph


@pytest.mark.parametrize("cfg", WAVE_CFGS)
def test_full_size_8192_one_fault_per_wave_tile(h, cfg):
    """8192^3 N(0,1), beta = 1, in the configuration the granularity benchmark
    times: one +1e5 fault in each of the 16384 wavefront tiles (must-detect at
    every k-step: the bound at full K is about 1e3 for 64 N(0,1) columns;
    16384 events and log entries fill the handle's device logs exactly);
    all are corrected, and on three sampled wavefront tiles the event log
    equals the oracle replay's and C matches it."""
    m = n = k = 8192
    A = W.normal((m, k), 2, W.STREAM_A)
    B = W.normal((k, n), 2, W.STREAM_B)
    C0 = W.normal((m, n), 2, W.STREAM_C)
    cm, cn, ku, g = check_cfg(cfg)
    sites = W.fault_sites(W.rng(8192, 64), m, n, k, cm, cn, ku, g, 0, payload=1e5, per_tile=1)
    F.ftgemm_set_config(h, cfg)
    F.ftgemm_set_injection(h, sites)
    try:
        st, C, rep = run(h, A, B, C0, beta=1.0, cap=32768)
        log = F.ftgemm_get_injection_log(h, 32768)
    finally:
        F.ftgemm_set_injection(h, None)
    assert st == F.OK and len(log) == len(sites) == (m // cm) * (n // cn)
    assert rep.report.corrected == len(sites) and rep.report.uncorrectable == 0
    assert rep.report.checks == _n_checks(m, n, k, cfg)
    tiles = [(0, 0), (m // cm - 1, n // cn - 1), (37, 90)]
    in_sample = lambda e: (int(e["tile_m"]), int(e["tile_n"])) in tiles
    part = log[np.array([in_sample(l) for l in log], dtype=bool)]
    res, cls, _, bad = replay_against_gpu(A, B, cfg, rep, part, C0=C0, beta=1.0, tiles=tiles)
    assert bad == 0 and len(part) == len(tiles)
    assert np.all(cls["cls"] == O.CLS_MUST)
    ev = rep.events[np.array([in_sample(e) for e in rep.events], dtype=bool)]
    assert event_keys(ev) == event_keys(res.events)
    for (tm, tn) in tiles:
        sl = (slice(tm * cm, (tm + 1) * cm), slice(tn * cn, (tn + 1) * cn))
        assert rel_fro(C[sl], res.C[sl]) <= TOL_F32, (tm, tn)
