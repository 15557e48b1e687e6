"""GPU tests of the non-fused ABFT path (ftgemm_run_nonfused: the same
256 x 256 tile checks, as separate launches around the plain FP32 kernel on
k-chunks).  Bar: C equal to the FP64 oracle product within 1e-5 (relative
Frobenius), no event on clean runs, and every injected fault (applied to C
after its chunk's GEMM) corrected at its site, so the event log equals the
injection sites exactly."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import dev, host, rel_fro

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-5
T = 256


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.F32, 0)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


def _run(h, A, B, check_k=0, sites=None):
    import torch
    m, k = A.shape
    n = B.shape[1]
    dA, dB = dev(A), dev(B)
    dC = torch.full((n, m), 7.0, device="cuda")     # beta = 0: the old C must not leak in
    F.ftgemm_set_injection(h, sites)
    try:
        rep = F.ReportBuffer(4096)
        st = F.ftgemm_run_nonfused(h, m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, dC.data_ptr(), m, check_k,
                                   stream=torch.cuda.current_stream().cuda_stream, report=rep)
        log = F.ftgemm_get_injection_log(h) if sites is not None else None
    finally:
        F.ftgemm_set_injection(h, None)
    return st, host(dC, m, n), rep, log


@pytest.mark.parametrize("shape,check_k", [((512, 512, 512), 0), ((300, 520, 200), 64), ((1000, 37, 999), 128),
                                           ((256, 256, 64), 0), ((1, 1, 1), 0)])
def test_clean_matches_oracle(h, shape, check_k):
    m, n, k = shape
    A = W.uniform((m, k), 501, 0)
    B = W.uniform((k, n), 501, 1)
    st, C, rep, _ = _run(h, A, B, check_k)
    assert st == F.OK and rep.report.n_events == 0 and rep.report.detected == 0
    ck = check_k or 256
    assert rep.report.checks == -(-m // T) * -(-n // T) * -(-k // ck)
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32


def test_one_fault_per_tile_corrected_at_its_site(h):
    """2048^3 N(0,1): one additive fault of +-1e4 (far above the threshold,
    ~3e2 at the last check) per tile at a seeded chunk, row and column; the
    event log equals the sites, all corrected."""
    m = n = k = 2048
    A = W.normal((m, k), 502, 0)
    B = W.normal((k, n), 502, 1)
    g = W.rng(502, W.STREAM_SITES)
    ntm, ntn, nch = m // T, n // T, k // 256
    sites = np.zeros(ntm * ntn, dtype=F.FAULT_DTYPE)
    q = 0
    for tm in range(ntm):
        for tn in range(ntn):
            sites[q] = (tm, tn, int(g.integers(0, nch)), int(g.integers(0, T)), int(g.integers(0, T)),
                        W.KIND_ADD, 1e4 if g.integers(0, 2) else -1e4, 0)
            q += 1
    st, C, rep, log = _run(h, A, B, 0, sites)
    assert len(log) == len(sites)
    want = sorted((int(x["tile_m"]), int(x["tile_n"]), int(x["kstep"]), int(x["row"]), int(x["col"]),
                   F.EV_CORRECTED) for x in sites)
    got = sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]), int(e["kind"]))
                 for e in rep.events)
    assert got == want
    assert st == F.OK and rep.report.corrected == len(sites) and rep.report.uncorrectable == 0
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32


def test_two_faults_in_one_chunk_are_uncorrectable(h):
    m = n = k = 512
    A = W.uniform((m, k), 503, 0)
    B = W.uniform((k, n), 503, 1)
    sites = np.zeros(2, dtype=F.FAULT_DTYPE)
    sites[0] = (1, 0, 1, 5, 7, W.KIND_ADD, 1e3, 0)
    sites[1] = (1, 0, 1, 40, 200, W.KIND_ADD, 1e3, 0)
    st, C, rep, log = _run(h, A, B, 0, sites)
    assert st == F.UNCORRECTABLE and rep.report.uncorrectable == 1
    e = rep.events[0]
    assert (int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"])) == (1, 0, 1)
    assert e["kind"] == F.EV_UNCORRECTABLE and e["n_rows"] == 2 and e["n_cols"] == 2
    assert rel_fro(C, O.gemm(A, B)) > 1e-3


def test_unsupported_arguments(h):
    import torch
    m = n = k = 64
    dA, dB = dev(W.uniform((m, k), 504, 0)), dev(W.uniform((k, n), 504, 1))
    dC = torch.zeros((n, m), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for alpha, beta in ((2.0, 0.0), (1.0, 1.0)):
        with pytest.raises(F.FtgemmError):
            F.ftgemm_run_nonfused(h, m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, dC.data_ptr(), m, stream=s,
                                  alpha=alpha, beta=beta)
    rep = F.ReportBuffer(1)
    with pytest.raises(F.FtgemmError):
        F.ftgemm_run_nonfused(h, m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, dC.data_ptr(), m, check_k=-1,
                              stream=s, report=rep)
    assert rep.report.bad_arg == 13
    hb = F.ftgemm_create(F.BF16, 0)
    try:
        with pytest.raises(F.FtgemmError):
            F.ftgemm_run_nonfused(hb, m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, dC.data_ptr(), m, stream=s)
    finally:
        F.ftgemm_destroy(hb)
