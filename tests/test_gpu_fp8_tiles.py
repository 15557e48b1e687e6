"""GPU tests of the FP8 E4M3 128 x 128 tile (the one automatic selection picks
for smaller problems): clean runs, plain and online, and an exact injection
site log against the oracle on the exactly decoded operands, element by
element.  Per-element bound: (k + 2) u (|A||B|)_ij with the FP8 matrix
instruction's accumulation model u = gpu_util.U_FP8_ACC."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import U_FP8_ACC, elementwise_ratio, event_keys, replay_against_gpu

pytestmark = pytest.mark.gpu
CFG = (128, 128, 64, 4)


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.F8E4M3, 0)
    F.ftgemm_set_config(handle, CFG)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


def _run(h, Ac, Bc, sa, sb, sites=None, level=F.FT_CORRECT, C0=None, alpha=1.0, beta=0.0):
    import torch
    m, k = Ac.shape
    n = Bc.shape[1]
    F.ftgemm_set_scales(h, sa, sb)
    dA = torch.from_numpy(np.ascontiguousarray(Ac.T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(Bc.T)).cuda()
    dC = (torch.from_numpy(np.ascontiguousarray(np.asarray(C0, np.float32).T)).cuda() if C0 is not None
          else torch.zeros((n, m), device="cuda"))
    F.ftgemm_set_injection(h, sites)
    try:
        rep = F.ReportBuffer(4096)
        st = F.ftgemm_run(h, m, n, k, alpha, dA.data_ptr(), m, dB.data_ptr(), k, beta, dC.data_ptr(), m,
                          level, 0.0, torch.cuda.current_stream().cuda_stream, rep)
        log = F.ftgemm_get_injection_log(h) if sites is not None else None
    finally:
        F.ftgemm_set_injection(h, None)
    return st, np.asfortranarray(dC.cpu().numpy().T), rep, log


def _operands(m, n, k, workload):
    Ac, sa = W.quantize_e4m3(W.normal((m, k), workload, 0))
    Bc, sb = W.quantize_e4m3(W.normal((k, n), workload, 1))
    return Ac, sa, Bc, sb, np.asfortranarray(O.decode_e4m3(Ac)), np.asfortranarray(O.decode_e4m3(Bc))


@pytest.mark.parametrize("level", [F.FT_OFF, F.FT_CORRECT])
@pytest.mark.parametrize("shape", [(512, 768, 640), (300, 520, 200), (1000, 37, 999), (1, 1, 1)])
def test_clean_matches_oracle(h, shape, level):
    m, n, k = shape
    Ac, sa, Bc, sb, A, B = _operands(m, n, k, 308)
    C0 = W.normal((m, n), 308, 2)
    st, C, rep, _ = _run(h, Ac, Bc, sa, sb, level=level, C0=C0, alpha=0.5, beta=-1.5)
    assert st == F.OK and rep.report.n_events == 0
    assert rep.report.config.as_tuple() == CFG + CFG[:2]
    ref = O.gemm(A, B, C0, alpha=0.5 * sa * sb, beta=-1.5)
    assert elementwise_ratio(C, ref, A, B, alpha=0.5 * sa * sb, beta=-1.5, C0=C0, acc_u=U_FP8_ACC) <= 1.0


def test_fault_injection_exact_site_log(h):
    m, n, k = 512, 384, 768
    Ac, sa, Bc, sb, A, B = _operands(m, n, k, 309)
    sites = W.fault_sites(W.rng(309, 3), m, n, k, *CFG, 12, payload=1e3 / (sa * sb))
    st, C, rep, log = _run(h, Ac, Bc, sa, sb, sites)
    assert len(log) == 12
    res, cls, n_grey, bad = replay_against_gpu(A, B, CFG, rep, log, alpha=sa * sb)
    assert bad == 0 and np.all(cls["cls"] == O.CLS_MUST)
    assert st == F.OK and rep.report.corrected == 12
    assert event_keys(rep.events) == event_keys(res.events)
    assert elementwise_ratio(C, res.C, A, B, CFG, alpha=sa * sb, events=rep.events, oracle_events=res.events,
                             log=log, acc_u=U_FP8_ACC) <= 1.0
