"""GPU tests of the BF16 128 x 128 tile (the one automatic selection picks
below 3072^3): clean runs and an exact injection site log against the oracle
on the exactly decoded operands.  Bar as for the 256 x 256 BF16 tile: the
FP32-accumulated product within 1e-5 (relative Frobenius) of the oracle's,
and element by element within (k + 2) 2^-24 (|A||B|)_ij (bf16 products are
exact, the accumulation binary32)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import elementwise_ratio, event_keys, rel_fro, replay_against_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5
CFG = (128, 128, 64, 4)


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.BF16, 0)
    F.ftgemm_set_config(handle, CFG)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


def _run(h, Ac, Bc, sa, sb, sites=None):
    import torch
    m, k = Ac.shape
    n = Bc.shape[1]
    F.ftgemm_set_scales(h, sa, sb)
    dA = torch.from_numpy(np.ascontiguousarray(Ac.T).view(np.int16)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(Bc.T).view(np.int16)).cuda()
    dC = torch.zeros((n, m), device="cuda")
    F.ftgemm_set_injection(h, sites)
    try:
        rep = F.ReportBuffer(4096)
        st = F.ftgemm_run(h, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                          F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
        log = F.ftgemm_get_injection_log(h) if sites is not None else None
    finally:
        F.ftgemm_set_injection(h, None)
    return st, np.asfortranarray(dC.cpu().numpy().T), rep, log


def _operands(m, n, k, workload):
    Ac, sa = W.quantize_bf16(W.normal((m, k), workload, 0))
    Bc, sb = W.quantize_bf16(W.normal((k, n), workload, 1))
    return Ac, sa, Bc, sb, np.asfortranarray(O.decode_bf16(Ac)), np.asfortranarray(O.decode_bf16(Bc))


@pytest.mark.parametrize("shape", [(512, 768, 640), (300, 520, 200), (1000, 37, 999), (1, 1, 1)])
def test_clean_matches_oracle(h, shape):
    m, n, k = shape
    Ac, sa, Bc, sb, A, B = _operands(m, n, k, 306)
    st, C, rep, _ = _run(h, Ac, Bc, sa, sb)
    assert st == F.OK and rep.report.n_events == 0
    assert rep.report.config.as_tuple() == CFG + CFG[:2]
    ref = O.gemm(A, B, alpha=sa * sb)
    assert rel_fro(C, ref) <= TOL
    assert elementwise_ratio(C, ref, A, B, alpha=sa * sb) <= 1.0


def test_fault_injection_exact_site_log(h):
    m, n, k = 512, 384, 768
    Ac, sa, Bc, sb, A, B = _operands(m, n, k, 307)
    sites = W.fault_sites(W.rng(307, 3), m, n, k, *CFG, 12, payload=1e3 / (sa * sb))
    st, C, rep, log = _run(h, Ac, Bc, sa, sb, sites)
    assert len(log) == 12
    res, cls, n_grey, bad = replay_against_gpu(A, B, CFG, rep, log, alpha=sa * sb)
    assert bad == 0 and np.all(cls["cls"] == O.CLS_MUST)
    assert st == F.OK and rep.report.corrected == 12
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, O.gemm(A, B, alpha=sa * sb)) <= TOL
    assert elementwise_ratio(C, res.C, A, B, CFG, alpha=sa * sb, events=rep.events, oracle_events=res.events,
                             log=log) <= 1.0
