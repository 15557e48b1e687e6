"""GPU parity of the BF16-input online ABFT GEMM (FP32 accumulation, FP32
checksums on the exactly decoded operands) against the FP64 oracle on the
same bf16 values.  Bar: relative Frobenius error <= 2e-2 against the oracle
on the quantised operands (the stated bound for BF16); event logs equal to
the oracle replay's exactly."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import event_keys, rel_fro, replay_against_gpu

pytestmark = pytest.mark.gpu
TOL_BF16 = 2e-2


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.BF16, 0)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


@pytest.fixture(autouse=True)
def _reset(h):
    F.ftgemm_set_config(h, None)
    F.ftgemm_set_injection(h, None)
    F.ftgemm_set_scales(h, 1.0, 1.0)
    yield


def _dev_codes(codes):
    import torch
    return torch.from_numpy(np.ascontiguousarray(codes.T).view(np.int16)).cuda()


def _run(h, Ac, Bc, C0=None, alpha=1.0, beta=0.0, level=F.FT_CORRECT, cap=16384):
    import torch
    m, k = Ac.shape
    n = Bc.shape[1]
    dA, dB = _dev_codes(Ac), _dev_codes(Bc)
    dC = (torch.from_numpy(np.ascontiguousarray(np.asarray(C0, np.float32).T)).cuda() if C0 is not None
          else torch.zeros((n, m), device="cuda"))
    rep = F.ReportBuffer(cap)
    st = F.ftgemm_run(h, m, n, k, alpha, dA.data_ptr(), m, dB.data_ptr(), k, beta, dC.data_ptr(), m,
                      level, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    return st, np.asfortranarray(dC.cpu().numpy().T), rep


def _oracle_inputs(Ac, Bc):
    return np.asfortranarray(O.decode_bf16(Ac)), np.asfortranarray(O.decode_bf16(Bc))


@pytest.mark.parametrize("shape", [(256, 256, 64), (512, 768, 640), (300, 520, 200), (1000, 37, 999), (1, 1, 1)])
def test_clean_matches_oracle(h, shape):
    m, n, k = shape
    Ac, _ = W.quantize_bf16(W.normal((m, k), 300, 0))
    Bc, _ = W.quantize_bf16(W.normal((k, n), 300, 1))
    A, B = _oracle_inputs(Ac, Bc)
    st, C, rep = _run(h, Ac, Bc)
    ref = O.gemm(A, B)
    assert st == F.OK and rep.report.n_events == 0
    err = rel_fro(C, ref)
    assert err <= TOL_BF16
    assert err <= 1e-5, err    # exact products, FP32 accumulation


def test_integer_operands_exact(h):
    Ac, _ = W.quantize_bf16(W.integers((320, 448), 301, 0))
    Bc, _ = W.quantize_bf16(W.integers((448, 288), 301, 1))
    A, B = _oracle_inputs(Ac, Bc)
    st, C, rep = _run(h, Ac, Bc)
    assert st == F.OK and rep.report.n_events == 0
    assert np.array_equal(C.astype(np.float64), O.gemm(A, B))


def test_scales_alpha_beta_ragged(h):
    m, n, k = 300, 520, 200
    Ac, _ = W.quantize_bf16(W.normal((m, k), 302, 0))
    Bc, _ = W.quantize_bf16(W.normal((k, n), 302, 1))
    C0 = W.normal((m, n), 302, 2)
    A, B = _oracle_inputs(Ac, Bc)
    F.ftgemm_set_scales(h, 2.0, 0.25)
    st, C, rep = _run(h, Ac, Bc, C0, alpha=1.5, beta=-0.5)
    assert st == F.OK and rep.report.n_events == 0
    assert rel_fro(C, O.gemm(A, B, C0, alpha=1.5 * 2.0 * 0.25, beta=-0.5)) <= 1e-5


def test_heavy_tailed_clean_no_false_positive(h):
    m = n = k = 1024
    Ac, _ = W.quantize_bf16(W.heavy_tailed((m, k), 4, W.STREAM_A))
    Bc, _ = W.quantize_bf16(W.heavy_tailed((k, n), 4, W.STREAM_B))
    A, B = _oracle_inputs(Ac, Bc)
    st, C, rep = _run(h, Ac, Bc)
    assert st == F.OK and rep.report.n_events == 0
    assert rel_fro(C, O.gemm(A, B)) <= 1e-5


@pytest.mark.parametrize("kind", [W.KIND_ADD, W.KIND_XOR])
def test_fault_injection_exact_site_log(h, kind):
    m, n, k = 768, 512, 1024
    Ac, _ = W.quantize_bf16(W.normal((m, k), 303, 0))
    Bc, _ = W.quantize_bf16(W.normal((k, n), 303, 1))
    A, B = _oracle_inputs(Ac, Bc)
    cfg = (256, 256, 64, 4)
    sites = W.fault_sites(W.rng(303, 3), m, n, k, 256, 256, 64, 4, 20, kind=kind, payload=1e3,
                          bits=range(23, 31))
    F.ftgemm_set_config(h, cfg)
    F.ftgemm_set_injection(h, sites)
    st, C, rep = _run(h, Ac, Bc)
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    assert len(log) == 20
    res, cls, n_grey, bad = replay_against_gpu(A, B, cfg, rep, log)
    assert bad == 0
    must = int(np.sum(cls["cls"] == O.CLS_MUST))
    assert rep.report.corrected >= must and (kind == W.KIND_XOR or must == 20)
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C, res.C) <= 1e-5


def test_full_size_8192_sampled_tiles(h):
    """BF16 8192^3, heavy-tailed N(0,1) operands: no event in a clean run, and
    sampled tiles match the oracle replay on the decoded operands."""
    m = n = k = 8192
    Ac, _ = W.quantize_bf16(W.heavy_tailed((m, k), 4, W.STREAM_A))
    Bc, _ = W.quantize_bf16(W.heavy_tailed((k, n), 4, W.STREAM_B))
    st, C, rep = _run(h, Ac, Bc)
    cfg = rep.report.config.as_tuple()
    assert st == F.OK and rep.report.n_events == 0
    tiles = [(0, 0), (m // cfg[0] - 1, n // cfg[1] - 1), (5, 17)]
    A, B = _oracle_inputs(Ac, Bc)
    res = O.replay(A, B, O.ReplayConfig(mc=cfg[0], nc=cfg[1], ku=cfg[2], g=cfg[3]), tiles=tiles)
    assert res.n_events == 0
    for (tm, tn) in tiles:
        sl = (slice(tm * cfg[0], (tm + 1) * cfg[0]), slice(tn * cfg[1], (tn + 1) * cfg[1]))
        assert rel_fro(C[sl], res.C[sl]) <= 1e-5, (tm, tn)
