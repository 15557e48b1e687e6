"""GPU tests of the recompute of tainted tiles (FT_RECOMPUTE OR-ed into the
detect-only or the online level): a tile that ends possibly wrong does not
write C, and the retry launch recomputes exactly those tiles.  The first
pass's event log must equal the oracle replay's; the final C must be the
clean oracle product (the retry runs without injection); the queue must be
empty again after every call."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import event_keys, rel_fro, replay_against_gpu, run

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-5
CFG = (256, 256, 32, 8)   # the benchmark's FP32 configuration


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
    F.ftgemm_set_config(h, CFG)
    F.ftgemm_set_injection(h, None)
    yield
    F.ftgemm_set_config(h, None)
    F.ftgemm_set_injection(h, None)


def _sites(rows):
    sites = np.zeros(len(rows), dtype=F.FAULT_DTYPE)
    for q, r in enumerate(rows):
        sites[q] = r
    return sites


def _pass(h, A, B, sites, level, C0=None, beta=0.0, cfg=CFG):
    F.ftgemm_set_injection(h, sites)
    st, C, rep = run(h, A, B, C0, beta=beta, ft_level=level)
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    base = level & ~F.FT_RECOMPUTE
    res, cls, n_grey, bad = replay_against_gpu(A, B, cfg, rep, log, C0=C0, beta=beta, ft_level=base)
    assert bad == 0
    return st, C, rep, res


def test_uncorrectable_tile_is_recomputed(h):
    """Two +1e3 faults in tile (1, 0) within one check interval: two rows and
    two columns flag, the online level cannot locate them.  With recompute the
    tile is redone and C is the clean product (beta = 1 keeps C0 for the retry);
    without it C stays wrong there."""
    m = n = k = 512
    A = W.normal((m, k), 401, 0)
    B = W.normal((k, n), 401, 1)
    C0 = W.normal((m, n), 401, 2)
    sites = _sites([(1, 0, 3, 5, 7, W.KIND_ADD, 1e3, 0), (1, 0, 5, 40, 200, W.KIND_ADD, 1e3, 0)])
    clean = O.gemm(A, B, C0, beta=1.0)

    st, C, rep, res = _pass(h, A, B, sites, F.FT_CORRECT, C0=C0, beta=1.0)
    assert st == F.UNCORRECTABLE and rep.report.uncorrectable == 1 and rep.report.recomputed == 0
    assert rel_fro(C, clean) > 1e-3

    st, C, rep, res = _pass(h, A, B, sites, F.FT_CORRECT | F.FT_RECOMPUTE, C0=C0, beta=1.0)
    assert event_keys(rep.events) == event_keys(res.events)
    assert rep.report.uncorrectable == 1
    assert rep.report.recomputed == 1 and rep.report.recompute_failed == 0
    assert st == F.OK
    assert rel_fro(C, clean) <= TOL_F32


def test_detect_only_with_recompute(h):
    """Offline scheme: one check per tile at the end; every tile that flags is
    recomputed, the others are written by the first pass."""
    m, n, k = 768, 512, 640
    A = W.uniform((m, k), 402, 0)
    B = W.uniform((k, n), 402, 1)
    sites = _sites([(0, 1, 2, 17, 3, W.KIND_ADD, 1e3, 0), (2, 0, 15, 100, 250, W.KIND_ADD, 1e3, 0),
                    (2, 1, 19, 255, 0, W.KIND_ADD, -5e2, 0)])
    st, C, rep, res = _pass(h, A, B, sites, F.FT_DETECT | F.FT_RECOMPUTE)
    assert event_keys(rep.events) == event_keys(res.events)
    assert rep.report.detected == 3 and rep.report.recomputed == 3 and rep.report.recompute_failed == 0
    assert st == F.OK
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32


def test_ragged_edge_tile_recomputed(h):
    """The tainted tile is the ragged corner tile of an odd shape."""
    m, n, k = 300, 520, 200
    A = W.uniform((m, k), 403, 0)
    B = W.uniform((k, n), 403, 1)
    sites = _sites([(1, 2, 1, 10, 1, W.KIND_ADD, 1e3, 0), (1, 2, 2, 30, 5, W.KIND_ADD, 1e3, 0)])
    st, C, rep, res = _pass(h, A, B, sites, F.FT_CORRECT | F.FT_RECOMPUTE)
    assert rep.report.uncorrectable == 1 and rep.report.recomputed == 1 and st == F.OK
    assert rel_fro(C, O.gemm(A, B)) <= TOL_F32


def test_queue_is_empty_after_every_call(h):
    """Clean, faulty, clean, faulty, clean: the recompute count follows the
    faults of each call only (the retry launch clears the queue it read)."""
    m = n = k = 512
    A = W.uniform((m, k), 404, 0)
    B = W.uniform((k, n), 404, 1)
    ref = O.gemm(A, B)
    bad = _sites([(0, 0, 0, 1, 1, W.KIND_ADD, 1e3, 0), (0, 0, 1, 2, 2, W.KIND_ADD, 1e3, 0),
                  (1, 1, 9, 3, 3, W.KIND_ADD, 1e3, 0), (1, 1, 10, 4, 4, W.KIND_ADD, 1e3, 0)])
    for sites, expect in ((None, 0), (bad, 2), (None, 0), (bad[:2], 1), (None, 0)):
        F.ftgemm_set_injection(h, sites)
        st, C, rep = run(h, A, B, ft_level=F.FT_CORRECT | F.FT_RECOMPUTE)
        F.ftgemm_set_injection(h, None)
        assert st == F.OK and rep.report.recomputed == expect
        assert rel_fro(C, ref) <= TOL_F32


def test_recompute_without_report_then_with(h):
    """No report (no synchronisation, no counter reset): the pair of launches
    still leaves C right and the queue empty for the next call."""
    import torch
    from gpu_util import dev, host
    m = n = k = 512
    A = W.uniform((m, k), 405, 0)
    B = W.uniform((k, n), 405, 1)
    bad = _sites([(0, 1, 0, 1, 1, W.KIND_ADD, 1e3, 0), (0, 1, 1, 2, 2, W.KIND_ADD, 1e3, 0)])
    F.ftgemm_set_injection(h, bad)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((n, m), device="cuda")
    st = F.ftgemm_run(h, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                      F.FT_CORRECT | F.FT_RECOMPUTE, 0.0, torch.cuda.current_stream().cuda_stream, None)
    F.ftgemm_set_injection(h, None)
    torch.cuda.synchronize()
    assert st == F.OK
    assert rel_fro(host(dC, m, n), O.gemm(A, B)) <= TOL_F32
    st, C, rep = run(h, A, B, ft_level=F.FT_CORRECT | F.FT_RECOMPUTE)
    assert st == F.OK and rep.report.recomputed == 0


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_low_precision_recompute(dtype):
    import torch
    kind, quant, dec, store = {"bf16": (F.BF16, W.quantize_bf16, O.decode_bf16, np.int16),
                               "fp8": (F.F8E4M3, W.quantize_e4m3, O.decode_e4m3, np.uint8)}[dtype]
    hd = F.ftgemm_create(kind, 0)
    try:
        m = n = k = 512
        Ac, sa = quant(W.normal((m, k), 406, 0))
        Bc, sb = quant(W.normal((k, n), 406, 1))
        F.ftgemm_set_scales(hd, sa, sb)
        F.ftgemm_set_config(hd, (256, 256, 64, 4))
        pay = 1e3 / (sa * sb)
        F.ftgemm_set_injection(hd, _sites([(1, 1, 0, 7, 9, W.KIND_ADD, pay, 0), (1, 1, 2, 70, 90, W.KIND_ADD, pay, 0)]))
        dA = torch.from_numpy(np.ascontiguousarray(Ac.T).view(store)).cuda()
        dB = torch.from_numpy(np.ascontiguousarray(Bc.T).view(store)).cuda()
        dC = torch.zeros((n, m), device="cuda")
        rep = F.ReportBuffer(64)
        st = F.ftgemm_run(hd, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                          F.FT_CORRECT | F.FT_RECOMPUTE, 0.0, torch.cuda.current_stream().cuda_stream, rep)
        assert st == F.OK and rep.report.uncorrectable == 1 and rep.report.recomputed == 1
        C = np.asfortranarray(dC.cpu().numpy().T)
        ref = O.gemm(np.asfortranarray(dec(Ac)), np.asfortranarray(dec(Bc)), alpha=sa * sb)
        assert rel_fro(C, ref) <= 1e-4
    finally:
        F.ftgemm_set_injection(hd, None)
        F.ftgemm_destroy(hd)


def test_recompute_flag_validation(h):
    """The flag needs a fault-tolerant level, and ftgemm_batched does not take it."""
    assert F.ftgemm_validate(8, 8, 8, 8, 8, 8, ft_level=F.FT_RECOMPUTE)[0] == F.INVALID
    assert F.ftgemm_validate(8, 8, 8, 8, 8, 8, ft_level=F.FT_RECOMPUTE)[1] == 13
    assert F.ftgemm_validate(8, 8, 8, 8, 8, 8, ft_level=F.FT_DETECT | F.FT_RECOMPUTE)[0] == F.OK
    rep = F.ReportBuffer(1)
    with pytest.raises(F.FtgemmError):
        F.ftgemm_batched(h, F.make_problems(0), ft_level=F.FT_CORRECT | F.FT_RECOMPUTE, report=rep)
    assert rep.report.bad_arg == 4


def test_recompute_pair_captured_in_a_graph(h):
    """With recompute on and no report, ftgemm_run issues two launches and
    no memset: after one eager call of the shape (which sizes the queue) the
    pair can be captured into a HIP graph.  Each of several replays, with
    eager work between them, reproduces the eager result bit for bit, and a
    later eager call finds the queue empty."""
    import torch
    from gpu_util import dev, host
    m = n = k = 512
    A = W.uniform((m, k), 407, 0)
    B = W.uniform((k, n), 407, 1)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((n, m), device="cuda")

    def call():
        return F.ftgemm_run(h, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                            F.FT_CORRECT | F.FT_RECOMPUTE, 0.0, torch.cuda.current_stream().cuda_stream, None)
    assert call() == F.OK
    torch.cuda.synchronize()
    eager = host(dC, m, n).copy()
    assert rel_fro(eager, O.gemm(A, B)) <= TOL_F32
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    for rep in range(3):
        dC.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(dC, m, n), eager), rep
        x = torch.randn(1024, 1024, device="cuda")
        (x @ x).sum().item()          # unrelated eager work between replays
    del graph
    st, C, rep = run(h, A, B, ft_level=F.FT_CORRECT | F.FT_RECOMPUTE)
    assert st == F.OK and rep.report.recomputed == 0
