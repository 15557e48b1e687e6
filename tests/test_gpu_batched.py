"""GPU tests of the batched persistent launch, its HIP-graph capture and the
autotuner, against the FP64 oracle.

Batched problems: M, N, K log-uniform (seeded), FP32 or BF16 by a seeded
coin, each problem checked against the oracle on its own (relative Frobenius
error <= 1e-5: exact products, FP32 accumulation), and the event log of an
injected run against the oracle replay of every problem with the
configuration the plan gave it."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import event_keys, rel_fro

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.F32, 0)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


class Batch:
    """Host operands, device buffers and the descriptor array of a batch."""

    def __init__(self, shapes, workload, beta=0.0, alpha=1.0):
        import torch
        self.torch = torch
        self.host = []
        self.dev = []
        self.probs = F.make_problems(len(shapes))
        for p, (m, n, k, dt) in enumerate(shapes):
            A = W.uniform((m, k), workload, 10 * p) if m * k else np.zeros((m, k), np.float32, order="F")
            B = W.uniform((k, n), workload, 10 * p + 1) if k * n else np.zeros((k, n), np.float32, order="F")
            C0 = W.normal((m, n), workload, 10 * p + 2) if m * n else np.zeros((m, n), np.float32, order="F")
            if dt == "bf16":
                Ac, _ = W.quantize_bf16(A)
                Bc, _ = W.quantize_bf16(B)
                A64, B64 = O.decode_bf16(Ac), O.decode_bf16(Bc)
                dA = torch.from_numpy(np.ascontiguousarray(Ac.T).view(np.int16)).cuda() if Ac.size else torch.zeros(1, device="cuda")
                dB = torch.from_numpy(np.ascontiguousarray(Bc.T).view(np.int16)).cuda() if Bc.size else torch.zeros(1, device="cuda")
            elif dt == "fp8":
                # codes of the unscaled operands (U[-1, 1] fits E4M3 as it is; scales 1)
                Ac = np.asfortranarray(W.to_e4m3_codes(A.astype(np.float64)))
                Bc = np.asfortranarray(W.to_e4m3_codes(B.astype(np.float64)))
                A64, B64 = O.decode_e4m3(Ac), O.decode_e4m3(Bc)
                dA = torch.from_numpy(np.ascontiguousarray(Ac.T)).cuda() if Ac.size else torch.zeros(1, device="cuda")
                dB = torch.from_numpy(np.ascontiguousarray(Bc.T)).cuda() if Bc.size else torch.zeros(1, device="cuda")
            else:
                A64, B64 = A.astype(np.float64), B.astype(np.float64)
                dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda() if A.size else torch.zeros(1, device="cuda")
                dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda() if B.size else torch.zeros(1, device="cuda")
            dC = torch.from_numpy(np.ascontiguousarray(C0.T)).cuda() if C0.size else torch.zeros(1, device="cuda")
            self.host.append((np.asfortranarray(A64), np.asfortranarray(B64), C0))
            self.dev.append((dA, dB, dC))
            q = self.probs[p]
            q["dtype"] = {"bf16": F.BF16, "fp8": F.F8E4M3}.get(dt, F.F32)
            q["m"], q["n"], q["k"] = m, n, k
            q["lda"], q["ldb"], q["ldc"] = max(1, m), max(1, k), max(1, m)
            q["alpha"], q["beta"], q["scale_a"], q["scale_b"] = alpha, beta, 1.0, 1.0
            q["A"], q["B"], q["C"] = dA.data_ptr(), dB.data_ptr(), dC.data_ptr()
        self.C0 = [d[2].clone() for d in self.dev]

    def reset(self):
        for (dA, dB, dC), c0 in zip(self.dev, self.C0):
            dC.copy_(c0)

    def result(self, p):
        m, n = int(self.probs[p]["m"]), int(self.probs[p]["n"])
        if m * n == 0:
            return np.zeros((m, n), np.float32)
        return np.asfortranarray(self.dev[p][2].cpu().numpy().reshape(n, m).T)

    def reference(self, p):
        A, B, C0 = self.host[p]
        q = self.probs[p]
        return O.gemm(A, B, C0 if q["beta"] != 0 else None, alpha=float(q["alpha"]), beta=float(q["beta"]))


def _shapes(count, lo, hi, workload):
    return [(b.m, b.n, b.k, b.dtype) for b in W.batched_problems(count, lo, hi, workload)]


def test_batched_matches_oracle_per_problem(h):
    import torch
    shapes = _shapes(40, 32, 700, 500) + [(0, 5, 7, "f32"), (9, 0, 3, "bf16"), (70, 33, 0, "f32"),
                                          (300, 257, 1, "bf16"), (1, 1, 1, "f32")]
    bt = Batch(shapes, 500, beta=0.5)
    rep = F.ReportBuffer(64)
    st = F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    assert st == F.OK and rep.report.n_events == 0 and rep.report.checks > 0
    for p in range(len(shapes)):
        assert rel_fro(bt.result(p), bt.reference(p)) <= TOL, (p, shapes[p])
    used = {F.ftgemm_batched_config(h, p).as_tuple()[:3] for p in range(len(shapes))}
    assert (128, 128, 32) in used and (128, 128, 64) in used


def test_batched_fp8_problems_match_oracle(h):
    """FP8 E4M3 problems in a batch with FP32 and BF16 ones: each FP8
    problem runs the FP8 128 x 128 variant and matches the oracle on its
    decoded codes (relative Frobenius 1e-4: the FP8 instruction sums its
    products below binary32 precision), the others as before."""
    import torch
    shapes = [(300, 200, 257, "fp8"), (64, 64, 64, "fp8"), (1, 130, 70, "fp8"), (256, 256, 512, "f32"),
              (200, 300, 100, "bf16"), (513, 129, 65, "fp8")]
    bt = Batch(shapes, 503, beta=0.5)
    rep = F.ReportBuffer(64)
    st = F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    assert st == F.OK and rep.report.n_events == 0 and rep.report.checks > 0
    for p, (m, n, k, dt) in enumerate(shapes):
        assert rel_fro(bt.result(p), bt.reference(p)) <= (1e-4 if dt == "fp8" else TOL), (p, shapes[p])
        if dt == "fp8":
            assert F.ftgemm_batched_config(h, p).as_tuple()[:3] == (128, 128, 64)


def test_batched_alpha_zero_and_beta_zero_quick_returns(h):
    import torch
    shapes = [(100, 90, 80, "f32"), (64, 64, 64, "bf16")]
    bt = Batch(shapes, 501, beta=0.0, alpha=0.0)
    bt.probs["beta"] = [2.0, 0.0]
    F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert np.array_equal(bt.result(0), 2.0 * bt.host[0][2])
    assert np.array_equal(bt.result(1), np.zeros((64, 64), np.float32))


def test_batched_invalid_problem_is_named(h):
    import torch
    bt = Batch([(64, 64, 64, "f32"), (64, 64, 64, "f32")], 502)
    bad = bt.probs.copy()
    bad[1]["lda"] = 10
    rep = F.ReportBuffer(4)
    with pytest.raises(F.FtgemmError):
        F.ftgemm_batched(h, bad, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    assert rep.report.bad_arg == 3 and rep.report.bad_problem == 1


def test_batched_injection_exact_site_log(h):
    """One additive 1e3 fault in every problem (a seeded tile, k-step and
    element), in one launch: every fault corrected at its site, nothing else
    flagged, each problem equal to the oracle replay."""
    import torch
    shapes = _shapes(24, 64, 600, 503)
    bt = Batch(shapes, 503)
    F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream)   # build the plan
    torch.cuda.synchronize()
    bt.reset()
    g = W.rng(503, W.STREAM_SITES)
    sites = []
    for p, (m, n, k, dt) in enumerate(shapes):
        c = F.ftgemm_batched_config(h, p).as_tuple()
        s = W.fault_sites(g, m, n, k, c[0], c[1], c[2], c[3], 1, payload=1e3)
        s["problem"] = p
        sites.append(s)
    sites = np.concatenate(sites)
    sites = sites[np.lexsort((sites["kstep"], sites["tile_n"], sites["tile_m"], sites["problem"]))]
    F.ftgemm_set_injection(h, sites)
    rep = F.ReportBuffer(4096)
    F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    assert len(log) == len(shapes)
    assert rep.report.corrected == len(shapes) and rep.report.uncorrectable == 0
    ev = rep.events
    for p, (m, n, k, dt) in enumerate(shapes):
        c = F.ftgemm_batched_config(h, p).as_tuple()
        A, B, C0 = bt.host[p]
        mine = log[log["problem"] == p]
        inj = O.make_injections([(int(x["tile_m"]), int(x["tile_n"]), int(x["kstep"]), int(x["row"]),
                                  int(x["col"]), float(x["old_v"]), float(x["new_v"])) for x in mine])
        res = O.replay(A, B, O.ReplayConfig(mc=c[0], nc=c[1], ku=c[2], g=c[3], c=float(rep.report.tol_used)),
                       injections=inj)
        assert int(np.sum(res.classes["cls"] == O.CLS_MUST)) == 1
        assert event_keys(ev[ev["problem"] == p]) == event_keys(res.events), p
        assert rel_fro(bt.result(p), res.C) <= TOL, p


def test_batched_fp8_injection_exact_site_log(h):
    """One additive 1e3 fault in every problem of a batch that holds FP8
    problems (so the launch runs the instantiation with the FP8 tile): every
    fault corrected at its site, the event log of each problem equal to the
    oracle replay's on its decoded operands, C within the FP8 accumulation
    bound of the replay."""
    import torch
    shapes = [(300, 200, 257, "fp8"), (128, 128, 512, "fp8"), (200, 300, 100, "bf16"), (256, 130, 70, "fp8"),
              (190, 256, 300, "f32"), (513, 129, 65, "fp8"), (96, 96, 640, "fp8"), (64, 200, 128, "f32")]
    bt = Batch(shapes, 505)
    F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream)   # build the plan
    torch.cuda.synchronize()
    bt.reset()
    g = W.rng(505, W.STREAM_SITES)
    sites = []
    for p, (m, n, k, dt) in enumerate(shapes):
        c = F.ftgemm_batched_config(h, p).as_tuple()
        if dt == "fp8":
            assert c[:3] == (128, 128, 64)
        s = W.fault_sites(g, m, n, k, c[0], c[1], c[2], c[3], 1, payload=1e3)
        s["problem"] = p
        sites.append(s)
    sites = np.concatenate(sites)
    sites = sites[np.lexsort((sites["kstep"], sites["tile_n"], sites["tile_m"], sites["problem"]))]
    F.ftgemm_set_injection(h, sites)
    rep = F.ReportBuffer(256)
    F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    assert len(log) == len(shapes)
    assert rep.report.corrected == len(shapes) and rep.report.uncorrectable == 0
    ev = rep.events
    for p, (m, n, k, dt) in enumerate(shapes):
        c = F.ftgemm_batched_config(h, p).as_tuple()
        A, B, C0 = bt.host[p]
        mine = log[log["problem"] == p]
        inj = O.make_injections([(int(x["tile_m"]), int(x["tile_n"]), int(x["kstep"]), int(x["row"]),
                                  int(x["col"]), float(x["old_v"]), float(x["new_v"])) for x in mine])
        res = O.replay(A, B, O.ReplayConfig(mc=c[0], nc=c[1], ku=c[2], g=c[3], c=float(rep.report.tol_used)),
                       injections=inj)
        assert int(np.sum(res.classes["cls"] == O.CLS_MUST)) == 1
        assert event_keys(ev[ev["problem"] == p]) == event_keys(res.events), p
        assert rel_fro(bt.result(p), res.C) <= (1e-4 if dt == "fp8" else TOL), p


def test_batched_graph_capture_replays(h):
    """The batched call captured into a HIP graph (same problem list as the
    eager call before it): each of several replays, with eager work and
    synchronisation between them, reproduces the eager result bit for bit."""
    import torch
    shapes = _shapes(32, 32, 512, 504)
    bt = Batch(shapes, 504, beta=1.0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, s.cuda_stream)
    torch.cuda.synchronize()
    eager = [bt.result(p) for p in range(len(shapes))]
    bt.reset()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        bt.reset()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for p in range(len(shapes)):
            assert np.array_equal(bt.result(p), eager[p]), (rep, p)
        x = torch.randn(1024, 1024, device="cuda")
        (x @ x).sum().item()          # unrelated eager work between replays
    del graph


def test_capture_with_a_new_problem_list_is_refused(h):
    import torch
    bt = Batch(_shapes(4, 32, 64, 505), 505)
    other = bt.probs.copy()
    other["beta"] = 3.0
    F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with pytest.raises(F.FtgemmError):
        with torch.cuda.graph(graph):
            F.ftgemm_batched(h, other, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()


def test_tune_picks_a_config_that_runs_used_and_persisted(h, tmp_path):
    import torch
    m, n, k = 384, 640, 512
    stream = torch.cuda.current_stream().cuda_stream
    cfg = F.ftgemm_tune(h, m, n, k, F.FT_CORRECT, 256, stream).as_tuple()
    assert cfg[2] * cfg[3] <= 256
    A = W.uniform((m, k), 506, 0)
    B = W.uniform((k, n), 506, 1)
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    dC = torch.zeros((n, m), device="cuda")
    rep = F.ReportBuffer(16)
    st = F.ftgemm_run(h, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                      F.FT_CORRECT, 0.0, stream, rep)
    assert st == F.OK and rep.report.config.as_tuple() == cfg
    C = np.asfortranarray(dC.cpu().numpy().T)
    assert rel_fro(C, O.gemm(A, B)) <= TOL
    path = str(tmp_path / "tuned.json")
    F.save_tuned(h, path)
    h2 = F.ftgemm_create(F.F32, 0)
    try:
        assert F.load_tuned(h2, path) >= 1
        assert (m, n, k, F.FT_CORRECT, cfg) in F.ftgemm_get_tuned(h2)
    finally:
        F.ftgemm_destroy(h2)


def test_tune_batched_measures_every_variant(h):
    import torch
    rates = F.ftgemm_tune_batched(h, torch.cuda.current_stream().cuda_stream)
    assert rates.shape == (4,) and np.all(rates > 1e11)


def test_full_size_1024_problems_sampled(h):
    """The benchmarked batch: 1024 problems, M, N, K log-uniform in
    [32, 2048], FP32 and BF16 mixed, one persistent launch.  No event in the
    clean run, every check counted, and 32 seeded sampled problems match the
    oracle product."""
    import torch
    shapes = _shapes(1024, 32, 2048, 5)
    bt = Batch(shapes, 5, beta=1.0)
    rep = F.ReportBuffer(64)
    st = F.ftgemm_batched(h, bt.probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    assert st == F.OK and rep.report.n_events == 0
    expect = 0
    for p, (m, n, k, _) in enumerate(shapes):
        c = F.ftgemm_batched_config(h, p).as_tuple()
        nk = -(-k // c[2])
        expect += -(-m // c[0]) * -(-n // c[1]) * -(-nk // c[3])
    assert rep.report.checks == expect
    for p in W.rng(5, W.STREAM_SHAPES).choice(len(shapes), 32, replace=False):
        assert rel_fro(bt.result(p), bt.reference(p)) <= TOL, (p, shapes[p])
