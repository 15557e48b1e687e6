"""GPU parity of the double-complex FT-GEMM (ftgemm_run_z64) against the
complex binary64 oracle, through the C ABI.  Bar: C within the element-wise
accumulation bound of binary64 (and relative Frobenius error 1e-12); event
logs (tile, k-step, row, col, kind, component) equal to the oracle replay's,
where the GPU's real products have k-steps of 2 ku real indices = ku complex
ones and events carry the component in `problem`."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import log_to_injections

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.C64, 0)
    yield handle
    F.ftgemm_set_injection(handle, None)
    F.ftgemm_destroy(handle)


@pytest.fixture(autouse=True)
def _reset(h):
    F.ftgemm_set_config(h, None)
    F.ftgemm_set_injection(h, None)
    yield


def _cnormal(shape, wl, st):
    return np.asfortranarray(W.normal64(shape, wl, 2 * st) + 1j * W.normal64(shape, wl, 2 * st + 1))


def _dev(X):
    """Column-major complex (rows, cols) -> device tensor of (re, im) pairs."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(X.T)).view(torch.float64).cuda()


def _host(d, rows, cols):
    import torch
    return np.asfortranarray(d.cpu().view(torch.complex128).numpy().reshape(cols, rows).T)


def _run(h, A, B, C0=None, alpha=1.0, beta=0.0, level=F.FT_CORRECT, cap=4096):
    import torch
    m, k = A.shape
    n = B.shape[1]
    dA, dB = _dev(A), _dev(B)
    dC = _dev(C0) if C0 is not None else torch.zeros((n, 2 * m), dtype=torch.float64, device="cuda")
    rep = F.ReportBuffer(cap)
    st = F.ftgemm_run_z64(h, m, n, k, alpha, dA.data_ptr(), max(m, 1), dB.data_ptr(), max(k, 1), beta, dC.data_ptr(),
                          max(m, 1), level, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    return st, _host(dC, m, n), rep


def _elementwise_ratio(C, ref, A, B, alpha=1.0, beta=0.0, C0=None, extra=None):
    """|C - ref|_ij over (2k + 3) u (|alpha| (|A||B|)_ij + |beta| |C0_ij|) per
    component: each component of a complex sum of k products is a real sum of
    2k products, plus the complex epilogue."""
    k = A.shape[1]
    bound = (2 * k + 3) * U64 * (abs(alpha) * (np.abs(A) @ np.abs(B)))
    if C0 is not None and beta != 0:
        bound = bound + (2 * k + 3) * U64 * abs(beta) * np.abs(C0)
    if extra is not None:
        bound = bound + extra
    err = np.maximum(np.abs((C - ref).real), np.abs((C - ref).imag))
    r = np.where(err == 0, 0.0, err / bound)
    return float(r.max()) if r.size else 0.0


def _keys_gpu(ev):
    return sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]),
                   int(e["kind"]), int(e["problem"])) for e in ev)


def _keys_oracle(ev):
    return sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]),
                   int(e["kind"]), int(e["comp"])) for e in ev)


def _cfg(rep):
    """The oracle configuration of a run: the GPU's k-step counts real inner
    indices (two per complex k)."""
    c = rep.report.config.as_tuple()
    return O.ReplayConfig(mc=c[0], nc=c[1], ku=c[2] // 2, g=c[3], u=O.U_FP64, c=float(rep.report.tol_used))


@pytest.mark.parametrize("shape", [(256, 256, 256), (300, 200, 130), (129, 257, 65), (1, 1, 1), (64, 300, 513)])
def test_clean_matches_oracle(h, shape):
    m, n, k = shape
    A = _cnormal((m, k), 700, 0)
    B = _cnormal((k, n), 700, 1)
    C0 = _cnormal((m, n), 700, 2)
    al, be = 0.75 - 0.5j, -1.0 + 2.0j
    st, C, rep = _run(h, A, B, C0, alpha=al, beta=be)
    ref = O.zgemm(A, B, C0, alpha=al, beta=be)
    assert st == F.OK and rep.report.n_events == 0
    assert np.linalg.norm(C - ref) <= 1e-12 * np.linalg.norm(ref)
    assert _elementwise_ratio(C, ref, A, B, al, be, C0) <= 1.0
    cfg = rep.report.config.as_tuple()
    per_tile = -(-(-(-2 * k // cfg[2])) // cfg[3])
    assert rep.report.checks == 2 * (-(-m // cfg[0])) * (-(-n // cfg[1])) * per_tile   # two real products


def test_gaussian_integers_exact(h):
    A = np.asfortranarray(W.integers((200, 150), 701, 0) + 1j * W.integers((200, 150), 701, 1)).astype(np.complex128)
    B = np.asfortranarray(W.integers((150, 90), 701, 2) + 1j * W.integers((150, 90), 701, 3)).astype(np.complex128)
    st, C, rep = _run(h, A, B)
    assert st == F.OK and rep.report.n_events == 0
    assert np.array_equal(C, O.zgemm(A, B))


def test_quick_returns_and_levels(h):
    A = _cnormal((40, 30), 702, 0)
    B = _cnormal((30, 20), 702, 1)
    C0 = _cnormal((40, 20), 702, 2)
    st, C, _ = _run(h, A[:, :0], B[:0], C0, alpha=1.0, beta=2j)            # k = 0: C = beta C
    assert st == F.OK and np.array_equal(C, 2j * C0)
    st, C, _ = _run(h, A, B, np.full((40, 20), np.nan + 0j), beta=0.0)    # beta = 0: C not read
    assert st == F.OK and np.isfinite(C).all()
    for level in (F.FT_OFF, F.FT_DETECT):
        st, C, rep = _run(h, A, B, level=level)
        assert st == F.OK and rep.report.n_events == 0
        assert np.linalg.norm(C - A @ B) <= 1e-12 * np.linalg.norm(A @ B)


def _inject(h, A, B, sites, level=F.FT_CORRECT):
    F.ftgemm_set_config(h, (128, 128, 16, 2))
    F.ftgemm_set_injection(h, sites)
    st, C, rep = _run(h, A, B, level=level)
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    inj = log_to_injections(log, comp_field="problem")
    res = O.zreplay(A, B, _cfg(rep), injections=inj)
    return st, C, rep, log, res


def test_one_fault_per_tile_and_component(h):
    """One +1e3 fault in every tile of each component, at seeded k-steps:
    all corrected at their sites, C equals the clean product."""
    m, n, k = 300, 260, 200
    A = _cnormal((m, k), 703, 0)
    B = _cnormal((k, n), 703, 1)
    g = W.rng(703, W.STREAM_SITES)
    rows = []
    for comp in (0, 1):
        s = W.fault_sites(g, m, n, 2 * k, 128, 128, 16, 2, 0, payload=1e3, per_tile=1)
        s["problem"] = comp
        rows.append(s)
    sites = np.sort(np.concatenate(rows), order=["problem", "tile_m", "tile_n", "kstep"])
    st, C, rep, log, res = _inject(h, A, B, sites)
    assert len(log) == len(sites) == 18
    assert np.all(res.classes["cls"] == O.CLS_MUST)
    assert st == F.OK and rep.report.corrected == 18
    assert _keys_gpu(rep.events) == _keys_oracle(res.events)
    ref = O.zgemm(A, B)
    assert np.linalg.norm(C - ref) <= 1e-12 * np.linalg.norm(ref)
    beta_row = max(float(e["tau_row"]) for e in res.events) / 2.0
    assert _elementwise_ratio(C, res.C, A, B, extra=beta_row) <= 1.0


def test_faults_in_both_components_same_interval_both_corrected(h):
    """The real part of one element and the imaginary part of another, same
    tile and check interval: two real products, one fault each, both fixed."""
    m, n, k = 256, 256, 256
    A = _cnormal((m, k), 704, 0)
    B = _cnormal((k, n), 704, 1)
    sites = np.zeros(2, dtype=F.FAULT_DTYPE)
    sites[0] = (0, 1, 3, 5, 7, W.KIND_ADD, 1e3, 0)
    sites[1] = (0, 1, 3, 9, 2, W.KIND_ADD, -1e3, 1)
    st, C, rep, log, res = _inject(h, A, B, sites)
    assert st == F.OK and rep.report.corrected == 2 and rep.report.uncorrectable == 0
    assert _keys_gpu(rep.events) == _keys_oracle(res.events)
    assert sorted(int(e["problem"]) for e in rep.events) == [0, 1]


def test_two_faults_in_one_component_uncorrectable(h):
    m, n, k = 256, 256, 256
    A = _cnormal((m, k), 705, 0)
    B = _cnormal((k, n), 705, 1)
    sites = np.zeros(2, dtype=F.FAULT_DTYPE)
    sites[0] = (1, 0, 4, 5, 7, W.KIND_ADD, 1e3, 1)
    sites[1] = (1, 0, 4, 9, 2, W.KIND_ADD, 1e3, 1)
    st, C, rep, log, res = _inject(h, A, B, sites)
    assert st == F.UNCORRECTABLE and rep.report.uncorrectable == 1
    assert _keys_gpu(rep.events) == _keys_oracle(res.events)
    assert np.linalg.norm(C - res.C) <= 1e-12 * np.linalg.norm(res.C)


def test_bit_flips_exact_site_log(h):
    """Bit flips in either component's accumulator (bits 20..62 of the
    binary64 value): must-detect flips corrected at their site, the event log
    equal to the replay's (grey flips follow the GPU's decision)."""
    m, n, k = 384, 256, 512
    A = _cnormal((m, k), 706, 0)
    B = _cnormal((k, n), 706, 1)
    g = W.rng(706, W.STREAM_SITES)
    parts = []
    for comp in (0, 1):
        s = W.fault_sites(g, m, n, 2 * k, 128, 128, 16, 2, 24, kind=W.KIND_XOR, bits=range(40, 63))
        s["problem"] = comp
        parts.append(s)
    sites = np.sort(np.concatenate(parts), order=["problem", "tile_m", "tile_n", "kstep"])
    st, C, rep, log, res = _inject(h, A, B, sites)
    assert len(log) == 48
    assert not np.any(res.classes["cls"] == O.CLS_GREY)   # at u = 2^-53 no flip of these bits is grey
    must = int(np.sum(res.classes["cls"] == O.CLS_MUST))
    assert must > 0 and rep.report.corrected >= must
    assert _keys_gpu(rep.events) == _keys_oracle(res.events)


def test_nonfinite_operand(h):
    m, n, k = 256, 256, 256
    A = _cnormal((m, k), 707, 0)
    B = _cnormal((k, n), 707, 1)
    A[130, 40] = complex(np.nan, 1.0)
    F.ftgemm_set_config(h, (128, 128, 16, 2))
    st, C, rep = _run(h, A, B)
    res = O.zreplay(A, B, _cfg(rep))
    assert st == F.NONFINITE_INPUT
    # each real product reports the two tiles of tile row 1 once; the oracle reports each tile once
    gk = sorted({(int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["kind"])) for e in rep.events})
    ok = sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["kind"])) for e in res.events)
    assert gk == ok == [(1, 0, 5, F.EV_NONFINITE), (1, 1, 5, F.EV_NONFINITE)]   # complex k 40: real step 5
    fin = np.isfinite(res.C)
    assert np.array_equal(np.isfinite(C), fin)
    assert np.linalg.norm(C[fin] - res.C[fin]) <= 1e-12 * np.linalg.norm(res.C[fin])
