"""GPU tests of the boundary's edge semantics, through the C ABI:

* non-finite operands: a check tile whose operands hold Inf or NaN is
  reported once (FTGEMM_EV_NONFINITE at the first check whose k prefix holds
  the value), nothing is located or corrected there, the tile is not queued
  for recomputation, C there is what IEEE arithmetic gives, and the call
  returns FTGEMM_NONFINITE_INPUT; every other tile is checked as usual.  The
  expected events come from the oracle replay, which follows the same reading
  of the fault model (section 4.1 covers faults in the computation on finite
  data);
* the row-major PyTorch entry point (C^T = B^T A^T with swapped operands),
  clean and with faults, against the oracle on the row-major problem;
* the check counter, taken on the device, against the number of check tiles
  times check steps."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import (check_cfg, corrected_value_errors, elementwise_ratio, event_keys, log_to_injections,
                      rel_fro, replay_against_gpu, run)

pytestmark = pytest.mark.gpu


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


def _same_ieee(C, ref):
    """NaN where the reference is NaN, the same infinities, and the finite
    elements close (relative 1e-5 of the finite part's norm)."""
    C = np.asarray(C, np.float64)
    ref = np.asarray(ref, np.float64)
    assert np.array_equal(np.isnan(C), np.isnan(ref))
    assert np.array_equal(np.isposinf(C), np.isposinf(ref)) and np.array_equal(np.isneginf(C), np.isneginf(ref))
    fin = np.isfinite(ref)
    return rel_fro(C[fin], ref[fin])


def _nonfinite_operands(m, n, k, seed):
    A = W.uniform((m, k), seed, 0)
    B = W.uniform((k, n), seed, 1)
    A[5, 40] = np.nan          # tile row 0 from k = 40 (k-step 1)
    B[300, 130] = np.inf       # tile column 1 (128-wide) from k = 300 (k-step 9)
    A[200, 10] = -np.inf       # tile row 1 from k-step 0
    return A, B


@pytest.mark.parametrize("level", [F.FT_CORRECT, F.FT_DETECT])
def test_nonfinite_operands_reported_once_per_tile(h, level):
    m, n, k = 384, 300, 400
    A, B = _nonfinite_operands(m, n, k, 400)
    cfg = (128, 128, 32, 2)
    F.ftgemm_set_config(h, cfg)
    st, C, rep = run(h, A, B, ft_level=level)
    rc = O.ReplayConfig(mc=128, nc=128, ku=32, g=2, ft_level=level)
    res = O.replay(A, B, rc)
    ev = rep.events
    assert len(ev) > 0 and all(int(e["kind"]) == F.EV_NONFINITE for e in ev)
    assert event_keys(ev) == event_keys(res.events)
    assert all(int(e["row"]) == -1 and int(e["col"]) == -1 for e in ev)
    assert rep.report.nonfinite_input == len(ev) and rep.report.detected == 0
    assert st == F.NONFINITE_INPUT
    # tiles reading row 5 or row 200 of A or column 130 of B: 3 tile rows x ... (oracle decides)
    tiles = {(int(e["tile_m"]), int(e["tile_n"])) for e in ev}
    assert (0, 0) in tiles and (1, 1) in tiles
    assert _same_ieee(C, res.C) <= 1e-5
    nk = -(-k // 32)
    per_tile = (-(-nk // 2)) if level == F.FT_CORRECT else 1
    assert rep.report.checks == 3 * 3 * per_tile


def test_nonfinite_tile_keeps_other_tiles_protected(h):
    """A fault in a finite tile is still corrected beside a NaN tile; a fault
    in the NaN tile is not located (the tile is reported, not decided on)."""
    m, n, k = 256, 256, 256
    A = W.uniform((m, k), 401, 0)
    B = W.uniform((k, n), 401, 1)
    A[3, 5] = np.nan           # tile row 0, k-step 0: tiles (0, 0) and (0, 1)
    sites = np.zeros(2, dtype=F.FAULT_DTYPE)
    sites[0] = (1, 1, 2, 7, 9, W.KIND_ADD, 1e3, 0)     # finite tile
    sites[1] = (0, 1, 4, 2, 3, W.KIND_ADD, 1e3, 0)     # NaN tile
    cfg = (128, 128, 32, 1)
    F.ftgemm_set_config(h, cfg)
    F.ftgemm_set_injection(h, sites)
    st, C, rep = run(h, A, B)
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    res, cls, n_grey, bad = replay_against_gpu(A, B, cfg, rep, log)
    assert event_keys(rep.events) == event_keys(res.events)
    kinds = sorted(int(e["kind"]) for e in rep.events)
    assert kinds == [F.EV_CORRECTED, F.EV_NONFINITE, F.EV_NONFINITE]
    assert st == F.NONFINITE_INPUT and rep.report.corrected == 1
    assert _same_ieee(C, res.C) <= 1e-5


def test_nonfinite_tiles_are_not_recomputed(h):
    m, n, k = 384, 300, 400
    A, B = _nonfinite_operands(m, n, k, 402)
    F.ftgemm_set_config(h, (128, 128, 32, 2))
    for level in (F.FT_DETECT, F.FT_CORRECT):
        st, C, rep = run(h, A, B, ft_level=level | F.FT_RECOMPUTE)
        assert st == F.NONFINITE_INPUT
        assert rep.report.recomputed == 0 and rep.report.recompute_failed == 0
        res = O.replay(A, B, O.ReplayConfig(mc=128, nc=128, ku=32, g=2, ft_level=level))
        assert _same_ieee(C, res.C) <= 1e-5


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_nonfinite_low_precision_codes(dtype):
    """A NaN code (bfloat16 0x7FC0, E4M3 0x7F) in A: the tiles reading it are
    reported, C there is NaN, the others match the oracle."""
    import torch
    fdt, quant, dec, view, nan_code = {
        "bf16": (F.BF16, W.quantize_bf16, O.decode_bf16, np.int16, 0x7FC0),
        "fp8": (F.F8E4M3, W.quantize_e4m3, O.decode_e4m3, np.uint8, 0x7F)}[dtype]
    m, n, k = 512, 512, 512
    Ac, _ = quant(W.normal((m, k), 403, 0))
    Bc, _ = quant(W.normal((k, n), 403, 1))
    Ac[300, 100] = nan_code
    A, B = np.asfortranarray(dec(Ac)), np.asfortranarray(dec(Bc))
    assert np.isnan(A[300, 100])
    hd = F.ftgemm_create(fdt, 0)
    try:
        F.ftgemm_set_config(hd, (256, 256, 64, 4))
        dA = torch.from_numpy(np.ascontiguousarray(Ac.T).view(view)).cuda()
        dB = torch.from_numpy(np.ascontiguousarray(Bc.T).view(view)).cuda()
        dC = torch.zeros((n, m), device="cuda")
        rep = F.ReportBuffer(64)
        st = F.ftgemm_run(hd, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                          F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
        C = np.asfortranarray(dC.cpu().numpy().T)
    finally:
        F.ftgemm_destroy(hd)
    res = O.replay(A, B, O.ReplayConfig(mc=256, nc=256, ku=64, g=4))
    assert st == F.NONFINITE_INPUT
    assert event_keys(rep.events) == event_keys(res.events)
    assert sorted((int(e["tile_m"]), int(e["tile_n"])) for e in rep.events) == [(1, 0), (1, 1)]
    # the accumulation bar of each operand type (the FP8 matrix instruction sums its products at
    # less than binary32 precision: 1e-4, as in the low-precision parity tests)
    assert _same_ieee(C, res.C) <= (1e-5 if dtype == "bf16" else 1e-4)


def test_nonfinite_wavefront_check_tiles(h):
    """64 x 64 wavefront check tiles: only the check tiles whose rows read the
    NaN are reported."""
    m, n, k = 256, 256, 256
    A = W.uniform((m, k), 404, 0)
    B = W.uniform((k, n), 404, 1)
    A[70, 33] = np.nan           # check-tile row 1 (rows 64..127)
    cfg = (128, 128, 32, 2, 64, 64)
    F.ftgemm_set_config(h, cfg)
    st, C, rep = run(h, A, B)
    res = O.replay(A, B, O.ReplayConfig(mc=64, nc=64, ku=32, g=2))
    assert st == F.NONFINITE_INPUT
    assert event_keys(rep.events) == event_keys(res.events)
    assert sorted((int(e["tile_m"]), int(e["tile_n"])) for e in rep.events) == [(1, j) for j in range(4)]
    assert rep.report.checks == 16 * 4
    assert _same_ieee(C, res.C) <= 1e-5


def test_nonfinite_f64():
    import torch
    m, n, k = 256, 256, 256
    A = W.uniform64((m, k), 405, 0)
    B = W.uniform64((k, n), 405, 1)
    B[200, 140] = np.nan         # check tile column 1 from k-step 12
    hd = F.ftgemm_create(F.F64, 0)
    try:
        dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
        dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
        dC = torch.zeros((n, m), dtype=torch.float64, device="cuda")
        rep = F.ReportBuffer(64)
        st = F.ftgemm_run_f64(hd, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                              F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
        C = np.asfortranarray(dC.cpu().numpy().T)
        cfg = rep.report.config.as_tuple()
    finally:
        F.ftgemm_destroy(hd)
    res = O.replay(A, B, O.ReplayConfig(mc=cfg[0], nc=cfg[1], ku=cfg[2], g=cfg[3], u=O.U_FP64))
    assert st == F.NONFINITE_INPUT
    assert event_keys(rep.events) == event_keys(res.events)
    assert sorted((int(e["tile_m"]), int(e["tile_n"])) for e in rep.events) == [(0, 1), (1, 1)]
    assert _same_ieee(C, res.C) <= 1e-12


def test_nonfinite_batched(h):
    """Batched: the problem with a NaN reports its tiles, its neighbours are clean."""
    import torch
    probs = F.make_problems(3)
    keep = []
    ops = []
    for p, (m, n, k) in enumerate([(200, 150, 300), (256, 256, 256), (90, 70, 500)]):
        A = W.uniform((m, k), 406, 2 * p)
        B = W.uniform((k, n), 406, 2 * p + 1)
        if p == 1:
            A[10, 20] = np.nan
        dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
        dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
        dC = torch.zeros((n, m), device="cuda")
        keep += [dA, dB, dC]
        ops.append((A, B, dC, m, n))
        probs[p] = (F.F32, 0, m, n, k, m, k, m, 1.0, 0.0, 1.0, 1.0, dA.data_ptr(), dB.data_ptr(), dC.data_ptr())
    rep = F.ReportBuffer(64)
    st = F.ftgemm_batched(h, probs, F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    assert st == F.NONFINITE_INPUT
    assert rep.report.nonfinite_input >= 1 and all(int(e["problem"]) == 1 for e in rep.events)
    for p, (A, B, dC, m, n) in enumerate(ops):
        cfg = F.ftgemm_batched_config(h, p).as_tuple()
        res = O.replay(A, B, O.ReplayConfig(mc=cfg[0], nc=cfg[1], ku=cfg[2], g=cfg[3]))
        mine = [e for e in rep.events if int(e["problem"]) == p]
        assert event_keys(mine) == event_keys(res.events), p
        C = np.asfortranarray(dC.cpu().numpy().T)
        assert _same_ieee(C, res.C) <= 1e-5


# ---------------------------------------------------------------------------
# row-major PyTorch entry point
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(300, 520, 200), (1000, 37, 999), (256, 256, 256)])
def test_row_major_entry_matches_oracle(h, shape):
    import torch
    m, n, k = shape
    A = W.normal((m, k), 410, 0)
    B = W.normal((k, n), 410, 1)
    C0 = W.normal((m, n), 410, 2)
    tA = torch.from_numpy(np.ascontiguousarray(A)).cuda()     # row-major: rows contiguous
    tB = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    tC = torch.from_numpy(np.ascontiguousarray(C0)).cuda()
    rep = F.ReportBuffer(16)
    Cout, st = F.ftgemm_matmul(h, tA, tB, tC, alpha=0.5, beta=-1.0, report=rep)
    assert Cout is tC and st == F.OK and rep.report.n_events == 0
    ref = O.gemm(A, B, C0, alpha=0.5, beta=-1.0)
    C = tC.cpu().numpy()
    assert elementwise_ratio(C, ref, A, B, alpha=0.5, beta=-1.0, C0=C0) <= 1.0
    # and against torch's own product of the same tensors (FP32 on the device)
    assert rel_fro(C, (0.5 * (tA.double() @ tB.double()) - torch.from_numpy(C0).double().cuda()).cpu().numpy()) <= 1e-5


def test_row_major_entry_strided_rows_and_validation(h):
    import torch
    m, n, k = 130, 70, 90
    A = W.normal((m, k), 411, 0)
    B = W.normal((k, n), 411, 1)
    big = torch.zeros((m, k + 6), device="cuda")
    big[:, :k] = torch.from_numpy(A).cuda()
    tA = big[:, :k]                                            # row stride k + 6
    tB = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    C, st = F.ftgemm_matmul(h, tA, tB)
    assert st == F.OK and rel_fro(C.cpu().numpy(), O.gemm(A, B)) <= 1e-5
    with pytest.raises(ValueError):
        F.ftgemm_matmul(h, tA.t(), tB)                         # column stride != 1
    with pytest.raises(ValueError):
        F.ftgemm_matmul(h, tA, tB[:80])                        # inner dimensions differ
    with pytest.raises(ValueError):
        F.ftgemm_matmul(h, tA.to(torch.bfloat16), tB.to(torch.bfloat16))   # F32 handle


def test_row_major_entry_faults_events_in_c_coordinates(h):
    """Faults set on the transposed problem C^T: the report's events, swapped
    back, equal the oracle replay of the row-major problem C = A B with the
    swapped fault log (tile_m / row index rows of C)."""
    import torch
    m, n, k = 384, 256, 512
    A = W.uniform((m, k), 412, 0)
    B = W.uniform((k, n), 412, 1)
    F.ftgemm_set_config(h, (128, 128, 32, 2))
    # sites in C^T coordinates (n x m problem): one per check tile
    sites = W.fault_sites(W.rng(412, 3), n, m, k, 128, 128, 32, 2, 0, payload=1e3, per_tile=1)
    F.ftgemm_set_injection(h, sites)
    rep = F.ReportBuffer(64)
    C, st = F.ftgemm_matmul(h, torch.from_numpy(np.ascontiguousarray(A)).cuda(),
                            torch.from_numpy(np.ascontiguousarray(B)).cuda(), report=rep)
    log = F.ftgemm_get_injection_log(h)
    F.ftgemm_set_injection(h, None)
    assert st == F.OK and len(log) == len(sites) == 6 and rep.report.corrected == 6
    assert rep.report.config.as_tuple()[:2] == (128, 128)
    sw = log.copy()
    for a, b in (("tile_m", "tile_n"), ("row", "col")):
        sw[a], sw[b] = log[b], log[a]
    res = O.replay(A, B, O.ReplayConfig(mc=128, nc=128, ku=32, g=2), injections=log_to_injections(sw))
    assert event_keys(rep.events) == event_keys(res.events)
    assert rel_fro(C.cpu().numpy(), O.gemm(A, B)) <= 1e-5
