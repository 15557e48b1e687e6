"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (no GPU).  Each test names the passage it pins.

A planted-mistake suite (test_oracle_mutants.py) re-runs these checks against
deliberately broken builds of the oracle and requires each break to be caught.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _int_matmul(A, B):
    """Brute-force exact integer product (pure Python ints)."""
    m, k = A.shape
    n = B.shape[1]
    Ai = [[int(A[i, p]) for p in range(k)] for i in range(m)]
    Bi = [[int(B[p, j]) for j in range(n)] for p in range(k)]
    return np.array([[sum(Ai[i][p] * Bi[p][j] for p in range(k)) for j in range(n)] for i in range(m)],
                    dtype=np.float64)


# ---------------------------------------------------------------------------
# plain GEMM (section 3.1: C += A B; BLAS alpha/beta)
# ---------------------------------------------------------------------------
def test_gemm_identity_gives_B():
    B = W.normal((7, 5), 90, 1).astype(np.float64)
    C = O.gemm(np.eye(7), B)
    assert np.array_equal(C, B)


def test_gemm_all_ones_gives_K():
    for (m, n, k) in [(3, 4, 5), (1, 1, 1), (9, 2, 17)]:
        C = O.gemm(np.ones((m, k)), np.ones((k, n)))
        assert np.array_equal(C, np.full((m, n), float(k)))


def test_gemm_integers_exact_vs_bruteforce():
    A = W.integers((5, 9), 91, 0).astype(np.float64)
    B = W.integers((9, 7), 91, 1).astype(np.float64)
    assert np.array_equal(O.gemm(A, B), _int_matmul(A, B))


def test_gemm_leading_dimensions():
    """A, B, C embedded in larger column-major arrays (lda > m, ldb > k)."""
    lib = O.load()
    m, n, k = 4, 3, 5
    Abig = np.asfortranarray(W.integers((m + 3, k), 92, 0).astype(np.float64))
    Bbig = np.asfortranarray(W.integers((k + 2, n), 92, 1).astype(np.float64))
    Cbig = np.asfortranarray(np.full((m + 1, n), 7.0))
    rc = lib.oracle_gemm(m, n, k, 1.0, O._dp(Abig), m + 3, O._dp(Bbig), k + 2, 0.0, O._dp(Cbig), m + 1)
    assert rc == 0
    assert np.array_equal(Cbig[:m], _int_matmul(Abig[:m], Bbig[:k]))
    assert np.all(Cbig[m] == 7.0)   # padding row untouched


def test_gemm_alpha_beta_semantics():
    A = W.integers((4, 6), 93, 0).astype(np.float64)
    B = W.integers((6, 5), 93, 1).astype(np.float64)
    C0 = W.integers((4, 5), 93, 2).astype(np.float64)
    assert np.array_equal(O.gemm(A, B, C0, alpha=2.0, beta=-0.5), 2.0 * _int_matmul(A, B) - 0.5 * C0)
    nan0 = np.full((4, 5), np.nan)
    assert np.array_equal(O.gemm(A, B, nan0, alpha=1.0, beta=0.0), _int_matmul(A, B))  # C0 not read
    Anan = np.full((4, 6), np.nan)
    assert np.array_equal(O.gemm(Anan, B, C0, alpha=0.0, beta=3.0), 3.0 * C0)       # AB not formed
    assert np.array_equal(O.gemm(np.zeros((4, 0)), np.zeros((0, 5)), C0, beta=2.0, k=0), 2.0 * C0)


def test_gemm_float_vs_numpy_float64():
    """Special case reducing to a library routine: numpy float64 matmul."""
    A = W.normal((33, 47), 94, 0).astype(np.float64)
    B = W.normal((47, 29), 94, 1).astype(np.float64)
    C = O.gemm(A, B)
    ref = A @ B
    assert np.linalg.norm(C - ref) / np.linalg.norm(ref) <= 1e-13


def test_gemm_rejects_bad_arguments():
    lib = O.load()
    a = np.zeros((4, 4))
    dp = O._dp(a)
    assert lib.oracle_gemm(-1, 1, 1, 1.0, dp, 1, dp, 1, 0.0, dp, 1) == -1
    assert lib.oracle_gemm(4, 1, 1, 1.0, dp, 3, dp, 1, 0.0, dp, 4) == -6
    assert lib.oracle_gemm(4, 1, 3, 1.0, dp, 4, dp, 2, 0.0, dp, 4) == -8
    assert lib.oracle_gemm(4, 1, 1, 1.0, dp, 4, dp, 1, 0.0, dp, 3) == -11


# ---------------------------------------------------------------------------
# checksum encodings (section 2.2, Eq. 1-3)
# ---------------------------------------------------------------------------
def _read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows.setdefault(key, []).append([float(v) for v in vals])
    return {k: np.array(v) for k, v in rows.items()}


def test_encode_golden_worked_example():
    g = _read_golden("encode_2x2.txt")
    A, B = g["A"], g["B"]
    assert np.array_equal(O.encode_col(A), g["eTA"][0])
    assert np.array_equal(O.encode_row(B), g["Be"][0])
    C = O.gemm(A, B)
    assert np.array_equal(C, g["C"])
    assert np.array_equal(O.encode_row(C), g["Ce"][0])     # C e, the row checksums
    assert np.array_equal(O.encode_col(C), g["eTC"][0])    # e^T C, the column checksums


@pytest.mark.parametrize("seed", range(5))
def test_encoded_product_identity_exact_on_integers(seed):
    """Eq. 3: e^T(AB) = (e^T A) B and (AB) e = A (B e), exact for integers."""
    m, k, n = 6 + seed, 11, 5 + 2 * seed
    A = W.integers((m, k), 95, 10 + seed).astype(np.float64)
    B = W.integers((k, n), 95, 20 + seed).astype(np.float64)
    C = _int_matmul(A, B)
    w = O.encode_col(A)
    v = O.encode_row(B)
    assert np.array_equal(O.encode_col(C), _int_matmul(w[None, :], B)[0])
    assert np.array_equal(O.encode_row(C), _int_matmul(A, v[:, None])[:, 0])


# ---------------------------------------------------------------------------
# online invariance (Eq. 4) and the threshold
# ---------------------------------------------------------------------------
def test_online_invariance_integers_zero_residual_every_step():
    """With integer operands every FP64 sum is exact, so after every
    rank-ku update the residuals are exactly zero: with tau = 0 (c = 0) and a
    check after every step, no row or column may be flagged."""
    m, n, k = 13, 11, 29
    A = W.integers((m, k), 96, 0)
    B = W.integers((k, n), 96, 1)
    cfg = O.ReplayConfig(mc=5, nc=4, ku=3, g=1, c=0.0)
    res = O.replay(A, B, cfg)
    assert res.n_events == 0
    assert np.array_equal(res.C, _int_matmul(A.astype(np.float64), B.astype(np.float64)))


def test_check_runs_and_flags_float_roundoff_when_tau_is_zero():
    """Counterpart of the test above: with non-integer data the FP64
    residuals are tiny but non-zero, so tau = 0 must flag (proves the check
    is evaluated at all)."""
    A = W.normal((8, 40), 97, 0)
    B = W.normal((40, 8), 97, 1)
    res = O.replay(A, B, O.ReplayConfig(mc=8, nc=8, ku=8, g=1, c=0.0))
    assert res.n_events > 0


def _fp32_residuals(A32, B32, ksteps):
    """Residuals of the row and column checks when everything runs in FP32
    (products and sums rounded to binary32), evaluated after the given
    prefixes of k.  Independent of the oracle's FP64 code."""
    m, K = A32.shape
    n = B32.shape[1]
    P = np.zeros((m, n), np.float32)
    R = np.zeros(m, np.float32)
    S = np.zeros(n, np.float32)
    v = B32.sum(axis=1, dtype=np.float32)
    w = A32.sum(axis=0, dtype=np.float32)
    out = {}
    for p in range(K):
        P = (P + np.outer(A32[:, p], B32[p, :]).astype(np.float32)).astype(np.float32)
        R = (R + (A32[:, p] * v[p]).astype(np.float32)).astype(np.float32)
        S = (S + (w[p] * B32[p, :]).astype(np.float32)).astype(np.float32)
        if p + 1 in ksteps:
            rr = P.sum(axis=1, dtype=np.float32).astype(np.float64) - R.astype(np.float64)
            cc = P.sum(axis=0, dtype=np.float32).astype(np.float64) - S.astype(np.float64)
            out[p + 1] = (rr, cc)
    return out


@pytest.mark.parametrize("dist", ["uniform", "positive", "normal", "heavy"])
def test_threshold_bounds_fp32_roundoff(dist):
    """The detection bound beta must exceed the residual produced by FP32
    arithmetic (zero false positives at tau = 2 beta, with margin)."""
    worst = 0.0
    for s in range(6):
        m, n, K = 24, 20, 256
        if dist == "uniform":
            A, B = W.uniform((m, K), 98, 2 * s), W.uniform((K, n), 98, 2 * s + 1)
        elif dist == "positive":
            A, B = W.uniform((m, K), 98, 2 * s, 0.0, 1.0), W.uniform((K, n), 98, 2 * s + 1, 0.0, 1.0)
        elif dist == "normal":
            A, B = W.normal((m, K), 98, 2 * s), W.normal((K, n), 98, 2 * s + 1)
        else:
            A, B = W.heavy_tailed((m, K), 98, 2 * s), W.heavy_tailed((K, n), 98, 2 * s + 1)
        A64, B64 = A.astype(np.float64), B.astype(np.float64)
        res = _fp32_residuals(A, B, {64, 128, 256})
        for kp, (rr, cc) in res.items():
            na = np.linalg.norm(A64[:, :kp], axis=1)
            nb = np.linalg.norm(B64[:kp, :], axis=0)
            for i in range(m):
                b = O.beta_bound(O.U_FP32, kp, n, na[i], nb.sum())
                worst = max(worst, abs(rr[i]) / b)
            for j in range(n):
                b = O.beta_bound(O.U_FP32, kp, m, nb[j], na.sum())
                worst = max(worst, abs(cc[j]) / b)
    assert worst < 1.0, worst
    # not vacuous: real FP32 residuals reach a visible fraction of the bound
    if dist == "positive":
        assert worst > 1e-3, worst


def test_threshold_closed_form_constant_operands():
    """A = 2 (all entries), B = 3: after K' indices ||a_i|| = 2 sqrt(K'),
    ||b_j|| = 3 sqrt(K'), so beta_row = 2u (K'+n+1) * 2 sqrt(K') * n * 3 sqrt(K')
    = 12 u n K' (K'+n+1) and symmetrically beta_col = 12 u m K' (K'+m+1)."""
    m, n, k, ku = 5, 3, 10, 4
    A = np.full((m, k), 2.0, dtype=np.float32)
    B = np.full((k, n), 3.0, dtype=np.float32)
    u = O.U_FP32
    for t, kp in [(0, 4), (1, 8), (2, 10)]:
        inj = O.make_injections([(0, 0, t, 1, 2, 0.0, 1e6)])
        c = O.replay(A, B, O.ReplayConfig(mc=m, nc=n, ku=ku, g=1), injections=inj).classes[0]
        assert c["check_step"] == t
        assert c["beta_row"] == pytest.approx(12 * u * n * kp * (kp + n + 1), rel=1e-12)
        assert c["beta_col"] == pytest.approx(12 * u * m * kp * (kp + m + 1), rel=1e-12)
        assert c["tau_row"] == pytest.approx(2.0 * c["beta_row"], rel=1e-15)


def test_beta_formula_closed_form():
    """beta = 2u (K' + count + 1) * own_norm * other_norm_sum."""
    assert O.beta_bound(2.0 ** -24, 100, 27, 3.0, 5.0) == pytest.approx(2 * 2.0 ** -24 * 128 * 15.0, rel=1e-15)
    assert O.beta_bound(0.5, 0, 0, 1.0, 1.0) == pytest.approx(1.0)


# ---------------------------------------------------------------------------
# locate + correct (section 4.2.1, section 5.3) under the SEU model (4.1)
# ---------------------------------------------------------------------------
def _tiny_problem():
    m, n, k = 6, 5, 7
    A = W.uniform((m, k), 99, 0)
    B = W.uniform((k, n), 99, 1)
    cfg = O.ReplayConfig(mc=4, nc=3, ku=3, g=1)   # ragged tiles 4+2 x 3+2, steps 3+3+1
    return A, B, cfg


@pytest.mark.parametrize("delta", [1e3, -1e3, math.inf, -math.inf, math.nan, 7.5])
def test_exhaustive_single_error_located_and_corrected(delta):
    """Brute force over every tile, every element and every k-step: one
    must-detect fault is reported exactly at its site and C equals the
    fault-free product."""
    A, B, cfg = _tiny_problem()
    m, n, k = A.shape[0], B.shape[1], A.shape[1]
    clean = O.gemm(A, B)
    nk = (k + cfg.ku - 1) // cfg.ku
    checked = 0
    for tm in range(2):
        for tn in range(2):
            rows = min(cfg.mc, m - tm * cfg.mc)
            cols = min(cfg.nc, n - tn * cfg.nc)
            for t in range(nk):
                for r in range(rows):
                    for c in range(cols):
                        inj = O.make_injections([(tm, tn, t, r, c, 0.0, delta)])
                        res = O.replay(A, B, cfg, injections=inj)
                        assert res.classes[0]["cls"] == O.CLS_MUST
                        assert res.n_events == 1
                        e = res.events[0]
                        assert (e["tile_m"], e["tile_n"], e["kstep"], e["row"], e["col"], e["kind"]) == \
                            (tm, tn, t, r, c, O.EV_CORRECTED)
                        assert np.allclose(res.C, clean, rtol=0, atol=1e-12)
                        checked += 1
    assert checked == (4 * 3 + 4 * 2 + 2 * 3 + 2 * 2) * nk


def test_sub_threshold_fault_is_benign_and_stays():
    A, B, cfg = _tiny_problem()
    clean = O.gemm(A, B)
    inj = O.make_injections([(1, 1, 2, 1, 1, 0.0, 1e-9)])
    res = O.replay(A, B, cfg, injections=inj)
    assert res.classes[0]["cls"] == O.CLS_BENIGN
    assert res.n_events == 0
    d = res.C - clean
    assert d[4 + 1, 3 + 1] == pytest.approx(1e-9, rel=1e-6)
    d[4 + 1, 3 + 1] = 0
    assert np.all(np.abs(d) < 1e-14)


def test_classes_follow_tau_and_beta():
    """must: |delta| > tau + beta on both sides; benign: |delta| < tau - beta
    on both sides; grey: in between (either outcome valid)."""
    A, B, cfg = _tiny_problem()
    probe = O.replay(A, B, cfg, injections=O.make_injections([(0, 0, 0, 1, 2, 0.0, 1e3)]))
    c = probe.classes[0]
    hi = max(c["tau_row"] + c["beta_row"], c["tau_col"] + c["beta_col"])
    lo = min(c["tau_row"] - c["beta_row"], c["tau_col"] - c["beta_col"])
    assert lo > 0
    for d, want in [(hi * 1.01, O.CLS_MUST), (lo * 0.99, O.CLS_BENIGN), (0.5 * (lo + hi), O.CLS_GREY)]:
        r = O.replay(A, B, cfg, injections=O.make_injections([(0, 0, 0, 1, 2, 0.0, d)]))
        assert r.classes[0]["cls"] == want, (d, lo, hi)


def _two(A, B, cfg, a, b):
    return O.replay(A, B, cfg, injections=O.make_injections([a, b]))


def test_two_faults_same_interval_are_uncorrectable_never_miscorrected():
    """SEU violated (section 4.1): two faults in one tile and one check
    interval must be reported UNCORRECTABLE and C left as computed."""
    A, B, cfg = _tiny_problem()
    cases = {
        "distinct rows and cols": ((0, 0, 1, 0, 0, 0.0, 1e3), (0, 0, 1, 2, 1, 0.0, 1e3), 2, 2),
        "same row": ((0, 0, 1, 1, 0, 0.0, 1e3), (0, 0, 1, 1, 2, 0.0, 1e3), 1, 2),
        "same col": ((0, 0, 1, 0, 1, 0.0, 1e3), (0, 0, 1, 3, 1, 0.0, 1e3), 2, 1),
        "cancelling in a row": ((0, 0, 1, 1, 0, 0.0, 1e3), (0, 0, 1, 1, 2, 0.0, -1e3), 0, 2),
    }
    clean = O.gemm(A, B)
    for name, (a, b, nr, nc) in cases.items():
        res = _two(A, B, cfg, a, b)
        assert res.n_events == 1, name
        e = res.events[0]
        assert e["kind"] == O.EV_UNCORRECTABLE, name
        assert (e["n_rows"], e["n_cols"]) == (nr, nc), name
        diff = res.C - clean                       # C left as computed: both faults remain
        assert diff[a[3], a[4]] == pytest.approx(a[6], rel=1e-9), name
        assert diff[b[3], b[4]] == pytest.approx(b[6], rel=1e-9), name


def test_one_fault_per_interval_many_per_run_all_corrected():
    """Online correction (section 2.2, Eq. 4): one fault per step is
    corrected, so a run survives as many faults as it has check intervals,
    and tiles are independent."""
    A, B, cfg = _tiny_problem()
    clean = O.gemm(A, B)
    faults = [(0, 0, 0, 1, 1, 0.0, 1e3), (0, 0, 1, 2, 0, 0.0, -5e2), (0, 0, 2, 3, 2, 0.0, math.inf),
              (1, 1, 0, 1, 1, 0.0, 1e3), (1, 0, 0, 0, 0, 0.0, 1e4), (0, 1, 0, 3, 1, 0.0, math.nan)]
    res = O.replay(A, B, cfg, injections=O.make_injections(faults))
    assert res.n_events == len(faults)
    assert all(e["kind"] == O.EV_CORRECTED for e in res.events)
    got = sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]))
                 for e in res.events)
    assert got == sorted(f[:5] for f in faults)
    assert np.allclose(res.C, clean, rtol=0, atol=1e-12)


def test_check_interval_delays_detection_to_next_check():
    A, B, _ = _tiny_problem()
    cfg = O.ReplayConfig(mc=4, nc=3, ku=2, g=3)   # k=7 -> steps 0..3, checks after 2 and 3
    res = O.replay(A, B, cfg, injections=O.make_injections([(0, 0, 0, 2, 1, 0.0, 1e3)]))
    assert res.n_events == 1 and res.events[0]["kstep"] == 2
    assert res.classes[0]["check_step"] == 2
    res = O.replay(A, B, cfg, injections=O.make_injections([(0, 0, 3, 2, 1, 0.0, 1e3)]))
    assert res.events[0]["kstep"] == 3


def test_forced_row_only_is_checksum_event_and_rebases():
    A, B, cfg = _tiny_problem()
    clean = O.gemm(A, B)
    inj = O.make_injections([(0, 0, 0, 1, 1, 0.0, 1e3, 1)])   # GPU saw the row only
    res = O.replay(A, B, cfg, injections=inj)
    # step 0: row only -> row checksum re-based; step 1: the column still sees
    # the fault -> column checksum re-based; step 2: nothing left to flag.
    assert res.n_events == 2
    assert [(int(e["kstep"]), int(e["kind"])) for e in res.events] == \
        [(0, O.EV_CHECKSUM_ROW), (1, O.EV_CHECKSUM_COL)]
    assert (res.events[0]["row"], res.events[1]["col"]) == (1, 1)
    assert res.C[1, 1] - clean[1, 1] == pytest.approx(1e3)


def test_detect_only_level_reports_at_final_check_and_keeps_error():
    A, B, _ = _tiny_problem()
    cfg = O.ReplayConfig(mc=4, nc=3, ku=3, g=1, ft_level=1)
    clean = O.gemm(A, B)
    res = O.replay(A, B, cfg, injections=O.make_injections([(0, 0, 0, 1, 1, 0.0, 1e3)]))
    assert res.n_events == 1
    e = res.events[0]
    assert e["kind"] == O.EV_DETECTED and e["kstep"] == 2 and (e["row"], e["col"]) == (1, 1)
    assert res.C[1, 1] - clean[1, 1] == pytest.approx(1e3)


def test_level_off_applies_faults_without_checks():
    A, B, _ = _tiny_problem()
    cfg = O.ReplayConfig(mc=4, nc=3, ku=3, g=1, ft_level=0)
    clean = O.gemm(A, B)
    res = O.replay(A, B, cfg, injections=O.make_injections([(1, 0, 1, 0, 2, 0.0, 1e3)]))
    assert res.n_events == 0
    assert res.C[4, 2] - clean[4, 2] == pytest.approx(1e3)


def test_replay_without_faults_equals_plain_gemm_with_alpha_beta():
    A = W.normal((37, 53), 100, 0)
    B = W.normal((53, 41), 100, 1)
    C0 = W.normal((37, 41), 100, 2)
    ref = O.gemm(A, B, C0, alpha=0.75, beta=-1.25)
    res = O.replay(A, B, O.ReplayConfig(mc=16, nc=16, ku=8, g=2), C0=C0, alpha=0.75, beta=-1.25)
    assert res.n_events == 0
    assert np.max(np.abs(res.C - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_replay_tile_subset_matches_full():
    A = W.normal((40, 30), 101, 0)
    B = W.normal((30, 50), 101, 1)
    cfg = O.ReplayConfig(mc=16, nc=16, ku=8, g=1)
    full = O.replay(A, B, cfg)
    part = O.replay(A, B, cfg, tiles=[(1, 2), (2, 0)])
    assert np.array_equal(part.C[16:32, 32:48], full.C[16:32, 32:48])
    assert np.array_equal(part.C[32:40, 0:16], full.C[32:40, 0:16])


# ---------------------------------------------------------------------------
# operand decoders
# ---------------------------------------------------------------------------
def test_decode_e4m3_known_codes():
    codes = np.array([0x00, 0x38, 0xB8, 0x7E, 0x08, 0x01, 0x07, 0x40, 0x3C])
    want = [0.0, 1.0, -1.0, 448.0, 2.0 ** -6, 2.0 ** -9, 7 * 2.0 ** -9, 2.0, 1.5]
    assert list(O.decode_e4m3(codes)) == want
    assert np.isnan(O.decode_e4m3(np.array([0x7F, 0xFF]))).all()


def test_decode_e4m3_all_codes_vs_torch():
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = O.decode_e4m3(codes)
    assert np.array_equal(np.isnan(ref), np.isnan(got))
    assert np.array_equal(ref[~np.isnan(ref)], got[~np.isnan(got)])


def test_decode_bf16_all_codes_vs_torch():
    torch = pytest.importorskip("torch")
    codes = np.arange(65536, dtype=np.uint16)
    ref = torch.from_numpy(codes.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    got = O.decode_bf16(codes)
    ok = ~np.isnan(ref)
    assert np.array_equal(np.isnan(ref), np.isnan(got))
    assert np.array_equal(ref[ok], got[ok])


# ---------------------------------------------------------------------------
# binary64 roundoff (the FP64 path replays with u = 2^-53)
# ---------------------------------------------------------------------------
def test_fp64_roundoff_clean_runs_raise_nothing():
    """At u = 2^-53 the threshold still bounds the oracle's own binary64
    residuals: no event on clean N(0,1), heavy-tailed and positive data,
    a check after every k-step, ragged tiles."""
    for s, gen in enumerate((W.normal64, W.heavy_tailed, W.uniform64)):
        A, B = gen((40, 200), 99, 2 * s), gen((200, 36), 99, 2 * s + 1)
        res = O.replay(A, B, O.ReplayConfig(mc=16, nc=16, ku=8, g=1, u=O.U_FP64, c=2.0))
        assert res.n_events == 0, gen.__name__


def test_fp64_threshold_sees_what_fp32_cannot():
    """A +1e-6 fault on N(0,1) data: far below the binary32 threshold (about
    1e-2 here, so benign and kept), far above the binary64 one (about 1e-10,
    so located and corrected at its site); u enters the threshold."""
    A, B = W.normal64((32, 64), 100, 0), W.normal64((64, 32), 100, 1)
    clean = O.gemm(A, B)
    inj = O.make_injections([(1, 0, 3, 5, 7, 0.0, 1e-6)])
    r32 = O.replay(A, B, O.ReplayConfig(mc=16, nc=16, ku=8, g=1, u=O.U_FP32, c=2.0), injections=inj)
    assert r32.n_events == 0 and r32.classes[0]["cls"] == O.CLS_BENIGN
    assert abs(r32.C[16 + 5, 7] - clean[16 + 5, 7] - 1e-6) < 1e-12
    r64 = O.replay(A, B, O.ReplayConfig(mc=16, nc=16, ku=8, g=1, u=O.U_FP64, c=2.0), injections=inj)
    assert r64.classes[0]["cls"] == O.CLS_MUST and r64.n_events == 1
    e = r64.events[0]
    assert (e["tile_m"], e["tile_n"], e["kstep"], e["row"], e["col"], e["kind"]) == (1, 0, 3, 5, 7, O.EV_CORRECTED)
    assert np.max(np.abs(r64.C - clean)) < 1e-12


# ---------------------------------------------------------------------------
# non-finite operands (the paper's checks assume finite data; reading: a tile
# whose operands hold Inf or NaN is reported once, nothing is located or
# corrected there, and C is what IEEE arithmetic gives)
# ---------------------------------------------------------------------------
def _py_gemm(A, B):
    """Brute-force product in pure Python floats (IEEE binary64, ascending k)."""
    m, k = A.shape
    n = B.shape[1]
    out = np.zeros((m, n))
    for i in range(m):
        for j in range(n):
            s = 0.0
            for p in range(k):
                s += float(A[i, p]) * float(B[p, j])
            out[i, j] = s
    return out


def _same_ieee(X, Y):
    return (np.array_equal(np.isnan(X), np.isnan(Y)) and np.array_equal(np.isinf(X), np.isinf(Y))
            and np.array_equal(X[np.isinf(X)], Y[np.isinf(Y)])
            and np.allclose(X[np.isfinite(X)], Y[np.isfinite(Y)], rtol=0, atol=1e-12))


@pytest.mark.parametrize("where,value", [("A", math.nan), ("A", math.inf), ("B", -math.inf), ("B", math.nan)])
def test_nonfinite_operand_reported_once_per_tile_and_c_is_ieee(where, value):
    A, B, cfg = _tiny_problem()            # 6 x 5 x 7, tiles 4+2 x 3+2, k-steps 3+3+1, a check every step
    A, B = A.astype(np.float64), B.astype(np.float64)
    if where == "A":
        A[5, 4] = value                    # row 5 -> tile row 1; k = 4 -> k-step 1
        want = {(1, 0), (1, 1)}
    else:
        B[3, 1] = value                    # column 1 -> tile column 0; k = 3 -> k-step 1
        want = {(0, 0), (1, 0)}
    res = O.replay(A, B, cfg)
    keys = sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]),
                   int(e["kind"])) for e in res.events)
    assert keys == sorted((tm, tn, 1, -1, -1, O.EV_NONFINITE) for (tm, tn) in want)
    assert _same_ieee(res.C, _py_gemm(A, B))


def test_nonfinite_tile_does_not_stop_corrections_elsewhere():
    A, B, cfg = _tiny_problem()
    A, B = A.astype(np.float64), B.astype(np.float64)
    A[5, 0] = math.nan                     # tile row 1 non-finite from k-step 0
    clean = _py_gemm(A, B)
    inj = O.make_injections([(0, 1, 2, 3, 1, 0.0, 1e3), (1, 0, 1, 0, 0, 0.0, 1e3)])
    res = O.replay(A, B, cfg, injections=inj)
    keys = sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]),
                   int(e["kind"])) for e in res.events)
    assert keys == [(0, 1, 2, 3, 1, O.EV_CORRECTED), (1, 0, 0, -1, -1, O.EV_NONFINITE),
                    (1, 1, 0, -1, -1, O.EV_NONFINITE)]
    # the finite tile is corrected; the fault in the non-finite tile stays (row 4, column 0
    # holds a finite value plus 1e3, since only row 5 carries the NaN)
    assert res.classes[0]["cls"] == O.CLS_MUST and res.classes[1]["cls"] == -1
    want = clean.copy()
    want[4, 0] += 1e3
    assert _same_ieee(res.C, want)


def test_nonfinite_operand_at_detect_only_level():
    A, B, cfg = _tiny_problem()
    A, B = A.astype(np.float64), B.astype(np.float64)
    B[6, 4] = math.inf                     # column 4 -> tile column 1; k = 6 -> last k-step
    res = O.replay(A, B, O.ReplayConfig(mc=cfg.mc, nc=cfg.nc, ku=cfg.ku, g=1, ft_level=1))
    keys = sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["kind"])) for e in res.events)
    assert keys == [(0, 1, 2, O.EV_NONFINITE), (1, 1, 2, O.EV_NONFINITE)]
