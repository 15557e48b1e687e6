"""Pins of the complex binary64 oracle (the double-complex FT-GEMM; section 6
names further data types as future work), against what mathematics fixes:
closed forms, exact Gaussian-integer products checked by brute force, the
encoded-product identities, zero residuals after every step on exact data,
the bound's closed form for constant operands (2K' products per component,
complex 2-norms), the bound against the residuals of binary32 and binary64
arithmetic, exhaustive single-fault injection in either component, and the
per-component reading of the single-event-upset model.  CPU only."""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import workloads as W


def _cnormal(shape, wl, st):
    return np.asfortranarray(W.normal(shape, wl, 2 * st).astype(np.float64) +
                             1j * W.normal(shape, wl, 2 * st + 1).astype(np.float64))


def _gauss_int(shape, wl, st, lo=-4, hi=4):
    return np.asfortranarray(W.integers(shape, wl, 2 * st, lo, hi).astype(np.float64) +
                             1j * W.integers(shape, wl, 2 * st + 1, lo, hi).astype(np.float64))


def _py_zgemm(A, B):
    """Brute force in Python's exact integer arithmetic (Gaussian integers)."""
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), dtype=np.complex128)
    for i in range(m):
        for j in range(n):
            re = im = 0
            for p in range(k):
                ar, ai = int(A[i, p].real), int(A[i, p].imag)
                br, bi = int(B[p, j].real), int(B[p, j].imag)
                re += ar * br - ai * bi
                im += ar * bi + ai * br
            C[i, j] = complex(re, im)
    return C


# ---------------------------------------------------------------------------
# plain complex product
# ---------------------------------------------------------------------------
def test_zgemm_identity_and_i_identity():
    B = _cnormal((7, 5), 600, 0)
    assert np.array_equal(O.zgemm(np.eye(7), B), B)
    assert np.array_equal(O.zgemm(1j * np.eye(7), B), 1j * B)
    assert np.array_equal(O.zgemm(B.T, 1j * np.eye(7)), 1j * B.T)


def test_zgemm_all_one_plus_i():
    """(1+i) everywhere: every element is K (1+i)^2 = 2iK."""
    K = 9
    A = np.full((4, K), 1 + 1j)
    B = np.full((K, 3), 1 + 1j)
    assert np.array_equal(O.zgemm(A, B), np.full((4, 3), 2j * K))


@pytest.mark.parametrize("seed", range(3))
def test_zgemm_gaussian_integers_exact_vs_bruteforce(seed):
    A = _gauss_int((13, 17), 601, seed)
    B = _gauss_int((17, 11), 602, seed)
    assert np.array_equal(O.zgemm(A, B), _py_zgemm(A, B))


def test_zgemm_vs_numpy_and_alpha_beta():
    A = _cnormal((30, 40), 603, 0)
    B = _cnormal((40, 20), 603, 1)
    C0 = _cnormal((30, 20), 603, 2)
    al, be = 0.5 - 2j, -1 + 0.25j
    ref = al * (A @ B) + be * C0
    got = O.zgemm(A, B, C0, alpha=al, beta=be)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13
    # beta == 0: C0 is not read (NaN there stays out)
    got = O.zgemm(A, B, np.full((30, 20), np.nan + 0j), alpha=1.0, beta=0.0)
    assert np.isfinite(got).all()


# ---------------------------------------------------------------------------
# encodings and the checksum relation (Eq. 1-4)
# ---------------------------------------------------------------------------
def test_zencodings_are_column_and_row_sums():
    A = _gauss_int((6, 5), 604, 0)
    B = _gauss_int((5, 4), 604, 1)
    assert np.array_equal(O.zencode_col(A), np.array([sum(A[:, p]) for p in range(5)]))
    assert np.array_equal(O.zencode_row(B), np.array([sum(B[p, :]) for p in range(5)]))


@pytest.mark.parametrize("seed", range(4))
def test_encoded_product_identity_exact_on_gaussian_integers(seed):
    """e^T (A B) = (e^T A) B and (A B) e = A (B e), exactly."""
    A = _gauss_int((9, 12), 605, seed)
    B = _gauss_int((12, 7), 606, seed)
    C = _py_zgemm(A, B)
    w = O.zencode_col(A)
    v = O.zencode_row(B)
    assert np.array_equal(C.sum(axis=0), _py_zgemm(w[None, :], B)[0])
    assert np.array_equal(C.sum(axis=1), _py_zgemm(A, v[:, None])[:, 0])


def test_online_invariance_zero_residual_every_step():
    """Gaussian-integer data: every partial sum is exact, so with tau = 0 (c = 0)
    no check of any step flags."""
    A = _gauss_int((12, 40), 607, 0)
    B = _gauss_int((40, 10), 607, 1)
    res = O.zreplay(A, B, O.ReplayConfig(mc=5, nc=4, ku=3, g=1, c=0.0))
    assert res.n_events == 0
    assert np.array_equal(res.C, _py_zgemm(A, B))


def test_check_flags_roundoff_when_tau_is_zero():
    A = _cnormal((8, 40), 608, 0)
    B = _cnormal((40, 8), 608, 1)
    res = O.zreplay(A, B, O.ReplayConfig(mc=8, nc=8, ku=8, g=1, c=0.0))
    assert res.n_events > 0
    assert {int(e["comp"]) for e in res.events} == {0, 1}


# ---------------------------------------------------------------------------
# the bound: 2K' products per component, complex 2-norms
# ---------------------------------------------------------------------------
def test_bound_closed_form_constant_operands():
    """A = 1+2i everywhere, B = 3-i: |a| = sqrt(5), |b| = sqrt(10); after K'
    indices ||a_i|| = sqrt(5 K'), ||b_j|| = sqrt(10 K'), so
    beta_row = 2u (2K'+n+1) sqrt(5K') n sqrt(10K') = 2u (2K'+n+1) n K' sqrt(50)."""
    m, n, k, ku = 5, 3, 10, 4
    A = np.full((m, k), 1 + 2j)
    B = np.full((k, n), 3 - 1j)
    u = O.U_FP64
    for t, kp in [(0, 4), (1, 8), (2, 10)]:
        for comp in (0, 1):
            inj = O.make_injections([(0, 0, t, 1, 2, 0.0, 1e6, -1, comp)])
            c = O.zreplay(A, B, O.ReplayConfig(mc=m, nc=n, ku=ku, g=1, u=u), injections=inj).classes[0]
            assert c["check_step"] == t
            assert c["beta_row"] == pytest.approx(2 * u * (2 * kp + n + 1) * n * kp * math.sqrt(50), rel=1e-12, abs=0)
            assert c["beta_col"] == pytest.approx(2 * u * (2 * kp + m + 1) * m * kp * math.sqrt(50), rel=1e-12, abs=0)


def _f32_complex_residuals(A, B, K):
    """Row and column residuals when every complex product and sum is formed
    component-wise in binary32 (re = ar br - ai bi, im = ar bi + ai br, each
    product and each addition rounded), independent of the oracle's code."""
    f = np.float32
    Ar, Ai = A.real.astype(f), A.imag.astype(f)
    Br, Bi = B.real.astype(f), B.imag.astype(f)
    m, n = A.shape[0], B.shape[1]
    Pr = np.zeros((m, n), f)
    Pi = np.zeros((m, n), f)
    vr, vi = Br.sum(axis=1, dtype=f), Bi.sum(axis=1, dtype=f)
    wr, wi = Ar.sum(axis=0, dtype=f), Ai.sum(axis=0, dtype=f)
    Rr, Ri = np.zeros(m, f), np.zeros(m, f)
    Sr, Si = np.zeros(n, f), np.zeros(n, f)
    for p in range(K):
        Pr = (Pr + np.outer(Ar[:, p], Br[p]).astype(f)).astype(f)
        Pr = (Pr - np.outer(Ai[:, p], Bi[p]).astype(f)).astype(f)
        Pi = (Pi + np.outer(Ar[:, p], Bi[p]).astype(f)).astype(f)
        Pi = (Pi + np.outer(Ai[:, p], Br[p]).astype(f)).astype(f)
        Rr = (Rr + (Ar[:, p] * vr[p]).astype(f)).astype(f)
        Rr = (Rr - (Ai[:, p] * vi[p]).astype(f)).astype(f)
        Ri = (Ri + (Ar[:, p] * vi[p]).astype(f)).astype(f)
        Ri = (Ri + (Ai[:, p] * vr[p]).astype(f)).astype(f)
        Sr = (Sr + (wr[p] * Br[p]).astype(f)).astype(f)
        Sr = (Sr - (wi[p] * Bi[p]).astype(f)).astype(f)
        Si = (Si + (wr[p] * Bi[p]).astype(f)).astype(f)
        Si = (Si + (wi[p] * Br[p]).astype(f)).astype(f)
    d = np.float64
    rows = [Pr.sum(axis=1, dtype=f).astype(d) - Rr.astype(d), Pi.sum(axis=1, dtype=f).astype(d) - Ri.astype(d)]
    cols = [Pr.sum(axis=0, dtype=f).astype(d) - Sr.astype(d), Pi.sum(axis=0, dtype=f).astype(d) - Si.astype(d)]
    return rows, cols


@pytest.mark.parametrize("dist", ["normal", "positive"])
def test_bound_covers_binary32_complex_residuals(dist):
    """The component bound with u = 2^-24 exceeds every residual of binary32
    complex arithmetic (so the 2K' count of products per component and the
    complex norms are enough), with a visible fraction reached on positive data."""
    worst = 0.0
    for s in range(4):
        m, n, K = 16, 12, 192
        if dist == "normal":
            A, B = _cnormal((m, K), 609, 2 * s), _cnormal((K, n), 609, 2 * s + 1)
        else:
            A = W.uniform((m, K), 610, 2 * s, 0.0, 1.0) + 1j * W.uniform((m, K), 611, 2 * s, 0.0, 1.0)
            B = W.uniform((K, n), 610, 2 * s + 1, 0.0, 1.0) + 1j * W.uniform((K, n), 611, 2 * s + 1, 0.0, 1.0)
        # the binary32 values are the operands
        A = A.real.astype(np.float32).astype(np.float64) + 1j * A.imag.astype(np.float32).astype(np.float64)
        B = B.real.astype(np.float32).astype(np.float64) + 1j * B.imag.astype(np.float32).astype(np.float64)
        rows, cols = _f32_complex_residuals(A, B, K)
        na = np.linalg.norm(A, axis=1)
        nb = np.linalg.norm(B, axis=0)
        for comp in (0, 1):
            for i in range(m):
                worst = max(worst, abs(rows[comp][i]) / O.beta_bound(O.U_FP32, 2 * K, n, na[i], nb.sum()))
            for j in range(n):
                worst = max(worst, abs(cols[comp][j]) / O.beta_bound(O.U_FP32, 2 * K, m, nb[j], na.sum()))
    assert worst < 1.0, worst
    if dist == "positive":
        assert worst > 1e-3, worst


def test_binary64_clean_runs_raise_nothing():
    A = _cnormal((64, 300), 612, 0)
    B = _cnormal((300, 48), 612, 1)
    res = O.zreplay(A, B, O.ReplayConfig(mc=32, nc=16, ku=8, g=2, u=O.U_FP64))
    assert res.n_events == 0
    assert np.linalg.norm(res.C - A @ B) / np.linalg.norm(A @ B) <= 1e-13


# ---------------------------------------------------------------------------
# locate + correct, per component
# ---------------------------------------------------------------------------
def _tiny():
    A = _cnormal((6, 7), 613, 0)
    B = _cnormal((7, 5), 613, 1)
    return A, B, O.ReplayConfig(mc=4, nc=3, ku=3, g=1, u=O.U_FP64)   # ragged 4+2 x 3+2, steps 3+3+1


@pytest.mark.parametrize("delta", [1e3, -1e3, math.inf, math.nan])
@pytest.mark.parametrize("comp", [0, 1])
def test_exhaustive_single_error_in_either_component(delta, comp):
    """Every tile, element, k-step and component: one must-detect fault is
    reported at its site with its component, and C equals the fault-free
    product (the other component untouched)."""
    A, B, cfg = _tiny()
    clean = O.zgemm(A, B)
    checked = 0
    for tm, tn in itertools.product(range(2), range(2)):
        rows = min(cfg.mc, 6 - tm * cfg.mc)
        cols = min(cfg.nc, 5 - tn * cfg.nc)
        for t in range(3):
            for r in range(rows):
                for c in range(cols):
                    inj = O.make_injections([(tm, tn, t, r, c, 0.0, delta, -1, comp)])
                    res = O.zreplay(A, B, cfg, injections=inj)
                    assert res.classes[0]["cls"] == O.CLS_MUST
                    assert res.n_events == 1
                    e = res.events[0]
                    assert (e["tile_m"], e["tile_n"], e["kstep"], e["row"], e["col"], e["kind"], e["comp"]) == \
                        (tm, tn, t, r, c, O.EV_CORRECTED, comp)
                    assert np.allclose(res.C, clean, rtol=0, atol=1e-12)
                    checked += 1
    assert checked == (12 + 8 + 6 + 4) * 3


def test_faults_in_both_components_of_one_interval_are_both_corrected():
    """A fault in the real part of one element and one in the imaginary part
    of another, in the same check interval: each component sees one fault,
    so both are corrected (a complex element is two real values)."""
    A, B, cfg = _tiny()
    inj = O.make_injections([(0, 0, 1, 1, 2, 0.0, 1e3, -1, 0), (0, 0, 1, 3, 0, 0.0, -1e3, -1, 1)])
    res = O.zreplay(A, B, cfg, injections=inj)
    keys = sorted((int(e["row"]), int(e["col"]), int(e["kind"]), int(e["comp"])) for e in res.events)
    assert keys == [(1, 2, O.EV_CORRECTED, 0), (3, 0, O.EV_CORRECTED, 1)]
    assert np.allclose(res.C, O.zgemm(A, B), rtol=0, atol=1e-12)


def test_two_faults_in_one_component_are_uncorrectable():
    A, B, cfg = _tiny()
    inj = O.make_injections([(0, 0, 1, 1, 2, 0.0, 1e3, -1, 1), (0, 0, 1, 3, 0, 0.0, 1e3, -1, 1)])
    res = O.zreplay(A, B, cfg, injections=inj)
    assert [(int(e["kind"]), int(e["comp"])) for e in res.events] == [(O.EV_UNCORRECTABLE, 1)]
    assert res.events[0]["n_rows"] == 2 and res.events[0]["n_cols"] == 2


def test_sub_threshold_fault_stays_in_its_component():
    """At the binary32 bound (u = 2^-24, ~1e-5 here) a 1e-9 fault is benign:
    not flagged, and it stays in its component of C."""
    A, B, _ = _tiny()
    cfg = O.ReplayConfig(mc=4, nc=3, ku=3, g=1, u=O.U_FP32)
    clean = O.zgemm(A, B)
    res = O.zreplay(A, B, cfg, injections=O.make_injections([(1, 1, 2, 1, 1, 0.0, 1e-9, -1, 1)]))
    assert res.classes[0]["cls"] == O.CLS_BENIGN and res.n_events == 0
    d = res.C - clean
    assert d[5, 4].imag == pytest.approx(1e-9, rel=1e-4) and abs(d[5, 4].real) < 1e-14
    d[5, 4] = 0
    assert np.all(np.abs(d) < 1e-14)


def test_detect_only_and_alpha_beta_epilogue():
    A, B, cfg = _tiny()
    C0 = _cnormal((6, 5), 614, 0)
    al, be = 2 - 1j, 0.5j
    inj = O.make_injections([(1, 0, 0, 0, 1, 0.0, 1e3, -1, 1)])
    det = O.zreplay(A, B, O.ReplayConfig(mc=4, nc=3, ku=3, g=1, u=O.U_FP64, ft_level=1), injections=inj)
    assert [(int(e["kind"]), int(e["kstep"]), int(e["comp"])) for e in det.events] == [(O.EV_DETECTED, 2, 1)]
    res = O.zreplay(A, B, cfg, C0=C0, alpha=al, beta=be)
    ref = al * (A @ B) + be * C0
    assert np.linalg.norm(res.C - ref) / np.linalg.norm(ref) <= 1e-13


def test_nonfinite_operand_reported_once():
    A, B, cfg = _tiny()
    A = A.copy()
    A[5, 3] = complex(np.nan, 0.0)     # tile row 1, k-step 1
    res = O.zreplay(A, B, cfg)
    ev = sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["kind"])) for e in res.events)
    assert ev == [(1, 0, 1, O.EV_NONFINITE), (1, 1, 1, O.EV_NONFINITE)]
