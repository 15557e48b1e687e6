"""Helpers for the GPU parity tests: column-major device operands, one call
through the C ABI, and comparison of the GPU result and event log with the
FP64 oracle replay."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F

torch = None


def _torch():
    global torch
    if torch is None:
        import torch as t
        torch = t
    return torch


def dev(x: np.ndarray):
    """Column-major (rows, cols) numpy -> device tensor of shape (cols, rows),
    i.e. the same bytes as a column-major matrix with ld = rows."""
    t = _torch()
    return t.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float32).T)).cuda()


def host(d, rows: int, cols: int) -> np.ndarray:
    return np.asfortranarray(d.cpu().numpy().reshape(cols, rows).T)


def run(h, A, B, C0=None, alpha=1.0, beta=0.0, ft_level=F.FT_CORRECT, tol=0.0, cap=16384):
    """One ftgemm_run call with a report; returns (status, C, ReportBuffer)."""
    t = _torch()
    m, k = A.shape
    n = B.shape[1]
    dA = dev(A) if A.size else t.zeros(1, device="cuda")
    dB = dev(B) if B.size else t.zeros(1, device="cuda")
    dC = dev(C0) if C0 is not None else t.zeros((max(n, 1), max(m, 1)), device="cuda")
    rep = F.ReportBuffer(cap)
    st = F.ftgemm_run(h, m, n, k, alpha, dA.data_ptr(), max(m, 1), dB.data_ptr(), max(k, 1), beta,
                      dC.data_ptr(), max(m, 1), ft_level, tol, t.cuda.current_stream().cuda_stream, rep)
    C = host(dC, max(m, 1), max(n, 1))[:m, :n] if m and n else np.zeros((m, n), np.float32)
    return st, C, rep


def rel_fro(C, ref) -> float:
    C = np.asarray(C, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(C - ref) / (den if den > 0 else 1.0))


def event_keys(ev) -> list:
    return sorted((int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]),
                   int(e["kind"])) for e in ev)


def _fault_values(l):
    """(old, new) for the oracle: a finite fault is applied as its exact offset
    (the log's binary64 delta, taken as old = 0, new = delta), a non-finite one
    as the value the accumulator took."""
    d = float(l["delta"])
    if np.isfinite(d) and np.isfinite(l["old_v"]) and np.isfinite(l["new_v"]):
        return 0.0, d
    return float(l["old_v"]), float(l["new_v"])


def log_to_injections(log, comp_field=None) -> np.ndarray:
    """Oracle injections from the GPU's applied-fault log (comp_field: the log
    field that names a complex component)."""
    rows = []
    for l in log:
        old, new = _fault_values(l)
        row = (int(l["tile_m"]), int(l["tile_n"]), int(l["kstep"]), int(l["row"]), int(l["col"]), old, new)
        rows.append(row + ((-1, int(l[comp_field])) if comp_field else ()))
    return O.make_injections(rows)


def _gpu_force(events, inj, check_step) -> int:
    """The flags the GPU raised for an injection's row/col at a check step,
    as the oracle's force bitmask, or None if the pattern is not a plain
    single-site outcome."""
    here = [e for e in events if int(e["tile_m"]) == inj["tile_m"] and int(e["tile_n"]) == inj["tile_n"]
            and int(e["kstep"]) == check_step]
    if not here:
        return 0
    if len(here) > 1:
        return None
    e = here[0]
    kind = int(e["kind"])
    if kind == F.EV_CORRECTED and (e["row"], e["col"]) == (inj["row"], inj["col"]):
        return 3
    if kind == F.EV_CHECKSUM_ROW and e["row"] == inj["row"]:
        return 1
    if kind == F.EV_CHECKSUM_COL and e["col"] == inj["col"]:
        return 2
    return None


def check_cfg(cfg):
    """(check_m, check_n, k_step, check_interval) of a configuration tuple:
    the check tile is the compute tile unless a check shape is given."""
    cm = cfg[4] if len(cfg) > 4 and cfg[4] else cfg[0]
    cn = cfg[5] if len(cfg) > 5 and cfg[5] else cfg[1]
    return (cm, cn, cfg[2], cfg[3])


def replay_against_gpu(A, B, cfg, rep, log, C0=None, alpha=1.0, beta=0.0, ft_level=2, tiles=None, u=O.U_FP32):
    """Replay the run on the oracle with the GPU's applied faults.  Faults the
    oracle classifies grey (either decision is valid) take the GPU's decision;
    returns (ReplayResult, classes of the first pass, n_grey, n_grey_invalid)."""
    cc = check_cfg(cfg)
    rc = O.ReplayConfig(mc=cc[0], nc=cc[1], ku=cc[2], g=cc[3], c=float(rep.report.tol_used),
                        ft_level=ft_level, u=u)
    inj = log_to_injections(log)
    res = O.replay(A, B, rc, C0=C0, alpha=alpha, beta=beta, injections=inj, tiles=tiles)
    grey = np.where(res.classes["cls"] == O.CLS_GREY)[0]
    invalid = 0
    if len(grey):
        ev = rep.events
        for q in grey:
            f = _gpu_force(ev, inj[q], int(res.classes[q]["check_step"]))
            if f is None:
                invalid += 1
            else:
                inj[q]["force"] = f
        first = res.classes.copy()
        res = O.replay(A, B, rc, C0=C0, alpha=alpha, beta=beta, injections=inj, tiles=tiles)
        return res, first, len(grey), invalid
    return res, res.classes, 0, 0


U32 = 2.0 ** -24      # unit roundoff of binary32
# Accumulation model of the FP8 matrix instruction for element-wise bounds:
# it sums its 64 products per instruction below binary32 precision (measured
# on clean N(0,1) data at K = 64, one instruction: |C - AB|_ij up to 2.6e-5
# (|A||B|)_ij, 1.6 times (k + 2) 2^-22), so the element-wise bound takes
# u = 2^-19 for it, a factor of about 5 above that measurement.
U_FP8_ACC = 2.0 ** -19


def _abs_product(A, B):
    return np.abs(np.asarray(A, np.float64)) @ np.abs(np.asarray(B, np.float64))


def elementwise_ratio(C, ref, A, B, cfg=None, alpha=1.0, beta=0.0, C0=None, u=U32, events=(), oracle_events=(),
                      log=(), tile=None, acc_u=None, c=2.0):
    """Largest per-element ratio |C - ref|_ij / bound_ij over C (or the check
    tile `tile` = (tm, tn) of C when given, with C, ref, C0 the full arrays).

    bound_ij = (k + 2) u_acc (|alpha| (|A||B|)_ij + |beta| |C0_ij|): the
    gamma_K bound of an accumulation in any order with one rounding per
    addition, plus the two roundings of the epilogue (u_acc = acc_u, else u).
    An element rebuilt by a correction comes from the row checksum, so its
    error is that of a clean residual, at most beta_row = tau_row / c of the
    oracle's event (c: the threshold factor of the run; its later k-steps
    accumulate as usual); an element
    that keeps a fault delta from the log adds (k + 2) u_acc |delta|.  Events
    and log entries are in check-tile coordinates (cfg gives the check tile)."""
    ua = u if acc_u is None else acc_u
    k = A.shape[1]
    i0 = j0 = 0
    if tile is not None:
        cm, cn = check_cfg(cfg)[:2]
        i0, j0 = tile[0] * cm, tile[1] * cn
        si, sj = slice(i0, min(i0 + cm, C.shape[0])), slice(j0, min(j0 + cn, C.shape[1]))
        C, ref, A, B = C[si, sj], ref[si, sj], A[si], B[:, sj]
        C0 = C0[si, sj] if C0 is not None else None
    bound = (k + 2) * ua * abs(alpha) * _abs_product(A, B)
    if C0 is not None and beta != 0.0:
        bound += (k + 2) * ua * abs(beta) * np.abs(np.asarray(C0, np.float64))
    if cfg is not None:
        cm, cn = check_cfg(cfg)[:2]
        tau_of = {}     # corrected element -> tau_row of its check (the oracle's where it has one)
        for e in list(events) + list(oracle_events):
            if int(e["kind"]) == F.EV_CORRECTED:
                tau_of[(int(e["tile_m"]), int(e["tile_n"]), int(e["row"]), int(e["col"]))] = \
                    abs(float(e["tau_row"]))
        for key, tau in tau_of.items():
            i, j = key[0] * cm + key[2] - i0, key[1] * cn + key[3] - j0
            if 0 <= i < bound.shape[0] and 0 <= j < bound.shape[1]:
                bound[i, j] += abs(alpha) * tau / c     # beta_row = tau_row / c
        for l in log:
            i, j = int(l["tile_m"]) * cm + int(l["row"]) - i0, int(l["tile_n"]) * cn + int(l["col"]) - j0
            if 0 <= i < bound.shape[0] and 0 <= j < bound.shape[1]:
                d = float(l["new_v"]) - float(l["old_v"])
                if np.isfinite(d):
                    bound[i, j] += (k + 2) * ua * abs(alpha) * abs(d)
    err = np.abs(np.asarray(C, np.float64) - np.asarray(ref, np.float64))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(err == 0.0, 0.0, err / bound)
    return float(np.max(r)) if r.size else 0.0


def corrected_value_errors(events, oracle_events, c):
    """For every CORRECTED event of the GPU, |value_after_gpu - value_after_oracle|
    in units of the oracle's beta_row = tau_row / c at that check (the rebuilt
    element's error is at most beta_row).  Returns the largest such ratio
    and the number of events compared."""
    ora = {(int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"])): e
           for e in oracle_events if int(e["kind"]) == F.EV_CORRECTED}
    worst, n = 0.0, 0
    for e in events:
        if int(e["kind"]) != F.EV_CORRECTED:
            continue
        key = (int(e["tile_m"]), int(e["tile_n"]), int(e["kstep"]), int(e["row"]), int(e["col"]))
        o = ora[key]
        beta_row = float(o["tau_row"]) / c
        worst = max(worst, abs(float(e["value_after"]) - float(o["value_after"])) / beta_row)
        n += 1
    return worst, n
