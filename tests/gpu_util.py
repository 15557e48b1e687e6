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


def log_to_injections(log) -> np.ndarray:
    return O.make_injections([(int(l["tile_m"]), int(l["tile_n"]), int(l["kstep"]), int(l["row"]),
                               int(l["col"]), float(l["old_v"]), float(l["new_v"])) for l in log])


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
