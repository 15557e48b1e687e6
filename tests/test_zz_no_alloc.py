"""The allocation-free entry point ftgemm_run_noalloc, called through the C
ABI, against ftgemm_run (the handle entry point it is a variant of) on the
same operands: C bitwise equal (the same kernels and configuration), the same
status, counts and event log.  Two calls in a row, the second on a smaller
problem, so the static workspace's leftovers from the first call must not
leak into the second; events come from non-finite operands (the no-alloc
entry has no injection hook)."""
import ctypes

import numpy as np
import pytest

from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

pytestmark = pytest.mark.gpu


def _operands(m, n, k, seed, nan_at=None):
    A = W.normal((m, k), seed, 0)
    B = W.normal((k, n), seed, 1)
    C0 = W.normal((m, n), seed, 2)
    if nan_at is not None:
        A[nan_at] = np.nan
    return A, B, C0


def _call(fn, first, m, n, k, A, B, C0, level):
    import torch
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    dC = torch.from_numpy(np.ascontiguousarray(C0.T)).cuda()
    rep = F.ReportBuffer(2048)
    st = fn(first, m, n, k, 0.75, ctypes.c_void_p(dA.data_ptr()), m, ctypes.c_void_p(dB.data_ptr()), k, 1.25,
            ctypes.c_void_p(dC.data_ptr()), m, level, 0.0, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
            rep.ptr())
    torch.cuda.synchronize()
    return st, dC.cpu().numpy(), rep


def _compare(h, m, n, k, seed, level, nan_at=None):
    A, B, C0 = _operands(m, n, k, seed, nan_at)
    st0, C0h, r0 = _call(F.lib().ftgemm_run, ctypes.c_void_p(h), m, n, k, A, B, C0, level)
    st1, C1, r1 = _call(F.lib().ftgemm_run_noalloc, F.F32, m, n, k, A, B, C0, level)
    assert st1 == st0 and st0 >= 0
    assert np.array_equal(C1, C0h, equal_nan=True)
    for f in ("checks", "detected", "corrected", "uncorrectable", "checksum_only", "nonfinite_input",
              "n_events", "recomputed", "recompute_failed"):
        assert getattr(r1.report, f) == getattr(r0.report, f), f
    assert r1.report.config.as_tuple() == r0.report.config.as_tuple()
    assert np.array_equal(np.sort(r1.events, order=["tile_m", "tile_n", "kstep"]),
                          np.sort(r0.events, order=["tile_m", "tile_n", "kstep"]))
    return st1, r1


@pytest.fixture(scope="module")
def h():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    handle = F.ftgemm_create(F.F32, 0)
    yield handle
    F.ftgemm_destroy(handle)


def test_noalloc_matches_run_two_calls_second_smaller(h):
    st, rep = _compare(h, 1536, 1280, 1024, 420, F.FT_CORRECT, nan_at=(700, 300))
    assert st == F.NONFINITE_INPUT and rep.report.nonfinite_input > 0
    st, rep = _compare(h, 300, 200, 130, 421, F.FT_CORRECT)
    assert st == F.OK and rep.report.n_events == 0 and rep.report.nonfinite_input == 0


def test_noalloc_levels_and_recompute(h):
    for level in (F.FT_OFF, F.FT_DETECT, F.FT_DETECT | F.FT_RECOMPUTE, F.FT_CORRECT | F.FT_RECOMPUTE):
        _compare(h, 640, 520, 300, 422, level)


def test_noalloc_rejects_a_recompute_queue_beyond_its_workspace():
    """More output tiles than the static queue holds, with recompute: a clear
    error before any launch (the host checks the size; nothing runs)."""
    rep = F.ReportBuffer(4)
    # 64x64 tiles are never picked for this shape; the default tile count is checked on the host
    m = n = 256 * 129
    st = F.lib().ftgemm_run_noalloc(F.F32, m, n, 64, 1.0, ctypes.c_void_p(16), m, ctypes.c_void_p(16), 64, 0.0,
                                    ctypes.c_void_p(16), m, F.FT_CORRECT | F.FT_RECOMPUTE, 0.0, None, rep.ptr())
    assert st == F.NO_MEMORY


def test_noalloc_argument_errors():
    rep = F.ReportBuffer(4)
    st = F.lib().ftgemm_run_noalloc(F.F32, 8, 8, 8, 1.0, None, 4, None, 8, 0.0, None, 8, 2, 0.0, None, rep.ptr())
    assert st == F.INVALID and rep.report.bad_arg == 7
    st = F.lib().ftgemm_run_noalloc(F.F64, 8, 8, 8, 1.0, None, 8, None, 8, 0.0, None, 8, 2, 0.0, None, rep.ptr())
    assert st == F.UNSUPPORTED
