"""GPU parity on the irregular FP32 shapes at full size: tall-skinny
(65536 x 256 x 4096, 256 x 65536 x 4096), small-K (16384 x 16384 x 64) and
odd sizes (3001 x 1999 x 4097), U[-1,1], beta = 0, under the fixed
256 x 256 x 32 / g = 8 configuration and under the autotuned one.  The oracle
replays sampled output tiles (first, last and interior ones, the ragged edge
included); exponent-bit flips in accumulator lanes must give the oracle's
event log on those tiles exactly."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

from gpu_util import check_cfg, event_keys, rel_fro, replay_against_gpu

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


@pytest.fixture(scope="module")
def operands():
    """Host and device operands of the four shapes, generated once."""
    import torch
    out = {}
    for idx, (m, n, k) in enumerate(W.irregular_shapes(3)):
        A = W.uniform((m, k), 3, 10 * idx)
        B = W.uniform((k, n), 3, 10 * idx + 1)
        dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
        dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
        out[(m, n, k)] = (A, B, dA, dB)
    return out


def _sample_tiles(m, n, cfg):
    cfg = check_cfg(cfg)
    ntm, ntn = -(-m // cfg[0]), -(-n // cfg[1])
    pick = {(0, 0), (ntm - 1, ntn - 1), (ntm // 2, ntn // 2), (0, ntn - 1), (ntm - 1, 0)}
    return sorted(pick)


def _run(h, m, n, k, dA, dB, cap=4096):
    import torch
    dC = torch.zeros((n, m), device="cuda")
    rep = F.ReportBuffer(cap)
    st = F.ftgemm_run(h, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k, 0.0, dC.data_ptr(), m,
                      F.FT_CORRECT, 0.0, torch.cuda.current_stream().cuda_stream, rep)
    return st, dC, rep


def _check_tiles(A, B, dC, m, n, cfg, rep, log=None):
    tiles = _sample_tiles(m, n, cfg)
    tset = set(tiles)
    if log is not None and len(log):
        keep = log[np.array([(int(x["tile_m"]), int(x["tile_n"])) in tset for x in log], dtype=bool)]
        res, cls, n_grey, bad = replay_against_gpu(A, B, cfg, rep, keep, tiles=tiles)
        assert bad == 0
    else:
        cc = check_cfg(cfg)
        res = O.replay(A, B, O.ReplayConfig(mc=cc[0], nc=cc[1], ku=cc[2], g=cc[3],
                                            c=float(rep.report.tol_used)), tiles=tiles)
    ev = rep.events
    if len(ev):
        ev = ev[np.array([(int(e["tile_m"]), int(e["tile_n"])) in tset for e in ev], dtype=bool)]
    assert event_keys(ev) == event_keys(res.events)
    C = dC.cpu().numpy()
    cc = check_cfg(cfg)
    for (tm, tn) in tiles:
        i0, j0 = tm * cc[0], tn * cc[1]
        i1, j1 = min(m, i0 + cc[0]), min(n, j0 + cc[1])
        got = C[j0:j1, i0:i1].T
        assert rel_fro(got, res.C[i0:i1, j0:j1]) <= TOL, (tm, tn)
    return res


@pytest.mark.parametrize("mode", ["fixed", "tuned"])
@pytest.mark.parametrize("shape", W.IRREGULAR_SHAPES)
def test_irregular_shape_clean(h, operands, shape, mode):
    import torch
    m, n, k = shape
    A, B, dA, dB = operands[shape]
    if mode == "fixed":
        F.ftgemm_set_config(h, (256, 256, 32, 8))
    else:
        F.ftgemm_set_config(h, None)
        F.ftgemm_tune(h, m, n, k, F.FT_CORRECT, 256, torch.cuda.current_stream().cuda_stream)
    try:
        st, dC, rep = _run(h, m, n, k, dA, dB)
    finally:
        F.ftgemm_set_config(h, None)
    cfg = rep.report.config.as_tuple()
    assert st == F.OK and rep.report.n_events == 0
    assert cfg[2] * cfg[3] <= 256
    _check_tiles(A, B, dC, m, n, cfg, rep)


@pytest.mark.parametrize("shape", W.IRREGULAR_SHAPES)
def test_irregular_shape_exponent_bit_flips(h, operands, shape):
    """Flips of exponent bits 23..30 in accumulator lanes, at most one per tile
    per check interval, 40 per launch: the sampled tiles' events and values
    equal the oracle replay of the logged faults."""
    m, n, k = shape
    A, B, dA, dB = operands[shape]
    cfg = F.ftgemm_select_config(F.F32, m, n, k).as_tuple()
    ntm, ntn = -(-m // cfg[0]), -(-n // cfg[1])
    nk = -(-k // cfg[2])
    slots = ntm * ntn * -(-nk // cfg[3])
    count = min(40, slots)
    g = W.rng(3, W.STREAM_SITES)
    sites = W.fault_sites(g, m, n, k, cfg[0], cfg[1], cfg[2], cfg[3], count, kind=W.KIND_XOR, bits=range(23, 31))
    # put a fault into every sampled tile as well, so the comparison sees some
    extra = []
    for (tm, tn) in _sample_tiles(m, n, cfg):
        if not np.any((sites["tile_m"] == tm) & (sites["tile_n"] == tn)):
            rows = min(cfg[0], m - tm * cfg[0])
            cols = min(cfg[1], n - tn * cfg[1])
            extra.append((tm, tn, int(g.integers(0, nk)), int(g.integers(0, rows)), int(g.integers(0, cols)),
                          W.KIND_XOR, float(g.integers(23, 31)), 0))
    if extra:
        sites = np.concatenate([sites, np.array(extra, dtype=F.FAULT_DTYPE)])
        sites = sites[np.lexsort((sites["kstep"], sites["tile_n"], sites["tile_m"]))]
    F.ftgemm_set_config(h, cfg)          # the sites are drawn for this tiling
    F.ftgemm_set_injection(h, sites)
    try:
        st, dC, rep = _run(h, m, n, k, dA, dB)
        log = F.ftgemm_get_injection_log(h)
    finally:
        F.ftgemm_set_injection(h, None)
        F.ftgemm_set_config(h, None)
    assert len(log) == len(sites)
    _check_tiles(A, B, dC, m, n, cfg, rep, log)
