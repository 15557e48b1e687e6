"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/ftgemm.h declares, its structs have the sizes the binding
assumes, and the host-only entry points (argument validation, configuration
selection, status strings) behave as documented."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2305_01024_amd import ftgemm as F
from paper_2305_01024_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftgemm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ftgemm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    assert os.path.exists(F.LIB_PATH), "build the library first"
    out = subprocess.run(["nm", "-D", "--defined-only", F.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (ftgemm_\w+)", out))
    declared = _declared_functions()
    assert len(declared) >= 10
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    lib = F.lib()
    for name in declared:
        assert hasattr(lib, name)


def test_struct_sizes_match_header_layout():
    # sizes implied by include/ftgemm.h on LP64
    assert F.EVENT_DTYPE.itemsize == 64
    assert F.FAULT_DTYPE.itemsize == 32
    assert F.FAULT_LOG_DTYPE.itemsize == 64
    assert ctypes.sizeof(F.Config) == 24
    assert ctypes.sizeof(F.Report) == 6 * 8 + 4 + 4 + 8 + 24 + 4 + 4 + 4 + 4 + 4 + 4
    assert F.Report.nonfinite_input.offset == 40
    assert F.PROBLEM_DTYPE.itemsize == 96
    assert ctypes.sizeof(F.Tuned) == 56
    assert W.SITE_DTYPE == F.FAULT_DTYPE


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """sizeof/offsetof of every ABI struct, as the host C++ compiler lays them
    out from include/ftgemm.h, against the ctypes / numpy mirrors."""
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        pytest.skip("no host compiler")
    structs = {
        "ftgemm_event_t": F.EVENT_DTYPE, "ftgemm_fault_t": F.FAULT_DTYPE,
        "ftgemm_fault_log_t": F.FAULT_LOG_DTYPE, "ftgemm_problem_t": F.PROBLEM_DTYPE,
    }
    ctypes_structs = {"ftgemm_report_t": F.Report, "ftgemm_config_t": F.Config, "ftgemm_tuned_t": F.Tuned}
    lines = ['#include <cstdio>', '#include <cstddef>', '#include "ftgemm.h"', 'int main() {']
    for name, dt in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fld in dt.names:
            lines.append(f'printf("{name} {fld} %zu\\n", offsetof({name}, {fld}));')
    for name, st in ctypes_structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fld, _ in st._fields_:
            lines.append(f'printf("{name} {fld} %zu\\n", offsetof({name}, {fld}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    r = subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include", "-I/opt/rocm/include",
                        str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        name, fld, val = line.split()
        got[(name, fld)] = int(val)
    for name, dt in structs.items():
        assert got[(name, "size")] == dt.itemsize, name
        for fld in dt.names:
            assert got[(name, fld)] == dt.fields[fld][1], (name, fld)
    for name, st in ctypes_structs.items():
        assert got[(name, "size")] == ctypes.sizeof(st), name
        for fld, _ in st._fields_:
            assert got[(name, fld)] == getattr(st, fld).offset, (name, fld)


def test_enum_values_match_header():
    """Status codes, event kinds, levels and dtypes of the binding equal the
    header's enumerators (parsed from include/ftgemm.h)."""
    text = open(os.path.join(ROOT, "include", "ftgemm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    vals = {k: int(v, 0) for k, v in re.findall(r"\b(FTGEMM_[A-Z0-9_]+)\s*=\s*(-?(?:0x)?[0-9A-Fa-f]+)", text)}
    mirror = {"FTGEMM_OK": F.OK, "FTGEMM_UNCORRECTABLE": F.UNCORRECTABLE,
              "FTGEMM_NONFINITE_INPUT": F.NONFINITE_INPUT, "FTGEMM_INVALID": F.INVALID,
              "FTGEMM_UNSUPPORTED": F.UNSUPPORTED, "FTGEMM_HIP_ERROR": F.HIP_ERROR,
              "FTGEMM_NO_MEMORY": F.NO_MEMORY, "FTGEMM_LOG_OVERFLOW": F.LOG_OVERFLOW,
              "FTGEMM_EV_CORRECTED": F.EV_CORRECTED, "FTGEMM_EV_CHECKSUM_ROW": F.EV_CHECKSUM_ROW,
              "FTGEMM_EV_CHECKSUM_COL": F.EV_CHECKSUM_COL, "FTGEMM_EV_UNCORRECTABLE": F.EV_UNCORRECTABLE,
              "FTGEMM_EV_DETECTED": F.EV_DETECTED, "FTGEMM_EV_NONFINITE": F.EV_NONFINITE,
              "FTGEMM_FT_OFF": F.FT_OFF, "FTGEMM_FT_DETECT": F.FT_DETECT, "FTGEMM_FT_CORRECT": F.FT_CORRECT,
              "FTGEMM_FT_RECOMPUTE": F.FT_RECOMPUTE, "FTGEMM_F32": F.F32, "FTGEMM_BF16": F.BF16,
              "FTGEMM_F8E4M3": F.F8E4M3, "FTGEMM_F64": F.F64, "FTGEMM_C64": F.C64, "FTGEMM_FAULT_ADD": F.FAULT_ADD,
              "FTGEMM_FAULT_XOR": F.FAULT_XOR}
    for name, v in mirror.items():
        assert vals[name] == v, name
    # the status strings distinguish every status
    strings = {F.ftgemm_status_string(v) for v in (F.OK, F.UNCORRECTABLE, F.NONFINITE_INPUT, F.INVALID,
                                                   F.UNSUPPORTED, F.HIP_ERROR, F.NO_MEMORY, F.LOG_OVERFLOW)}
    assert len(strings) == 8 and "unknown status" not in strings


@pytest.mark.parametrize("args,bad", [
    ((-1, 4, 4, 4, 4, 4), 2),
    ((4, -1, 4, 4, 4, 4), 3),
    ((4, 4, -1, 4, 4, 4), 4),
    ((4, 4, 4, 3, 4, 4), 7),
    ((4, 4, 4, 4, 3, 4), 9),
    ((4, 4, 4, 4, 4, 3), 12),
    ((0, 0, 0, 1, 1, 1), 0),
    ((5, 7, 0, 5, 1, 5), 0),
    ((2 ** 31, 4, 4, 2 ** 31, 4, 2 ** 31), 2),
])
def test_validate_reports_blas_argument_positions(args, bad):
    st, got = F.ftgemm_validate(*args)
    assert got == bad
    assert st == (F.OK if bad == 0 else F.INVALID)


def test_validate_level_and_tol():
    assert F.ftgemm_validate(4, 4, 4, 4, 4, 4, ft_level=3)[1] == 13
    assert F.ftgemm_validate(4, 4, 4, 4, 4, 4, ft_level=-1)[1] == 13
    assert F.ftgemm_validate(4, 4, 4, 4, 4, 4, tol=float("nan"))[1] == 14
    assert F.ftgemm_validate(4, 4, 4, 4, 4, 4, tol=-1.0)[1] == 0   # <= 0 selects the default


def test_validate_recompute_flag():
    """FTGEMM_FT_RECOMPUTE is accepted on the fault-tolerant levels only."""
    for lvl in (F.FT_DETECT, F.FT_CORRECT):
        assert F.ftgemm_validate(4, 4, 4, 4, 4, 4, ft_level=lvl | F.FT_RECOMPUTE) == (F.OK, 0)
    assert F.ftgemm_validate(4, 4, 4, 4, 4, 4, ft_level=F.FT_OFF | F.FT_RECOMPUTE)[1] == 13
    assert F.ftgemm_validate(4, 4, 4, 4, 4, 4, ft_level=3 | F.FT_RECOMPUTE)[1] == 13
    assert F.ftgemm_validate(4, 4, 4, 4, 4, 4, ft_level=F.FT_CORRECT | 0x20)[1] == 13


def test_nonfused_and_batched_with_null_handle_are_invalid():
    rep = F.ReportBuffer(4)
    st = F.lib().ftgemm_run_nonfused(None, 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 0, 0.0, None, rep.ptr())
    assert st == F.INVALID and rep.report.bad_arg == 1
    st = F.lib().ftgemm_batched(None, 0, None, F.FT_CORRECT, 0.0, None, rep.ptr())
    assert st == F.INVALID and rep.report.bad_arg == 1


def test_select_config_follows_the_measured_best_tile_and_checks_every_256_k():
    """Automatic selection (a modelled time per FP32 tile: waves of resident
    workgroups at each tile's measured full-load rate) picks, for online FT at
    these square sizes, the tile that was fastest when every compute-tile
    variant was timed on MI355X; compute-tile checks, a check every 256 k."""
    measured_best = {1024: 128, 2048: 128, 2560: 128, 3072: 128, 3584: 256, 4096: 256, 5120: 128, 6144: 128,
                     8192: 256}
    for N, t in measured_best.items():
        c = F.ftgemm_select_config(F.F32, N, N, N, F.FT_CORRECT)
        assert (c.m_tile, c.n_tile) == (t, t), (N, c.as_tuple())
    for (m, n) in [(8192, 8192), (4096, 4096), (2048, 2048), (65536, 256), (256, 65536), (3001, 1999),
                   (100, 100), (1, 1)]:
        for level in (F.FT_OFF, F.FT_DETECT, F.FT_CORRECT, F.FT_CORRECT | F.FT_RECOMPUTE):
            c = F.ftgemm_select_config(F.F32, m, n, 1024, level)
            assert c.k_step * c.check_interval == 256
            assert (c.check_m, c.check_n) == (c.m_tile, c.n_tile)    # automatic selection: compute-tile checks
    for dtype in (F.BF16, F.F8E4M3):
        c = F.ftgemm_select_config(dtype, 8192, 8192, 8192)
        assert (c.check_m, c.check_n) == (c.m_tile, c.n_tile)
    # BF16, the same model with the BF16 tiles' measured rates: 128 x 128 where
    # 256 x 256 tiles would leave most compute units idle (2048^3: 0.079 against
    # 0.144 ms online), 256 x 256 from 3072 on (0.212 against 0.266 ms)
    for N, t in {2048: 128, 3072: 256, 4096: 256, 8192: 256}.items():
        for level in (F.FT_OFF, F.FT_CORRECT):
            c = F.ftgemm_select_config(F.BF16, N, N, N, level)
            assert (c.m_tile, c.n_tile, c.k_step * c.check_interval) == (t, t, 256), (N, level, c.as_tuple())
    # FP8, the same model with the FP8 tiles' measured rates: 128 x 128 up to
    # 2560^3 (2048^3 online: 0.090 against 0.145 ms), 256 x 256 from 3072^3
    # (0.209 against 0.273 ms)
    for N, t in {1024: 128, 2048: 128, 2560: 128, 3072: 256, 4096: 256, 8192: 256}.items():
        for level in (F.FT_OFF, F.FT_CORRECT):
            c = F.ftgemm_select_config(F.F8E4M3, N, N, N, level)
            assert (c.m_tile, c.n_tile, c.k_step * c.check_interval) == (t, t, 256), (N, level, c.as_tuple())
    # FP64: the one compiled configuration, a check every 256 k, for any shape and level
    for (m, n) in [(8192, 8192), (1, 1), (3001, 1999)]:
        for level in (F.FT_OFF, F.FT_DETECT, F.FT_CORRECT):
            assert F.ftgemm_select_config(F.F64, m, n, 512, level).as_tuple() == (128, 128, 16, 16, 128, 128)


def test_status_strings():
    assert F.ftgemm_status_string(F.OK) == "ok"
    assert "invalid" in F.ftgemm_status_string(F.INVALID)


def test_run_with_null_handle_is_invalid_not_a_crash():
    rep = F.ReportBuffer(4)
    st = F.lib().ftgemm_run(None, 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 2, 0.0, None, rep.ptr())
    assert st == F.INVALID and rep.report.bad_arg == 1


def test_create_without_gfx950_is_unsupported():
    """On a host with no gfx950 device the handle is refused, not faked."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert F.lib().ftgemm_create(ctypes.byref(h), F.F32, 0) == F.UNSUPPORTED
    assert h.value is None


def test_fault_sites_respect_one_per_tile_interval():
    g = np.random.default_rng(7)
    m, n, k, mc, nc, ku, gi = 600, 500, 1000, 128, 128, 32, 8
    sites = W.fault_sites(g, m, n, k, mc, nc, ku, gi, count=60, kind=W.KIND_XOR)   # 80 slots
    key = set()
    nk = -(-k // ku)
    for s in sites:
        tile_rows = min(mc, m - s["tile_m"] * mc)
        tile_cols = min(nc, n - s["tile_n"] * nc)
        assert 0 <= s["row"] < tile_rows and 0 <= s["col"] < tile_cols
        assert 0 <= s["kstep"] < nk and 0 <= s["payload"] <= 30
        k_ = (s["tile_m"], s["tile_n"], s["kstep"] // gi)
        assert k_ not in key
        key.add(k_)
