"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code.

Two builds, both with gcc's sanitizer runtimes and no recovery (the first
report aborts the process):

* the oracle (oracle/ftgemm_oracle.c), run under its own pin suites
  (test_oracle_pins.py, test_oracle_complex.py): every GEMM, encoding, tile
  replay, injection, complex and non-finite path the pins exercise;
* the library's host API (csrc/ftgemm_api.cpp) linked with the unchanged HIP
  kernel objects, run under the ABI suite (test_abi.py): argument
  validation with BLAS argument positions, configuration selection, status
  strings, NULL-handle and no-device paths, and the fault-site helpers.

The suites run in a subprocess with the ASan runtime preloaded (the Python
interpreter itself is not instrumented) and with FTGEMM_ORACLE_LIB /
FTGEMM_LIB pointing at the sanitized builds.  No GPU is needed or used; the
GPU kernels themselves are outside what a host sanitizer can see.  CPU only.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

from oracle import oracle as O
from paper_2305_01024_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]

pytestmark = pytest.mark.skipif(os.environ.get("FTGEMM_SANITIZED") == "1",
                                reason="already running under the sanitizers")


def _asan_runtime():
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("gcc/g++ not available")
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("gcc's ASan runtime is not installed")
    return rt


def _run_suites(files, env_extra, rt):
    env = dict(os.environ, LD_PRELOAD=rt, FTGEMM_SANITIZED="1", OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join(ROOT, "tests", f) for f in files]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, f"sanitized run failed:\n{out}"
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out


def test_oracle_under_asan_ubsan(tmp_path):
    rt = _asan_runtime()
    lib = O.build(extra_flags=SAN, out=str(tmp_path / "liboracle_san.so"))
    _run_suites(["test_oracle_pins.py", "test_oracle_complex.py"], {"FTGEMM_ORACLE_LIB": lib}, rt)


def test_host_api_under_asan_ubsan(tmp_path):
    rt = _asan_runtime()
    objs = [os.path.join(B.LIBDIR, "obj", s + ".o") for s in B.HIP_SOURCES]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        pytest.skip(f"HIP objects not built ({os.path.basename(missing[0])}): run the package build first")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not glob.glob(os.path.join(rocm, "lib", "libamdhip64.so*")):
        pytest.skip("HIP runtime library not found")
    api = str(tmp_path / "ftgemm_api_san.o")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fPIC", *SAN, "-D__HIP_PLATFORM_AMD__",
                    f"-I{rocm}/include", f"-I{B.INCLUDE}", f"-I{B.CSRC}", "-c",
                    os.path.join(B.CSRC, "ftgemm_api.cpp"), "-o", api], check=True)
    lib = str(tmp_path / "libftgemm_san.so")
    subprocess.run(["g++", "-shared", *SAN, api, *objs, f"-L{rocm}/lib", "-lamdhip64",
                    f"-Wl,-rpath,{rocm}/lib", "-o", lib], check=True)
    _run_suites(["test_abi.py"], {"FTGEMM_LIB": lib}, rt)
