"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message, and every dtype the bench accepts names kernel sources that
exist (the hash that ties a hardware-counter summary to its build)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_source_hashes():
    import bench
    seen = set()
    for dtype in bench.KERNEL_SOURCES:
        h = bench.kernel_source_hash(dtype)
        assert len(h) == 64
        seen.add(h)
    assert len(seen) == len(bench.KERNEL_SOURCES)
