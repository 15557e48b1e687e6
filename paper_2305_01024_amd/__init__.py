"""Online algorithm-based fault-tolerant GEMM for AMD MI355X (gfx950).

The compute path is the HIP library ``lib/libftgemm.so`` (C ABI declared in
``include/ftgemm.h``); :mod:`paper_2305_01024_amd.ftgemm` is its thin ctypes
binding.  :mod:`paper_2305_01024_amd.workloads` holds the seeded synthetic
input generators shared by tests and benchmark.
"""
