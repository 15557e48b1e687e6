"""FP64 CPU oracle for online ABFT GEMM.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.
"""
