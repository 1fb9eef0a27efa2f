"""CPU oracle for the condensed-space IPM hot path (FP64).

TEST INFRASTRUCTURE ONLY: a plain, slow, independent reference used by the
tests, the smoke check and the CPU-baseline leg of the benchmark.  The product
path (the HIP library and its Python binding) never imports it.
"""
