"""MI355X QTT finite-element elasticity solver (HIP library + thin binding).

The solver lives in libtnfem.so (C ABI: include/tnfem.h); ``tnfem`` is its ctypes
binding.  ``workloads`` holds the seeded problem generators shared by tests and
the benchmark.
"""
