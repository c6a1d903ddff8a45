"""FP64 CPU oracle for the curved-space D3Q19 lattice Boltzmann path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product path never does.  See ``lbm_oracle.cpp``
for the method and its conventions.
"""
from .oracle import Oracle, dual_forces, lib_path, run_forces, set_threads, threads  # noqa: F401
