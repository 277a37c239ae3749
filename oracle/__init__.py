"""CPU FP64 oracle for the tiled Cholesky hot path (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library.

Submodules: oracle (the C FP64 factorization and solve, bound with ctypes)
and mixed (low-precision trailing products, scaling, shift, iterative
refinement and preconditioned conjugate gradients, plain numpy).
"""
from .oracle import (  # noqa: F401
    build, potrf, potrf_crout, solve, num_threads, scaled_residual,
    backward_error, row_scaled_error, lib_path, U64,
)
