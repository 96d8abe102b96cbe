"""Oracle: a plain, slow, obviously correct FP64 CPU implementation of the
method of "Faster Kernel Interpolation for Gaussian Processes" (Yadav,
Sheldon, Musco).

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  It shares no code with
the HIP library: the O(n) pass is plain serial C (``precompute.c``), the
m-space algebra is NumPy/SciPy in FP64 following the paper's definitions and
algorithms step by step.

Readings of the paper that the oracle fixes (the paper is silent or garbled):
  * cubic interpolation is Keys' cubic convolution with a = -1/2;
  * the kernel is s * exp(-1/2 sum_d (x_d - x'_d)^2 / l_d^2) (s not squared),
    sigma is the noise standard deviation and sigma^2 sits on the diagonal;
  * the CG stop test is relative: ||r|| <= tol * ||b||;
  * the simplified factorized CG loop starts at k = 0;
  * the MLL uses stochastic Lanczos quadrature with Lanczos tridiagonals taken
    from the CG coefficients, and its gradient is the implicit adjoint with a
    Hutchinson trace estimate (or the exact trace on small problems).
"""
from .native import (  # noqa: F401
    stencils, precompute, probe_sketches, probe_values, interpolate,
    wtw_matvec, lib_path, splitmix64,
)
from .ski import *  # noqa: F401,F403
