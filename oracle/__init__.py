"""Plain, slow FP64 CPU oracle for the stabilised parareal-like method of
H. Nguyen and R. Tsai, "A stable parareal-like method for the second order
wave equation" (arXiv 1905.00473).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it.  The HIP library
never calls it, links it or falls back to it, and the two share no code.

Every routine is numpy in float64 and follows the paper's definitions in
the paper's order: the discretisation of Sec. 3.1, the data matrices
(eqs. matrixF / matrixG), the discrete wave energy (eq.
discrete-wave-energy), the Procrustes solution of Sec. 3.3, the
incremental SVD of Algorithm 1, the gradient-to-function map of eq.
gradient2coordinate / Algorithm 2 and the iteration of Algorithm 3 /
eq. thetarelation.

Parity status of every function is listed in the header of `wave.py`.
"""

from .wave import *  # noqa: F401,F403
from . import adjoint  # noqa: F401
