"""FP64 CPU oracle for the preconditioned MLBA deblurring iteration.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library itself never does, and this package imports nothing from the library.

Every function follows a passage of Cai, Donatelli, Bianchi, Huang,
"Regularization preconditioners for frame-based image deblurring with reduced
boundary artifacts" (arXiv:1504.07234), cited in its docstring.  Arithmetic is
float64 throughout.

Modules
  blur      the blur A and its transpose for the rectangular model and the
            imposed boundary conditions (section 2, eq. (Arect), Table 1)
  framelet  undecimated linear B-spline tight framelet W and W^T (section 6.1)
  precond   spectral Tikhonov preconditioners (Algorithms 1 and 3)
  mlba      soft threshold, the iteration (MLBA2), schedules, ||A^T P A||
  adjoint   reverse-mode gradient of K unrolled iterations
  alg2      Algorithm 2, the PCG-approximated preconditioner (section 4.2)
  alg4      Algorithm 4 and Algorithm 4-NS (section 5)
"""
from . import adjoint, alg2, alg4, blur, framelet, precond, mlba  # noqa: F401

RECT, REFLECT, PERIODIC, ZERO = blur.RECT, blur.REFLECT, blur.PERIODIC, blur.ZERO
BCCB, DCT, NONE = precond.BCCB, precond.DCT, precond.NONE
