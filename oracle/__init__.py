"""FP64 CPU oracle for the maximum-likelihood map-maker (test infrastructure).

This package is a slow, plain, obviously-correct statement of what the
map-maker computes, written from the MADmap paper (Cantalupo et al.,
arXiv:0906.1775).  It exists only to check the HIP library: the tests, the
smoke check and the benchmark's CPU-baseline leg may import it; the library and
its Python binding never do, and the two share no code.

Contents
--------
pointing  the sparse pointing matrix A (Formalism section) and hit counts.
noise     the 1/f power spectrum p(f) (Algorithm section), the inverse-noise
          lag kernel f(|t - t'|) of the banded Toeplitz N^-1 (Weighting
          section) and its application by plain linear convolution.
fftlen    the FFT-length rule of the Weighting section and Appendix A.
solver    H = A^T N^-1 A, b = A^T N^-1 d (eq. pcgSystem), the white-noise
          block preconditioner (A^T W^-1 A)^-1 and point-Jacobi
          (Implementation section), and the preconditioned conjugate-gradient
          iteration that returns the lowest-residual iterate.
gradient  gradients of a quadratic map loss with respect to the TOD and the
          noise parameters (f_knee, alpha), by one adjoint solve.

Everything is float64.  Inputs given as float32 (TOD, polarisation weights)
are upcast exactly, so the oracle sees the same numbers the library sees.
"""

from . import fftlen, gradient, noise, pointing, solver  # noqa: F401
from .solver import Oracle  # noqa: F401
