"""FP64 CPU oracle for the expanded-encoding compressed-sensing reconstruction.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is a plain,
slow, obviously correct NumPy implementation of what the GPU library
computes, written from the paper (Varela-Mattatall, Dubovan et al.,
"High-resolution single-shot spiral diffusion-weighted imaging at 7T using
expanded encoding with compressed sensing"):

* ``encoding``  -- the expanded encoding operator A_exp and its adjoint
  (eq. 1; Introduction and Methods 2.1 name its ingredients: B0 map,
  spherical-harmonic field dynamics up to 2nd/3rd order, coil
  sensitivities, arbitrary trajectory), plus the field-parameter
  vector-Jacobian products;
* ``wavelet``   -- periodised orthonormal 2D wavelet transform W (Haar and
  8-tap Daubechies, derived here by spectral factorisation) and the
  soft-threshold proximal map of lambda*||W x||_1 (eq. 1);
* ``solve``     -- FISTA / ISTA on eq. 1 (Methods 2.1), the objective,
  the Lipschitz power iteration, the lambda rule from W A^H y
  (Methods 2.1), NRMSE (Methods 2.2.2) and conjugate-gradient least
  squares with early stopping (Methods 2.1);
* ``splitemu``  -- round-to-nearest-even bf16/fp16 emulation of the
  hi/lo split products, for error-level checks on tiny sizes.

It shares no code with the HIP path and imports nothing from it.  Every
function works in float64/complex128.
"""
from . import encoding, wavelet, solve, splitemu  # noqa: F401
