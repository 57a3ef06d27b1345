"""FP64 CPU oracle for the wavelet / blur / FISTA / convolution-adjoint path.

TEST INFRASTRUCTURE ONLY. Plain, slow, obviously-correct NumPy float64 code
written from the paper (Folberth & Becker, "Efficient Adjoint Computation for
Wavelet and Convolution Operators", IEEE SPM Lecture Notes 2016). Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it. The GPU library never calls it and shares no code with it.

Modules:
  filters    Daubechies scaling filters by spectral factorization (Sec. "The
             adjoint for orthogonal wavelets": Haar and Daubechies).
  extension  Extension operators E (zero, half-point symmetric, periodic),
             their multiplicities and the adjoint of the pseudoinverse
             (Sec. "A few signal extensions").
  wavelet    Zero-boundary core Phi, one-level and multi-level 2-D
             W (synthesis), W^dagger (analysis), W^* (true adjoint, eq. 2).
  blur       Gaussian PSF R with reflexive boundaries and its adjoint R^*.
  fista      Objective of eq. 1, its gradient, soft threshold and FISTA.
  conv       Blind-channel convolution and its two adjoints (Sec. "Example 2").
  cnn        Reference conv3x3 network used by the learned warm start.
"""
