"""Plain, slow, FP64 CPU oracle for RA-FEAST (test infrastructure only).

This package is test infrastructure.  It exists to check the GPU library, and
only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  The GPU library never calls it and shares no code with it.

It follows the paper step by step (FEAST Algorithm 1, RA-FEAST Algorithm 2,
eq. projector-quad, eq. rand-range), in numpy float64, using library
primitives (dense/sparse LU solves, Householder QR, symmetric eigensolver) as
single steps, with no blocking or fusion.

Modules
-------
contour   Gauss-Legendre quadrature on the half circle and the rational filter.
feast     Rayleigh-Ritz, FEAST iteration (literal and residual-correction
          forms), the randomized warmstart and RA-FEAST.
philox    Philox4x32-10 counter-based generator and the Box-Muller map.
subspace  Canonical angles / sin-Theta between subspaces.
spectrum  Gershgorin bounds and reference spectra for window fixtures.
cocg      Plain COCG for complex-symmetric systems.
mlp       Forward/backward of the small preconditioner MLP and its loss.
stats     Sample covariance, its spectrum through X X^T, the variance-explained
          rule and top windows (Section 4).
"""
