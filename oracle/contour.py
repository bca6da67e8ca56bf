"""Quadrature for the FEAST spectral projector (Section 2.1, eq. projector and
eq. projector-quad).

The projector onto the eigenvectors with eigenvalues inside a contour is the
contour integral of the resolvent divided by 2*pi*i.  For a circle with centre
c = (lmin+lmax)/2 and radius r = (lmax-lmin)/2, write z = c + r e^{i phi}.
For real symmetric A the integrand at phi and -phi are complex conjugates, so
the full-circle integral equals twice the real part of the upper-half
integral.  Gauss-Legendre on phi in [0, pi] with N_c nodes gives

    P  ~  sum_j Re[ w_j (z_j I - A)^{-1} ],
    z_j = c + r e^{i phi_j},   w_j = (omega_j / 2) r e^{i phi_j},
    phi_j = (pi/2)(1 - x_j),

with (x_j, omega_j) the Legendre nodes and weights on [-1, 1].  N_c counts the
nodes on the upper half (the conjugate lower half is implied), which is the
reading of "N_c contour points" adopted throughout.
"""

from __future__ import annotations

import numpy as np


def gauss_legendre(N: int):
    """Legendre nodes (ascending) and weights on [-1, 1] by Golub-Welsch.

    The nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix of
    the Legendre three-term recurrence (off-diagonal k / sqrt(4k^2 - 1)); the
    weights are 2 * (first eigenvector component)^2.
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    k = np.arange(1, N, dtype=np.float64)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    J = np.diag(beta, 1) + np.diag(beta, -1)
    x, V = np.linalg.eigh(J)
    w = 2.0 * V[0, :] ** 2
    return x, w


def half_circle(lmin: float, lmax: float, nc: int):
    """Nodes z_j and weights w_j (complex arrays of length nc) for the filter."""
    if not lmax > lmin:
        raise ValueError("need lmax > lmin")
    c = 0.5 * (lmin + lmax)
    r = 0.5 * (lmax - lmin)
    x, om = gauss_legendre(nc)
    phi = 0.5 * np.pi * (1.0 - x)
    e = np.exp(1j * phi)
    z = c + r * e
    w = 0.5 * om * r * e
    return z, w


def filter_value(lam, z, w):
    """Rational filter rho(lam) = sum_j Re[w_j / (z_j - lam)] (real array)."""
    lam = np.asarray(lam, dtype=np.float64)
    return np.real(np.sum(w[:, None] / (z[:, None] - lam.reshape(1, -1)), axis=0)).reshape(lam.shape)
