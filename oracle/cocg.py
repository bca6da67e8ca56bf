"""Conjugate Orthogonal Conjugate Gradient (COCG) for complex-symmetric systems.

van der Vorst and Melissen (IEEE Trans. Magn. 1990): CG with the unconjugated
bilinear form x^T y in place of the inner product; it applies to
M = M^T complex, here M = zI - A with A real symmetric and z off the real axis
(the shifted systems of Section 2.1).  Plain loop, FP64/complex128.

    x = x0, r = b - M x, p = r, rho = r^T r
    repeat: w = M p; mu = p^T w; alpha = rho / mu
            x += alpha p; r -= alpha w
            stop if ||r||_2 <= tol ||b||_2
            rho' = r^T r; beta = rho'/rho; p = r + beta p; rho = rho'
"""

from __future__ import annotations

import numpy as np


def cocg(A, z, b, tol=1e-10, maxiter=100000, x0=None):
    """Solve (z I - A) x = b.  Returns (x, iterations, converged)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.complex128).copy()

    def M(v):
        return z * v - A @ v

    r = b - M(x) if x0 is not None else b.copy()
    p = r.copy()
    rho = np.dot(r, r)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, True
    for k in range(1, maxiter + 1):
        w = M(p)
        mu = np.dot(p, w)
        alpha = rho / mu
        x += alpha * p
        r -= alpha * w
        if np.linalg.norm(r) <= tol * bn:
            return x, k, True
        rho_new = np.dot(r, r)
        beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
    return x, maxiter, False
