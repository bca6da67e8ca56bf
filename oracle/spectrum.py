"""Spectral bounds and reference spectra (window fixtures)."""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def gershgorin(A):
    """Gershgorin interval [sigma_lo, sigma_hi] containing every eigenvalue."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    rad = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    return float(np.min(d - rad)), float(np.max(d + rad))


def dense_eigvalsh(A):
    """All eigenvalues (ascending) of a sparse symmetric matrix, densely (small n)."""
    M = A.toarray() if sp.issparse(A) else np.asarray(A)
    return np.linalg.eigvalsh(M)


def dense_eigh(A):
    M = A.toarray() if sp.issparse(A) else np.asarray(A)
    return np.linalg.eigh(M)


def bottom_eigvalsh(A, k: int):
    """The k smallest eigenvalues by shift-invert Lanczos (larger n)."""
    from scipy.sparse.linalg import eigsh

    lo, _ = gershgorin(A)
    vals = eigsh(sp.csc_matrix(A), k=k, sigma=lo - 1e-3, which="LM",
                 return_eigenvectors=False, tol=1e-14)
    return np.sort(vals)


def count_below(A, sigma: float) -> int:
    """Number of eigenvalues of the symmetric matrix A below sigma, exactly,
    by Sylvester's law of inertia: A - sigma I = P^T L D L^T P for a
    permutation P and unit lower triangular L, and the count is the number of
    negative entries of D.  The factorization is sparse Gaussian elimination
    with a symmetric fill-reducing permutation and no pivoting, so U = D L^T;
    a factorization that pivoted anyway (the row order differs from the
    column order) or that solves a random system with a backward error above
    1e-10 (large element growth) is refused.  Assumes
    sigma is not an eigenvalue (a mid-gap point).  Independent of the Lanczos
    routine above: it is the check on the window fixtures it writes."""
    from scipy.sparse.linalg import splu

    A = sp.csr_matrix(A, dtype=np.float64)
    n = A.shape[0]
    M = (A - sigma * sp.identity(n, format="csr")).tocsc()
    lu = splu(M, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
              options=dict(SymmetricMode=True))
    if not np.array_equal(lu.perm_r, lu.perm_c):
        raise RuntimeError("elimination pivoted: not a symmetric factorization")
    d = lu.U.diagonal()
    if not np.all(np.isfinite(d)) or np.any(d == 0.0):
        raise RuntimeError("zero or non-finite pivot: sigma is (nearly) an eigenvalue")
    b = np.random.default_rng(0).standard_normal(n)
    x = lu.solve(b)
    norm1 = float(abs(M).sum(axis=0).max())
    berr = np.abs(M @ x - b).max() / (norm1 * np.abs(x).max() + np.abs(b).max())
    if not berr <= 1e-10:
        raise RuntimeError(f"unstable factorization (backward error {berr:.1e})")
    return int(np.count_nonzero(d < 0.0))
