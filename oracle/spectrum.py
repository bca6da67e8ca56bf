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
