"""The statistical applications of Section 4, written out (test
infrastructure: the oracle side only).

* ``sample_covariance``  eq. sample-cov: Sigma = X^T X / (n - 1) for an
  n x p data matrix X (rows are samples).
* ``covariance_spectrum``  the nonzero spectrum of Sigma through the n x n
  matrix X X^T / (n - 1), which has the same nonzero eigenvalues (the squared
  singular values of X / sqrt(n - 1)): a route to the reference values that
  never forms the p x p matrix.
* ``variance_count``  the variance-explained rule stated for kernel PCA
  (Section 4.2): the smallest k with sum_{i<=k} lambda_i / tr >= frac, the
  eigenvalues taken in decreasing order.
* ``top_window``  the search interval of a top window of k eigenvalues: from
  the midpoint of the gap below lambda_k to a given upper end.
"""

from __future__ import annotations

import numpy as np


def sample_covariance(X):
    """eq. sample-cov: X^T X / (n - 1), X n x p (dense, FP64)."""
    X = np.asarray(X, dtype=np.float64)
    return (X.T @ X) / (X.shape[0] - 1)


def covariance_spectrum(X):
    """Eigenvalues of X X^T / (n - 1) in decreasing order: the nonzero
    eigenvalues of the sample covariance (eq. sample-cov), and zeros."""
    X = np.asarray(X, dtype=np.float64)
    G = (X @ X.T) / (X.shape[0] - 1)
    return np.sort(np.linalg.eigvalsh(G))[::-1]


def dense_spectrum(K):
    """All eigenvalues of a dense symmetric matrix in decreasing order."""
    return np.sort(np.linalg.eigvalsh(np.asarray(K, dtype=np.float64)))[::-1]


def variance_count(eigs_desc, trace, frac=0.95):
    """Smallest k with sum of the k largest eigenvalues >= frac * trace
    (Section 4.2's rule for kernel PCA; the same rule serves the covariance).
    eigs_desc: eigenvalues in decreasing order (enough of them to reach the
    fraction); trace: the trace of the matrix."""
    c = np.cumsum(np.asarray(eigs_desc, dtype=np.float64))
    idx = np.nonzero(c >= frac * trace)[0]
    if len(idx) == 0:
        raise ValueError("the eigenvalues given do not reach the requested fraction")
    return int(idx[0]) + 1


def top_window(eigs_desc, k, upper):
    """[lmin, lmax] holding exactly the k largest eigenvalues: lmin at the
    midpoint of (lambda_{k+1}, lambda_k), lmax = upper (>= lambda_1)."""
    e = np.asarray(eigs_desc, dtype=np.float64)
    if upper < e[0]:
        raise ValueError("upper end below the largest eigenvalue")
    return 0.5 * (e[k - 1] + e[k]), float(upper)
