"""Canonical angles between subspaces (Section 3.2.1, the angle matrix Theta;
Lemma 2: the 2-norm distance of the two orthogonal projectors equals the
largest sine of the canonical angles)."""

from __future__ import annotations

import numpy as np


def orthonormal_basis(X):
    """Orthonormal basis of range(X) by Householder QR (X of full column rank)."""
    Q, _ = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    return Q


def sin_theta(U, V):
    """Sines of the canonical angles between range(U) and range(V).

    Both are orthonormalised first.  The cosines are the singular values of
    U^T V; sines are returned in decreasing order, clipped to [0, 1].
    """
    Uq = orthonormal_basis(U)
    Vq = orthonormal_basis(V)
    if Uq.shape[1] != Vq.shape[1]:
        raise ValueError("subspaces of different dimension")
    s = np.linalg.svd(Uq.T @ Vq, compute_uv=False)
    s = np.clip(s, 0.0, 1.0)
    # sin from the complementary projection is more accurate for tiny angles
    R = Vq - Uq @ (Uq.T @ Vq)
    sn = np.linalg.svd(R, compute_uv=False)
    sn = np.sort(np.clip(sn, 0.0, 1.0))[::-1]
    small = np.sqrt(np.maximum(0.0, 1.0 - np.sort(s) ** 2))
    return np.where(sn < 0.5, sn, small)


def projector_distance(U, V):
    """||P_U - P_V||_2 computed from the explicit projectors (dense, small n)."""
    Uq = orthonormal_basis(U)
    Vq = orthonormal_basis(V)
    D = Uq @ Uq.T - Vq @ Vq.T
    return float(np.linalg.norm(D, 2))
