"""Checks shared by the end-to-end GPU tests: eigenvalues against a reference,
scaled residuals, orthonormality, subspace angle within the Davis-Kahan bound,
and the sign convention."""

import numpy as np

from oracle.subspace import sin_theta


def gap_out(all_eigs, lmin, lmax):
    inside = all_eigs[(all_eigs >= lmin) & (all_eigs <= lmax)]
    outside = all_eigs[(all_eigs < lmin) | (all_eigs > lmax)]
    return np.min(np.abs(outside[:, None] - inside[None, :]))


def check_against(out, A, lam_ref, V_ref, lmin, lmax, tol_eig, gap):
    s_win = max(abs(lmin), abs(lmax))
    assert out["M"] == len(lam_ref)
    assert np.abs(out["lam"] - lam_ref).max() <= 1e-10 * s_win
    X = out["X"]
    R = A @ X - X * out["lam"][None, :]
    res = np.linalg.norm(R, axis=0) / s_win
    assert res.max() <= tol_eig * 1.0001
    # the two sides evaluate A x - lambda x in FP64 in different orders: they
    # agree to rounding, about u ||A||_inf ||x|| per column, relative to s_win
    floor = 16 * np.finfo(np.float64).eps * abs(A).sum(axis=1).max() / s_win
    np.testing.assert_allclose(out["resid"], res, rtol=1e-3, atol=floor)
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() < 1e-12
    st = sin_theta(X, V_ref).max()
    assert st <= max(1e-8, 2 * np.linalg.norm(R) / gap), st
    # sign convention: largest-magnitude entry positive
    idx = np.argmax(np.abs(X), axis=0)
    assert np.all(X[idx, np.arange(X.shape[1])] > 0)
