"""Pins for the oracle's quadrature and rational filter (eq. projector,
eq. projector-quad)."""

import math
import os

import numpy as np
import pytest

from oracle.contour import filter_value, gauss_legendre, half_circle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_gl():
    rows = {}
    with open(os.path.join(GOLDEN, "gauss_legendre.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            N, xe, we = line.split()
            rows.setdefault(int(N), []).append((eval(xe, {"math": math}), eval(we, {"math": math})))
    return rows


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_gauss_legendre_closed_form(N):
    x, w = gauss_legendre(N)
    ref = _golden_gl()[N]
    np.testing.assert_allclose(x, [r[0] for r in ref], atol=1e-15)
    np.testing.assert_allclose(w, [r[1] for r in ref], rtol=1e-14)


@pytest.mark.parametrize("N", [1, 2, 3, 6, 8, 16, 32])
def test_gauss_legendre_exact_on_polynomials(N):
    # exact for degree <= 2N-1: int_{-1}^{1} x^k dx = 2/(k+1) (k even), 0 (k odd)
    x, w = gauss_legendre(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * N):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, x ** k) - exact) < 1e-13, (N, k)
    # and not exact at degree 2N (the error constant is still visible for N <= 8)
    if N <= 8:
        assert abs(np.dot(w, x ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-10


@pytest.mark.parametrize("nc", [1, 2, 3, 4, 8, 16, 32])
def test_filter_centre_one_edges_half(nc):
    lmin, lmax = -0.3, 2.7
    z, w = half_circle(lmin, lmax, nc)
    vals = filter_value(np.array([0.5 * (lmin + lmax), lmin, lmax]), z, w)
    assert abs(vals[0] - 1.0) < 1e-14
    # at the edges the nodes nearest the real axis lose a few digits to
    # cancellation in z_j - lam
    assert abs(vals[1] - 0.5) < 1e-13
    assert abs(vals[2] - 0.5) < 1e-13
    # nodes lie on the upper half circle
    c, r = 0.5 * (lmin + lmax), 0.5 * (lmax - lmin)
    np.testing.assert_allclose(np.abs(z - c), r, rtol=1e-15)
    assert np.all(z.imag > 0)


def test_filter_tends_to_window_indicator():
    # Residue theorem: (1/2 pi i) \oint dz/(z - lam) is 1 inside, 0 outside.
    lmin, lmax = 0.0, 1.0
    lam_in = np.array([0.1, 0.3, 0.5, 0.7, 0.9])
    lam_out = np.array([-0.5, -0.2, -0.1, 1.1, 1.2, 3.0])
    prev = None
    for nc in (8, 16, 32):
        z, w = half_circle(lmin, lmax, nc)
        err = max(np.abs(filter_value(lam_in, z, w) - 1).max(),
                  np.abs(filter_value(lam_out, z, w)).max())
        if prev is not None:
            assert err < prev * 0.05
        prev = err
    assert prev < 1e-9


def test_filter_equals_projector_on_small_matrix():
    # One exact filter application equals V rho(Lambda) V^T Q.
    from oracle.feast import ShiftedSolver, filter_block

    rng = np.random.default_rng(3)
    n = 40
    B = rng.standard_normal((n, n))
    A = 0.5 * (B + B.T)
    lam, V = np.linalg.eigh(A)
    lmin, lmax = lam[10] - 0.05, lam[20] + 0.05
    z, w = half_circle(lmin, lmax, 6)
    Q = rng.standard_normal((n, 5))
    import scipy.sparse as sp

    solver = ShiftedSolver(sp.csr_matrix(A), z, method="dense")
    got = filter_block(solver, z, w, Q, form="literal")
    ref = V @ (filter_value(lam, z, w)[:, None] * (V.T @ Q))
    np.testing.assert_allclose(got, ref, atol=1e-12)
