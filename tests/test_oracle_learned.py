"""Pins of the learned-preconditioner oracle (oracle/learned.py) against
closed forms, exact polynomial interpolation and finite differences."""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import learned as Lr
from workloads import grid_laplacian
from workloads.learned import init_weights, parameter_count


def test_spectral_map_and_features():
    a, b = Lr.spectral_map(2.0, 10.0)
    assert a * 2.0 + b == -1.0 and a * 10.0 + b == 1.0
    x = Lr.features(6.0 + 2.0j, 2.0, 10.0, 2.0, 10.0)
    np.testing.assert_allclose(x, [0.0, 0.5, -1.0, 1.0], atol=1e-15)


def test_chebyshev_vectors_closed_form():
    # diagonal A: T_k(A^) r = cos(k arccos t_i) r_i with t_i the mapped entries
    lam = np.linspace(1.0, 9.0, 17)
    r = np.random.default_rng(0).standard_normal(17)
    T = Lr.cheb_vectors(sp.diags(lam), 1.0, 9.0, r)
    t = (2 * lam - 10.0) / 8.0
    for k in range(Lr.K):
        np.testing.assert_allclose(T[k], np.cos(k * np.arccos(t)) * r, atol=1e-13)


def test_quadratic_loss_matches_direct_residual():
    A = grid_laplacian((9, 7), 0.01).to_scipy()
    rng = np.random.default_rng(1)
    r = rng.standard_normal(A.shape[0]) + 0.3j * rng.standard_normal(A.shape[0])
    z = 1.3 + 0.2j
    G, h, rr = Lr.sample_data(A, 0.0, 8.01, z, r)
    assert np.abs(G - G.conj().T).max() <= 1e-12 * np.abs(G).max()
    assert np.linalg.eigvalsh(G).min() > 0
    c = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    direct = z * Lr.apply_poly(A, 0.0, 8.01, c, r) - A @ Lr.apply_poly(A, 0.0, 8.01, c, r) - r
    assert abs(Lr.quad_loss(c, G, h, rr) - np.vdot(direct, direct).real / rr) <= 1e-10
    cs = Lr.c_star(G, h)
    best = Lr.quad_loss(cs, G, h, rr)
    assert abs(best - (1.0 - np.vdot(h, np.linalg.solve(G, h)).real / rr)) <= 1e-10
    for _ in range(5):
        d = 1e-3 * (rng.standard_normal(8) + 1j * rng.standard_normal(8))
        assert Lr.quad_loss(cs + d, G, h, rr) > best


def test_exact_inverse_for_eight_eigenvalues():
    # with 8 distinct eigenvalues a degree-7 polynomial interpolates 1/(z - t)
    # on the spectrum: p(A) = (zI - A)^{-1}, zero loss, one-step solve
    lam = np.array([0.5, 1.0, 2.0, 3.0, 4.5, 5.0, 6.5, 8.0])
    A = sp.diags(np.repeat(lam, 3))
    z = 2.4 + 0.5j
    r = np.random.default_rng(2).standard_normal(24)
    G, h, rr = Lr.sample_data(A, 0.0, 8.5, z, r)
    cs = Lr.c_star(G, h)
    assert Lr.quad_loss(cs, G, h, rr) <= 1e-10
    x, it, res = Lr.pc_cocg(A, z, r, cs, 0.0, 8.5, tol=1e-10)
    assert it == 1 and res <= 1e-10
    np.testing.assert_allclose(x, r / (z - np.repeat(lam, 3)), rtol=1e-9)


def test_gelu_values_and_derivative():
    phi1 = 0.5 * (1.0 + math.erf(1.0 / math.sqrt(2.0)))
    np.testing.assert_allclose(Lr.gelu(np.array([0.0, 1.0, -1.0])), [0.0, phi1, -(1.0 - phi1)],
                               atol=1e-16)
    x = np.linspace(-4, 4, 33)
    fd = (Lr.gelu(x + 1e-6) - Lr.gelu(x - 1e-6)) / 2e-6
    np.testing.assert_allclose(Lr.gelu_grad(x), fd, atol=1e-8)


def _samples(count=12, seed=3):
    A = grid_laplacian((8, 8), 0.01).to_scipy()
    rng = np.random.default_rng(seed)
    X, G, h, rr = [], [], [], []
    for s in range(count):
        z = rng.uniform(0.1, 2.0) + 1j * rng.uniform(0.01, 0.5)
        r = rng.standard_normal(64)
        g_, h_, rr_ = Lr.sample_data(A, 0.0, 8.01, z, r)
        X.append(Lr.features(z, 0.0, 8.01, 0.04, 1.5))
        G.append(g_)
        h.append(h_)
        rr.append(rr_)
    return np.array(X), np.array(G), np.array(h), np.array(rr)


@pytest.mark.parametrize("standardize", [False, True])
def test_network_gradient_against_finite_differences(standardize):
    params = [(W.astype(np.float64), b.astype(np.float64) + 0.01) for W, b in init_weights(7)]
    assert sum(W.size + b.size for W, b in params) == parameter_count() == 9680
    X, G, h, rr = _samples()
    # the input standardization of the training features (a fixed affine map
    # of the inputs: the gradient with respect to the weights goes through it)
    norm = None
    if standardize:  # constant features (the Ritz values here) keep sd = 1
        mu, sd = X.mean(axis=0), X.std(axis=0)
        sd[sd <= 1e-9 * np.maximum(1.0, np.abs(mu))] = 1.0
        norm = (mu, sd)
    grads = Lr.batch_grad(params, X, G, h, rr, norm=norm)
    rng = np.random.default_rng(4)
    for l in range(len(params)):
        for which in (0, 1):
            P = params[l][which]
            idx = tuple(rng.integers(0, s) for s in P.shape)
            old = P[idx]
            eps = 1e-6 * max(1.0, abs(old))
            P[idx] = old + eps
            lp = Lr.batch_loss(params, X, G, h, rr, norm=norm)
            P[idx] = old - eps
            lm = Lr.batch_loss(params, X, G, h, rr, norm=norm)
            P[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = grads[l][which][idx]
            assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-6), (l, which, an, fd)


def test_network_outputs_are_scaled_coefficients():
    # c_k = (y_2k + i y_2k+1) / Im z^: a network whose outputs equal
    # Im z^ times the optimal coefficients reaches the per-sample optimum
    X, G, h, rr = _samples(count=3)
    Y = np.zeros((3, 16))
    for s in range(3):
        c = Lr.c_star(G[s], h[s]) * X[s, 1]
        Y[s, 0::2], Y[s, 1::2] = c.real, c.imag
    C = Lr.coeffs(Y, X)
    for s in range(3):
        np.testing.assert_allclose(C[s], Lr.c_star(G[s], h[s]), rtol=1e-12)
        assert Lr.quad_loss(C[s], G[s], h[s], rr[s]) <= Lr.quad_loss(0 * C[s], G[s], h[s], rr[s])
    # and the standardization is (x - mu) / sd before the first layer
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in init_weights(2)]
    mu, sd = X.mean(axis=0), np.array([0.5, 2.0, 4.0, 8.0])
    np.testing.assert_allclose(Lr.mlp_forward(params, X, (mu, sd))[0],
                               Lr.mlp_forward(params, (X - mu) / sd)[0], rtol=1e-14)


def test_preconditioned_cocg_against_direct_solve():
    A = grid_laplacian((12, 12), 0.01).to_scipy()
    n = A.shape[0]
    z = 0.9 + 0.05j
    b = np.random.default_rng(5).standard_normal(n)
    ref = np.linalg.solve(z * np.eye(n) - A.toarray(), b)
    kappa = 8.01 / 0.05
    x0, it0, r0 = Lr.pc_cocg(A, z, b, None, 0.0, 8.01)
    G, h, _ = Lr.sample_data(A, 0.0, 8.01, z, b)
    x1, it1, r1 = Lr.pc_cocg(A, z, b, Lr.c_star(G, h), 0.0, 8.01)
    for x, r in ((x0, r0), (x1, r1)):
        assert r <= 1e-10
        assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1.1 * kappa * 1e-10
    assert it1 < it0  # the fitted polynomial cuts the iteration count


def test_bf16_round_is_nearest_even():
    # hand cases: ties go to the even neighbour, 1 + 2^-7 is the next value
    # above 1, 65504 rounds up to 65536
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -1 - 2.0 ** -8, 65504.0,
                  1 + 2.0 ** -7 + 2.0 ** -9])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, -1.0, 65536.0, 1 + 2.0 ** -7])
    np.testing.assert_array_equal(Lr.bf16_round(x).astype(np.float64), want)
    # against torch's own bfloat16 conversion (an independent implementation)
    import torch

    r = np.random.default_rng(3).standard_normal(20000).astype(np.float32) * 10.0 ** np.arange(
        -10, 10).repeat(1000).astype(np.float32)
    ref = torch.from_numpy(r).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(Lr.bf16_round(r), ref)


def test_bf16_network_stays_near_the_fp64_one():
    # the reduced-precision network differs from the FP64 one by bfloat16
    # rounding (8 significant bits), not by more
    params = init_weights(4)
    X = np.random.default_rng(8).standard_normal((40, 4))
    norm = (X.mean(axis=0), X.std(axis=0))
    Y64 = Lr.mlp_forward(params, X, norm)[0]
    Y16 = Lr.mlp_forward(params, X, norm, bf16=True)[0]
    rel = np.linalg.norm(Y16 - Y64) / np.linalg.norm(Y64)
    assert 1e-5 < rel < 3e-2
    # identity weights through one layer: bf16 rounding of the input only
    P1 = [(np.eye(4, dtype=np.float32), np.zeros(4, dtype=np.float32))]
    x = np.array([[1 + 3 * 2.0 ** -8, 2.0, -0.5, 1 + 2.0 ** -9]])
    np.testing.assert_array_equal(Lr.mlp_forward(P1, x, bf16=True)[0],
                                  Lr.bf16_round(x).astype(np.float64))
