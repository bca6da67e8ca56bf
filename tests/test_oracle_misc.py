"""Pins for the oracle's Philox/Box-Muller sketch, COCG and subspace metric."""

import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.cocg import cocg
from oracle.philox import gaussian_sketch, philox4x32_10
from oracle.subspace import projector_distance, sin_theta
from workloads import grid_laplacian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for row in rows:
        v = [int(x, 16) for x in row]
        ctr = [np.array([c], dtype=np.uint64) for c in v[0:4]]
        out = philox4x32_10(ctr, (np.uint64(v[4]), np.uint64(v[5])))
        assert [int(o[0]) for o in out] == v[6:10]


def test_box_muller_special_values_and_moments():
    # rad = 1 when u1 = exp(-1/2); angle 0 gives (1, 0)
    u1 = math.exp(-0.5)
    rad = math.sqrt(-2 * math.log(u1))
    assert abs(rad - 1.0) < 1e-15
    G = gaussian_sketch(200000, 6, seed=1234)
    assert G.shape == (200000, 6)
    m = G.mean(axis=0)
    v = G.var(axis=0)
    se = 1 / math.sqrt(200000)
    assert np.all(np.abs(m) < 5 * se)
    assert np.all(np.abs(v - 1) < 5 * math.sqrt(2) * se)
    C = np.corrcoef(G.T)
    assert np.abs(C - np.eye(6)).max() < 5 * se
    # fourth moment of N(0,1) is 3
    assert abs((G ** 4).mean() - 3.0) < 0.05
    # deterministic in the seed, different across seeds, odd widths truncate
    np.testing.assert_array_equal(gaussian_sketch(50, 5, 7), gaussian_sketch(50, 6, 7)[:, :5])
    assert np.abs(gaussian_sketch(50, 4, 7) - gaussian_sketch(50, 4, 8)).max() > 0.1


def test_sin_theta_equals_projector_distance_lemma2():
    rng = np.random.default_rng(0)
    for _ in range(5):
        U = rng.standard_normal((60, 7))
        V = U + 0.05 * rng.standard_normal((60, 7))
        assert abs(sin_theta(U, V).max() - projector_distance(U, V)) < 1e-12
    # identical subspaces, orthogonal subspaces
    U = rng.standard_normal((30, 4))
    assert sin_theta(U, U @ rng.standard_normal((4, 4))).max() < 1e-13
    E = np.eye(30)
    assert abs(sin_theta(E[:, :4], E[:, 4:8]).max() - 1.0) < 1e-15


def test_cocg_matches_direct_solve():
    A = grid_laplacian((30, 30), 0.01).to_scipy()
    rng = np.random.default_rng(0)
    b = rng.standard_normal(900)
    for z in (0.1 + 0.05j, 0.3 + 0.002j):
        x, it, ok = cocg(A, z, b, tol=1e-12)
        assert ok
        M = (z * sp.identity(900) - A).toarray()
        np.testing.assert_allclose(x, np.linalg.solve(M, b), rtol=0, atol=1e-9 * np.abs(x).max())
        assert np.linalg.norm(z * x - A @ x - b) <= 1.01e-12 * np.linalg.norm(b)
    # a smaller imaginary part needs more iterations
    _, it_far, _ = cocg(A, 0.1 + 0.05j, b, tol=1e-10)
    _, it_near, _ = cocg(A, 0.1 + 0.002j, b, tol=1e-10)
    assert it_near > it_far
