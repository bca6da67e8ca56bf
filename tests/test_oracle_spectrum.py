"""Pins for the oracle's spectral helpers and for the window fixtures they
wrote (tests/golden/windows.json).

The reference spectra of the kNN workloads come from shift-invert Lanczos
(oracle.spectrum.bottom_eigvalsh).  They are checked here against two
independent routes: a dense symmetric eigensolve where n is small enough,
and an exact eigenvalue count by Sylvester's law of inertia (sparse LDL^T of
A - sigma I) at the window edges, which catches a missed or doubled
eigenvalue that would silently move a window edge.
"""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import feast as F
from oracle.cocg import cocg
from oracle.contour import filter_value, half_circle
from oracle.learned import pc_cocg
from oracle.spectrum import bottom_eigvalsh, count_below, dense_eigvalsh, gershgorin
from workloads import grid_laplacian, knn_laplacian, rgg_laplacian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _windows():
    with open(os.path.join(GOLDEN, "windows.json")) as f:
        return json.load(f)


# ------------------------------------------------------------- Gershgorin ---

def test_gershgorin_hand_computed():
    # rows: 4 - (|-1| + |2|) = 1 .. 4 + 3 = 7;  -2 - (1 + 0.5) .. -2 + 1.5;
    # 1 - (2 + 0.5) .. 1 + 2.5  ->  [min(1, -3.5, -1.5), max(7, -0.5, 3.5)]
    A = np.array([[4.0, -1.0, 2.0],
                  [-1.0, -2.0, 0.5],
                  [2.0, 0.5, 1.0]])
    lo, hi = gershgorin(sp.csr_matrix(A))
    assert lo == -3.5 and hi == 7.0
    ev = np.linalg.eigvalsh(A)
    assert lo <= ev[0] and ev[-1] <= hi


def test_gershgorin_diagonal_is_exact():
    d = np.array([-3.0, 0.25, 9.5])
    assert gershgorin(sp.diags(d)) == (-3.0, 9.5)


# -------------------------------------------------------- sign convention ---

def test_normalise_signs_tie_and_flip():
    X = np.array([[3.0, -1.0, 0.0],
                  [-3.0, 2.0, 4.0],
                  [0.0, -2.0, -4.0]])
    Y = F.normalise_signs(X)
    # column 0: |3| ties at rows 0 and 1 -> the lower index (row 0, +3) rules
    np.testing.assert_allclose(Y[:, 0], np.array([3.0, -3.0, 0.0]) / np.sqrt(18.0), rtol=0, atol=1e-16)
    # column 1: |2| ties at rows 1 (+2) and 2 (-2) -> row 1 positive, unchanged
    np.testing.assert_allclose(Y[:, 1], np.array([-1.0, 2.0, -2.0]) / 3.0, rtol=0, atol=1e-16)
    # column 2: tie between +4 (row 1) and -4 (row 2) -> row 1 positive
    np.testing.assert_allclose(Y[:, 2], np.array([0.0, 4.0, -4.0]) / np.sqrt(32.0), rtol=0, atol=1e-16)
    # a column whose first largest entry is negative is flipped
    Z = F.normalise_signs(np.array([[1.0], [-5.0], [5.0]]))
    np.testing.assert_allclose(Z[:, 0], np.array([-1.0, 5.0, -5.0]) / np.sqrt(51.0), rtol=0, atol=1e-16)
    np.testing.assert_allclose(np.linalg.norm(Y, axis=0), 1.0, rtol=1e-15)


# ----------------------------------------------------------- inertia count ---

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_count_below_matches_dense(seed):
    rng = np.random.default_rng(seed)
    n = 300
    B = sp.random(n, n, density=0.02, random_state=seed, format="csr")
    A = (B + B.T) * 0.5 + sp.diags(rng.uniform(-2.0, 2.0, n))  # indefinite
    ev = dense_eigvalsh(A)
    for i in (0, 7, 120, 150, 299):
        lo = ev[i - 1] if i > 0 else ev[0] - 1.0
        sigma = 0.5 * (lo + ev[i]) if i > 0 else ev[0] - 0.5
        assert count_below(A, sigma) == i
    assert count_below(A, ev[-1] + 1.0) == n


def test_count_below_grid_closed_form():
    # Dirichlet 40 x 40 + 0.01 I: 20 eigenvalues below the mid-gap window
    # edge of the 40 x 40 workload (closed form 2 - 2 cos(pi k / 41) sums)
    A = grid_laplacian((40, 40), 0.01).to_scipy()
    k = np.arange(1, 41)
    e1 = 2.0 - 2.0 * np.cos(np.pi * k / 41.0)
    ev = np.sort((e1[:, None] + e1[None, :]).ravel()) + 0.01
    assert count_below(A, 0.20200934091026512) == 20
    # the first gap at or after index 100 (the spectrum has degenerate pairs)
    i = next(i for i in range(100, 200) if ev[i + 1] - ev[i] > 1e-8)
    assert count_below(A, 0.5 * (ev[i] + ev[i + 1])) == i + 1


def test_bottom_eigvalsh_matches_dense():
    A = knn_laplacian(1500, 2, 10, seed=3, weighted=True, shift=1e-3).to_scipy()
    ev = dense_eigvalsh(A)
    got = bottom_eigvalsh(A, 30)
    np.testing.assert_allclose(got, ev[:30], rtol=0, atol=1e-12 * ev[-1])


# ------------------------------------------------------ window fixtures -----

def test_knn8000_fixture_dense():
    """The headline window: 50 eigenvalues below lmax, and the 52 stored
    values, against a dense eigensolve of the n = 8000 matrix."""
    win = _windows()["knn8000"]
    A = knn_laplacian(8000, 2, 10, seed=1, weighted=True, shift=1e-3).to_scipy()
    assert A.nnz == win["nnz"]
    assert count_below(A, win["lmax"]) == win["count"] == 50
    ev = dense_eigvalsh(A)
    np.testing.assert_allclose(win["eigenvalues"], ev[:52], rtol=0, atol=1e-12)
    assert ev[49] < win["lmax"] < ev[50]


def test_batch32_fixture_counts():
    """Every member of the 32-graph batch: the stored count equals the exact
    number of eigenvalues below its window edge lmax, and (except the six 3D
    members above 20,000 rows, whose factorizations take 5-12 s each) one
    more lies below the mid-gap after the first outside eigenvalue.  The
    lower edge -0.1 u lies below the spectrum of these semidefinite
    Laplacians.  Members
    up to n = 8000 also have every stored value checked against a dense
    eigensolve."""
    for w in _windows()["batch32"]:
        A = knn_laplacian(w["n"], w["dim"], w["k"], seed=w["seed"], weighted=False).to_scipy()
        assert A.nnz == w["nnz"]
        c, ev = w["count"], w["eigenvalues"]
        assert count_below(A, w["lmax"]) == c, w["recipe"]
        assert w["lmin"] < 0.0
        if not (w["dim"] == 3 and w["n"] > 20000):
            assert count_below(A, 0.5 * (ev[c] + ev[c + 1])) == c + 1, w["recipe"]
        if w["n"] <= 8000:
            ref = dense_eigvalsh(A)[: len(ev)]
            np.testing.assert_allclose(ev, ref, rtol=0, atol=1e-12 * max(1.0, abs(ref[-1])))


@pytest.mark.parametrize("n", [2000, 4000, 8000, 16000])
def test_rgg_fixture_counts(n):
    """The paper's sweep windows [0.001, 5.0] (seeds 0-4 per size): the
    stored in-window count, and the stored values below 0.001, against exact
    counts at both edges."""
    for w in [w for w in _windows()["rgg"] if w["n"] == n and w["seed"] < 5]:
        A = rgg_laplacian(n, w["seed"]).to_scipy()
        assert A.nnz == w["nnz"]
        below = count_below(A, 0.001)
        assert below == len(w["below"])
        assert count_below(A, 5.0) - below == w["count"]


# -------------------------------------------------------------- filter ------

@pytest.mark.parametrize("nc", list(range(1, 17)) + [24, 32])
def test_filter_at_least_half_inside_window(nc):
    """The spurious-pair rule counts a Ritz pair when its filter gain is at
    least 1/4; it relies on |rho| >= 1/2 on the whole closed window (1/2 at
    the edges) for every node count, and on |rho| < 1/2 just outside."""
    lmin, lmax = 0.7, 2.3
    z, w = half_circle(lmin, lmax, nc)
    lam = np.linspace(lmin, lmax, 4001)
    rho = filter_value(lam, z, w)
    assert np.all(np.abs(rho) >= 0.5 - 1e-12), (nc, float(np.abs(rho).min()))
    r = 0.5 * (lmax - lmin)
    out = np.concatenate([np.linspace(lmin - 3 * r, lmin - 1e-6 * r, 2000),
                          np.linspace(lmax + 1e-6 * r, lmax + 3 * r, 2000)])
    assert np.all(np.abs(filter_value(out, z, w)) < 0.5)


# ------------------------------------------------- true-residual branch -----

def test_pc_cocg_replaces_drifted_residual():
    """With a tolerance below the rounding floor the recursive residual keeps
    falling below tol ||b|| while the true one cannot, so every check takes
    the replacement branch (r <- b - (zI - A) x).  The solver must then run
    to its iteration cap without claiming convergence, report the true
    residual, and keep it at the rounding floor (a wrong sign or a missed
    replacement lets it drift up by orders of magnitude)."""
    A = grid_laplacian((12, 12), 0.01).to_scipy()
    z = 1.3 + 0.05j
    b = np.random.default_rng(4).standard_normal(A.shape[0])
    x, it, res = pc_cocg(A, z, b, None, 0.0, 8.01, tol=1e-30, maxit=600)
    true = np.linalg.norm(b - (z * x - A @ x)) / np.linalg.norm(b)
    assert it == 600
    assert res == pytest.approx(true, rel=1e-12)
    assert true < 1e-13
    # the same system converges normally at a reachable tolerance, like the
    # unpreconditioned oracle COCG
    x2, it2, res2 = pc_cocg(A, z, b, None, 0.0, 8.01, tol=1e-10)
    assert res2 <= 1e-10 and it2 < 600
    x3, _, _ = cocg(A, z, b, tol=1e-12)
    assert np.linalg.norm(x2 - x3) <= 1e-8 * np.linalg.norm(x3)
