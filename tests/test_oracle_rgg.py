"""The paper's experiment (Section 5.1): random geometric graph Laplacians,
window [0.001, 5.0].  Pins of the oracle against the stored reference spectra
(shift-invert Lanczos, an independent method), and of the fixture recipe."""

import json
import os

import numpy as np
import pytest

from oracle import feast as F
from oracle.philox import gaussian_sketch
from workloads import rgg_laplacian

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixture(n, seed):
    with open(os.path.join(HERE, "golden", "windows.json")) as f:
        for w in json.load(f)["rgg"]:
            if w["n"] == n and w["seed"] == seed:
                return w
    raise KeyError((n, seed))


def test_rgg_fixture_recipe():
    w = _fixture(2000, 0)
    csr = rgg_laplacian(2000, 0)
    assert csr.nnz == w["nnz"]
    ev = np.array(w["eigenvalues"])
    assert w["count"] == len(ev) and np.all((ev >= 0.001) & (ev <= 5.0))
    assert w["m0"] == (40 if w["count"] < 40 else -(-3 * w["count"] // 2))
    # L = D - A of a connected graph: one zero eigenvalue just below the window
    assert len(w["below"]) == 1 and abs(w["below"][0]) < 1e-10
    # every row sums to zero
    A = csr.to_scipy()
    assert np.abs(A @ np.ones(2000)).max() < 1e-12


@pytest.mark.parametrize("nc,max_iter,bound", [(2, 4, 1e-9), (4, 4, 1e-9), (8, 2, 1e-9)])
def test_rgg_ra_feast_max_error(nc, max_iter, bound):
    # Max Error over the window's eigenvalues after a few iterations below
    # the paper's 1e-9 (Section 5.2, accuracy and robustness)
    w = _fixture(2000, 0)
    A = rgg_laplacian(2000, 0).to_scipy()
    m0 = w["m0"]
    p = F.default_oversampling(m0)
    out = F.ra_feast(A, w["lmin"], w["lmax"], m0, nc, gaussian_sketch(2000, m0 + p, 0), q=2,
                     max_iter=max_iter)
    ref = np.array(w["eigenvalues"])
    assert out["M"] == len(ref)
    assert np.abs(out["lam"] - ref).max() < bound


def test_rgg_standard_feast_converges():
    w = _fixture(2000, 0)
    A = rgg_laplacian(2000, 0).to_scipy()
    m0 = w["m0"]
    out = F.feast(A, w["lmin"], w["lmax"], m0, 8, gaussian_sketch(2000, m0, 0), tol=1e-10)
    ref = np.array(w["eigenvalues"])
    assert out["status"] == "ok" and out["M"] == len(ref)
    assert np.abs(out["lam"] - ref).max() < 1e-10 * 5.0
