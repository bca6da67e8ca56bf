"""The paper's experiment (Section 5.1) on the GPU path through the C ABI:
random geometric graph Laplacians, window [0.001, 5.0], Max Error of the
returned eigenvalues against the stored reference spectra."""

import json
import os

import numpy as np
import pytest

from oracle.philox import gaussian_sketch
from workloads import rgg_laplacian

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixture(n, seed):
    with open(os.path.join(HERE, "golden", "windows.json")) as f:
        for w in json.load(f)["rgg"]:
            if w["n"] == n and w["seed"] == seed:
                return w
    raise KeyError((n, seed))


@pytest.mark.parametrize("n,nc,max_iter,engine", [(2000, 2, 4, "resident"), (2000, 8, 2, "resident"),
                                                  (16000, 2, 4, "stream")])
def test_rgg_ra_feast_max_error(gpu_lib, n, nc, max_iter, engine):
    # RA-FEAST with few contour points and iterations: every window
    # eigenvalue found, Max Error below the paper's 1e-9 (Section 5.2)
    w = _fixture(n, 0)
    csr = rgg_laplacian(n, 0)
    with gpu_lib.Plan(csr, w["lmin"], w["lmax"], w["m0"], nc=nc, q=2, p=-1, max_iter=max_iter,
                      precision="fp32", seed=0) as plan:
        assert plan.engine == engine
        plan.warmstart(omega=gaussian_sketch(n, plan.w, 0))
        out = plan.solve(want_vectors=False)
    ref = np.array(w["eigenvalues"])
    assert out["M"] == len(ref)
    assert out["iters"] <= max_iter
    assert np.abs(out["lam"] - ref).max() < 1e-9


def test_rgg_standard_feast(gpu_lib):
    # standard FEAST (N_c = 8, random start) to residual 1e-10
    w = _fixture(2000, 0)
    csr = rgg_laplacian(2000, 0)
    with gpu_lib.Plan(csr, w["lmin"], w["lmax"], w["m0"], nc=8, q=0, p=-1, ws_op="none",
                      precision="fp32", seed=0) as plan:
        plan.warmstart()
        out = plan.solve(want_vectors=False)
    ref = np.array(w["eigenvalues"])
    assert out["status"] == "OK" and out["M"] == len(ref)
    assert np.abs(out["lam"] - ref).max() < 1e-10 * 5.0
