"""GPU parity of the direct engine (standard FEAST with exact solves, the
baseline of Section 5.1): band LDL^T of every z_j I - A in the reverse
Cuthill-McKee order, through the C ABI, against exact solves, closed-form
spectra, the stored kNN and RGG spectra and the oracle's FEAST, whose solves
are sparse LU."""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import feast as F
from oracle.contour import half_circle
from oracle.philox import gaussian_sketch
from tests.closed_forms import grid_eigs, window_basis
from tests.feast_checks import check_against, gap_out
from workloads import gaussian, grid_laplacian, knn_laplacian, rgg_laplacian

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CFG1_WIN = (0.0, 0.20200934091026512)


@pytest.mark.parametrize("name", ["grid40", "knn2000", "grid12x7"])
def test_direct_solve_matches_exact(gpu_lib, name):
    import torch

    if name == "grid40":
        csr = grid_laplacian((40, 40), 0.01)  # bandwidth 40: panels of 32
    elif name == "knn2000":
        csr = knn_laplacian(2000, 2, 10, seed=3, weighted=True, shift=1e-3)
    else:
        csr = grid_laplacian((12, 7), 0.5)    # n = 84: a ragged last solve block
    A = csr.to_scipy()
    n = csr.n
    lam = np.linalg.eigvalsh(A.toarray())
    z, _ = half_circle(0.0, 0.2, 4)
    z = np.concatenate([z, [0.3 + 1e-3j]])
    k = 6
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, k))
    B[:, 1] = 0.0
    B[:, 2] *= 1e6
    with gpu_lib.Plan(csr, 0.0, 0.2, 4, nc=2, q=1, p=4, precision="fp64",
                      engine="direct") as plan:
        assert plan.engine == "direct"
        X = torch.zeros((n, len(z) * k), dtype=torch.complex128, device="cuda")
        its, rs = plan.shifted_solve(z, torch.from_numpy(B).cuda(), X, 1e-10)
    Xh = X.cpu().numpy()
    assert np.all(its == 0)
    for j, zj in enumerate(z):
        lu = spla.splu((zj * sp.identity(n, format="csc") - A.tocsc()).astype(complex))
        kappa = np.abs(zj - lam).max() / np.abs(zj - lam).min()
        for c in range(k):
            col = j * k + c
            if c == 1:
                assert np.abs(Xh[:, col]).max() == 0 and rs[col] == 0
                continue
            ref = lu.solve(B[:, c].astype(complex))
            err = np.linalg.norm(Xh[:, col] - ref) / np.linalg.norm(ref)
            # backward stable substitution with bounded growth: forward
            # error within a modest multiple of kappa u
            assert err <= 1e3 * kappa * U + 1e-14, (name, j, c, err, kappa)
            assert rs[col] <= 1e3 * kappa * U, (name, j, c, rs[col])


@pytest.mark.parametrize("form", ["literal", "residual"])
def test_direct_plain_feast_grid40(gpu_lib, form):
    # cfg1 as standard FEAST: N_c = 16, random start, exact solves
    dims, shift = (40, 40), 0.01
    csr = grid_laplacian(dims, shift)
    A = csr.to_scipy()
    lmin, lmax = CFG1_WIN
    vals, V = window_basis(dims, shift, lmin, lmax)
    allv, _ = grid_eigs(dims, shift)
    with gpu_lib.Plan(csr, lmin, lmax, 30, nc=16, q=2, p=10, precision="fp64", ws_op="none",
                      engine="direct", rhs_form=form) as plan:
        om = gaussian(csr.n, plan.w, 0)
        plan.warmstart(omega=om)
        out = plan.solve()
    assert out["status"] == "OK" and out["M"] == 20
    check_against(out, A, vals, V, lmin, lmax, 1e-10, gap_out(allv, lmin, lmax))
    assert out["cocg_iters"] == 0
    ref = F.feast(A, lmin, lmax, 30, 16, om[:, :30], form=form)
    assert np.abs(out["lam"] - ref["lam"]).max() <= 1e-10 * lmax
    # exact solves on both sides: the same iterations
    assert out["iters"] == ref["iters"]


def test_direct_plain_feast_knn8000(gpu_lib):
    # cfg2's plain FEAST with exact factorizations (the paper's comparison)
    with open(os.path.join(GOLDEN, "windows.json")) as f:
        win = json.load(f)["knn8000"]
    csr = knn_laplacian(8000, 2, 10, seed=1, weighted=True, shift=1e-3)
    with gpu_lib.Plan(csr, win["lmin"], win["lmax"], 64, nc=16, q=0, p=20, precision="fp64",
                      ws_op="none", engine="direct") as plan:
        plan.warmstart()
        out = plan.solve()
    assert out["status"] == "OK" and out["M"] == win["count"]
    ev = np.array(win["eigenvalues"][: win["count"]])
    s_win = max(abs(win["lmin"]), abs(win["lmax"]))
    assert np.abs(out["lam"] - ev).max() <= 1e-10 * s_win
    A = csr.to_scipy()
    R = A @ out["X"] - out["X"] * out["lam"][None, :]
    assert np.linalg.norm(R, axis=0).max() / s_win <= 1.5e-10


def test_direct_ra_feast_rgg2000(gpu_lib):
    # RA-FEAST with exact solves on the paper's RGG graph (Section 5.1):
    # the eigenvalues and the iteration count of the oracle, whose solves
    # are exact as well
    with open(os.path.join(GOLDEN, "windows.json")) as f:
        w = next(x for x in json.load(f)["rgg"] if x["n"] == 2000 and x["seed"] == 0)
    csr = rgg_laplacian(2000, 0)
    A = csr.to_scipy()
    with gpu_lib.Plan(csr, w["lmin"], w["lmax"], w["m0"], nc=4, q=2, p=-1, max_iter=4,
                      precision="fp64", engine="direct") as plan:
        om = gaussian_sketch(csr.n, plan.w, 0)
        plan.warmstart(omega=om)
        out = plan.solve(want_vectors=False)
    ref = np.array(w["eigenvalues"])
    assert out["M"] == len(ref)
    assert np.abs(out["lam"] - ref).max() < 1e-9
    orc = F.ra_feast(A, w["lmin"], w["lmax"], w["m0"], 4, om, q=2, max_iter=4)
    assert out["iters"] == orc["iters"]
    assert np.abs(np.sort(out["lam"]) - np.sort(orc["lam"])).max() <= 1e-10 * 5.0
