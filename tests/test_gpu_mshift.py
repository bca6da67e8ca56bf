"""GPU parity of the multi-shift COCG engine through the C ABI: one real CG on
the positive definite seed A - s I per right-hand side drives every shifted
system (z_j I - A) d = b.  Stage solves against exact solves and the oracle's
single-shift COCG, and whole FEAST runs against closed-form spectra and the
stored kNN spectrum."""

import json
import os

import numpy as np
import pytest

from oracle.cocg import cocg
from oracle.contour import half_circle
from oracle.feast import ShiftedSolver
from tests.closed_forms import grid_eigs, window_basis
from tests.feast_checks import check_against, gap_out
from workloads import gaussian, grid_laplacian, knn_laplacian

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    return torch


# k = 5: one column per lane; k = 70 and 150: two and three per lane (the
# padded width 128 / 192); n = 4913 and 2197 are not multiples of the rows a
# workgroup takes
@pytest.mark.parametrize("dims,k", [((40, 40), 5), ((17, 17, 17), 70), ((13, 13, 13), 150)])
def test_multishift_solve_matches_exact(gpu_lib, torch_dev, dims, k):
    torch = torch_dev
    csr = grid_laplacian(dims, 0.01)
    A = csr.to_scipy()
    n = csr.n
    z, _ = half_circle(0.0, 0.2, 4)
    z = np.concatenate([z, [0.3 + 1e-3j]])
    rng = np.random.default_rng(k)
    B = rng.standard_normal((n, k))
    B[:, 0] *= 1e3
    B[:, 1] = 0.0
    B[:, 2] *= 1e-9
    tol = 1e-10
    with gpu_lib.Plan(csr, 0.0, 0.2, 8, nc=2, q=1, p=4, precision="fp64",
                      engine="multishift") as plan:
        assert plan.engine == "multishift"
        X = torch.zeros((n, len(z) * k), dtype=torch.complex128, device="cuda")
        its, rs = plan.shifted_solve(z, torch.from_numpy(B).cuda(), X, tol)
    Xh = X.cpu().numpy()
    lam = np.linalg.eigvalsh(A.toarray()) if n <= 2500 else grid_eigs(dims, 0.01)[0]
    solver = ShiftedSolver(A, z)
    for j in range(len(z)):
        ref = solver.solve(j, B)
        kappa = np.abs(z[j] - lam).max() / np.abs(z[j] - lam).min()
        for c in range(k):
            col = j * k + c
            x, b = Xh[:, col], B[:, c]
            if c == 1:  # zero right-hand side: zero solution, no iterations
                assert np.abs(x).max() == 0 and its[col] == 0 and rs[col] == 0
                continue
            assert rs[col] <= 1.01 * tol, (j, c, rs[col])
            # the true residual recomputed here in FP64
            r = b - (z[j] * x - A @ x)
            assert np.linalg.norm(r) <= (1.01 * tol + 16 * U * np.linalg.norm(x)
                                         * 8.1 / np.linalg.norm(b)) * np.linalg.norm(b)
            err = np.linalg.norm(x - ref[:, c]) / np.linalg.norm(ref[:, c])
            assert err <= 1.1 * kappa * tol + 1e-13, (j, c, err)
    # each shifted system takes no more iterations than single-shift COCG on
    # it (the same Krylov space, the same Galerkin condition)
    for j in range(len(z)):
        for c in (0, 3):
            _, it_o, _ = cocg(A, z[j], B[:, c], tol=tol)
            assert its[j * k + c] <= 1.05 * it_o + 5, (j, c, its[j * k + c], it_o)
    assert its.max() > 10


@pytest.mark.parametrize("form", ["residual", "literal"])
def test_multishift_feast_grid40(gpu_lib, form):
    dims, shift = (40, 40), 0.01
    csr = grid_laplacian(dims, shift)
    A = csr.to_scipy()
    lmin, lmax = 0.0, 0.20200934091026512
    vals, V = window_basis(dims, shift, lmin, lmax)
    allv, _ = grid_eigs(dims, shift)
    tol_solve = 1e-6 if form == "residual" else 1e-12
    with gpu_lib.Plan(csr, lmin, lmax, 30, nc=4, q=2, p=10, precision="fp64",
                      engine="multishift", rhs_form=form, tol_solve=tol_solve) as plan:
        plan.warmstart(omega=gaussian(csr.n, 40, 0))
        out = plan.solve()
    assert out["status"] == "OK" and out["M"] == 20
    check_against(out, A, vals, V, lmin, lmax, 1e-10, gap_out(allv, lmin, lmax))
    assert sum(out["cocg_node"]) == out["cocg_iters"]


def test_multishift_feast_knn8000(gpu_lib):
    with open(os.path.join(GOLDEN, "windows.json")) as f:
        win = json.load(f)["knn8000"]
    csr = knn_laplacian(8000, 2, 10, seed=1, weighted=True, shift=1e-3)
    assert csr.nnz == win["nnz"]
    with gpu_lib.Plan(csr, win["lmin"], win["lmax"], 64, nc=4, q=2, p=20, precision="fp64",
                      engine="multishift", tol_solve=1e-6) as plan:
        plan.warmstart()
        out = plan.solve()
    assert out["status"] == "OK" and out["M"] == win["count"]
    ev = np.array(win["eigenvalues"][: win["count"]])
    s_win = max(abs(win["lmin"]), abs(win["lmax"]))
    assert np.abs(out["lam"] - ev).max() <= 1e-10 * s_win
    A = csr.to_scipy()
    R = A @ out["X"] - out["X"] * out["lam"][None, :]
    assert np.linalg.norm(R, axis=0).max() / s_win <= 1.5e-10


def test_multishift_plan_checks(gpu_lib):
    csr = grid_laplacian((10, 10), 0.01)
    with pytest.raises(gpu_lib.RafeastError) as e:
        gpu_lib.Plan(csr, 0.0, 0.5, 8, nc=2, precision="fp32", engine="multishift")
    assert e.value.name == "INVALID_ARG"
