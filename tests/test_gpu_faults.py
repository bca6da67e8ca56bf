"""Forced faults and determinism through the C ABI.

Breakdown: with b = e_i and the real shift z = A_ii, the first COCG pivot
p^T (zI - A) p = z - A_ii is exactly zero in every precision (A_ii = 4.5 is a
float), so the system breaks down at once; every restart from the true
residual s = b repeats it.  The engines must stop that system after their
breakdown budget with its FP64 solution (zero) and residual (one) reported,
while the other systems of the same launch converge as usual.  The
multi-shift engine divides by the seed's residual polynomial at z and takes
shifts off the real axis only.

Determinism: Phase 1 and Phase 2 run twice on one plan give bit-identical
results on every engine (fixed-order reductions, no floating-point atomics).
"""

import numpy as np
import pytest

from tests.closed_forms import grid_eigs
from workloads import gaussian, grid_laplacian

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    return torch


# 10 x 12 Dirichlet grid + 0.5: diagonal 4.5 everywhere; 4.5 is not an
# eigenvalue (13 j + 11 k = 143 has no solution with 1 <= j <= 10)
DIMS, SHIFT, ROW = (10, 12), 0.5, 37


@pytest.mark.parametrize("engine,precision", [("resident", "fp32"), ("resident", "fp64"),
                                              ("stream", "fp32"), ("stream", "fp64")])
def test_forced_breakdown_is_reported(gpu_lib, torch_dev, engine, precision):
    torch = torch_dev
    csr = grid_laplacian(DIMS, SHIFT)
    A = csr.to_scipy()
    n = csr.n
    assert A[ROW, ROW] == 4.5
    z = np.array([4.5 + 0.0j, 1.0 + 0.3j, 7.0 + 0.05j])
    rng = np.random.default_rng(3)
    B = np.zeros((n, 3))
    B[ROW, 0] = 1.0
    B[:, 1] = rng.standard_normal(n)
    B[:, 2] = rng.standard_normal(n)
    tol = 1e-9
    with gpu_lib.Plan(csr, 0.0, 1.0, 4, nc=2, q=1, p=4, precision=precision,
                      engine=engine) as plan:
        assert plan.engine == engine
        want = torch.complex64 if precision == "fp32" else torch.complex128
        X = torch.zeros((n, len(z) * 3), dtype=want, device="cuda")
        its, rs = plan.shifted_solve(z, torch.from_numpy(B).cuda(), X, tol)
    Xh = X.cpu().numpy().astype(np.complex128)
    assert np.isfinite(Xh).all() and np.isfinite(rs).all()
    # the forced breakdown: no step taken, the solution stays zero, the
    # reported residual is that of x = 0
    assert its[0] == 0, its[:3]
    assert np.abs(Xh[:, 0]).max() == 0.0
    assert rs[0] == pytest.approx(1.0, abs=1e-15)
    # the shifts off the real axis converge in the same launch, to the
    # exact solution within the condition bound
    lam = grid_eigs(DIMS, SHIFT)[0]
    M = A.toarray()
    for j in (1, 2):
        kappa = np.abs(z[j] - lam).max() / np.abs(z[j] - lam).min()
        for c in range(3):
            col = j * 3 + c
            assert rs[col] <= 1.01 * tol, (j, c, rs[col])
            ref = np.linalg.solve(z[j] * np.eye(n) - M, B[:, c])
            err = np.linalg.norm(Xh[:, col] - ref) / np.linalg.norm(ref)
            out_round = 2.0 ** -24 if precision == "fp32" else 0.0
            assert err <= 1.1 * kappa * tol + out_round * 4 + 1e-13, (j, c, err)
    # the real shift with generic right-hand sides (an indefinite real
    # system): whatever the engine reached, the residual it reports is the
    # FP64 solution's
    for c in (1, 2):
        x = Xh[:, c]
        if precision == "fp64":
            r = np.linalg.norm(B[:, c] - (z[0] * x - A @ x)) / np.linalg.norm(B[:, c])
            assert abs(r - rs[c]) <= 1e-12 + 64 * U * (1 + np.linalg.norm(x) * 16.0
                                                      / np.linalg.norm(B[:, c])), (c, r, rs[c])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_zero_right_hand_sides_among_others(gpu_lib, torch_dev, precision):
    # more systems than workgroups on the resident engine (3 shifts x 100
    # columns), every other right-hand side zero: a workgroup that meets a
    # zero column ends that item early and takes the next one; zero columns
    # give zero solutions, zero iterations and zero residuals, and the others
    # converge in the same launch
    torch = torch_dev
    dims, shift = (20, 20), 0.01
    csr = grid_laplacian(dims, shift)
    A = csr.to_scipy()
    n = csr.n
    z = np.array([0.3 + 0.05j, 1.0 + 0.2j, 4.0 + 0.1j])
    k = 100
    B = np.random.default_rng(5).standard_normal((n, k))
    B[:, 0::2] = 0.0
    tol = 1e-8
    with gpu_lib.Plan(csr, 0.0, 0.2, 4, nc=2, q=1, p=4, precision=precision,
                      engine="resident") as plan:
        assert plan.engine == "resident"
        want = torch.complex64 if precision == "fp32" else torch.complex128
        X = torch.zeros((n, len(z) * k), dtype=want, device="cuda")
        its, rs = plan.shifted_solve(z, torch.from_numpy(B).cuda(), X, tol)
    Xh = X.cpu().numpy().astype(np.complex128)
    for j in range(len(z)):
        for c in range(k):
            col = j * k + c
            if c % 2 == 0:
                assert its[col] == 0 and rs[col] == 0.0, (j, c, its[col], rs[col])
                assert np.abs(Xh[:, col]).max() == 0.0, (j, c)
            else:
                assert its[col] > 0 and rs[col] <= 1.01 * tol, (j, c, its[col], rs[col])
    lam = grid_eigs(dims, shift)[0]
    M = A.toarray()
    out_round = 2.0 ** -24 if precision == "fp32" else 0.0
    for j in range(len(z)):
        kappa = np.abs(z[j] - lam).max() / np.abs(z[j] - lam).min()
        for c in (1, 51, 99):
            ref = np.linalg.solve(z[j] * np.eye(n) - M, B[:, c])
            err = np.linalg.norm(Xh[:, j * k + c] - ref) / np.linalg.norm(ref)
            assert err <= 1.1 * kappa * tol + out_round * 4 + 1e-13, (j, c, err)


def test_multishift_rejects_real_shifts(gpu_lib, torch_dev):
    torch = torch_dev
    csr = grid_laplacian(DIMS, SHIFT)
    n = csr.n
    with gpu_lib.Plan(csr, 0.0, 1.0, 4, nc=2, q=1, p=4, precision="fp64",
                      engine="multishift") as plan:
        B = torch.ones((n, 1), dtype=torch.float64, device="cuda")
        X = torch.zeros((n, 2), dtype=torch.complex128, device="cuda")
        with pytest.raises(gpu_lib.RafeastError) as e:
            plan.shifted_solve(np.array([1.0 + 0.2j, 4.5 + 0.0j]), B, X, 1e-8)
        assert e.value.name == "INVALID_ARG"
        # the plan stays usable
        its, rs = plan.shifted_solve(np.array([1.0 + 0.2j, 4.5 + 0.1j]), B, X, 1e-8)
        assert (rs <= 1.01e-8).all()


@pytest.mark.parametrize("engine,precision", [("resident", "fp32"), ("resident", "fp64"),
                                              ("stream", "fp32"), ("multishift", "fp64")])
def test_single_plan_runs_are_bit_identical(gpu_lib, engine, precision):
    dims, shift = (30, 30), 0.01
    csr = grid_laplacian(dims, shift)
    lmin, lmax = 0.0, 0.25
    omega = gaussian(csr.n, 24, 5)
    with gpu_lib.Plan(csr, lmin, lmax, 16, nc=4, q=2, p=8, precision=precision,
                      engine=engine, tol_solve=1e-6) as plan:
        assert plan.engine == engine
        runs = []
        for _ in range(2):
            ws = plan.warmstart(omega=omega, want_q0=True)
            out = plan.solve()
            runs.append((ws, out))
        # the plan's own device sketch (Philox) as well
        ws_a = plan.warmstart(want_q0=True)
        ws_b = plan.warmstart(want_q0=True)
    (wa, a), (wb, b) = runs
    assert a["status"] == "OK" and a["M"] > 0
    assert np.array_equal(wa["Q0"], wb["Q0"])
    assert wa["beta_m0"] == wb["beta_m0"] and wa["ratio"] == wb["ratio"]
    for key in ("M", "iters", "cocg_iters", "cocg_max", "refinements", "cocg_node"):
        assert a[key] == b[key], key
    for key in ("lam", "resid", "X"):
        assert np.array_equal(a[key], b[key]), key
    assert a["max_resid"] == b["max_resid"]
    assert np.array_equal(ws_a["Q0"], ws_b["Q0"])
