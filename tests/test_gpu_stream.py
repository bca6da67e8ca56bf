"""GPU parity of the streaming COCG engine (vectors in HBM, all systems in lock
step) through the C ABI: every column-group width it instantiates, and the
64^3 interior window (Dirichlet 7-point Laplacian + 0.01 I, n = 262144) against
the closed-form spectrum."""

import os

import numpy as np
import pytest

from tests.closed_forms import grid_eigs, window_basis
from tests.feast_checks import check_against, gap_out
from workloads import gaussian, grid_laplacian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    return torch


# FP32 takes two columns per lane (groups of 128) from 128 columns on, one
# below; FP64 one.  k = 30: 60 columns, padded; k = 40: 80 columns in a
# group of 128 mixing both shifts; k = 128 / 256: several groups.
@pytest.mark.parametrize("precision,k", [("fp32", 30), ("fp32", 40), ("fp32", 128),
                                         ("fp32", 256), ("fp64", 30), ("fp64", 128)])
def test_stream_column_groups(gpu_lib, torch_dev, precision, k):
    torch = torch_dev
    dims = (17, 17, 17)  # n = 4913, not a multiple of the workgroup's rows
    csr = grid_laplacian(dims, 0.01)
    A = csr.to_scipy()
    n = csr.n
    z = np.array([0.5 + 0.05j, 2.0 + 0.01j])
    rng = np.random.default_rng(k)
    B = rng.standard_normal((n, k))
    B[:, 3] = 0.0
    B[:, 5] *= 1e-9
    tol = 1e-10
    with gpu_lib.Plan(csr, 0.0, 0.6, 8, nc=2, q=1, p=4, precision=precision,
                      engine="stream") as plan:
        assert plan.engine == "stream"
        ct = torch.complex64 if precision == "fp32" else torch.complex128
        X = torch.zeros((n, len(z) * k), dtype=ct, device="cuda")
        its, rs = plan.shifted_solve(z, torch.from_numpy(B).cuda(), X, tol)
    Xh = X.cpu().numpy().astype(np.complex128)
    u_out = 2.0 ** -24 if precision == "fp32" else 2.0 ** -53
    lam = grid_eigs(dims, 0.01)[0]
    for j in range(len(z)):
        dist = np.abs(z[j] - lam).min()  # ||(zI - A)^{-1}|| = 1 / dist
        for c in range(k):
            col = j * k + c
            x, b = Xh[:, col], B[:, c]
            if c == 3:
                assert np.abs(x).max() == 0 and its[col] == 0 and rs[col] == 0
                continue
            assert rs[col] <= tol, (j, c, rs[col])
            r = b - (z[j] * x - A @ x)
            bound = tol + 8.1 * np.linalg.norm(x) * 2 * u_out / np.linalg.norm(b)
            assert np.linalg.norm(r) <= 1.01 * bound * np.linalg.norm(b), (j, c)
            assert np.linalg.norm(x) <= 1.01 * np.linalg.norm(b) / dist
    assert its.max() > 10


# The precision form as specified (complex-FP32 COCG with FP64 reliable
# updates, fixed 1e-6 tolerance): about two and a half minutes on one MI355X
# (four rounds of 512 FP32 COCG solves of up to 20000 iterations each).
@pytest.mark.slow
def test_grid3d_64_interior_window(gpu_lib):
    dims, shift = (64, 64, 64), 0.01
    csr = grid_laplacian(dims, shift)
    A = csr.to_scipy()
    lmin, lmax = 0.493673151133, 0.506687779116
    vals, V = window_basis(dims, shift, lmin, lmax)
    assert len(vals) == 39
    allv, _ = grid_eigs(dims, shift)
    gap = gap_out(allv, lmin, lmax)
    m0, nc, p = 64, 8, 20
    with gpu_lib.Plan(csr, lmin, lmax, m0, nc=nc, q=2, p=p, precision="fp32",
                      tol_solve=1e-6, tol_eig=1e-10) as plan:
        assert plan.engine == "stream"
        om = gaussian(csr.n, m0 + p, 0)
        ws = plan.warmstart(omega=om)
        out = plan.solve()
    assert ws["op"] == "fold"
    assert out["status"] == "OK"
    check_against(out, A, vals, V, lmin, lmax, 1e-10, gap)


# The same window with relaxed Phase-2 solves (COCG starting at 1e-2, tightened
# by the contraction control): about a minute and a half, so it runs by default.
def test_grid3d_64_interior_window_relaxed(gpu_lib):
    dims, shift = (64, 64, 64), 0.01
    csr = grid_laplacian(dims, shift)
    A = csr.to_scipy()
    lmin, lmax = 0.493673151133, 0.506687779116
    vals, V = window_basis(dims, shift, lmin, lmax)
    assert len(vals) == 39
    allv, _ = grid_eigs(dims, shift)
    gap = gap_out(allv, lmin, lmax)
    m0, nc, p = 64, 8, 20
    with gpu_lib.Plan(csr, lmin, lmax, m0, nc=nc, q=2, p=p, precision="fp32",
                      tol_solve=1e-6, tol_eig=1e-10, tol_solve_relaxed=1e-2) as plan:
        assert plan.engine == "stream"
        om = gaussian(csr.n, m0 + p, 0)
        ws = plan.warmstart(omega=om)
        out = plan.solve()
    assert ws["op"] == "fold"
    assert out["status"] == "OK"
    check_against(out, A, vals, V, lmin, lmax, 1e-10, gap)


# The same window with the FP64 multi-shift engine at the fixed 1e-6
# tolerance (about half a minute).
def test_grid3d_64_interior_window_multishift(gpu_lib):
    dims, shift = (64, 64, 64), 0.01
    csr = grid_laplacian(dims, shift)
    A = csr.to_scipy()
    lmin, lmax = 0.493673151133, 0.506687779116
    vals, V = window_basis(dims, shift, lmin, lmax)
    allv, _ = grid_eigs(dims, shift)
    gap = gap_out(allv, lmin, lmax)
    with gpu_lib.Plan(csr, lmin, lmax, 64, nc=8, q=2, p=20, precision="fp64",
                      engine="multishift", tol_solve=1e-6, tol_eig=1e-10) as plan:
        assert plan.engine == "multishift"
        ws = plan.warmstart(omega=gaussian(csr.n, 84, 0))
        out = plan.solve()
    assert ws["op"] == "fold"
    assert out["status"] == "OK"
    check_against(out, A, vals, V, lmin, lmax, 1e-10, gap)
