"""The engines at more than 2^20 rows (the 64-bit offsets of the n x k
blocks): shifted solves on a 102^3 grid Laplacian (n = 1,061,208) by the
streaming engine (FP32 and FP64), the multi-shift engine and the FP64
preconditioned solver, against the oracle's FP64 COCG on the CPU."""

import numpy as np
import pytest

from oracle.cocg import cocg
from oracle.learned import c_star, sample_data
from oracle.spectrum import gershgorin
from workloads import grid_laplacian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    csr = grid_laplacian((102, 102, 102), 0.01)
    assert csr.n > 1 << 20
    A = csr.to_scipy()
    rng = np.random.default_rng(3)
    B = rng.standard_normal((csr.n, 2))
    z = np.array([3.0 + 2.0j, 8.0 + 3.0j])
    ref = {}
    for j, zj in enumerate(z):
        for c in range(2):
            x, it, ok = cocg(A, zj, B[:, c], tol=1e-13)
            assert ok
            ref[(j, c)] = x
    return csr, A, B, z, ref


def _check(X, B, z, ref, tol, out_u):
    # distance of z_j from the spectrum [0.01, 12.01] bounds ||(zI - A)^{-1}||
    for j, zj in enumerate(z):
        kappa = 12.01 / abs(zj.imag)
        for c in range(B.shape[1]):
            x = X[:, j * B.shape[1] + c]
            e = np.linalg.norm(x - ref[(j, c)]) / np.linalg.norm(ref[(j, c)])
            assert e <= 1.1 * kappa * tol + 8 * out_u, (j, c, e)


@pytest.mark.parametrize("precision,engine", [("fp32", "stream"), ("fp64", "stream"),
                                              ("fp64", "multishift")])
def test_engines_beyond_2_20_rows(gpu_lib, big, precision, engine):
    import torch

    csr, A, B, z, ref = big
    tol = 1e-9
    with gpu_lib.Plan(csr, 0.0, 0.1, 4, nc=2, q=0, p=4, precision=precision,
                      engine=engine) as plan:
        assert plan.engine == engine
        ct = torch.complex64 if precision == "fp32" else torch.complex128
        X = torch.zeros((csr.n, 4), dtype=ct, device="cuda")
        its, rs = plan.shifted_solve(z, torch.from_numpy(np.ascontiguousarray(B)).cuda(), X, tol)
    assert np.all(rs <= 1.01 * tol), rs
    u = 2.0 ** -24 if precision == "fp32" else 2.0 ** -53
    _check(X.cpu().numpy().astype(np.complex128), B, z, ref, tol, u)


@pytest.mark.parametrize("precond", [False, True])
def test_preconditioned_solver_beyond_2_20_rows(gpu_lib, big, precond):
    import torch

    csr, A, B, z, ref = big
    lo, hi = gershgorin(A)
    coef = [c_star(*sample_data(A, lo, hi, zj, B[:, 0])[:2]) for zj in z] if precond else None
    tol = 1e-10
    with gpu_lib.Plan(csr, 0.0, 0.1, 4, nc=2, q=0, p=4, precision="fp64") as plan:
        X = torch.zeros((csr.n, 4), dtype=torch.complex128, device="cuda")
        its, rs = plan.pc_solve(z, torch.from_numpy(np.ascontiguousarray(B)).cuda(), X, tol,
                                coef=coef)
    assert np.all(rs <= tol), rs
    _check(X.cpu().numpy(), B, z, ref, tol, 2.0 ** -53)
