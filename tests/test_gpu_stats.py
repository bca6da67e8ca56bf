"""GPU parity of the statistical workloads (Section 4) through the C ABI:
top windows of a sample covariance (rafeast_plan_gram) and of a Gaussian
kernel matrix (rafeast_plan_dense) against the stored spectra and the oracle's
RA-FEAST, the dense products against host products, and the dense streaming
COCG against LU."""

import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import feast as F
from oracle.stats import sample_covariance
from oracle.subspace import sin_theta
from workloads import gaussian
from workloads.stats import rbf_kernel, spiked_data

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fixture(name):
    with open(os.path.join(GOLDEN, "windows.json")) as f:
        return json.load(f)["stats"][name]


def _operator(fx):
    if fx["kind"] == "covariance":
        X = spiked_data(fx["rows"], fx["p"], seed=1)
        return X, sample_covariance(X)
    K = rbf_kernel(fx["n"], bandwidth=0.4, seed=2)
    return K, K


def _plan(gpu_lib, fx, data, **kw):
    make = gpu_lib.Plan.from_covariance if fx["kind"] == "covariance" else gpu_lib.Plan.from_dense
    return make(data, fx["lmin"], fx["lmax"], fx["m0"], nc=fx["nc"], q=2, ws_op="literal", **kw)


@pytest.mark.parametrize("name", ["cov_small", "kpca_small"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_top_window_parity(gpu_lib, name, precision):
    fx = _fixture(name)
    data, A = _operator(fx)
    n = A.shape[0]
    k = fx["count"]
    ref = np.array(fx["eigenvalues"][:k])
    s_win = max(abs(fx["lmin"]), abs(fx["lmax"]))
    with _plan(gpu_lib, fx, data, precision=precision) as plan:
        assert plan.engine == "stream"
        om = gaussian(n, plan.w, 0)
        ws = plan.warmstart(omega=om)
        out = plan.solve()
    assert ws["op"] == "literal"
    assert out["status"] == "OK" and out["M"] == k
    lam = out["lam"]
    np.testing.assert_allclose(np.sort(lam)[::-1], ref, rtol=0, atol=1e-10 * s_win)
    X = out["X"]
    R = A @ X - X * lam[None, :]
    res = np.linalg.norm(R, axis=0) / s_win
    assert res.max() <= 1.0001e-10
    assert np.abs(X.T @ X - np.eye(k)).max() < 1e-12
    orc = F.ra_feast(A, fx["lmin"], fx["lmax"], fx["m0"], fx["nc"], om, q=2, ws_op="literal")
    assert orc["M"] == k
    np.testing.assert_allclose(lam, orc["lam"], rtol=0, atol=1e-10 * s_win)
    ev = np.array(fx["eigenvalues"])
    gap = ev[k - 1] - ev[k]
    assert sin_theta(X, orc["X"]).max() <= max(1e-8, 2 * np.linalg.norm(R) / gap)
    assert abs(out["iters"] - orc["iters"]) <= 2


def test_top_window_relaxed_solves(gpu_lib):
    fx = _fixture("kpca_small")
    data, A = _operator(fx)
    k = fx["count"]
    s_win = abs(fx["lmax"])
    with _plan(gpu_lib, fx, data, tol_solve_relaxed=1e-2) as plan:
        plan.warmstart(omega=gaussian(A.shape[0], plan.w, 0))
        out = plan.solve()
    assert out["status"] == "OK" and out["M"] == k
    np.testing.assert_allclose(np.sort(out["lam"])[::-1], fx["eigenvalues"][:k], rtol=0,
                               atol=1e-10 * s_win)


@pytest.mark.parametrize("name", ["cov_small", "kpca_small"])
def test_dense_products(gpu_lib, name):
    import torch

    fx = _fixture(name)
    data, A = _operator(fx)
    n = A.shape[0]
    rng = np.random.default_rng(7)
    Xh = rng.standard_normal((n, 37))
    Yh = rng.standard_normal((n, 37))
    X = torch.tensor(Xh, device="cuda")
    Y = torch.tensor(Yh, device="cuda")
    with _plan(gpu_lib, fx, data) as plan:
        plan.spmm(X, Y, alpha=0.5, beta=-2.0)
        got = Y.cpu().numpy()
    want = 0.5 * (A @ Xh) - 2.0 * Xh  # Y = alpha A X + beta X; Y's old values unused
    # both sides round inner products of length m (gamma_m = m u bounds
    # each): m = n with |K| |X| for the kernel; X^T (X V) / (rows - 1) with
    # m = rows + p and |X|^T (|X| |V|) / (rows - 1) for the covariance
    u = np.finfo(np.float64).eps / 2
    if fx["kind"] == "covariance":
        m = fx["rows"] + fx["p"]
        mag = np.abs(data).T @ (np.abs(data) @ np.abs(Xh)) / (fx["rows"] - 1)
    else:
        m = n
        mag = np.abs(A) @ np.abs(Xh)
    bound = 2 * m * u * 0.5 * mag + 4 * u * (0.5 * np.abs(A @ Xh) + 2.0 * np.abs(Xh))
    assert np.all(np.abs(got - want) <= bound)


def test_covariance_products_split_inner_dimension(gpu_lib):
    # p = 2501 features: the product X V runs as two chunks of 1250 and a
    # remainder of 1, summed; FP64 (spmm) and FP32 (inside COCG) paths
    import torch

    X = spiked_data(150, 2501, spikes=5, seed=9)
    A = sample_covariance(X)
    n = A.shape[0]
    Vh = np.random.default_rng(3).standard_normal((n, 20))
    V = torch.tensor(Vh, device="cuda")
    Y = torch.zeros_like(V)
    ev = np.sort(np.linalg.eigvalsh(X @ X.T / 149))[::-1]
    with gpu_lib.Plan.from_covariance(X, 0.5 * (ev[4] + ev[5]), 1.05 * ev[0], 10, nc=8,
                                      ws_op="literal") as plan:
        plan.spmm(V, Y)
        got = Y.cpu().numpy()
        plan.warmstart(omega=gaussian(n, plan.w, 1))
        out = plan.solve()
    u = np.finfo(np.float64).eps / 2
    mag = np.abs(X).T @ (np.abs(X) @ np.abs(Vh)) / 149
    assert np.all(np.abs(got - A @ Vh) <= 2 * (150 + 2501) * u * mag)
    assert out["status"] == "OK" and out["M"] == 5
    np.testing.assert_allclose(np.sort(out["lam"])[::-1], ev[:5], rtol=0, atol=1e-10 * 1.05 * ev[0])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_dense_shifted_solves(gpu_lib, precision):
    import torch

    fx = _fixture("kpca_small")
    data, A = _operator(fx)
    n = A.shape[0]
    z = np.array([0.5 * (fx["lmin"] + fx["lmax"]) + 0.3j * fx["lmax"], fx["lmin"] + 5.0j])
    B = gaussian(n, 5, 3)
    want = torch.complex64 if precision == "fp32" else torch.complex128
    Xd = torch.zeros((n, len(z) * 5), dtype=want, device="cuda")
    with _plan(gpu_lib, fx, data, precision=precision) as plan:
        its, rs = plan.shifted_solve(z, torch.tensor(np.ascontiguousarray(B), device="cuda"),
                                     Xd, 1e-8)
    got = Xd.cpu().numpy().astype(np.complex128)
    u_out = 2.0 ** -24 if precision == "fp32" else 2.0 ** -53
    ev = np.linalg.eigvalsh(A)
    tol = 1e-8
    for j, zj in enumerate(z):
        M = zj * np.eye(n) - A
        ref = sla.solve(M, B)
        norm_m = np.abs(zj - ev).max()
        kappa = norm_m / np.abs(zj - ev).min()
        for c in range(5):
            x = got[:, j * 5 + c]
            b = B[:, c]
            # the library's FP64 solution met the tolerance ...
            assert rs[j * 5 + c] <= tol, (j, c, rs[j * 5 + c])
            # ... so the returned (output-rounded) x is within kappa * tol of
            # the exact solve, plus the output rounding
            err = np.linalg.norm(x - ref[:, c]) / np.linalg.norm(ref[:, c])
            assert err <= 1.1 * kappa * tol + 4 * u_out, (j, c, err)
            r = np.linalg.norm(b - M @ x)
            assert r <= (tol + 2.1 * norm_m * np.linalg.norm(x) * u_out / np.linalg.norm(b)) * \
                np.linalg.norm(b), (j, c, r)
    assert np.all(its > 0)


def test_dense_plan_rejects_learned_preconditioner(gpu_lib):
    import torch

    fx = _fixture("kpca_small")
    data, A = _operator(fx)
    R = torch.zeros((A.shape[0], 2), dtype=torch.float64, device="cuda")
    with _plan(gpu_lib, fx, data) as plan:
        with pytest.raises(gpu_lib.RafeastError) as e:
            plan.pc_samples([fx["lmin"] + 1j], R, 0.0, 1.0)
    assert e.value.name == "UNSUPPORTED"
