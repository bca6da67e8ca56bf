"""GPU parity of the individual stages, through the C ABI, against the oracle
or against bounds fixed by the arithmetic."""

import numpy as np
import pytest

from oracle import philox
from oracle.contour import half_circle
from oracle.feast import ShiftedSolver
from oracle.subspace import sin_theta
from workloads import gaussian, grid_laplacian, knn_laplacian, random_symmetric

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    return torch


def _plan(native, csr, **kw):
    args = dict(lmin=0.0, lmax=0.2, m0=16, nc=4, q=1, p=10)
    args.update(kw)
    return native.Plan(csr, **args)


@pytest.fixture(scope="module")
def small_plan(gpu_lib):
    csr = knn_laplacian(3000, 2, 10, seed=4, weighted=True, shift=1e-3)
    p = _plan(gpu_lib, csr, m0=64, p=20)
    yield csr, p
    p.close()


@pytest.mark.parametrize("n,k1,k2,same", [(1000, 30, 45, False), (4096, 64, 64, False),
                                          (777, 1, 17, False), (130, 148, 148, False),
                                          (3000, 192, 7, False), (100_003, 128, 128, False),
                                          (5003, 84, 84, True), (262_147, 192, 192, True)])
def test_gram_parity(small_plan, torch_dev, n, k1, k2, same):
    # same: X^T X with one buffer for both operands (one LDS slab serves both)
    torch = torch_dev
    _, plan = small_plan
    rng = np.random.default_rng(n + k1)
    X = rng.standard_normal((n, k1))
    Y = X if same else rng.standard_normal((n, k2))
    Xd = torch.from_numpy(X).cuda()
    Yd = Xd if same else torch.from_numpy(Y).cuda()
    G = torch.zeros((k1, k2), dtype=torch.float64, device="cuda")
    plan.gram(Xd, Yd, G)
    ref = X.T @ Y
    bound = 1.01 * n * U * (np.abs(X).T @ np.abs(Y)) + 1e-300
    assert np.all(np.abs(G.cpu().numpy() - ref) <= bound)


def test_spmm_parity(small_plan, torch_dev):
    torch = torch_dev
    csr, plan = small_plan
    A = csr.to_scipy()
    rng = np.random.default_rng(0)
    for k in (84, 1, 64, 130):
        X = rng.standard_normal((csr.n, k))
        Y = torch.zeros((csr.n, k), dtype=torch.float64, device="cuda")
        plan.spmm(torch.from_numpy(X).cuda(), Y, alpha=-0.5, beta=2.0)
        ref = -0.5 * (A @ X) + 2.0 * X
        maxrow = int(np.diff(csr.rowptr).max())
        bound = 1.01 * (maxrow + 2) * U * (0.5 * (abs(A) @ np.abs(X)) + 2.0 * np.abs(X))
        assert np.all(np.abs(Y.cpu().numpy() - ref) <= bound + 1e-300), k


def test_spmm_column_groups(gpu_lib, torch_dev):
    # a 64 x 64 x 40 grid in natural order: a row reaches 4096 rows either
    # side, so wide blocks are swept in column groups (64 -> 2 x 32,
    # 84 -> 2 x 42, 130 -> 44 + 44 + 42), narrow ones in one; odd k takes the
    # one-column kernel
    torch = torch_dev
    csr = grid_laplacian((64, 64, 40), 0.01)
    plan = _plan(gpu_lib, csr, engine="stream")
    A = csr.to_scipy()
    rng = np.random.default_rng(7)
    try:
        for k in (64, 84, 130, 16, 9):
            X = rng.standard_normal((csr.n, k))
            Y = torch.full((csr.n, k), float("nan"), dtype=torch.float64, device="cuda")
            plan.spmm(torch.from_numpy(X).cuda(), Y, alpha=0.75, beta=-1.5)
            ref = 0.75 * (A @ X) - 1.5 * X
            bound = 1.01 * 10 * U * (0.75 * (abs(A) @ np.abs(X)) + 1.5 * np.abs(X))
            got = Y.cpu().numpy()
            assert np.isfinite(got).all(), k
            assert np.all(np.abs(got - ref) <= bound + 1e-300), k
    finally:
        plan.close()


# the last three have n >= 2^17, where the TSMM stages S in LDS (ragged
# row count; k not a multiple of 4; 113 KiB of S)
@pytest.mark.parametrize("n,k,cond", [(5000, 64, 1e2), (5000, 64, 1e10), (999, 37, 1e6),
                                      (20000, 148, 1e4), (300, 1, 1.0), (131077, 84, 1e4),
                                      (140001, 37, 1e6), (131113, 148, 1e2)])
def test_cholqr2(small_plan, torch_dev, n, k, cond):
    torch = torch_dev
    _, plan = small_plan
    rng = np.random.default_rng(k)
    Uq, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Vq, _ = np.linalg.qr(rng.standard_normal((k, k)))
    s = np.logspace(0, -np.log10(cond), k)
    X = (Uq * s) @ Vq.T
    X = X * rng.uniform(0.01, 100.0, k)[None, :]  # column scaling on top
    Yd = torch.from_numpy(X.copy()).cuda()
    info = plan.cholqr2(Yd)
    Q = Yd.cpu().numpy()
    assert info in (0, 1)
    if cond > 1e7:
        assert info == 1  # shifted first pass
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-13
    # span(Q) = span(X): Q^T X reproduces X
    resid = np.linalg.norm(X - Q @ (Q.T @ X)) / np.linalg.norm(X)
    assert resid < 1e-15 * cond * 10


def test_cholqr2_rank_deficient(small_plan, torch_dev):
    torch = torch_dev
    _, plan = small_plan
    rng = np.random.default_rng(1)
    X = rng.standard_normal((2000, 10))
    X[:, 7] = 0.0
    Yd = torch.from_numpy(X).cuda()
    assert plan.cholqr2(Yd) == 2
    # a failed pass writes nothing back: Y is the input, bit for bit
    assert np.array_equal(Yd.cpu().numpy(), X)


# H and V in LDS up to k = 98, H alone up to 128, both in global memory above
@pytest.mark.parametrize("k", [1, 2, 7, 33, 64, 65, 98, 99, 128, 129, 148, 192])
def test_syev_jacobi(small_plan, torch_dev, k):
    torch = torch_dev
    _, plan = small_plan
    rng = np.random.default_rng(k)
    B = rng.standard_normal((k, k))
    H = B + B.T
    if k >= 7:  # repeated eigenvalues
        Qr, _ = np.linalg.qr(rng.standard_normal((k, k)))
        ev = np.round(rng.uniform(-3, 3, k), 1)
        H = (Qr * ev) @ Qr.T
    th = torch.zeros(k, dtype=torch.float64, device="cuda")
    S = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    plan.syev(torch.from_numpy(H).cuda(), th, S)
    theta = th.cpu().numpy()
    Sv = S.cpu().numpy()
    nrm = np.linalg.norm(H, 2)
    np.testing.assert_allclose(theta, np.linalg.eigvalsh(H), atol=1e-13 * nrm * max(1, k / 16))
    assert np.all(np.diff(theta) >= 0)
    assert np.abs(Sv.T @ Sv - np.eye(k)).max() < 1e-13 * max(1, k / 16)
    assert np.abs(H @ Sv - Sv * theta[None, :]).max() < 1e-13 * nrm * max(1, k / 16)


@pytest.mark.parametrize("k", [64, 84])
def test_syev_jacobi_nearly_diagonal(small_plan, torch_dev, k):
    # the reduced matrix of a late FEAST iteration: diagonal up to a small
    # symmetric perturbation, with a cluster of close diagonal entries
    torch = torch_dev
    _, plan = small_plan
    rng = np.random.default_rng(100 + k)
    d = np.sort(rng.uniform(0.0, 0.06, k))
    d[10:14] = d[10] + 1e-9 * np.arange(4)
    E = 1e-7 * rng.standard_normal((k, k))
    H = np.diag(d) + E + E.T
    th = torch.zeros(k, dtype=torch.float64, device="cuda")
    S = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    plan.syev(torch.from_numpy(H).cuda(), th, S)
    theta = th.cpu().numpy()
    Sv = S.cpu().numpy()
    nrm = np.linalg.norm(H, 2)
    np.testing.assert_allclose(theta, np.linalg.eigvalsh(H), atol=1e-14 * nrm * k)
    assert np.abs(Sv.T @ Sv - np.eye(k)).max() < 1e-14 * k
    assert np.abs(H @ Sv - Sv * theta[None, :]).max() < 1e-14 * nrm * k


@pytest.mark.parametrize("seed", [0, 12345, (1 << 40) + 7])
def test_gaussian_matches_oracle_philox(small_plan, torch_dev, seed):
    torch = torch_dev
    csr, plan = small_plan
    for w in (21, 84):
        O = torch.zeros((csr.n, w), dtype=torch.float64, device="cuda")
        plan.gaussian(O, seed)
        ref = philox.gaussian_sketch(csr.n, w, seed)
        np.testing.assert_allclose(O.cpu().numpy(), ref, rtol=1e-14, atol=1e-14)


def test_plan_waits_for_torch_stream(small_plan, torch_dev):
    # a plan made without a stream runs on its own; an output tensor whose
    # fill torch has queued behind long work on its current stream must be
    # filled before the plan writes it (else the late fill overwrites it)
    torch = torch_dev
    csr, plan = small_plan
    M = torch.randn((4096, 4096), dtype=torch.float32, device="cuda")
    for _ in range(6):
        M = torch.tanh(M @ M)
    O = torch.full((csr.n, 21), 7.0, dtype=torch.float64, device="cuda")
    plan.gaussian(O, 99)
    ref = philox.gaussian_sketch(csr.n, 21, 99)
    np.testing.assert_allclose(O.cpu().numpy(), ref, rtol=1e-14, atol=1e-14)
    assert torch.isfinite(M).all()


@pytest.mark.parametrize("engine", ["resident", "stream"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-6), ("fp32", 1e-10)])
def test_shifted_solve_cocg(gpu_lib, torch_dev, precision, tol, engine):
    torch = torch_dev
    csr = grid_laplacian((40, 40), 0.01)
    A = csr.to_scipy()
    lmin, lmax = 0.0, 0.20200934091026512
    z, _ = half_circle(lmin, lmax, 4)
    z = np.concatenate([z, [0.3 + 1e-3j]])
    rng = np.random.default_rng(5)
    k = 5
    B = rng.standard_normal((csr.n, k)) * np.array([1, 1e-8, 1e3, 1, 0])[None, :]
    with _plan(gpu_lib, csr, precision=precision, m0=8, engine=engine) as plan:
        assert plan.engine == engine
        ct = torch.complex64 if precision == "fp32" else torch.complex128
        X = torch.zeros((csr.n, len(z) * k), dtype=ct, device="cuda")
        its, rs = plan.shifted_solve(z, torch.from_numpy(B).cuda(), X, tol)
    Xh = X.cpu().numpy().astype(np.complex128)
    solver = ShiftedSolver(A, z, method="dense")
    u_out = 2.0 ** -24 if precision == "fp32" else U
    for j in range(len(z)):
        ref = solver.solve(j, B)
        for c in range(k):
            x = Xh[:, j * k + c]
            b = B[:, c]
            if np.linalg.norm(b) == 0:
                assert np.abs(x).max() == 0 and its[j * k + c] == 0 and rs[j * k + c] == 0
                continue
            # the library's FP64 solution met the tolerance ...
            assert rs[j * k + c] <= tol, (j, c, rs[j * k + c])
            # ... and its (output-rounded) solution is within the forward-error bound
            # kappa * tol of the exact solve, plus the output rounding
            kappa = np.abs(z[j] - np.array([0.0, 8.0])).max() / abs(z[j].imag)
            err = np.linalg.norm(x - ref[:, c]) / np.linalg.norm(ref[:, c])
            assert err <= 1.1 * kappa * tol + 4 * u_out, (j, c, err)
            # the true residual of the returned x, recomputed here in FP64
            r = b - (z[j] * x - A @ x)
            assert np.linalg.norm(r) <= (tol + 8.1 * np.linalg.norm(x) * 2 * u_out
                                         / np.linalg.norm(b)) * np.linalg.norm(b)
    assert its.max() > 10
