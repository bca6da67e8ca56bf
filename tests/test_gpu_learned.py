"""GPU parity of the learned polynomial preconditioner through the C ABI:
training samples, the BF16 network (forward and gradient) against the FP64
oracle, training, and the preconditioned COCG against the oracle's."""

import numpy as np
import pytest

from oracle import learned as Lr
from oracle.spectrum import gershgorin
from workloads import grid_laplacian, knn_laplacian
from workloads.learned import (flatten, init_weights, minibatch_order, normalization,
                               residual_samples, unflatten)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    return torch


def _plan(lib, csr, **kw):
    args = dict(lmin=0.0, lmax=0.5, m0=8, nc=4, q=1, p=4, precision="fp64")
    args.update(kw)
    return lib.Plan(csr, **args)


def _host_samples(A, lo, hi, z, R, th):
    X, G, h, rr = [], [], [], []
    for zj in z:
        for i in range(R.shape[1]):
            g_, h_, rr_ = Lr.sample_data(A, lo, hi, zj, R[:, i])
            X.append(Lr.features(zj, lo, hi, *th))
            G.append(g_)
            h.append(h_)
            rr.append(rr_)
    return np.array(X), np.array(G), np.array(h), np.array(rr)


def _c(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def test_samples_match_oracle(gpu_lib, torch_dev):
    torch = torch_dev
    csr = knn_laplacian(900, 2, 8, seed=3, weighted=True, shift=1e-3)
    A = csr.to_scipy()
    lo, hi = gershgorin(A)
    R = residual_samples(csr.n, 5, 11)
    z = np.array([0.05 + 0.02j, 0.3 + 0.1j, 0.9 + 0.004j])
    with _plan(gpu_lib, csr) as plan:
        X, G, h, rr = plan.pc_samples(z, torch.from_numpy(np.ascontiguousarray(R)).cuda(),
                                      0.01, 0.4)
    Xr, Gr, hr, rrr = _host_samples(A, lo, hi, z, R, (0.01, 0.4))
    np.testing.assert_allclose(X.cpu().numpy(), Xr, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(rr.cpu().numpy(), rrr, rtol=1e-12)
    Gg, hg = _c(G), _c(h)
    for s in range(len(rrr)):
        assert np.abs(Gg[s] - Gr[s]).max() <= 1e-10 * np.abs(Gr[s]).max()
        assert np.abs(hg[s] - hr[s]).max() <= 1e-10 * np.abs(hr[s]).max()


def _training_set(torch, plan, A, n, count=48, seed=5):
    lo, hi = gershgorin(A)
    rng = np.random.default_rng(seed)
    z = rng.uniform(0.0, 0.5, 6) + 1j * rng.uniform(0.005, 0.2, 6)
    R = residual_samples(n, count // 6, seed)
    X, G, h, rr = plan.pc_samples(z, torch.from_numpy(np.ascontiguousarray(R)).cuda(), 0.01, 0.4)
    return (X, G, h, rr), _host_samples(A, lo, hi, z, R, (0.01, 0.4))


def test_network_forward_and_gradient_bf16(gpu_lib, torch_dev):
    torch = torch_dev
    csr = knn_laplacian(600, 2, 8, seed=4, weighted=True, shift=1e-3)
    A = csr.to_scipy()
    params = init_weights(21)
    P64 = [(w.astype(np.float64), b.astype(np.float64)) for w, b in params]
    with _plan(gpu_lib, csr) as plan:
        dev, host = _training_set(torch, plan, A, csr.n)
        # the input standardization the library sets from the features
        W = torch.from_numpy(flatten(params)).cuda()
        plan.pc_normalize(dev[0], W)
        mu, sd = normalization(W.cpu().numpy())
        Y = plan.pc_forward(dev[0], W).cpu().numpy().astype(np.float64)
        g, loss = plan.pc_gradient(*dev, W)
    np.testing.assert_allclose(mu, host[0].mean(axis=0), rtol=1e-6, atol=1e-7)
    ref_sd = host[0].std(axis=0)
    ref_sd[ref_sd <= 1e-9 * np.maximum(1.0, np.abs(host[0].mean(axis=0)))] = 1.0
    np.testing.assert_allclose(sd, ref_sd, rtol=1e-6)
    norm = (mu, sd)
    # against the oracle's bfloat16 network (weights, biases and layer inputs
    # rounded to nearest even, FP32 sums): what remains is FP32 summation
    # order, the GELU's erf implementations and the rare bfloat16 rounding
    # they flip, so the bound is 1e-3 rather than the 2e-2 that bfloat16
    # rounding itself would need against the FP64 network
    Yr = Lr.mlp_forward(P64, host[0], norm, bf16=True)[0]
    assert np.linalg.norm(Y - Yr) <= 1e-3 * np.linalg.norm(Yr)
    Y64 = Lr.mlp_forward(P64, host[0], norm)[0]
    assert np.linalg.norm(Y - Y64) <= 2e-2 * np.linalg.norm(Y64)
    ref = Lr.batch_grad(P64, *host, norm=norm, bf16=True)
    gr = np.concatenate([np.concatenate([dw.ravel(), db]) for dw, db in ref])
    gg = g.cpu().numpy().astype(np.float64)
    assert np.all(gg[len(gr):] == 0.0)  # the standardization is not trained
    gg = gg[: len(gr)]
    assert np.linalg.norm(gg - gr) <= 1e-3 * np.linalg.norm(gr)
    for l, (dw, db) in enumerate(unflatten(gg)):  # layer by layer, weights and biases
        assert np.linalg.norm(dw - ref[l][0]) <= 2e-3 * np.linalg.norm(ref[l][0]), l
        assert np.linalg.norm(db - ref[l][1]) <= 2e-3 * np.linalg.norm(ref[l][1]), l
    lr = Lr.batch_loss(P64, *host, norm=norm, bf16=True)
    assert abs(loss - lr) <= 1e-3 * abs(lr)


def test_training_lowers_the_loss(gpu_lib, torch_dev):
    torch = torch_dev
    csr = knn_laplacian(800, 3, 8, seed=6, weighted=True, shift=1e-3)
    A = csr.to_scipy()
    W = torch.from_numpy(flatten(init_weights(3))).cuda()
    with _plan(gpu_lib, csr) as plan:
        dev, host = _training_set(torch, plan, A, csr.n, count=96)
        _, before = plan.pc_gradient(*dev, W)
        order = minibatch_order(96, 60, 9)  # 60 epochs
        losses = plan.pc_train(*dev, W, order, batch=32, lr=3e-3)
        _, after = plan.pc_gradient(*dev, W)
    assert np.all(np.isfinite(losses))
    # the per-sample optimum c* bounds every coefficient choice from below
    bound = np.mean([Lr.quad_loss(Lr.c_star(G, h), G, h, rr) for G, h, rr in zip(*host[1:])])
    assert after < 0.5 * before and after >= bound - 1e-6


@pytest.mark.parametrize("precond", [False, True])
def test_pc_solve_matches_oracle(gpu_lib, torch_dev, precond):
    torch = torch_dev
    csr = grid_laplacian((14, 13), 0.01)
    A = csr.to_scipy()
    lo, hi = gershgorin(A)
    n = csr.n
    z = np.array([0.9 + 0.05j, 0.2 + 0.01j])
    B = residual_samples(n, 3, 13)
    coef = None
    if precond:
        coef = [Lr.c_star(*Lr.sample_data(A, lo, hi, zj, B[:, 0])[:2]) for zj in z]
    with _plan(gpu_lib, csr, max_cocg=5000) as plan:
        X = torch.zeros((n, len(z) * 3), dtype=torch.complex128, device="cuda")
        its, rs = plan.pc_solve(z, torch.from_numpy(np.ascontiguousarray(B)).cuda(), X, 1e-10,
                                coef=coef)
    Xh = X.cpu().numpy()
    Ad = A.toarray()
    for j, zj in enumerate(z):
        kappa = np.abs(zj - np.array([lo, hi])).max() / abs(zj.imag)
        for c in range(3):
            col = j * 3 + c
            ref = np.linalg.solve(zj * np.eye(n) - Ad, B[:, c])
            assert rs[col] <= 1e-10
            assert np.linalg.norm(Xh[:, col] - ref) <= 1.1 * kappa * 1e-10 * np.linalg.norm(ref)
            _, it_o, _ = Lr.pc_cocg(A, zj, B[:, c], None if coef is None else coef[j], lo, hi,
                                    tol=1e-10)
            assert abs(int(its[col]) - it_o) <= 2, (j, c, its[col], it_o)
