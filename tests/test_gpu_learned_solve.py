"""The learned polynomial preconditioner inside rafeast_solve (precond
LEARNED), on the kNN n = 8000 workload: training samples harvested from the
solver's own Ritz residuals, the network trained on the GPU, the eigenpairs
against the stored spectrum and the unpreconditioned solve, and what the
network gains over plain FP64 COCG on the same systems."""

import json
import os

import numpy as np
import pytest

from workloads import knn_laplacian
from workloads.learned import flatten, init_weights, minibatch_order

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def knn8000():
    with open(os.path.join(GOLDEN, "windows.json")) as f:
        win = json.load(f)["knn8000"]
    csr = knn_laplacian(8000, 2, 10, seed=1, weighted=True, shift=1e-3)
    assert csr.nnz == win["nnz"]
    return csr, win


def _kw(win, **extra):
    kw = dict(lmin=win["lmin"], lmax=win["lmax"], m0=64, nc=4, q=2, p=20, tol_eig=1e-10,
              tol_solve=1e-6, seed=0)
    kw.update(extra)
    return kw


def test_learned_preconditioner_inside_the_solve(gpu_lib, knn8000):
    import torch

    native = gpu_lib
    csr, win = knn8000
    # training data: COCG residuals of the solver's own shifted systems (the
    # right-hand sides and the residuals after 32 and 128 iterations) in the
    # first two FEAST iterations (the warm start's Ritz residuals, max_iter
    # 0, and those after one filter application), at the plan's own nodes
    samples = []
    for it in (0, 1):
        with native.Plan(csr, **_kw(win, max_iter=it, precision="fp32")) as plan:
            plan.warmstart()
            plan.solve(want_vectors=False)
            samples.append(plan.pc_harvest(steps=(0, 32, 128)))
    X, G, h, rr = (torch.cat([s[i] for s in samples]) for i in range(4))
    ns = X.shape[0]
    assert ns == 2 * 5 * 4 * 64 and bool((rr > 0).all())
    print(f"harvested {X.shape[0]} samples", flush=True)
    W = torch.from_numpy(flatten(init_weights(17, out_scale=0.0))).cuda()
    with native.Plan(csr, **_kw(win, max_iter=0, precision="fp32")) as plan:
        plan.pc_normalize(X, W)
        _, before = plan.pc_gradient(X, G, h, rr, W)
        losses = plan.pc_train(X, G, h, rr, W, minibatch_order(ns, 80, 3), batch=64, lr=1e-3)
        _, after = plan.pc_gradient(X, G, h, rr, W)
    print(f"trained: mean loss {before:.4f} -> {after:.4f}", flush=True)
    assert np.all(np.isfinite(losses)) and after < 0.5 * before

    ev = np.array(win["eigenvalues"][: win["count"]])
    s_win = max(abs(win["lmin"]), abs(win["lmax"]))
    runs = {}
    for name, extra in (("learned", dict(precision="fp64", precond="learned", max_cocg=4000)),
                        ("plain_fp64", dict(precision="fp64", engine="stream")),
                        ("plain_fp32_resident", dict(precision="fp32"))):
        with native.Plan(csr, **_kw(win, **extra)) as plan:
            if name == "learned":
                plan.pc_attach(W)
            plan.warmstart()
            out = plan.solve()
        print(f"{name}: {out['status']} M={out['M']} iters={out['iters']} "
              f"cocg={out['cocg_iters']} solve={out['t_ms']['solve']:.1f} ms "
              f"fallbacks={out['pc_fallbacks']}", flush=True)
        assert out["status"] == "OK" and out["M"] == win["count"], (name, out["status"])
        assert np.abs(out["lam"] - ev).max() <= 1e-10 * s_win, name
        assert out["max_resid"] <= 1e-10
        A = csr.to_scipy()
        R = A @ out["X"] - out["X"] * out["lam"][None, :]
        assert np.linalg.norm(R, axis=0).max() / s_win <= 1.5e-10
        assert sum(out["cocg_node"]) == out["cocg_iters"]
        runs[name] = out
    L, P64 = runs["learned"], runs["plain_fp64"]
    # a preconditioned iteration costs one operator product plus seven for
    # the Clenshaw recurrence of the degree-7 polynomial
    spmv_learned = 8 * L["cocg_iters"]
    report = dict(
        feast_iters={k: v["iters"] for k, v in runs.items()},
        cocg_iters={k: v["cocg_iters"] for k, v in runs.items()},
        cocg_node={k: v["cocg_node"] for k, v in runs.items()},
        spmv=dict(learned=spmv_learned, plain_fp64=P64["cocg_iters"]),
        solve_ms={k: round(v["t_ms"]["solve"], 2) for k, v in runs.items()},
        fallbacks=L["pc_fallbacks"],
        train_loss=dict(before=before, after=after),
        iteration_gain=P64["cocg_iters"] / L["cocg_iters"],
        spmv_gain=P64["cocg_iters"] / spmv_learned,
        time_gain=P64["t_ms"]["solve"] / L["t_ms"]["solve"])
    print("learned-preconditioner gain:", json.dumps(report))
    # what the trained network gains over the same FP64 COCG without it:
    # fewer iterations (each one more expensive; the SpMV and time ratios
    # above are reported whatever their sign)
    assert L["iters"] <= P64["iters"] + 1
    assert report["iteration_gain"] > 1.5, report
