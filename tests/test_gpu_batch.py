"""GPU parity of the batching form (rafeast_plan_batch / rafeast_batch_solve)
through the C ABI: members of different sizes, windows and engines solved in
lock step, each against reference eigenpairs and against the same member
solved alone (rafeast_solve).  The shared resident launch is replayed from a
captured graph on every iteration, so the comparison with the single-member
runs (eager launches) checks every replay."""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import eigsh

from oracle.spectrum import gershgorin
from oracle.subspace import sin_theta
from tests.closed_forms import grid_eigs, window_basis
from workloads import gaussian, grid_laplacian, knn_laplacian, random_symmetric

pytestmark = pytest.mark.gpu


def _bottom(A, k):
    """The k smallest eigenpairs (shift-invert Lanczos), ascending."""
    lo, _ = gershgorin(A)
    vals, vecs = eigsh(sp.csc_matrix(A), k=k, sigma=lo - 1e-3, which="LM", tol=1e-14)
    o = np.argsort(vals)
    return vals[o], vecs[:, o]


def _members():
    out = []
    # closed-form grids: bottom windows at mid-gaps
    for dims, count in (((30, 30), 11), ((100, 100), 10)):
        vals, _ = grid_eigs(dims, 0.01)
        u = 0.5 * (vals[count - 1] + vals[count])
        lam, V = window_basis(dims, 0.01, 0.0, u)
        out.append(dict(csr=grid_laplacian(dims, 0.01), lmin=0.0, lmax=u, m0=int(1.5 * count) + 2,
                        ref=(lam, V, vals[count] - vals[count - 1])))
    # unweighted kNN Laplacians, no shift (window [-0.1 u, u] as in the batch workload)
    for n, dim, k, count in ((1500, 2, 8, 10), (2500, 3, 12, 20), (4000, 2, 16, 40)):
        csr = knn_laplacian(n, dim, k, seed=300 + n, weighted=False)
        A = csr.to_scipy()
        vals, vecs = _bottom(A, count + 2)
        u = 0.5 * (vals[count - 1] + vals[count])
        out.append(dict(csr=csr, lmin=-0.1 * u, lmax=u, m0=int(np.ceil(1.5 * count)),
                        ref=(vals[:count], vecs[:, :count], vals[count] - vals[count - 1])))
    # an interior window (fold warm start)
    csr = random_symmetric(700, 3, density=0.02)
    lam_all, V_all = np.linalg.eigh(csr.to_scipy().toarray())
    lo, hi = 0.5 * (lam_all[99] + lam_all[100]), 0.5 * (lam_all[115] + lam_all[116])
    out.append(dict(csr=csr, lmin=lo, lmax=hi, m0=26,
                    ref=(lam_all[100:116], V_all[:, 100:116],
                         min(lam_all[100] - lam_all[99], lam_all[116] - lam_all[115]))))
    return out


# relaxed Phase-2 solves, a different starting tolerance per member (0.5
# forces the tolerance down during the solve) in the one shared launch
RELAXED = [0.5, 1e-2, 1e-2, 0.0, 0.5, 1e-2]


@pytest.mark.parametrize("precision,relaxed", [("fp32", False), ("fp64", False), ("fp32", True)])
def test_batch_parity(gpu_lib, precision, relaxed, monkeypatch):
    members = _members()
    rel = RELAXED if relaxed else [0.0] * len(members)
    probs = [{k: m[k] for k in ("csr", "lmin", "lmax", "m0")} for m in members]
    for pr, r in zip(probs, rel):
        pr["tol_solve_relaxed"] = r
    with gpu_lib.Batch(probs, nc=4, q=2, p=10, precision=precision) as B:
        assert B.resident_count == len(members) - 1
        # the 100 x 100 grid is too large for the shared launch: multi-shift, FP64
        engines = [m.engine for m in B.members]
        assert engines == ["resident", "multishift"] + ["resident"] * 4
        # the shared launch gives every resident member the largest slot
        # count the members' own tunings chose
        slots = max(m.tuning["chosen"] for m in B.members if m.engine == "resident")
        for g, m in enumerate(B.members):
            m.warmstart(omega=gaussian(m.n, m.w, g))
        outs, t_ms, status = B.solve()
    assert status == "OK", [o["status"] for o in outs]
    assert t_ms["solve"] > 0 and t_ms["total"] >= t_ms["solve"]
    for g, (m, out) in enumerate(zip(members, outs)):
        A = m["csr"].to_scipy()
        lam_ref, V_ref, gap = m["ref"]
        s_win = max(abs(m["lmin"]), abs(m["lmax"]))
        assert out["status"] == "OK" and out["M"] == len(lam_ref), g
        assert np.abs(out["lam"] - lam_ref).max() <= 1e-10 * s_win, g
        X = out["X"]
        R = A @ X - X * out["lam"][None, :]
        assert (np.linalg.norm(R, axis=0) / s_win).max() <= 1.0001e-10, g
        assert np.abs(X.T @ X - np.eye(X.shape[1])).max() < 1e-12, g
        assert sin_theta(X, V_ref).max() <= max(1e-8, 2 * np.linalg.norm(R) / gap), g
    # each member alone, on the eager single-plan path with the slot layout it
    # had in the shared launch (so the same summation order): same iteration
    # counts, same eigenvalues
    monkeypatch.setenv("RAFEAST_RESIDENT_SLOTS", str(slots))
    for g, (m, out) in enumerate(zip(members, outs)):
        ms = engines[g] == "multishift"
        with gpu_lib.Plan(m["csr"], m["lmin"], m["lmax"], m["m0"], nc=4, q=2, p=10,
                          precision="fp64" if ms else precision, tol_solve_relaxed=rel[g],
                          engine="multishift" if ms else "auto") as plan:
            plan.warmstart(omega=gaussian(plan.n, plan.w, g))
            alone = plan.solve()
        s_win = max(abs(m["lmin"]), abs(m["lmax"]))
        assert alone["iters"] == out["iters"], g
        assert alone["tol_solve_last"] == out["tol_solve_last"], g
        assert 1e-6 <= out["tol_solve_last"] <= max(rel[g], 1e-6), g
        assert np.abs(alone["lam"] - out["lam"]).max() <= 1e-11 * s_win, g


def test_batch_repeated_solves_agree(gpu_lib):
    # the captured launch is replayed again by a second solve (same item count)
    members = _members()[:1] + _members()[2:4]
    probs = [{k: m[k] for k in ("csr", "lmin", "lmax", "m0")} for m in members]
    with gpu_lib.Batch(probs, nc=4, q=2, p=10) as B:
        res = []
        for _ in range(2):
            for g, m in enumerate(B.members):
                m.warmstart(omega=gaussian(m.n, m.w, g))
            outs, _, status = B.solve()
            assert status == "OK"
            res.append(outs)
    for a, b in zip(*res):
        assert np.array_equal(a["lam"], b["lam"]) and a["iters"] == b["iters"]
        assert np.array_equal(a["X"], b["X"])


def test_batch32_workload(gpu_lib):
    # the batching form at its full size: the 32 stored graphs (n from 2000 to
    # 60000, 9 in the shared resident launch), each member's eigenvalues
    # against its stored spectrum
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "windows.json")) as f:
        wins = json.load(f)["batch32"]
    probs = []
    for wn in wins:
        csr = knn_laplacian(wn["n"], wn["dim"], wn["k"], seed=wn["seed"], weighted=False)
        assert csr.nnz == wn["nnz"]
        probs.append(dict(csr=csr, lmin=wn["lmin"], lmax=wn["lmax"], m0=wn["m0"]))
    with gpu_lib.Batch(probs, nc=4, q=2, tol_eig=1e-10, tol_solve=1e-6, precision="fp32",
                       seed=0) as B:
        assert B.resident_count == 9
        for m in B.members:
            m.warmstart()
        outs, _, status = B.solve(want_vectors=False)
    assert status == "OK"
    for wn, o in zip(wins, outs):
        ev = np.array(wn["eigenvalues"][: wn["count"]])
        assert o["M"] == wn["count"]
        s_win = max(abs(wn["lmin"]), wn["lmax"])
        assert np.abs(o["lam"] - ev).max() <= 1e-10 * s_win
        assert o["max_resid"] <= 1e-10
