"""Pins for the oracle FEAST / RA-FEAST against closed forms, brute force and
invariants (Algorithm 1, Algorithm 2, Theorem 2)."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import feast as F
from oracle.contour import filter_value, half_circle
from oracle.subspace import sin_theta
from tests.closed_forms import grid_eigs, path_eigs, window_basis
from workloads import gaussian, grid_laplacian, random_symmetric

CFG1_WIN = (0.0, 0.20200934091026512)


def _check_pairs(out, A, lmin, lmax, tol):
    X, lam = out["X"], out["lam"]
    s_win = max(abs(lmin), abs(lmax))
    R = A @ X - X * lam[None, :]
    assert np.linalg.norm(R, axis=0).max() / s_win <= tol
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() < 1e-13
    assert np.all(lam >= lmin) and np.all(lam <= lmax)
    assert np.all(np.diff(lam) >= 0)


@pytest.mark.parametrize("nc,start", [(16, "plain"), (4, "ra")])
def test_grid2d_closed_form(nc, start):
    dims, shift = (40, 40), 0.01
    A = grid_laplacian(dims, shift).to_scipy()
    lmin, lmax = CFG1_WIN
    Om = gaussian(A.shape[0], 40, 0)
    if start == "plain":
        out = F.feast(A, lmin, lmax, 30, nc, Om[:, :30], tol=1e-10)
    else:
        out = F.ra_feast(A, lmin, lmax, 30, nc, Om, q=2)
    assert out["status"] == "ok"
    ref_vals, Vref = window_basis(dims, shift, lmin, lmax)
    assert out["M"] == 20 == len(ref_vals)
    np.testing.assert_allclose(out["lam"], ref_vals, atol=1e-12 * lmax)
    _check_pairs(out, A, lmin, lmax, 1e-10)
    assert sin_theta(out["X"], Vref).max() < 1e-8


def test_path_closed_form_interior_window():
    m = 300
    A = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1], format="csr")
    ev = path_eigs(m)
    lmin, lmax = 0.5 * (ev[99] + ev[100]), 0.5 * (ev[109] + ev[110])
    Om = gaussian(m, 20, 5)
    out = F.ra_feast(A, lmin, lmax, 14, 8, Om, q=1)
    assert out["status"] == "ok" and out["M"] == 10
    np.testing.assert_allclose(out["lam"], ev[100:110], atol=1e-12)


def test_grid3d_interior_fold_warmstart():
    dims, shift = (8, 8, 8), 0.01
    A = grid_laplacian(dims, shift).to_scipy()
    vals, _ = grid_eigs(dims, shift)
    # window of whole clusters around 3.0
    uniq = np.unique(np.round(vals, 12))
    lo_i = np.searchsorted(uniq, 2.6)
    hi_i = np.searchsorted(uniq, 3.0)
    lmin = 0.5 * (uniq[lo_i - 1] + uniq[lo_i])
    lmax = 0.5 * (uniq[hi_i - 1] + uniq[hi_i])
    ref = vals[(vals >= lmin) & (vals <= lmax)]
    m0 = int(len(ref) * 1.5) + 2
    Om = gaussian(A.shape[0], m0 + 10, 1)
    out = F.ra_feast(A, lmin, lmax, m0, 8, Om, q=2)
    assert out["ws_info"]["op"] == "fold"
    assert out["status"] == "ok"
    np.testing.assert_allclose(out["lam"], ref, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_matrix_brute_force(seed):
    Acsr = random_symmetric(150, seed, density=0.06)
    A = Acsr.to_scipy()
    lam, V = np.linalg.eigh(A.toarray())
    # interior window cut at mid-gaps around the 30th..45th eigenvalue
    lmin = 0.5 * (lam[29] + lam[30])
    lmax = 0.5 * (lam[44] + lam[45])
    Om = gaussian(150, 36, seed)
    for form in ("residual", "literal"):
        out = F.ra_feast(A, lmin, lmax, 26, 8, Om, q=2, form=form, max_iter=40)
        assert out["status"] == "ok", form
        np.testing.assert_allclose(out["lam"], lam[30:45], atol=1e-10 * abs(lmax))
        _check_pairs(out, A, lmin, lmax, 1e-10)
        assert sin_theta(out["X"], V[:, 30:45]).max() < 1e-8


def test_residual_form_equals_literal_form():
    A = grid_laplacian((20, 20), 0.01).to_scipy()
    lmin, lmax = 0.0, 0.5
    z, w = half_circle(lmin, lmax, 4)
    solver = F.ShiftedSolver(A, z, method="dense")
    Q = F.orth(gaussian(400, 12, 7))
    theta, Q, R, _ = F.rayleigh_ritz(A, Q, lmax)
    lit = F.filter_block(solver, z, w, Q, form="literal")
    res = F.filter_block(solver, z, w, Q, theta, R, form="residual")
    np.testing.assert_allclose(res, lit, atol=1e-12 * np.abs(lit).max())


def test_dense_and_sparse_solvers_agree():
    A = grid_laplacian((15, 15), 0.01).to_scipy()
    z, w = half_circle(0.0, 0.4, 3)
    B = gaussian(225, 4, 2)
    d = F.ShiftedSolver(A, z, method="dense")
    s = F.ShiftedSolver(A, z, method="sparse")
    for j in range(3):
        np.testing.assert_allclose(d.solve(j, B), s.solve(j, B), atol=1e-12)
        # and the solution satisfies the shifted system
        X = d.solve(j, B)
        np.testing.assert_allclose(z[j] * X - A @ X, B, atol=1e-12)


def test_empty_window_and_too_small_subspace():
    A = grid_laplacian((12, 12), 0.01).to_scipy()
    Om = gaussian(144, 8, 0)
    out = F.feast(A, -1.0, -0.5, 8, 8, Om, tol=1e-10, max_iter=6)
    assert out["status"] == "empty_window" and out["M"] == 0
    vals, _ = grid_eigs((12, 12), 0.01)
    lmax = 0.5 * (vals[9] + vals[10])  # 10 eigenvalues inside, subspace of 6
    out = F.feast(A, 0.0, lmax, 6, 8, Om[:, :6], tol=1e-10, max_iter=6)
    assert out["M"] >= 6
    assert out["status"] in ("subspace_too_small", "no_convergence")


def test_literal_operator_is_poor_for_bottom_window():
    # eq. B-def taken literally amplifies the top of A's spectrum.
    A = grid_laplacian((20, 20), 0.01).to_scipy()
    vals, _ = grid_eigs((20, 20), 0.01)
    lmin, lmax = 0.0, 0.5 * (vals[9] + vals[10])
    _, V = np.linalg.eigh(A.toarray())
    Om = gaussian(400, 22, 0)
    q_flip, _ = F.warmstart(A, lmin, lmax, 12, Om, 2, "flip")
    q_lit, _ = F.warmstart(A, lmin, lmax, 12, Om, 2, "literal")
    # fraction of the target space captured by each start (a random 12-column
    # block captures 12/400 = 0.03 on average)
    cap = lambda Q: np.linalg.norm(V[:, :10].T @ Q) ** 2 / 10
    assert cap(q_flip) > 0.4
    assert cap(q_lit) < 1e-10
    q8, _ = F.warmstart(A, lmin, lmax, 12, Om, 8, "flip")
    assert cap(q8) > cap(q_flip)


def test_warmstart_davis_kahan_lemma2():
    # ||sin Theta(Q0, V1)|| <= ||(I - Q0 Q0^T) B||_2 / delta_gap (Lemma 2),
    # for the flipped operator B on a bottom window.
    A = grid_laplacian((14, 14), 0.01).to_scipy()
    lam, V = np.linalg.eigh(A.toarray())
    lmin, lmax = 0.0, 0.5 * (lam[7] + lam[8])
    m0 = 8
    op, phi, _ = F.warmstart_operator(A, lmin, lmax, "flip")
    Bm = op(np.eye(196))
    beta = np.sort(phi(lam))[::-1]
    gap = beta[m0 - 1] - beta[m0]
    for seed in range(5):
        Q0, _ = F.warmstart(A, lmin, lmax, m0, gaussian(196, m0 + 10, seed), 3, "flip")
        st = sin_theta(Q0, V[:, :m0]).max()
        bound = np.linalg.norm(Bm - Q0 @ (Q0.T @ Bm), 2) / gap
        assert st <= bound * (1 + 1e-12)


def test_theorem1_statistics_top_window():
    # Theorem 1: ||P - P~||_2 <= R_Halko / delta_gap with probability >= 1 - delta.
    rng = np.random.default_rng(11)
    n, m0, p, q, delta = 300, 10, 10, 1, 0.1
    spec = np.concatenate([np.linspace(1.0, 0.9, m0), rng.uniform(0.0, 0.3, n - m0)])
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = sp.csr_matrix(U @ np.diag(spec) @ U.T)
    # Assumption 1.3 needs B's spectrum in [0, 1] with the targets on top: the
    # interval of eq. B-def spans A's whole spectrum here
    lmin, lmax = 0.0, 1.0
    beta = np.sort((spec - lmin) / (lmax - lmin))[::-1]
    b_m0, b_m1 = beta[m0 - 1], beta[m0]
    gap = b_m0 - b_m1
    R = F.r_halko(b_m0, b_m1, m0, p, q, delta)
    fails = 0
    for seed in range(40):
        Q0, _ = F.warmstart(A, lmin, lmax, m0, gaussian(n, m0 + p, seed), q, "literal")
        Q0o = F.orth(Q0)
        dist = np.linalg.norm(Q0o @ Q0o.T - U[:, :m0] @ U[:, :m0].T, 2)
        fails += dist > R / gap
    assert fails / 40 <= delta


def test_r_halko_hand_value():
    # m0 = 10, p = 10, q = 1, delta = 0.1, beta_m0 = 0.9, beta_m0+1 = 0.3:
    # C1 = 1 + 5 ln 200 = 27.491586832740182, sqrt(1 + 10/9) = sqrt(19)/3
    # = 1.4529663145135578, 0.3 (1/3)^2 = 1/30; product 1.3314783200165317
    assert F.r_halko(0.9, 0.3, 10, 10, 1, 0.1) == pytest.approx(1.3314783200165317, rel=1e-14)
    # q = 0 drops the power factor (x 9); a larger delta lowers C1
    assert F.r_halko(0.9, 0.3, 10, 10, 0, 0.1) == pytest.approx(11.983304880148786, rel=1e-14)
    assert F.r_halko(0.9, 0.3, 10, 10, 1, 0.5) < F.r_halko(0.9, 0.3, 10, 10, 1, 0.1)


def test_warmstart_reports_theorem1_bound():
    # the warmstart's own estimates satisfy Theorem 1 on a top window: the
    # projector error is below r_halko / gap (and Remark 1's 1/2 here)
    rng = np.random.default_rng(5)
    n, m0, p, q = 200, 8, 10, 2
    spec = np.concatenate([np.linspace(1.0, 0.95, m0), rng.uniform(0.0, 0.1, n - m0)])
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = sp.csr_matrix(U @ np.diag(spec) @ U.T)
    Q0, info = F.warmstart(A, 0.0, 1.0, m0, gaussian(n, m0 + p, 1), q, "literal")
    assert info["gap"] == pytest.approx(info["beta_m0"] - info["beta_m0p1"])
    assert info["proj_bound"] == pytest.approx(info["r_halko"] / info["gap"])
    Qo = F.orth(Q0)
    dist = np.linalg.norm(Qo @ Qo.T - U[:, :m0] @ U[:, :m0].T, 2)
    assert dist <= info["proj_bound"]
    assert info["proj_bound"] < 0.5


def test_theorem2_perturbed_iteration_floor():
    # e_{m+1} <= rho e_m + eps + O(u) with ||E||_F = eps injected each step.
    A = grid_laplacian((12, 12), 0.01).to_scipy()
    lam, V = np.linalg.eigh(A.toarray())
    lmin, lmax = 0.0, 0.5 * (lam[5] + lam[6])
    P = V[:, :6] @ V[:, :6].T
    z, w = half_circle(lmin, lmax, 4)
    r = np.abs(filter_value(lam, z, w))
    m0 = 10
    rho = np.sort(r)[::-1][m0] / r[:6].min()  # contraction of the ideal map
    floors = []
    for eps in (1e-4, 1e-6, 1e-8):
        rng = np.random.default_rng(1)

        def pert(m, Qt, eps=eps):
            E = rng.standard_normal(Qt.shape)
            return Qt + E * (eps / np.linalg.norm(E))

        out = F.feast(A, lmin, lmax, m0, 4, gaussian(144, m0, 0), tol=0.0, max_iter=10,
                      perturb=pert, record=True)
        errs = []
        for h in out["history"]:
            ins = (h["theta"] >= lmin) & (h["theta"] <= lmax)
            Q = h["Q"][:, ins]
            errs.append(np.linalg.norm(Q @ Q.T - P) if Q.shape[1] == 6 else np.inf)
        e = np.array(errs)
        for m in range(1, len(e) - 1):
            if np.isfinite(e[m]):
                assert e[m + 1] <= rho * e[m] + 3 * eps + 1e-12
        floors.append(e[-1])
    # the floor tracks eps
    for eps, fl in zip((1e-4, 1e-6, 1e-8), floors):
        assert 0.05 * eps <= fl <= 3 * eps


def test_default_oversampling_remark1():
    assert F.default_oversampling(30) == 10
    assert F.default_oversampling(50) == 10
    assert F.default_oversampling(64) == 20
    assert F.default_oversampling(128) == 20


# --- spurious Ritz values (filter gain) -------------------------------------

def _spurious_case():
    """Diagonal A with window [-1, 1] and outside pairs +-1.3, +-1.8 that the
    symmetric half-circle filter cannot tell apart; with m0 = 8 the subspace
    holds the 5 window vectors, the +-1.3 pair and one fixed mixture of the
    +-1.8 pair, whose Ritz value can fall inside the window."""
    inside = [-0.7, -0.3, 0.1, 0.5, 0.8]
    lam = np.array(inside + [-1.3, 1.3, -1.8, 1.8] + list(np.linspace(3.0, 20.0, 191)))
    return sp.diags(lam).tocsr(), np.array(inside), lam


def test_filter_gain_closed_form():
    lam = np.array([0.2, 0.9, 1.4, 2.5])
    z, w = half_circle(-1.0, 1.0, 4)
    rho = filter_value(lam, z, w)
    E = np.eye(4)
    # eigenvectors: the gain is |rho(lambda)|
    np.testing.assert_allclose(F.filter_gain(E * rho[None, :], E), np.abs(rho), rtol=1e-14)
    # an equal mixture of e_0 and e_3: 1 / sqrt((1/rho_0^2 + 1/rho_3^2) / 2)
    q = (E[:, [0]] + E[:, [3]]) / np.sqrt(2.0)
    Qt = E[:, [0, 3]] * rho[[0, 3]][None, :]
    g = F.filter_gain(Qt, q)[0]
    assert abs(g - 1.0 / np.sqrt(0.5 / rho[0] ** 2 + 0.5 / rho[3] ** 2)) <= 1e-14 * g


def test_spurious_ritz_value_is_excluded(monkeypatch):
    A, inside, lam = _spurious_case()
    n = A.shape[0]
    z, w = half_circle(-1.0, 1.0, 4)
    Q0 = np.random.default_rng(0).standard_normal((n, 8))
    # counting every in-window Ritz value: the mixture of the +-1.8 pair stays
    # in the window (its Ritz value does not move) and blocks convergence
    monkeypatch.setattr(F, "SPURIOUS_GAIN", 0.0)
    bad = F.feast(A, -1.0, 1.0, 8, 4, Q0, tol=1e-12, max_iter=25)
    assert bad["status"] == "no_convergence" and bad["M"] == 6
    spur = [i for i, t in enumerate(bad["theta_all"])
            if -1 <= t <= 1 and np.min(np.abs(t - inside)) > 1e-6]
    assert len(spur) == 1
    g = abs(filter_value(np.array([1.8]), z, w)[0])
    assert abs(bad["mu_all"][spur[0]] - g) <= 1e-8 * g
    monkeypatch.undo()
    # with the gain test: the five window eigenvalues, converged
    out = F.feast(A, -1.0, 1.0, 8, 4, Q0, tol=1e-12, max_iter=25)
    assert out["status"] == "ok" and out["M"] == 5
    np.testing.assert_allclose(out["lam"], inside, atol=1e-12)
    sel = (out["theta_all"] >= -1) & (out["theta_all"] <= 1) & (out["mu_all"] >= F.SPURIOUS_GAIN)
    np.testing.assert_allclose(out["mu_all"][sel], np.abs(filter_value(inside, z, w)), rtol=1e-6)


class _RelativeErrorSolver:
    """Exact shifted solves plus a random error of relative size tau in every
    column: a stand-in for an iterative solver stopped at tolerance tau."""

    def __init__(self, A, z, tau, seed):
        self.exact = F.ShiftedSolver(A, z)
        self.tau = tau
        self.rng = np.random.default_rng(seed)

    def solve(self, j, B):
        X = self.exact.solve(j, B)
        E = self.rng.standard_normal(X.shape) + 1j * self.rng.standard_normal(X.shape)
        E *= self.tau * np.linalg.norm(X, axis=0) / np.linalg.norm(E, axis=0)
        return X + E


@pytest.mark.parametrize("tau", [1e-2, 1e-4])
def test_relaxed_solves_residual_form(tau):
    # Phase 2 with relaxed solves (Section 3.3, k_inexact; Theorem 2): in the
    # residual-correction form the error a solve of relative accuracy tau
    # puts into the filtered block is tau times the Ritz residual, so
    # eps^(m) shrinks with e_m and the iteration still reaches 1e-10; with
    # the solves taken against Q the same tau leaves a floor near tau.
    dims, shift = (40, 40), 0.01
    A = grid_laplacian(dims, shift).to_scipy()
    lmin, lmax = CFG1_WIN
    vals, _ = window_basis(dims, shift, lmin, lmax)
    z, _ = half_circle(lmin, lmax, 4)
    om = gaussian(1600, 40, 0)
    exact = F.ra_feast(A, lmin, lmax, 30, 4, om, q=2)
    got = F.ra_feast(A, lmin, lmax, 30, 4, om, q=2, solver=_RelativeErrorSolver(A, z, tau, 3))
    assert exact["status"] == "ok" and got["status"] == "ok"
    assert got["M"] == len(vals)
    np.testing.assert_allclose(got["lam"], vals, rtol=0, atol=1e-10 * lmax)
    assert got["iters"] <= exact["iters"] + 1
    _check_pairs(got, A, lmin, lmax, 1e-10)
    lit = F.ra_feast(A, lmin, lmax, 30, 4, om, q=2, max_iter=12, form="literal",
                     solver=_RelativeErrorSolver(A, z, tau, 3))
    assert lit["status"] == "no_convergence"
    assert lit["res_all"][: len(vals)].max() > 1e-3 * tau
