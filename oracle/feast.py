"""FEAST and RA-FEAST, written out step by step in FP64 (oracle).

Follows FEAST Algorithm 1 and RA-FEAST Algorithm 2 of the paper, with the
readings listed below where the paper is silent or ambiguous.

Readings
--------
* Contour: Gauss-Legendre on the upper half circle, N_c upper nodes
  (``contour.half_circle``); the filtered block is the real part of the
  weighted sum of resolvent solves (eq. projector-quad).
* Iteration body (Algorithm 1): filter -> QR -> Rayleigh-Ritz -> rotate
  Q <- Q V.  Here each iteration starts with the Rayleigh-Ritz step on the
  current orthonormal Q (equivalent ordering), which also yields the residual
  used by the convergence test.  Algorithm 2 omits the rotation; it is kept,
  as in Algorithm 1.
* Convergence test (the paper states none): with Ritz pairs (theta_i, q_i),
  res_i = ||A q_i - theta_i q_i|| / (s_win ||q_i||), s_win = max(|lmin|, |lmax|);
  stop when every Ritz value inside [lmin, lmax] has res_i <= tol, or after
  max_iter filter steps.
* Residual-correction form of the shifted solves.  With A q = theta q + r,
  (zI - A)^{-1} q = (q + (zI - A)^{-1} r) / (z - theta) exactly, so the filter
  can solve against the Ritz residuals r_i instead of the q_i
  (form="residual"); the literal form (form="literal") solves against Q as in
  Algorithm 1.  With exact solves both give the same block.
* Warmstart operator (eq. B-def, Assumption 1.2-1.3).  The literal
  B = (A - lmin I)/(lmax - lmin) puts the targets on top of B's spectrum only
  for a window at the top of A's spectrum.  ws_op="auto" picks an
  SpMM-only map with the targets dominant:
    bottom window (lmin <= sigma_lo): C = (sigma_hi I - A)/(sigma_hi - lmin)
    top window    (lmax >= sigma_hi): the literal B
    interior:     F = I - ((A - cI)/R)^2, c the window centre,
                  R = max(c - sigma_lo, sigma_hi - c)
  with [sigma_lo, sigma_hi] the Gershgorin interval.  "literal", "flip",
  "fold" force one map; "none" is plain FEAST's random start.
* Power iteration (eq. rand-range): for symmetric op, (op op^T)^q op Omega =
  op^{2q+1} Omega; the block is orthonormalised after every application
  (same span, numerically stable).
* Warmstart size: the sketch has m0 + p columns; Rayleigh-Ritz of A on its
  span keeps the m0 Ritz vectors whose op-values |phi(theta)| are largest
  (ties to the lower index in ascending theta order).
* Output: Ritz pairs with theta in the closed window, ascending; each
  eigenvector has unit 2-norm and its largest-magnitude entry positive
  (lowest index on ties).  M >= m0 is reported as "subspace_too_small".
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .contour import half_circle
from .spectrum import gershgorin


# ---------------------------------------------------------------- solves ----

class ShiftedSolver:
    """Exact solves with (z_j I - A) for every node, factored once per node.

    Dense LU with partial pivoting for small n, sparse LU (SuperLU) otherwise.
    """

    def __init__(self, A, z, method: str = "auto"):
        A = sp.csr_matrix(A, dtype=np.float64)
        n = A.shape[0]
        if method == "auto":
            method = "dense" if n <= 2500 else "sparse"
        self.method = method
        self.z = np.asarray(z)
        self.f = []
        I = sp.identity(n, dtype=np.complex128, format="csc")
        for zj in self.z:
            M = zj * I - A.astype(np.complex128)
            if method == "dense":
                self.f.append(sla.lu_factor(M.toarray(), check_finite=False))
            else:
                self.f.append(spla.splu(sp.csc_matrix(M)))

    def solve(self, j: int, B):
        B = np.asarray(B, dtype=np.complex128)
        if self.method == "dense":
            return sla.lu_solve(self.f[j], B, check_finite=False)
        return self.f[j].solve(B)


# --------------------------------------------------------- building blocks --

def orth(X):
    """Orthonormal basis of range(X) by Householder QR (Algorithm 1, QR step)."""
    Q, _ = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    return Q


def rayleigh_ritz(A, Q, s_win: float):
    """Rayleigh-Ritz on span(Q) (Algorithm 1, Rayleigh-Ritz and rotation).

    Returns ascending Ritz values theta, rotated Q <- Q S, the residual block
    R = A Q - Q diag(theta) and the scaled residual norms res_i.
    """
    W = A @ Q
    H = Q.T @ W
    H = 0.5 * (H + H.T)
    theta, S = np.linalg.eigh(H)
    Q = Q @ S
    W = W @ S
    R = W - Q * theta[None, :]
    res = np.linalg.norm(R, axis=0) / (s_win * np.linalg.norm(Q, axis=0))
    return theta, Q, R, res


def filter_block(solver, z, w, Q, theta=None, R=None, form: str = "residual"):
    """Q~ = sum_j Re[w_j (z_j I - A)^{-1} Q] (eq. projector-quad).

    form="literal": solve against Q directly.
    form="residual": solve against the Ritz residuals R and use
      (zI - A)^{-1} q_i = (q_i + (zI - A)^{-1} r_i) / (z - theta_i).
    """
    Qt = np.zeros(Q.shape, dtype=np.float64)
    for j in range(len(z)):
        if form == "literal":
            X = solver.solve(j, Q)
            Qt += np.real(w[j] * X)
        elif form == "residual":
            D = solver.solve(j, R)
            Qt += np.real(w[j] * (Q + D) / (z[j] - theta)[None, :])
        else:
            raise ValueError(form)
    return Qt


def normalise_signs(X):
    """Unit columns with the largest-|entry| positive (lowest index on ties)."""
    X = X / np.linalg.norm(X, axis=0)[None, :]
    idx = np.argmax(np.abs(X), axis=0)  # argmax returns the first maximum
    s = np.sign(X[idx, np.arange(X.shape[1])])
    s[s == 0] = 1.0
    return X * s[None, :]


# ------------------------------------------------------------------ FEAST ---

# Ritz pairs whose filter gain is below this are spurious (see filter_gain).
SPURIOUS_GAIN = 0.25


def filter_gain(Qt, Q):
    """Filter gain mu_i of each Ritz vector q_i of Q, a basis of span(Qt).

    Qt = rho(A) Qprev is the filtered block of an orthonormal block Qprev
    (Section 2.1: the filter approximates the spectral projector).  Writing
    q_i = Qt y_i, the vector u_i = Qprev y_i satisfies rho(A) u_i = q_i, so
    mu_i = ||q_i|| / ||y_i|| = ||rho(A) u_i|| / ||u_i||.  For an eigenvector
    with eigenvalue lam it is |rho(lam)|, at least 1/2 inside the window (the
    filter is 1/2 at the edges); a mixture of eigenvectors from outside the
    window, which can put a Ritz value inside it, has the small gain of its
    parts.  y_i is the least-squares solution of Qt y = q_i.
    """
    Y = np.linalg.lstsq(Qt, Q, rcond=None)[0]
    return np.linalg.norm(Q, axis=0) / np.linalg.norm(Y, axis=0)


def feast(A, lmin, lmax, m0, nc, Q0, tol=1e-10, max_iter=20, form="residual",
          solver=None, perturb=None, record=False):
    """FEAST iteration from the start block Q0 (n x m0).

    perturb(m, Qt) -> Qt', if given, is applied to the filtered block of
    iteration m before orthonormalisation (perturbation E^(m) of Section 3.2.4).

    The pairs counted (M) and tested for convergence are the Ritz pairs with
    theta in the closed window whose filter gain (filter_gain) is at least
    SPURIOUS_GAIN; before the first filter step every gain counts as 1.  The
    window is reported empty when no Ritz value lies in it from iteration 2 on.
    """
    A = sp.csr_matrix(A, dtype=np.float64)
    s_win = max(abs(lmin), abs(lmax))
    z, w = half_circle(lmin, lmax, nc)
    if solver is None:
        solver = ShiftedSolver(A, z)
    Q = orth(Q0)
    hist = []
    status = "no_convergence"
    it = 0
    Qt = None  # the filtered block whose span Q is
    while True:
        theta, Q, R, res = rayleigh_ritz(A, Q, s_win)
        mu = filter_gain(Qt, Q) if Qt is not None else np.ones(Q.shape[1])
        inside = (theta >= lmin) & (theta <= lmax) & (mu >= SPURIOUS_GAIN)
        M = int(inside.sum())
        if record:
            hist.append(dict(Q=Q.copy(), theta=theta.copy(), res=res.copy(), M=M, mu=mu.copy()))
        if M > 0 and float(res[inside].max()) <= tol:
            status = "ok"
            break
        # empty: no Ritz value in the window at all (early gains can be small
        # for true window vectors that the previous block held only weakly)
        if not np.any((theta >= lmin) & (theta <= lmax)) and it >= 2:
            status = "empty_window"
            break
        if it >= max_iter:
            break
        Qt = filter_block(solver, z, w, Q, theta, R, form)
        if perturb is not None:
            Qt = perturb(it, Qt)
        Q = orth(Qt)
        it += 1
    if M >= m0 and status == "ok":
        status = "subspace_too_small"
    X = normalise_signs(Q[:, inside]) if M > 0 else np.zeros((A.shape[0], 0))
    return dict(lam=theta[inside], X=X, res=res[inside], M=M, iters=it,
                status=status, theta_all=theta, res_all=res, mu_all=mu, Q=Q, history=hist)


# -------------------------------------------------------------- warmstart ---

def warmstart_operator(A, lmin, lmax, ws_op="auto", bounds=None):
    """The map op(.) for Phase 1 and its scalar form phi(theta)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    lo, hi = gershgorin(A) if bounds is None else bounds
    if ws_op == "auto":
        if lmin <= lo:
            ws_op = "flip"
        elif lmax >= hi:
            ws_op = "literal"
        else:
            ws_op = "fold"
    if ws_op == "literal":
        s = 1.0 / (lmax - lmin)
        return (lambda X: s * (A @ X - lmin * X)), (lambda t: s * (t - lmin)), ws_op
    if ws_op == "flip":
        s = 1.0 / (hi - lmin)
        return (lambda X: s * (hi * X - A @ X)), (lambda t: s * (hi - t)), ws_op
    if ws_op == "fold":
        c = 0.5 * (lmin + lmax)
        Rr = max(c - lo, hi - c)

        def op(X):
            T = (A @ X - c * X) / Rr
            return X - (A @ T - c * T) / Rr

        return op, (lambda t: 1.0 - ((t - c) / Rr) ** 2), ws_op
    raise ValueError(ws_op)


def warmstart(A, lmin, lmax, m0, Omega, q, ws_op="auto", bounds=None):
    """Phase 1 of Algorithm 2: Q0 from the sketch Omega (n x (m0+p)).

    Returns (Q0, info) with info holding the op-Ritz estimates of
    beta_{m0} and beta_{m0+1} (Remark 1's post-hoc check).
    """
    A = sp.csr_matrix(A, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    if ws_op == "none":
        return orth(Omega[:, :m0]), dict(op="none")
    op, phi, name = warmstart_operator(A, lmin, lmax, ws_op, bounds)
    Y = Omega
    for _ in range(2 * q + 1):
        Y = orth(op(Y))
    H = Y.T @ (A @ Y)
    theta, S = np.linalg.eigh(0.5 * (H + H.T))
    f = np.abs(phi(theta))
    order = np.argsort(-f, kind="stable")
    sel = np.sort(order[:m0])
    Q0 = Y @ S[:, sel]
    info = dict(op=name, beta_m0=float(f[order[m0 - 1]]),
                beta_m0p1=float(f[order[m0]]) if len(f) > m0 else float("nan"),
                theta=theta, phi=f)
    p = Omega.shape[1] - m0
    info["gap"] = info["beta_m0"] - info["beta_m0p1"]
    info["r_halko"] = (float(r_halko(info["beta_m0"], info["beta_m0p1"], m0, p, q))
                       if p >= 2 else float("nan"))
    info["proj_bound"] = info["r_halko"] / info["gap"] if info["gap"] > 0 else float("nan")
    return Q0, info


def ra_feast(A, lmin, lmax, m0, nc, Omega, q, tol=1e-10, max_iter=20,
             form="residual", ws_op="auto", solver=None):
    """RA-FEAST (Algorithm 2): warmstart, then FEAST with N_c nodes."""
    Q0, info = warmstart(A, lmin, lmax, m0, Omega, q, ws_op)
    out = feast(A, lmin, lmax, m0, nc, Q0, tol=tol, max_iter=max_iter, form=form, solver=solver)
    out["ws_info"] = info
    out["Q0"] = Q0
    return out


def r_halko(beta_m0, beta_m0p1, m0: int, p: int, q: int, delta: float = 0.01):
    """R_Halko of the randomized range-finder lemma (eq. R-Halko):
    C1(delta) sqrt(1 + m0/(p-1)) beta_{m0+1} (beta_{m0+1}/beta_{m0})^(2q), with
    C1(delta) = 1 + (p/2) ln(2 m0 / delta).  Theorem 1 bounds the warmstart's
    projector error by R_Halko / delta_gap, delta_gap = beta_m0 - beta_{m0+1}
    (eq. gap-def), with probability at least 1 - delta."""
    c1 = 1.0 + 0.5 * p * np.log(2.0 * m0 / delta)
    return c1 * np.sqrt(1.0 + m0 / (p - 1.0)) * beta_m0p1 * (beta_m0p1 / beta_m0) ** (2 * q)


def default_oversampling(m0: int) -> int:
    """Remark 1: p = 10 for m0 <= 50, else min(20, ceil(m0/2))."""
    return 10 if m0 <= 50 else min(20, -(-m0 // 2))
