"""Learned polynomial preconditioner for the shifted solves: the plain FP64
definitions (test infrastructure; see oracle/__init__.py).

The paper's dominant cost is the shifted solves (z_j I - A) d = r of the
filter (Section 2.1).  This part, which the paper does not have, accelerates
them with a polynomial preconditioner p(A) ~ (zI - A)^{-1}:

* Spectral map: A^ = a A + b I with a = 2 / (hi - lo), b = -(hi + lo)/(hi - lo)
  for an interval [lo, hi] containing the spectrum (Gershgorin), so the
  spectrum of A^ lies in [-1, 1]; z^ = a z + b likewise.
* p(A) = sum_{k<8} c_k T_k(A^), c_k complex, T_k the Chebyshev polynomials
  (T_0 = 1, T_1 = t, T_{k+1} = 2 t T_k - T_{k-1}).  p(A) is a polynomial in
  A, so it is complex symmetric and commutes with zI - A.
* Training data: for a residual vector r at shift z, v_k = (zI - A) T_k(A^) r,
  G_kl = <v_k, v_l> (Hermitian inner product), h_k = <v_k, r>, rr = <r, r>.
  The loss of coefficients c is ||(zI - A) p(A) r - r||^2 / ||r||^2
  = (c^H G c - 2 Re(c^H h) + rr) / rr, minimised by c* = G^{-1} h.
* Coefficient network: features x = (Re z^, Im z^, theta^_lo, theta^_hi) (the
  mapped shift and the mapped smallest and largest current Ritz values),
  standardized as (x - mu) / sd with the training set's mean and standard
  deviation, -> 4 x 64 x 64 x 64 x 16 MLP with exact GELU (x Phi(x)) on the hidden
  layers -> outputs (Re c_0, Im c_0, ..., Re c_7, Im c_7).
* Preconditioned COCG: COCG on (zI - A) x = b with the preconditioner p(A):
  rho = r^T p(A) r, the search direction from p(A) r.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.special import erf

K = 8  # Chebyshev terms (degree 7)


def spectral_map(lo: float, hi: float):
    """(a, b) with A^ = a A + b I mapping [lo, hi] onto [-1, 1]."""
    return 2.0 / (hi - lo), -(hi + lo) / (hi - lo)


def cheb_vectors(A, lo, hi, r, K=K):
    """[T_k(A^) r for k < K] by the three-term recurrence."""
    a, b = spectral_map(lo, hi)
    A = sp.csr_matrix(A)

    def Ahat(v):
        return a * (A @ v) + b * v

    out = [np.asarray(r, dtype=np.complex128)]
    if K > 1:
        out.append(Ahat(out[0]))
    while len(out) < K:
        out.append(2.0 * Ahat(out[-1]) - out[-2])
    return out


def sample_data(A, lo, hi, z, r):
    """(G, h, rr) of residual r at shift z (definitions in the module doc)."""
    A = sp.csr_matrix(A)
    T = cheb_vectors(A, lo, hi, r)
    V = np.stack([z * t - A @ t for t in T], axis=1)  # n x K
    r = np.asarray(r, dtype=np.complex128)
    G = V.conj().T @ V
    h = V.conj().T @ r
    rr = float(np.vdot(r, r).real)
    return G, h, rr


def c_star(G, h):
    """The per-sample optimal coefficients G^{-1} h."""
    return np.linalg.solve(G, h)


def quad_loss(c, G, h, rr):
    """(c^H G c - 2 Re(c^H h) + rr) / rr (real)."""
    c = np.asarray(c, dtype=np.complex128)
    return float((np.vdot(c, G @ c).real - 2.0 * np.vdot(c, h).real + rr) / rr)


def features(z, lo, hi, th_lo, th_hi):
    """(Re z^, Im z^, theta^_lo, theta^_hi)."""
    a, b = spectral_map(lo, hi)
    zh = a * z + b
    return np.array([zh.real, zh.imag, a * th_lo + b, a * th_hi + b])


# ---------------------------------------------------------------- network ---

def gelu(x):
    """Exact GELU x Phi(x), Phi the standard normal distribution function."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def bf16_round(x):
    """x rounded to bfloat16 (the upper 16 bits of an IEEE binary32, round to
    nearest, ties to even), returned as float32 values."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _layer_fp32(W, b, H):
    """b + W h per row of H in float32, the inputs summed in index order (a
    product of two bfloat16 values is exact in float32)."""
    W = np.asarray(W, dtype=np.float32)
    Z = np.repeat(np.asarray(b, dtype=np.float32)[None, :], H.shape[0], axis=0)
    for i in range(W.shape[1]):
        Z = (Z + H[:, i:i + 1] * W[:, i][None, :]).astype(np.float32)
    return Z


def mlp_forward(params, X, norm=None, bf16=False):
    """Outputs Y (N x 16) of features X (N x 4); params = [(W, b)] with W
    (out x in); norm = (mu, sd): the network sees (X - mu) / sd (None: X).
    bf16: the reduced-precision network (weights, biases and every layer's
    input rounded to bfloat16, sums and GELU in float32), else float64
    throughout.  Returns (Y, cache) with the pre-activations for backward."""
    H = np.asarray(X, dtype=np.float64)
    if norm is not None:
        H = (H - np.asarray(norm[0], dtype=np.float64)) / np.asarray(norm[1], dtype=np.float64)
    cache = []
    if bf16:
        H = bf16_round(H)
        for l, (W, b) in enumerate(params):
            Zp = _layer_fp32(bf16_round(W), bf16_round(b), H)
            cache.append((H.astype(np.float64), Zp.astype(np.float64)))
            if l < len(params) - 1:
                g = (np.float32(0.5) * Zp *
                     (np.float32(1.0) + erf(Zp * np.float32(0.70710678118654752))).astype(np.float32))
                H = bf16_round(g)
            else:
                H = Zp
        return H.astype(np.float64), cache
    for l, (W, b) in enumerate(params):
        Zp = H @ np.asarray(W, dtype=np.float64).T + np.asarray(b, dtype=np.float64)
        cache.append((H, Zp))
        H = gelu(Zp) if l < len(params) - 1 else Zp
    return H, cache


def mlp_backward(params, cache, dY, bf16=False):
    """Gradients [(dW, db)] of sum(dY * Y) with respect to every layer (with
    the bfloat16 weights when bf16, the cache then from the bf16 forward)."""
    grads = [None] * len(params)
    D = np.asarray(dY, dtype=np.float64)
    for l in range(len(params) - 1, -1, -1):
        H, Zp = cache[l]
        if l < len(params) - 1:
            D = D * gelu_grad(Zp)
        W = np.asarray(bf16_round(params[l][0]) if bf16 else params[l][0], dtype=np.float64)
        grads[l] = (D.T @ H, D.sum(axis=0))
        D = D @ W
    return grads


def coeffs(Y, X):
    """Complex coefficients (N x 8) from network outputs Y (N x 16) of
    features X (N x 4): c_k = (y_2k + i y_2k+1) / Im z^, the outputs being the
    coefficients scaled by the shift's distance from the real axis."""
    Y = np.asarray(Y, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    return (Y[:, 0::2] + 1j * Y[:, 1::2]) / X[:, 1:2]


def batch_loss(params, X, G, h, rr, norm=None, bf16=False):
    """Mean loss over samples: X (N x 4), G (N x 8 x 8), h (N x 8), rr (N)."""
    C = coeffs(mlp_forward(params, X, norm, bf16)[0], X)
    return float(np.mean([quad_loss(C[s], G[s], h[s], rr[s]) for s in range(len(rr))]))


def batch_grad(params, X, G, h, rr, norm=None, bf16=False):
    """Gradients of batch_loss: dL/dRe c = 2 Re(Gc - h)/rr, dL/dIm c =
    2 Im(Gc - h)/rr per sample, times dc/dy = 1 / Im z^, averaged, then back
    through the network."""
    Y, cache = mlp_forward(params, X, norm, bf16)
    C = coeffs(Y, X)
    N = len(rr)
    dY = np.zeros_like(Y)
    for s in range(N):
        g = 2.0 * (G[s] @ C[s] - h[s]) / rr[s] / float(X[s][1])
        dY[s, 0::2] = g.real / N
        dY[s, 1::2] = g.imag / N
    return mlp_backward(params, cache, dY, bf16)


# -------------------------------------------------- preconditioned solve ---

def apply_poly(A, lo, hi, c, v):
    """p(A) v = sum_k c_k T_k(A^) v."""
    return sum(ck * t for ck, t in zip(c, cheb_vectors(A, lo, hi, v, len(c))))


def pc_cocg(A, z, b, c, lo, hi, tol=1e-10, maxit=10000):
    """Preconditioned COCG in FP64 for (zI - A) x = b, preconditioner p(A)
    with coefficients c (None: no preconditioner).  Stops when the true
    residual ||b - (zI - A) x|| <= tol ||b||, checked whenever the recursive
    one is.  Returns (x, iterations, relative true residual)."""
    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    M = (lambda v: v) if c is None else (lambda v: apply_poly(A, lo, hi, c, v))
    x = np.zeros_like(b)
    r = b.copy()
    u = M(r)
    p = u.copy()
    rho = r @ u
    it = 0
    while it < maxit:
        w = z * p - A @ p
        alpha = rho / (p @ w)
        x += alpha * p
        r -= alpha * w
        it += 1
        if np.linalg.norm(r) <= tol * nb:
            true = np.linalg.norm(b - (z * x - A @ x)) / nb
            if true <= tol:
                return x, it, true
            r = b - (z * x - A @ x)  # replace the drifted recursive residual
        u = M(r)
        rho_new = r @ u
        p = u + (rho_new / rho) * p
        rho = rho_new
    return x, it, np.linalg.norm(b - (z * x - A @ x)) / nb
