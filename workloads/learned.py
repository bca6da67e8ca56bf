"""Seeded draws for the learned polynomial preconditioner: the initial MLP
weights, the training-sample residuals and the minibatch order.  Random
numbers only; the network and the loss live with their users."""

from __future__ import annotations

import numpy as np

# Layer widths of the coefficient network: 4 features -> 3 hidden layers of
# 64 (GELU) -> 16 outputs (8 complex Chebyshev coefficients).
MLP_SIZES = (4, 64, 64, 64, 16)


def init_weights(seed: int, sizes=MLP_SIZES, out_scale: float = 0.1):
    """[(W_l, b_l)]: W_l (out x in) ~ N(0, 1/in) (float32), b_l = 0, except
    the last layer, scaled by out_scale so the untrained outputs start small
    (0: they start at zero, the choice for training a preconditioner)."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(len(sizes) - 1):
        fan_in, fan_out = sizes[l], sizes[l + 1]
        W = rng.standard_normal((fan_out, fan_in)) / np.sqrt(fan_in)
        if l == len(sizes) - 2:
            W = W * out_scale
        out.append((W.astype(np.float32), np.zeros(fan_out, dtype=np.float32)))
    return out


def flatten(params, norm=None) -> np.ndarray:
    """All weights and biases in layer order (W row-major, then b), then the
    input standardization mu[4], sd[4] (default 0 and 1), float32."""
    mu, sd = norm if norm is not None else (np.zeros(4), np.ones(4))
    parts = [np.concatenate([W.ravel(), b.ravel()]) for W, b in params] + [mu, sd]
    return np.concatenate(parts).astype(np.float32)


def normalization(flat, sizes=MLP_SIZES):
    """(mu, sd) stored after the weights of a flat parameter vector."""
    o = parameter_count(sizes)
    return (np.asarray(flat[o:o + sizes[0]], dtype=np.float64),
            np.asarray(flat[o + sizes[0]:o + 2 * sizes[0]], dtype=np.float64))


def unflatten(flat, sizes=MLP_SIZES):
    out, o = [], 0
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        W = np.asarray(flat[o:o + fo * fi], dtype=np.float64).reshape(fo, fi)
        o += fo * fi
        b = np.asarray(flat[o:o + fo], dtype=np.float64)
        o += fo
        out.append((W, b))
    return out


def parameter_count(sizes=MLP_SIZES) -> int:
    """Trained weights and biases (the standardization is not counted)."""
    return sum(sizes[l + 1] * sizes[l] + sizes[l + 1] for l in range(len(sizes) - 1))


def residual_samples(n: int, count: int, seed: int) -> np.ndarray:
    """count real n-vectors (columns, Fortran order) with standard normal entries."""
    g = np.random.default_rng(seed).standard_normal((count, n))
    return np.asfortranarray(g.T)


def minibatch_order(count: int, epochs: int, seed: int) -> np.ndarray:
    """epochs concatenated random permutations of range(count) (int32)."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.permutation(count) for _ in range(epochs)]).astype(np.int32)
