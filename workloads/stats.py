"""Dense inputs of the statistical applications (Section 4): a data matrix for
the sample covariance (eq. sample-cov, p >> n) and a Gaussian kernel matrix for
kernel PCA (eq. kernel-eig).  Seeded and synthetic; no eigensolver arithmetic."""

import numpy as np


def spiked_data(rows: int, p: int, spikes: int = 16, top: float = 100.0, decay: float = 0.8,
                noise: float = 0.01, seed: int = 0) -> np.ndarray:
    """rows x p data matrix (column-major): `spikes` latent directions with
    variances top * decay^i along random orthonormal loadings, plus isotropic
    Gaussian noise of standard deviation `noise`; columns centred."""
    rng = np.random.default_rng(seed)
    W, _ = np.linalg.qr(rng.standard_normal((p, spikes)))
    sd = np.sqrt(top * decay ** np.arange(spikes))
    S = rng.standard_normal((rows, spikes)) * sd[None, :]
    X = S @ W.T + noise * rng.standard_normal((rows, p))
    X -= X.mean(axis=0, keepdims=True)
    return np.asfortranarray(X)


def rbf_kernel(n: int, dim: int = 3, clusters: int = 6, spread: float = 0.15,
               bandwidth: float = 0.5, seed: int = 0) -> np.ndarray:
    """n x n Gaussian kernel matrix K_ij = exp(-|x_i - x_j|^2 / (2 h^2)) of
    points drawn from a mixture of `clusters` isotropic Gaussians (centres
    uniform in the unit cube, standard deviation `spread`), h = bandwidth.
    Exactly symmetric with unit diagonal."""
    rng = np.random.default_rng(seed)
    centres = rng.random((clusters, dim))
    lab = rng.integers(0, clusters, n)
    x = centres[lab] + spread * rng.standard_normal((n, dim))
    sq = (x * x).sum(axis=1)
    d2 = sq[:, None] + sq[None, :] - 2.0 * (x @ x.T)
    d2 = np.maximum(0.5 * (d2 + d2.T), 0.0)
    K = np.exp(-d2 / (2.0 * bandwidth * bandwidth))
    np.fill_diagonal(K, 1.0)
    return np.asfortranarray(K)
