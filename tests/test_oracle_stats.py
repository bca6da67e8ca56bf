"""Pins for the statistical workloads of Section 4 on the oracle side: the
variance-explained rule on a closed-form spectrum, the covariance spectrum
through X X^T against the p x p eigensolve, and the oracle's RA-FEAST on top
windows of a sample covariance and a kernel matrix against those spectra."""

import json
import os

import numpy as np
import pytest

from oracle import feast as F
from oracle.stats import (covariance_spectrum, dense_spectrum, sample_covariance, top_window,
                          variance_count)
from workloads import gaussian
from workloads.stats import rbf_kernel, spiked_data

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fixture(name):
    with open(os.path.join(GOLDEN, "windows.json")) as f:
        return json.load(f)["stats"][name]


def test_variance_count_closed_form():
    # lambda_i = 2^-i, i = 0..39: the k largest hold 2 (1 - 2^-k) of the
    # trace 2 (1 - 2^-40); 95% needs 2^-k <= 0.05 + 0.95 * 2^-40, so k = 5
    ev = 0.5 ** np.arange(40)
    assert variance_count(ev, ev.sum(), 0.95) == 5
    assert variance_count(ev, ev.sum(), 0.5) == 1
    assert variance_count(ev, ev.sum(), 0.75) == 2
    with pytest.raises(ValueError):
        variance_count(ev[:3], ev.sum(), 0.95)


def test_top_window_cuts_mid_gap():
    ev = np.array([9.0, 5.0, 3.0, 1.0])
    assert top_window(ev, 2, 10.0) == (4.0, 10.0)
    with pytest.raises(ValueError):
        top_window(ev, 2, 8.0)


def test_covariance_spectrum_duality():
    # the nonzero eigenvalues of X^T X / (n - 1) (p x p) are those of
    # X X^T / (n - 1) (n x n); centred columns leave one zero among the n
    X = spiked_data(30, 80, spikes=4, seed=5)
    big = np.sort(np.linalg.eigvalsh(sample_covariance(X)))[::-1]
    small = covariance_spectrum(X)
    np.testing.assert_allclose(small[:29], big[:29], rtol=1e-11, atol=1e-12 * big[0])
    assert abs(small[29]) <= 1e-12 * big[0]
    assert np.abs(big[29:]).max() <= 1e-12 * big[0]
    # trace of the covariance is ||X||_F^2 / (n - 1)
    assert np.isclose(big.sum(), (X * X).sum() / 29, rtol=1e-12)


def _check(out, A, ref, lmin, lmax):
    s_win = max(abs(lmin), abs(lmax))
    assert out["status"] == "ok" and out["M"] == len(ref)
    np.testing.assert_allclose(np.sort(out["lam"])[::-1], ref, rtol=0, atol=1e-10 * s_win)
    X = out["X"]
    R = A @ X - X * out["lam"][None, :]
    assert (np.linalg.norm(R, axis=0) / s_win).max() <= 1e-10


def test_oracle_ra_feast_covariance_top_window():
    fx = _fixture("cov_small")
    X = spiked_data(fx["rows"], fx["p"], seed=1)
    A = sample_covariance(X)
    k = fx["count"]
    ref = np.array(fx["eigenvalues"][:k])
    w = fx["m0"] + F.default_oversampling(fx["m0"])
    out = F.ra_feast(A, fx["lmin"], fx["lmax"], fx["m0"], fx["nc"], gaussian(fx["p"], w, 0),
                     q=2, ws_op="literal")
    _check(out, A, ref, fx["lmin"], fx["lmax"])


def test_oracle_ra_feast_kernel_top_window():
    fx = _fixture("kpca_small")
    K = rbf_kernel(fx["n"], bandwidth=0.4, seed=2)
    k = fx["count"]
    ref = np.array(fx["eigenvalues"][:k])
    # the stored spectrum is the dense eigensolve of this K
    np.testing.assert_allclose(dense_spectrum(K)[:k], ref, rtol=1e-13)
    w = fx["m0"] + F.default_oversampling(fx["m0"])
    out = F.ra_feast(K, fx["lmin"], fx["lmax"], fx["m0"], fx["nc"], gaussian(fx["n"], w, 0),
                     q=2, ws_op="literal")
    _check(out, K, ref, fx["lmin"], fx["lmax"])
    # the 95% rule holds for the stored count and fails for one less
    ev = dense_spectrum(K)
    assert ev[:k].sum() >= 0.95 * np.trace(K) > ev[: k - 1].sum()
