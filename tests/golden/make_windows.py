"""Writes windows.json: search intervals cut at mid-gaps of reference spectra.

Calls only oracle/ (spectra) and workloads/ (the seeded matrices).  Run from
the repository root:  python tests/golden/make_windows.py [entry ...]
(entries: knn8000, batch32, learned, rgg, stats; default all; others are kept).
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.spectrum import bottom_eigvalsh  # noqa: E402
from oracle.stats import (covariance_spectrum, dense_spectrum, top_window,  # noqa: E402
                          variance_count)
from workloads import knn_laplacian, rgg_laplacian  # noqa: E402
from workloads.graphs import batch_graph_specs  # noqa: E402


def knn8000():
    # kNN Laplacian, n = 8000, 2D points (stream 1), k = 10, Gaussian weights,
    # + 1e-3 I; window holding the 50 smallest eigenvalues.
    A = knn_laplacian(8000, 2, 10, seed=1, weighted=True, shift=1e-3).to_scipy()
    ev = bottom_eigvalsh(A, 60)
    return dict(
        recipe="knn_laplacian(8000, dim=2, k=10, seed=1, weighted=True, shift=1e-3)",
        count=50, lmin=0.0, lmax=float(0.5 * (ev[49] + ev[50])),
        eigenvalues=[float(v) for v in ev[:52]], nnz=int(A.nnz))


def batch32():
    # 32 unweighted kNN Laplacians (no shift) of the batching workload: member
    # g keeps its `count` smallest eigenvalues in [-0.1 u, u], u at the mid-gap
    out = []
    for s in batch_graph_specs():
        A = knn_laplacian(s["n"], s["dim"], s["k"], seed=s["seed"], weighted=False).to_scipy()
        c = s["count"]
        ev = bottom_eigvalsh(A, c + 2)
        u = float(0.5 * (ev[c - 1] + ev[c]))
        out.append(dict(
            recipe=f"knn_laplacian({s['n']}, dim={s['dim']}, k={s['k']}, seed={s['seed']}, "
                   "weighted=False)",
            n=s["n"], dim=s["dim"], k=s["k"], seed=s["seed"], count=c, lmin=-0.1 * u, lmax=u,
            m0=int(-(-3 * c // 2)), eigenvalues=[float(v) for v in ev], nnz=int(A.nnz)))
    return out


def learned():
    # 3D 16-NN Laplacians, Gaussian weights, + 1e-3 I (points stream 5): the
    # window edge u = mid-gap of eigenvalues 100 and 101 at n = 1e4, 2e4, 5e4;
    # at n = 1e6 (too large for shift-invert here) u follows the power law
    # u ~ C n^-p fitted to those three (the kNN Laplacian with sigma = median
    # neighbour distance scales its low spectrum like n^(-2/3)).
    ns, us = [10000, 20000, 50000], []
    for n in ns:
        ev = bottom_eigvalsh(knn_laplacian(n, 3, 16, seed=5, weighted=True, shift=1e-3).to_scipy(),
                             102)
        us.append(float(0.5 * (ev[99] + ev[100])))
    slope, icpt = np.polyfit(np.log(ns), np.log(us), 1)
    u6 = float(np.exp(icpt + slope * np.log(1e6)))
    return dict(
        recipe="knn_laplacian(n, dim=3, k=16, seed=5, weighted=True, shift=1e-3)",
        measured=dict(n=ns, u=us), fit_exponent=float(slope),
        train=dict(n=20000, seed=5, u=us[1]),
        test=dict(n=1000000, seed=5, u=u6,
                  method="power law fitted to the mid-gap lambda_100/101 at n=1e4, 2e4, 5e4"))


def rgg():
    # The paper's sweep (Section 5.1): random geometric graph Laplacians
    # L = D - A, n points in the unit square, radius 1.5 sqrt(ln n / n),
    # window [0.001, 5.0]; 40 seeds per n.  Stored per graph: the eigenvalues
    # in the window, the ones just outside it, and the subspace size: the
    # paper's m0 = 40, or ceil(1.5 count) where the window holds 40 or more
    # eigenvalues (at n = 16000).
    out = []
    for n in (2000, 4000, 8000, 16000):
        for seed in range(40):
            A = rgg_laplacian(n, seed).to_scipy()
            ev = bottom_eigvalsh(A, 64)
            inside = ev[(ev >= 0.001) & (ev <= 5.0)]
            c = int(len(inside))
            if c >= 60:
                raise RuntimeError(f"rgg n={n} seed={seed}: window holds {c} >= 60 eigenvalues")
            out.append(dict(
                recipe=f"rgg_laplacian({n}, seed={seed})", n=n, seed=seed, count=c,
                lmin=0.001, lmax=5.0, m0=40 if c < 40 else -(-3 * c // 2),
                below=[float(v) for v in ev[ev < 0.001]],
                eigenvalues=[float(v) for v in inside],
                above=[float(v) for v in ev[ev > 5.0][:2]], nnz=int(A.nnz)))
            print(f"rgg n={n} seed={seed} count={c}", flush=True)
    return out


def stats():
    # Section 4 workloads: top windows chosen by the 95%-variance rule, from
    # the midpoint of the gap below lambda_k to 1.05 lambda_1; m0 = 2k.
    # Sample covariance of spiked data (spectrum through X X^T) and Gaussian
    # kernel matrices (dense spectrum).
    from workloads.stats import rbf_kernel, spiked_data

    out = {}
    for name, rows, p, nc in (("cov_small", 200, 2400, 8), ("cov_bench", 1024, 65536, 8)):
        X = spiked_data(rows, p, seed=1)
        ev = covariance_spectrum(X)
        tr = float((X * X).sum() / (rows - 1))
        k = variance_count(ev, tr)
        lo, hi = top_window(ev, k, 1.05 * ev[0])
        out[name] = dict(recipe=f"spiked_data({rows}, {p}, seed=1), scale 1/(rows-1)",
                         kind="covariance", rows=rows, p=p, count=k, lmin=float(lo),
                         lmax=float(hi), m0=2 * k, nc=nc, trace=tr,
                         eigenvalues=[float(v) for v in ev[: 2 * k + 2]])
    for name, n, nc in (("kpca_small", 1200, 16), ("kpca_bench", 8192, 16)):
        K = rbf_kernel(n, bandwidth=0.4, seed=2)
        ev = dense_spectrum(K)
        tr = float(np.trace(K))
        k = variance_count(ev, tr)
        lo, hi = top_window(ev, k, 1.05 * ev[0])
        out[name] = dict(recipe=f"rbf_kernel({n}, bandwidth=0.4, seed=2)", kind="kernel", n=n,
                         count=k, lmin=float(lo), lmax=float(hi), m0=2 * k, nc=nc, trace=tr,
                         eigenvalues=[float(v) for v in ev[: 2 * k + 2]])
    return out


ENTRIES = dict(knn8000=knn8000, batch32=batch32, learned=learned, rgg=rgg, stats=stats)


def main(names):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "windows.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    for name in names or list(ENTRIES):
        out[name] = ENTRIES[name]()
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
