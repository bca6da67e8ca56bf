"""Writes windows.json: search intervals cut at mid-gaps of reference spectra.

Calls only oracle/ (spectra) and workloads/ (the seeded matrices).  Run from
the repository root:  python tests/golden/make_windows.py
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.spectrum import bottom_eigvalsh  # noqa: E402
from workloads import knn_laplacian  # noqa: E402
from workloads.graphs import batch_graph_specs  # noqa: E402


def main():
    out = {}
    # kNN Laplacian, n = 8000, 2D points (stream 1), k = 10, Gaussian weights,
    # + 1e-3 I; window holding the 50 smallest eigenvalues.
    A = knn_laplacian(8000, 2, 10, seed=1, weighted=True, shift=1e-3).to_scipy()
    ev = bottom_eigvalsh(A, 60)
    out["knn8000"] = dict(
        recipe="knn_laplacian(8000, dim=2, k=10, seed=1, weighted=True, shift=1e-3)",
        count=50, lmin=0.0, lmax=float(0.5 * (ev[49] + ev[50])),
        eigenvalues=[float(v) for v in ev[:52]], nnz=int(A.nnz))
    # 32 unweighted kNN Laplacians (no shift) of the batching workload: member
    # g keeps its `count` smallest eigenvalues in [-0.1 u, u], u at the mid-gap
    out["batch32"] = []
    for s in batch_graph_specs():
        A = knn_laplacian(s["n"], s["dim"], s["k"], seed=s["seed"], weighted=False).to_scipy()
        c = s["count"]
        ev = bottom_eigvalsh(A, c + 2)
        u = float(0.5 * (ev[c - 1] + ev[c]))
        out["batch32"].append(dict(
            recipe=f"knn_laplacian({s['n']}, dim={s['dim']}, k={s['k']}, seed={s['seed']}, "
                   "weighted=False)",
            n=s["n"], dim=s["dim"], k=s["k"], seed=s["seed"], count=c, lmin=-0.1 * u, lmax=u,
            m0=int(-(-3 * c // 2)), eigenvalues=[float(v) for v in ev], nnz=int(A.nnz)))
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "windows.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
