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
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "windows.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
