"""Matrix and random-draw generators (inputs only, no eigensolver arithmetic)."""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree


@dataclass
class CSR:
    """A square symmetric matrix in CSR form, zero-based, sorted unique columns."""

    n: int
    rowptr: np.ndarray  # int32 [n+1]
    colind: np.ndarray  # int32 [nnz]
    values: np.ndarray  # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.values, self.colind, self.rowptr), shape=(self.n, self.n))


def csr_from_scipy(A) -> CSR:
    """Canonical CSR (sorted, duplicate-free, explicit zeros removed)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return CSR(
        n=A.shape[0],
        rowptr=np.ascontiguousarray(A.indptr, dtype=np.int32),
        colind=np.ascontiguousarray(A.indices, dtype=np.int32),
        values=np.ascontiguousarray(A.data, dtype=np.float64),
    )


def _path_laplacian(m: int) -> sp.csr_matrix:
    """Dirichlet second-difference matrix tridiag(-1, 2, -1) of order m."""
    e = np.ones(m)
    return sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1], format="csr")


def grid_laplacian(dims, shift: float = 0.0) -> CSR:
    """Dirichlet grid Laplacian on a lexicographically ordered box grid.

    ``dims=(40, 40)`` gives the 5-point operator (diagonal 4, off-diagonal -1);
    ``dims=(64, 64, 64)`` the 7-point operator (diagonal 6).  The first index
    varies slowest.  ``shift`` is added to the diagonal.
    """
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    A = sp.csr_matrix((n, n))
    for axis, m in enumerate(dims):
        left = int(np.prod(dims[:axis])) if axis > 0 else 1
        right = int(np.prod(dims[axis + 1:])) if axis + 1 < len(dims) else 1
        A = A + sp.kron(sp.kron(sp.identity(left), _path_laplacian(m)), sp.identity(right))
    A = A + shift * sp.identity(n)
    return csr_from_scipy(A)


def _uniform_points(n: int, dim: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random((n, dim))


def knn_laplacian(n: int, dim: int, k: int, seed: int, weighted: bool = True,
                  shift: float = 0.0) -> CSR:
    """Union-symmetrised k-nearest-neighbour graph Laplacian L = D - W + shift*I.

    Points are uniform in [0,1)^dim (numpy PCG64 stream ``seed``).  Neighbours
    are exact (k-d tree), self excluded.  Weighted: w_ij = exp(-d_ij^2/sigma^2)
    with sigma the median of all n*k neighbour distances; unweighted: w_ij = 1.
    An edge exists if either endpoint lists the other.
    """
    pts = _uniform_points(n, dim, seed)
    tree = cKDTree(pts)
    dist, idx = tree.query(pts, k=k + 1)
    dist, idx = dist[:, 1:], idx[:, 1:]
    rows = np.repeat(np.arange(n), k)
    cols = idx.reshape(-1)
    d = dist.reshape(-1)
    if weighted:
        sigma = float(np.median(d))
        w = np.exp(-(d * d) / (sigma * sigma))
    else:
        w = np.ones_like(d)
    W = sp.csr_matrix((w, (rows, cols)), shape=(n, n))
    W.sum_duplicates()
    W = W.maximum(W.T)  # union symmetrisation (weights are symmetric in d)
    deg = np.asarray(W.sum(axis=1)).ravel()
    L = sp.diags(deg + shift) - W
    return csr_from_scipy(L)


def rgg_laplacian(n: int, seed: int, radius_factor: float = 1.5) -> CSR:
    """Random geometric graph Laplacian L = D - A (Section 5.1).

    n points uniform in the unit square, edges between pairs closer than
    r = radius_factor * sqrt(ln n / n) (natural log), unweighted.
    """
    pts = _uniform_points(n, 2, seed)
    r = radius_factor * math.sqrt(math.log(n) / n)
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    W = sp.csr_matrix((np.ones(len(i)), (i, j)), shape=(n, n))
    W = W + W.T
    deg = np.asarray(W.sum(axis=1)).ravel()
    return csr_from_scipy(sp.diags(deg) - W)


def random_symmetric(n: int, seed: int, density: float = 0.05, shift: float = 0.0) -> CSR:
    """Small random sparse symmetric matrix (diagonally dominant), for edge cases."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, data_rvs=rng.standard_normal)
    M = M + M.T
    off = np.asarray(abs(M).sum(axis=1)).ravel()
    return csr_from_scipy(M + sp.diags(off + shift + rng.random(n)))


def gaussian(n: int, w: int, seed: int) -> np.ndarray:
    """Standard-normal n x w sketch, column-major (Fortran order), float64."""
    g = np.random.default_rng(seed).standard_normal((w, n))
    return np.asfortranarray(g.T)


def batch_graph_specs(count: int = 32, seed_base: int = 100):
    """Specs of the many-small-graphs workload.

    Graph g: dimension 2 if g is even else 3; k = (8, 12, 16)[g % 3];
    n_g = round(exp(U[ln 2000, ln 60000])) from stream ``seed_base + g``;
    target count ~ U{10..40} from stream ``200 + g``.  Unweighted kNN
    Laplacians, no shift.
    """
    specs = []
    for g in range(count):
        rng = np.random.default_rng(seed_base + g)
        n_g = int(round(math.exp(rng.uniform(math.log(2000), math.log(60000)))))
        cnt = int(np.random.default_rng(200 + g).integers(10, 41))
        specs.append(dict(g=g, n=n_g, dim=2 if g % 2 == 0 else 3, k=(8, 12, 16)[g % 3],
                          seed=seed_base + g, count=cnt))
    return specs
