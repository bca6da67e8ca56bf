"""Closed-form spectra of Dirichlet grid Laplacians (test pins).

The Dirichlet second-difference matrix tridiag(-1, 2, -1) of order m has
eigenvalues 2 - 2 cos(pi k / (m + 1)) and eigenvectors sin(pi k i / (m + 1)),
k, i = 1..m.  The d-dimensional grid Laplacian is a Kronecker sum, so its
eigenvalues are sums over axes and its eigenvectors tensor products.
"""

import itertools

import numpy as np


def path_eigs(m):
    k = np.arange(1, m + 1)
    return 2.0 - 2.0 * np.cos(np.pi * k / (m + 1))


def grid_eigs(dims, shift=0.0):
    """All eigenvalues (ascending) with their mode tuples."""
    per = [path_eigs(m) for m in dims]
    modes = list(itertools.product(*[range(1, m + 1) for m in dims]))
    vals = np.array([sum(per[a][k[a] - 1] for a in range(len(dims))) for k in modes]) + shift
    order = np.argsort(vals, kind="stable")
    return vals[order], [modes[i] for i in order]


def grid_eigvec(dims, mode):
    """Unit eigenvector for a mode tuple, lexicographic order (first index slowest)."""
    v = np.ones(1)
    for m, k in zip(dims, mode):
        i = np.arange(1, m + 1)
        v = np.kron(v, np.sin(np.pi * k * i / (m + 1)))
    return v / np.linalg.norm(v)


def window_basis(dims, shift, lmin, lmax):
    vals, modes = grid_eigs(dims, shift)
    sel = [(v, md) for v, md in zip(vals, modes) if lmin <= v <= lmax]
    V = np.stack([grid_eigvec(dims, md) for _, md in sel], axis=1)
    return np.array([v for v, _ in sel]), V
