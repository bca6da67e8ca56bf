"""Host-side reverse Cuthill-McKee order used by the streaming COCG engine
(exported as rafeast_rcm_order; runs without a device)."""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, reverse_cuthill_mckee

from workloads import csr_from_scipy, grid_laplacian, knn_laplacian


@pytest.fixture(scope="module")
def native():
    from paper_2512_01257_amd import native as nat

    return nat


def _bandwidth(A, perm):
    B = A[perm][:, perm].tocoo()
    return int(np.abs(B.row - B.col).max()) if B.nnz else 0


def _shuffled(A, seed):
    p = np.random.default_rng(seed).permutation(A.shape[0])
    return A[p][:, p].tocsr()


def _check_perm(perm, n):
    assert perm.dtype == np.int32 and perm.shape == (n,)
    assert np.array_equal(np.sort(perm), np.arange(n))


def test_path_graph_gets_bandwidth_one(native):
    n = 500
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    A = _shuffled(A, 3)
    perm = native.rcm_order(csr_from_scipy(A))
    _check_perm(perm, n)
    assert _bandwidth(A, perm) == 1  # a path traversed from an end


def test_grid_and_knn_bandwidth_against_scipy(native):
    for A in (grid_laplacian((30, 20), 0.0).to_scipy().tocsr(),
              knn_laplacian(3000, 2, 8, seed=4).to_scipy().tocsr()):
        A = _shuffled(A, 7)
        perm = native.rcm_order(csr_from_scipy(A))
        _check_perm(perm, A.shape[0])
        ref = reverse_cuthill_mckee(A, symmetric_mode=True)
        bw, bw_ref = _bandwidth(A, perm), _bandwidth(A, ref)
        assert bw <= 1.25 * bw_ref + 2, (bw, bw_ref)
        assert bw < _bandwidth(A, np.arange(A.shape[0])) / 5


def test_components_are_contiguous(native):
    g1 = grid_laplacian((7, 5), 0.0).to_scipy()
    g2 = grid_laplacian((4, 4, 3), 0.0).to_scipy()
    iso = sp.identity(3)  # three isolated vertices (diagonal only)
    A = _shuffled(sp.block_diag([g1, iso, g2]).tocsr(), 11)
    perm = native.rcm_order(csr_from_scipy(A))
    _check_perm(perm, A.shape[0])
    _, lab = connected_components(A, directed=False)
    seq = lab[perm]
    # each label appears in one run
    runs = 1 + np.count_nonzero(seq[1:] != seq[:-1])
    assert runs == len(np.unique(lab))


def test_invalid_input_rejected(native):
    A = grid_laplacian((5, 5), 0.0)
    bad = type(A)(n=A.n, rowptr=A.rowptr.copy(), colind=A.colind.copy(), values=A.values.copy())
    bad.colind[0], bad.colind[1] = bad.colind[1], bad.colind[0]
    with pytest.raises(native.RafeastError) as e:
        native.rcm_order(bad)
    assert e.value.name == "BAD_CSR"
