"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module builds matrices and random draws only; it holds none of the
eigensolver's arithmetic.  Every generator is deterministic in its seed.

Workload families (all sparse symmetric graph Laplacians, the problem class of
the paper's experiments, Section 5.1):

* ``grid_laplacian``  Dirichlet 5-point (2D) / 7-point (3D) grid Laplacian plus
  a diagonal shift.
* ``knn_laplacian``   k-nearest-neighbour graph on uniform points, union
  symmetrised, Gaussian weights exp(-d^2/sigma^2) with sigma the median kNN
  distance (or unweighted), plus a diagonal shift.
* ``rgg_laplacian``   random geometric graph in the unit square with radius
  1.5*sqrt(log n / n), unweighted L = D - A (Section 5.1).
* ``gaussian``        the n x w standard-normal sketch used by the randomized
  warmstart (Algorithm 2, Phase 1); drawn here and passed to both the oracle
  and the GPU library so that both sides start from the same numbers.
"""

from .graphs import (  # noqa: F401
    CSR,
    csr_from_scipy,
    grid_laplacian,
    knn_laplacian,
    rgg_laplacian,
    random_symmetric,
    gaussian,
    batch_graph_specs,
)
