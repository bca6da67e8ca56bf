"""GPU parity of the matrix-core GEMM behind the dense operators of the
statistical workloads (Section 4: K X for the kernel matrix, Xd^T (Xd X) for
the sample covariance) through rafeast_gemm, against float64 host products.

Bound: every entry is an inner product of length K plus the alpha/beta
update, so |C - C_exact| <= (K + 2) u (|alpha| |op(A)| |B| + |beta| |C0|)
(u = 2^-53 in FP64; in FP32, u = 2^-24 against the exact product of the
float32 inputs), for any order of the sums (the chunked inner dimension
included)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (M, N, K): one partial tile; ragged tiles on every side; a long inner
# dimension with few output tiles (split into chunks); tiles cut by M and N
# (multiples of the vector width) over whole inner steps, the fast path with
# its edge reads redirected; a narrow product (32-column blocks, split); a
# single element; an empty inner dimension
SHAPES = [(100, 60, 40), (257, 131, 333), (200, 70, 4099), (196, 100, 2048), (300, 24, 1536),
          (1, 1, 1), (65, 33, 0)]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("a_cols", [False, True])
@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_matches_host(gpu_lib, dtype, a_cols, shape):
    import torch

    M, N, K = shape
    rng = np.random.default_rng(M * 1000 + N + K)
    npdt = np.float64 if dtype == "float64" else np.float32
    A = rng.standard_normal((K, M) if a_cols else (M, K)).astype(npdt)
    B = rng.standard_normal((K, N)).astype(npdt)
    C0 = rng.standard_normal((M, N)).astype(npdt)
    alpha, beta = 0.75, -1.25
    tdt = getattr(torch, dtype)
    Cd = torch.tensor(C0, device="cuda")
    gpu_lib.gemm(torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda"), Cd,
                 alpha=alpha, beta=beta, a_cols=a_cols)
    got = Cd.cpu().numpy().astype(np.float64)
    opA = (A.T if a_cols else A).astype(np.float64)
    B64, C64 = B.astype(np.float64), C0.astype(np.float64)
    want = alpha * (opA @ B64) + beta * C64
    u = 2.0 ** -53 if dtype == "float64" else 2.0 ** -24
    bound = (K + 2) * u * (abs(alpha) * (np.abs(opA) @ np.abs(B64)) + abs(beta) * np.abs(C64))
    assert Cd.dtype == tdt
    assert np.all(np.abs(got - want) <= bound + 1e-300), np.abs(got - want).max()


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_gemm_beta_zero_ignores_c(gpu_lib, dtype):
    import torch

    rng = np.random.default_rng(5)
    tdt = getattr(torch, dtype)
    A = torch.tensor(rng.standard_normal((150, 1100)), dtype=tdt, device="cuda")
    B = torch.tensor(rng.standard_normal((1100, 20)), dtype=tdt, device="cuda")
    Cd = torch.full((150, 20), float("nan"), dtype=tdt, device="cuda")
    gpu_lib.gemm(A, B, Cd, alpha=2.0, beta=0.0)
    got = Cd.cpu().numpy().astype(np.float64)
    assert np.isfinite(got).all()
    want = 2.0 * (A.cpu().double().numpy() @ B.cpu().double().numpy())
    u = 2.0 ** -53 if dtype == "float64" else 2.0 ** -24
    Ah, Bh = A.cpu().double().numpy(), B.cpu().double().numpy()
    assert np.all(np.abs(got - want) <= 1102 * u * 2.0 * (np.abs(Ah) @ np.abs(Bh)))
