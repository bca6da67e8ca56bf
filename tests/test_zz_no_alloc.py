"""The allocation-free Gram entry point (rafeast_gram_noalloc) against the
plan's Gram (rafeast_gram), through the C ABI."""

import ctypes as C

import pytest

from workloads import grid_laplacian


def test_gram_noalloc_rejects_oversized_tiles_on_host():
    # validated before any HIP call: k1 * k2 = 2^21 + 1450 doubles exceeds the
    # fixed scratch (and null pointers are refused first)
    from paper_2512_01257_amd import native

    L = native.lib()
    fake = C.c_void_p(256)
    s = L.rafeast_gram_noalloc(None, 1000, 1450, 1447, fake, 1450, fake, 1447, fake, 1447)
    assert native.STATUS[s] == "INVALID_ARG"
    assert "exceeds the scratch" in L.rafeast_last_error(None).decode()
    s = L.rafeast_gram_noalloc(None, 1000, 4, 4, None, 4, fake, 4, fake, 4)
    assert native.STATUS[s] == "INVALID_ARG"
    s = L.rafeast_gram_noalloc(None, 0, 4, 4, fake, 4, fake, 4, fake, 4)
    assert native.STATUS[s] == "INVALID_ARG"


@pytest.mark.gpu
def test_gram_noalloc_matches_plan_gram(gpu_lib):
    import torch

    native = gpu_lib
    torch.cuda.set_device(0)
    csr = grid_laplacian((10, 10), 0.01)
    # one non-null stream for the inputs, the plan and the entry point, so
    # the products are ordered after the generation of their operands (with
    # the null stream the plan would run on a stream of its own)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st), native.Plan(csr, 0.0, 0.5, 4, nc=2, q=0, p=4, engine="stream",
                                            stream=st.cuda_stream) as plan:
        g = torch.Generator(device="cuda").manual_seed(7)
        # two calls in a row, the second smaller; the first large enough that
        # the scratch holds fewer row chunks than the plan's Gram uses (256 x
        # 160 x 144 doubles > 2^21), so its sums are split differently
        for n, k1, k2, same_chunks in ((400_000, 160, 144, False), (3_001, 37, 21, True)):
            X = torch.randn((n, k1), dtype=torch.float64, device="cuda", generator=g)
            Y = torch.randn((n, k2), dtype=torch.float64, device="cuda", generator=g)
            G_ref = torch.empty((k1, k2), dtype=torch.float64, device="cuda")
            plan.gram(X, Y, G_ref)
            G = torch.full((k1, k2), float("nan"), dtype=torch.float64, device="cuda")
            native.gram_noalloc(X, Y, G, stream=st)
            torch.cuda.synchronize()
            assert torch.isfinite(G).all()
            if same_chunks:
                assert torch.equal(G, G_ref)
            else:
                # both are sums of the same n products in different orders:
                # |G - G_ref| <= 2 n u (|X|^T |Y|)
                bound = 2.0 * n * 2.0 ** -53 * (X.abs().T @ Y.abs())
                assert bool(((G - G_ref).abs() <= bound).all())
            # and the product itself, in float64 on the GPU by torch
            ref = X.T @ Y
            bound = 2.0 * n * 2.0 ** -53 * (X.abs().T @ Y.abs())
            assert bool(((G - ref).abs() <= 2.0 * bound).all())
            del X, Y
