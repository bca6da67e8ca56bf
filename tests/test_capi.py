"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid input before touching the device."""

import ctypes as C
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from workloads import CSR, grid_laplacian

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def native():
    from paper_2512_01257_amd import native as nat

    if not os.path.exists(nat.LIB_PATH):
        subprocess.run([sys.executable, os.path.join(ROOT, "paper_2512_01257_amd", "build.py")],
                       check=True)
    nat.lib()
    return nat


def _has_gpu():
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def test_every_declared_symbol_is_exported(native):
    L = native.lib()
    names = native.exported_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_params_default_and_status_strings(native):
    p = native.default_params()
    assert (p.nc, p.q, p.p, p.max_iter, p.max_cocg) == (8, 2, -1, 20, 20000)
    assert p.tol_eig == 1e-10 and p.tol_solve == 1e-6 and p.tol_solve_relaxed == 0.0
    assert p.precision == native.PRECISION["fp32"] and p.ws_op == 0 and p.rhs_form == 0
    L = native.lib()
    for code, name in native.STATUS.items():
        assert L.rafeast_status_string(code).decode() == name
    assert L.rafeast_status_string(99).decode() == "UNKNOWN"
    L.rafeast_destroy(None)  # no-op


def _plan_status(native, csr, **kw):
    args = dict(lmin=0.0, lmax=0.5, m0=8)
    args.update(kw)
    try:
        p = native.Plan(csr, **args)
        p.close()
        return "OK"
    except native.RafeastError as e:
        return e.name


def _copy(csr, **over):
    d = dict(n=csr.n, rowptr=csr.rowptr.copy(), colind=csr.colind.copy(), values=csr.values.copy())
    d.update(over)
    return CSR(**d)


def test_bad_csr_rejected(native):
    csr = grid_laplacian((6, 6), 0.01)
    rp = csr.rowptr.copy()
    rp[3], rp[4] = rp[4], rp[3]
    assert _plan_status(native, _copy(csr, rowptr=rp)) == "BAD_CSR"
    ci = csr.colind.copy()
    ci[0], ci[1] = ci[1], ci[0]
    assert _plan_status(native, _copy(csr, colind=ci)) == "BAD_CSR"
    ci = csr.colind.copy()
    ci[5] = 36
    assert _plan_status(native, _copy(csr, colind=ci)) == "BAD_CSR"
    v = csr.values.copy()
    v[7] = np.nan
    assert _plan_status(native, _copy(csr, values=v)) == "BAD_CSR"
    rp = csr.rowptr.copy()
    rp[0] = 1
    assert _plan_status(native, _copy(csr, rowptr=rp)) == "BAD_CSR"


def test_nonsymmetric_rejected(native):
    csr = grid_laplacian((6, 6), 0.01)
    v = csr.values.copy()
    v[1] += 1e-6  # an off-diagonal entry of row 0
    assert _plan_status(native, _copy(csr, values=v)) == "NOT_SYMMETRIC"
    # lower triangle only: pattern not symmetric
    import scipy.sparse as sp

    from workloads import csr_from_scipy

    low = csr_from_scipy(sp.tril(csr.to_scipy()))
    assert _plan_status(native, low) == "NOT_SYMMETRIC"


def test_invalid_params_rejected(native):
    csr = grid_laplacian((6, 6), 0.01)
    assert _plan_status(native, csr, lmin=0.5, lmax=0.5) == "INVALID_ARG"
    assert _plan_status(native, csr, lmin=math.nan) == "INVALID_ARG"
    assert _plan_status(native, csr, m0=0) == "INVALID_ARG"
    assert _plan_status(native, csr, m0=37) == "INVALID_ARG"
    assert _plan_status(native, csr, nc=0) == "INVALID_ARG"
    assert _plan_status(native, csr, nc=65) == "INVALID_ARG"
    assert _plan_status(native, csr, p=3) == "INVALID_ARG"
    assert _plan_status(native, csr, q=-1) == "INVALID_ARG"
    assert _plan_status(native, csr, tol_eig=0.0) == "INVALID_ARG"
    assert _plan_status(native, csr, tol_solve=1.0) == "INVALID_ARG"
    assert _plan_status(native, csr, tol_solve_relaxed=-1e-3) == "INVALID_ARG"
    assert _plan_status(native, csr, tol_solve_relaxed=1.0) == "INVALID_ARG"
    assert _plan_status(native, csr, tol_solve_relaxed=math.nan) == "INVALID_ARG"


def test_precond_validated_before_the_device(native):
    import ctypes as C

    csr = grid_laplacian((6, 6), 0.01)
    L = native.lib()
    A, keep = native._csr_struct(csr)
    prm = native._params(0.0, 0.5, 8, 4, 1, -1, 1e-10, 1e-6, 20, 20000, "fp32", "auto",
                         "residual", "auto", 0, None)
    prm.precond = 2
    h = C.c_void_p()
    assert L.rafeast_plan(C.byref(A), C.byref(prm), C.byref(h)) == 1
    assert b"precond" in L.rafeast_last_error(None)
    # dense plans and the batching form refuse the learned preconditioner
    prm.precond = native.PRECOND["learned"]
    prm.m0 = 2
    K = np.eye(4) * 2.0
    assert native.STATUS[L.rafeast_plan_dense(4, K.ctypes.data_as(C.POINTER(C.c_double)), 4,
                                              C.byref(prm), C.byref(h))] == "UNSUPPORTED"
    prm.m0 = 8
    As = (native.Csr * 1)(A)
    assert native.STATUS[L.rafeast_plan_batch(1, As, (native.Params * 1)(prm),
                                              C.byref(h))] == "UNSUPPORTED"
    assert b"precond" in L.rafeast_batch_last_error(None)
    # step-level learned calls refuse null plans and buffers
    assert L.rafeast_pc_harvest(None, 0, None, None, None, None, None, None) == 1
    assert L.rafeast_pc_attach(None, None) == 1


def test_dense_plans_validated_before_the_device(native):
    import ctypes as C

    L = native.lib()
    prm = native.default_params()
    prm.lmin, prm.lmax, prm.m0 = 0.5, 2.0, 2
    h = C.c_void_p()

    def dense(K, ld=None, **over):
        for k, v in over.items():
            setattr(prm, k, v)
        K = np.asfortranarray(K, dtype=np.float64)
        st = L.rafeast_plan_dense(K.shape[0], native._dptr(K), ld or K.shape[0], C.byref(prm),
                                  C.byref(h))
        prm.engine = 0
        return native.STATUS[st]

    def gram(X, scale=0.5, ld=None):
        X = np.asfortranarray(X, dtype=np.float64)
        st = L.rafeast_plan_gram(X.shape[0], X.shape[1], native._dptr(X), ld or X.shape[0],
                                 scale, C.byref(prm), C.byref(h))
        return native.STATUS[st]

    K = np.eye(5)
    K[0, 3] = 1e-3
    assert dense(K) == "NOT_SYMMETRIC"
    K[3, 0] = 1e-3
    assert dense(K, ld=4) == "INVALID_ARG"
    assert dense(K, engine=native.ENGINE["resident"]) == "UNSUPPORTED"
    K[1, 1] = np.inf
    assert dense(K) == "BAD_CSR"
    assert L.rafeast_plan_dense(5, None, 5, C.byref(prm), C.byref(h)) == 1
    X = np.arange(12.0).reshape(3, 4)
    assert gram(np.zeros((3, 4))) == "INVALID_ARG"
    assert gram(X, scale=0.0) == "INVALID_ARG"
    assert gram(X, ld=2) == "INVALID_ARG"
    X[1, 2] = np.nan
    assert gram(X) == "BAD_CSR"
    if not _has_gpu():
        assert gram(np.arange(12.0).reshape(3, 4)) == "DEVICE"


def test_oversized_subspace_unsupported(native):
    csr = grid_laplacian((20, 20), 0.01)
    assert _plan_status(native, csr, m0=180, p=20) == "UNSUPPORTED"


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_valid_input_without_device(native):
    csr = grid_laplacian((6, 6), 0.01)
    assert _plan_status(native, csr) == "DEVICE"
    # one-based input passes validation as well
    one = _copy(csr, rowptr=csr.rowptr + 1, colind=csr.colind + 1)
    L = native.lib()
    A = native.Csr(one.n, one.rowptr.ctypes.data_as(C.POINTER(C.c_int32)),
                   one.colind.ctypes.data_as(C.POINTER(C.c_int32)),
                   one.values.ctypes.data_as(C.POINTER(C.c_double)), 1)
    prm = native.default_params()
    prm.lmin, prm.lmax, prm.m0 = 0.0, 0.5, 8
    h = C.c_void_p()
    assert L.rafeast_plan(C.byref(A), C.byref(prm), C.byref(h)) == 5
    assert h.value is None
    assert b"device" in L.rafeast_last_error(None)


def test_batch_argument_errors(native):
    L = native.lib()
    assert L.rafeast_batch_plan(None, 0) is None
    assert L.rafeast_batch_resident_count(None) == 0
    L.rafeast_batch_destroy(None)  # no-op
    csr = grid_laplacian((6, 6), 0.01)
    A, keep = native._csr_struct(csr)
    As = (native.Csr * 2)(A, A)
    p0 = native._params(0.0, 0.5, 8, 4, 1, -1, 1e-10, 1e-6, 20, 20000, "fp32", "auto",
                        "residual", "auto", 0, None)
    p1 = native._params(0.0, 0.5, 8, 4, 1, -1, 1e-10, 1e-6, 20, 20000, "fp64", "auto",
                        "residual", "auto", 0, None)
    h = C.c_void_p()
    # members must share the precision (checked before any device call)
    assert L.rafeast_plan_batch(2, As, (native.Params * 2)(p0, p1), C.byref(h)) == 1
    assert h.value is None
    assert b"precision" in L.rafeast_batch_last_error(None)
    assert L.rafeast_plan_batch(0, As, (native.Params * 2)(p0, p0), C.byref(h)) == 1
    if not _has_gpu():
        assert L.rafeast_plan_batch(2, As, (native.Params * 2)(p0, p0), C.byref(h)) == 5


def test_plan_tuning_argument_errors(native):
    L = native.lib()
    ch, cnt = C.c_int32(), C.c_int32()
    cand = (C.c_int32 * 4)()
    ms = (C.c_float * 4)()
    assert L.rafeast_plan_tuning(None, C.byref(ch), C.byref(cnt), cand, ms, 4) == 1


def test_bench_refuses_more_than_one_gpu():
    # this build runs on one GPU: --gpus N > 1 (or a WORLD_SIZE > 1) exits with
    # a message before touching a device
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
    env = dict(os.environ, WORLD_SIZE="4")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True,
                       text=True, timeout=120, env=env)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_gemm_arguments_checked_before_the_device(native):
    L = native.lib()
    p = C.c_void_p(16)  # never dereferenced: every call fails its checks first
    # short leading dimension of B, unknown precision, bad a_cols, null A,
    # negative size, short lda for a column-stored A
    assert L.rafeast_gemm(None, 0, 0, 4, 4, 4, p, 4, p, 3, p, 4, 1.0, 0.0) == 1
    assert L.rafeast_gemm(None, 7, 0, 4, 4, 4, p, 4, p, 4, p, 4, 1.0, 0.0) == 1
    assert L.rafeast_gemm(None, 0, 2, 4, 4, 4, p, 4, p, 4, p, 4, 1.0, 0.0) == 1
    assert L.rafeast_gemm(None, 0, 0, 4, 4, 4, None, 4, p, 4, p, 4, 1.0, 0.0) == 1
    assert L.rafeast_gemm(None, 0, 0, -1, 4, 4, p, 4, p, 4, p, 4, 1.0, 0.0) == 1
    assert L.rafeast_gemm(None, 1, 1, 8, 4, 4, p, 4, p, 4, p, 4, 1.0, 0.0) == 1
    assert "rafeast_gemm" in L.rafeast_last_error(None).decode()


def test_direct_engine_validated_before_the_device(native):
    # the direct engine: FP64 only, CSR plans only, no preconditioner, not in
    # the batching form; all refused before any device call
    L = native.lib()
    csr = grid_laplacian((6, 6), 0.01)
    A, keep = native._csr_struct(csr)
    h = C.c_void_p()
    p32 = native._params(0.0, 0.5, 8, 4, 1, -1, 1e-10, 1e-6, 20, 20000, "fp32", "auto",
                         "residual", "direct", 0, None)
    assert L.rafeast_plan(C.byref(A), C.byref(p32), C.byref(h)) == 1
    assert b"direct engine runs in FP64" in L.rafeast_last_error(None)
    p64 = native._params(0.0, 0.5, 8, 4, 1, -1, 1e-10, 1e-6, 20, 20000, "fp64", "auto",
                         "residual", "direct", 0, None)
    p64.precond = native.PRECOND["learned"]
    assert native.STATUS[L.rafeast_plan(C.byref(A), C.byref(p64), C.byref(h))] == "UNSUPPORTED"
    p64.precond = native.PRECOND["none"]
    p64.m0 = 2
    K = np.eye(4) * 2.0
    assert native.STATUS[L.rafeast_plan_dense(4, K.ctypes.data_as(C.POINTER(C.c_double)), 4,
                                              C.byref(p64), C.byref(h))] == "UNSUPPORTED"
    p64.m0 = 8
    As = (native.Csr * 1)(A)
    assert native.STATUS[L.rafeast_plan_batch(1, As, (native.Params * 1)(p64),
                                              C.byref(h))] == "UNSUPPORTED"
    assert b"direct" in L.rafeast_batch_last_error(None)
    p64.engine = 5
    assert L.rafeast_plan(C.byref(A), C.byref(p64), C.byref(h)) == 1
