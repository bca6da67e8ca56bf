"""ctypes binding of librafeast.so (include/rafeast.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Importing this module does not touch the GPU; the library is loaded
on first use and a missing library raises immediately (there is no fallback).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RAFEAST_LIB selects another build of the library (the sanitizer build of
# the CPU tests); by default the in-tree one
LIB_PATH = os.environ.get("RAFEAST_LIB") or os.path.join(_HERE, "librafeast.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "rafeast.h")

STATUS = {
    0: "OK", 1: "INVALID_ARG", 2: "BAD_CSR", 3: "NOT_SYMMETRIC", 4: "OOM", 5: "DEVICE",
    6: "NO_CONVERGENCE", 7: "SUBSPACE_TOO_SMALL", 8: "BREAKDOWN", 9: "EMPTY_WINDOW",
    10: "UNSUPPORTED",
}
# statuses that still come with results
RESULT_STATUSES = {0, 6, 7, 8, 9}

PRECISION = {"fp64": 0, "fp32": 1}
WS_OP = {"auto": 0, "literal": 1, "flip": 2, "fold": 3, "none": 4}
RHS_FORM = {"residual": 0, "literal": 1}
ENGINE = {"auto": 0, "resident": 1, "stream": 2, "multishift": 3, "direct": 4}
PRECOND = {"none": 0, "learned": 1}
NPHASE = 5
PHASES = ("rr", "solve", "combine", "orth", "total")


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("rowptr", C.POINTER(C.c_int32)),
                ("colind", C.POINTER(C.c_int32)), ("values", C.POINTER(C.c_double)),
                ("index_base", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("lmin", C.c_double), ("lmax", C.c_double), ("m0", C.c_int32),
                ("nc", C.c_int32), ("q", C.c_int32), ("p", C.c_int32),
                ("tol_eig", C.c_double), ("tol_solve", C.c_double), ("max_iter", C.c_int32),
                ("max_cocg", C.c_int32), ("precision", C.c_int32), ("ws_op", C.c_int32),
                ("rhs_form", C.c_int32), ("engine", C.c_int32), ("seed", C.c_uint64),
                ("hip_stream", C.c_void_p), ("tol_solve_relaxed", C.c_double),
                ("precond", C.c_int32)]


class WsInfo(C.Structure):
    _fields_ = [("beta_m0", C.c_double), ("beta_m0p1", C.c_double), ("ratio", C.c_double),
                ("op", C.c_int32), ("t_ms", C.c_double), ("r_halko", C.c_double),
                ("gap", C.c_double), ("proj_bound", C.c_double)]


class Result(C.Structure):
    _fields_ = [("flags", C.c_int32), ("lam", C.c_void_p), ("resid", C.c_void_p),
                ("X", C.c_void_p), ("M", C.c_int32), ("iters", C.c_int32),
                ("cocg_iters", C.c_int64), ("cocg_max", C.c_int32), ("refinements", C.c_int32),
                ("max_resid", C.c_double), ("t_ms", C.c_double * NPHASE),
                ("tol_solve_last", C.c_double), ("cocg_node", C.c_int64 * 64),
                ("pc_fallbacks", C.c_int32)]


_lib = None


class RafeastError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {msg}")


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with __graft_entry__.build()")
    # torch ships its own HIP runtime: load it first so that the library binds
    # to the same one (a second runtime in the process sees no device)
    import torch  # noqa: F401

    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    L.rafeast_params_default.argtypes = [C.POINTER(Params)]
    L.rafeast_params_default.restype = None
    L.rafeast_plan.argtypes = [C.POINTER(Csr), C.POINTER(Params), C.POINTER(P)]
    L.rafeast_plan.restype = C.c_int
    L.rafeast_plan_dense.argtypes = [C.c_int64, dp, C.c_int64, C.POINTER(Params), C.POINTER(P)]
    L.rafeast_plan_dense.restype = C.c_int
    L.rafeast_plan_gram.argtypes = [C.c_int64, C.c_int64, dp, C.c_int64, C.c_double,
                                    C.POINTER(Params), C.POINTER(P)]
    L.rafeast_plan_gram.restype = C.c_int
    L.rafeast_warmstart.argtypes = [P, dp, dp, C.POINTER(WsInfo)]
    L.rafeast_warmstart.restype = C.c_int
    L.rafeast_solve.argtypes = [P, dp, C.POINTER(Result)]
    L.rafeast_solve.restype = C.c_int
    L.rafeast_destroy.argtypes = [P]
    L.rafeast_destroy.restype = None
    L.rafeast_last_error.argtypes = [P]
    L.rafeast_last_error.restype = C.c_char_p
    L.rafeast_status_string.argtypes = [C.c_int]
    L.rafeast_status_string.restype = C.c_char_p
    L.rafeast_plan_info.argtypes = [P, dp, dp, dp, C.POINTER(C.c_int64), dp, dp]
    L.rafeast_plan_info.restype = C.c_int
    L.rafeast_plan_engine.argtypes = [P]
    L.rafeast_plan_engine.restype = C.c_int32
    L.rafeast_plan_tuning.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_float), C.c_int32]
    L.rafeast_plan_tuning.restype = C.c_int
    L.rafeast_rcm_order.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32)]
    L.rafeast_rcm_order.restype = C.c_int
    L.rafeast_pc_param_count.argtypes = []
    L.rafeast_pc_param_count.restype = C.c_int32
    L.rafeast_pc_samples.argtypes = [P, C.c_int32, dp, C.c_int32, P, C.c_int32, C.c_double,
                                     C.c_double, P, P, P, P]
    L.rafeast_pc_samples.restype = C.c_int
    L.rafeast_pc_forward.argtypes = [P, C.c_int32, P, P, P]
    L.rafeast_pc_forward.restype = C.c_int
    L.rafeast_pc_gradient.argtypes = [P, C.c_int32, P, P, P, P, P, P, dp]
    L.rafeast_pc_gradient.restype = C.c_int
    L.rafeast_pc_train.argtypes = [P, C.c_int32, P, P, P, P, P, C.c_int32, C.c_int32,
                                   C.POINTER(C.c_int32), C.c_float, dp]
    L.rafeast_pc_train.restype = C.c_int
    L.rafeast_pc_solve.argtypes = [P, C.c_int32, dp, C.c_int32, P, C.c_int32, dp, P, C.c_double,
                                   C.POINTER(C.c_int32), dp]
    L.rafeast_pc_solve.restype = C.c_int
    L.rafeast_pc_harvest.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), P, P, P, P,
                                     C.POINTER(C.c_int32)]
    L.rafeast_pc_harvest.restype = C.c_int
    L.rafeast_pc_attach.argtypes = [P, P]
    L.rafeast_pc_attach.restype = C.c_int
    L.rafeast_pc_normalize.argtypes = [P, C.c_int32, P, P]
    L.rafeast_pc_normalize.restype = C.c_int
    L.rafeast_plan_batch.argtypes = [C.c_int32, C.POINTER(Csr), C.POINTER(Params), C.POINTER(P)]
    L.rafeast_plan_batch.restype = C.c_int
    L.rafeast_batch_plan.argtypes = [P, C.c_int32]
    L.rafeast_batch_plan.restype = P
    L.rafeast_batch_solve.argtypes = [P, C.POINTER(dp), C.POINTER(Result), C.POINTER(C.c_int),
                                      dp]
    L.rafeast_batch_solve.restype = C.c_int
    L.rafeast_batch_resident_count.argtypes = [P]
    L.rafeast_batch_resident_count.restype = C.c_int32
    L.rafeast_batch_destroy.argtypes = [P]
    L.rafeast_batch_destroy.restype = None
    L.rafeast_batch_last_error.argtypes = [P]
    L.rafeast_batch_last_error.restype = C.c_char_p
    L.rafeast_spmm.argtypes = [P, C.c_int32, P, C.c_int32, P, C.c_int32, C.c_double, C.c_double]
    L.rafeast_spmm.restype = C.c_int
    L.rafeast_gram.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, P, C.c_int32, P, C.c_int32,
                               P, C.c_int32]
    L.rafeast_gram.restype = C.c_int
    L.rafeast_gram_noalloc.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, P, C.c_int32, P,
                                       C.c_int32, P, C.c_int32]
    L.rafeast_gram_noalloc.restype = C.c_int
    L.rafeast_gemm.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P,
                               C.c_int64, P, C.c_int64, P, C.c_int64, C.c_double, C.c_double]
    L.rafeast_gemm.restype = C.c_int
    L.rafeast_cholqr2.argtypes = [P, C.c_int64, C.c_int32, P, C.c_int32, C.POINTER(C.c_int32)]
    L.rafeast_cholqr2.restype = C.c_int
    L.rafeast_syev.argtypes = [P, C.c_int32, P, P, P]
    L.rafeast_syev.restype = C.c_int
    L.rafeast_shifted_solve.argtypes = [P, C.c_int32, dp, C.c_int32, P, C.c_int32, P, C.c_double,
                                        C.POINTER(C.c_int32), dp]
    L.rafeast_shifted_solve.restype = C.c_int
    L.rafeast_gaussian.argtypes = [P, C.c_int32, C.c_uint64, P, C.c_int32]
    L.rafeast_gaussian.restype = C.c_int
    _lib = L
    return L


def exported_symbols():
    """Names of the rafeast_* functions declared in include/rafeast.h."""
    import re

    with open(HEADER_PATH) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(rafeast_[a-z0-9_]+)\s*\(", txt)))


def kernel_source_sha(name):
    """SHA-256 of a kernel source under csrc/ (ties stored profiles to a kernel version)."""
    import hashlib

    with open(os.path.join(_HERE, "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _tptr(t, dtype=None):
    """Device pointer of a contiguous CUDA/HIP torch tensor."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def gram_noalloc(X, Y, G, stream=None, n=None, k1=None, k2=None):
    """G = X^T Y through rafeast_gram_noalloc (no plan, no device allocation),
    enqueued on `stream` (a torch stream; None: the current stream) without
    waiting.  X, Y, G: contiguous float64 device tensors (n x k1, n x k2,
    k1 x k2); n, k1, k2 override the sizes (for host-side argument checks)."""
    import torch

    st = stream if stream is not None else torch.cuda.current_stream()
    n = X.shape[0] if n is None else n
    k1 = X.shape[1] if k1 is None else k1
    k2 = Y.shape[1] if k2 is None else k2
    s = lib().rafeast_gram_noalloc(C.c_void_p(st.cuda_stream), n, k1, k2,
                                   _tptr(X, torch.float64), X.stride(0),
                                   _tptr(Y, torch.float64), Y.stride(0),
                                   _tptr(G, torch.float64), G.stride(0))
    if s != 0:
        raise RafeastError(s, lib().rafeast_last_error(None).decode())


def gemm(A, B, Cm, alpha=1.0, beta=0.0, a_cols=False, stream=None):
    """Cm = alpha op(A) B + beta Cm through rafeast_gemm.  B, Cm: contiguous
    row-major device tensors (float64 or float32, K x N and M x N); A: the
    same dtype, op(A) = A (M x K, a_cols False) or op(A) = A^T with A stored
    K x M (a_cols True: op(A)(i, k) = A[k, i])."""
    import torch

    dt = Cm.dtype
    prec = PRECISION["fp64"] if dt == torch.float64 else PRECISION["fp32"]
    M, N = Cm.shape
    K = A.shape[0] if a_cols else A.shape[1]
    st = stream if stream is not None else torch.cuda.current_stream()

    def ld(t):  # an empty tensor may report stride 0: its row length then
        return t.stride(0) if t.numel() else max(1, t.shape[1])

    s = lib().rafeast_gemm(C.c_void_p(st.cuda_stream), prec, int(bool(a_cols)), M, N, K,
                           _tptr(A, dt), ld(A), _tptr(B, dt), ld(B), _tptr(Cm, dt), ld(Cm),
                           alpha, beta)
    if s != 0:
        raise RafeastError(s, lib().rafeast_last_error(None).decode())


def rcm_order(csr):
    """Reverse Cuthill-McKee permutation (perm[new] = old) the streaming engine uses."""
    L = lib()
    rowptr = np.ascontiguousarray(csr.rowptr, dtype=np.int32)
    colind = np.ascontiguousarray(csr.colind, dtype=np.int32)
    values = np.ascontiguousarray(csr.values, dtype=np.float64)
    A = Csr(int(csr.n), rowptr.ctypes.data_as(C.POINTER(C.c_int32)),
            colind.ctypes.data_as(C.POINTER(C.c_int32)),
            values.ctypes.data_as(C.POINTER(C.c_double)), 0)
    perm = np.zeros(int(csr.n), dtype=np.int32)
    st = L.rafeast_rcm_order(C.byref(A), perm.ctypes.data_as(C.POINTER(C.c_int32)))
    if st != 0:
        raise RafeastError(st, L.rafeast_last_error(None).decode())
    return perm


def _csr_struct(csr):
    rowptr = np.ascontiguousarray(csr.rowptr, dtype=np.int32)
    colind = np.ascontiguousarray(csr.colind, dtype=np.int32)
    values = np.ascontiguousarray(csr.values, dtype=np.float64)
    A = Csr(int(csr.n), rowptr.ctypes.data_as(C.POINTER(C.c_int32)),
            colind.ctypes.data_as(C.POINTER(C.c_int32)),
            values.ctypes.data_as(C.POINTER(C.c_double)), 0)
    return A, (rowptr, colind, values)


def _params(lmin, lmax, m0, nc, q, p, tol_eig, tol_solve, max_iter, max_cocg, precision,
            ws_op, rhs_form, engine, seed, stream, tol_solve_relaxed=0.0, precond="none"):
    prm = default_params()
    prm.lmin, prm.lmax, prm.m0, prm.nc, prm.q, prm.p = lmin, lmax, m0, nc, q, p
    prm.tol_eig, prm.tol_solve, prm.max_iter, prm.max_cocg = tol_eig, tol_solve, max_iter, max_cocg
    prm.precision = PRECISION[precision]
    prm.ws_op = WS_OP[ws_op]
    prm.rhs_form = RHS_FORM[rhs_form]
    prm.engine = ENGINE[engine]
    prm.seed = seed
    prm.hip_stream = stream
    prm.tol_solve_relaxed = tol_solve_relaxed
    prm.precond = PRECOND[precond]
    return prm


def default_params() -> Params:
    p = Params()
    lib().rafeast_params_default(C.byref(p))
    return p


class Plan:
    """A planned RA-FEAST problem (rafeast_plan) on the current HIP device."""

    def __init__(self, csr, lmin, lmax, m0, nc=8, q=2, p=-1, tol_eig=1e-10, tol_solve=1e-6,
                 max_iter=20, max_cocg=20000, precision="fp32", ws_op="auto",
                 rhs_form="residual", engine="auto", seed=0, stream=None, tol_solve_relaxed=0.0,
                 precond="none"):
        L = lib()
        A, keep = _csr_struct(csr)
        prm = _params(lmin, lmax, m0, nc, q, p, tol_eig, tol_solve, max_iter, max_cocg,
                      precision, ws_op, rhs_form, engine, seed, stream, tol_solve_relaxed,
                      precond)
        h = C.c_void_p()
        st = L.rafeast_plan(C.byref(A), C.byref(prm), C.byref(h))
        if st != 0:
            raise RafeastError(st, L.rafeast_last_error(None).decode())
        self._setup(h, int(csr.n), m0, nc, lmin, lmax, precision, p, owned=True,
                    own_stream=stream is None)

    @classmethod
    def _from_dense(cls, make, n, lmin, lmax, m0, kw):
        opts = dict(_PLAN_DEFAULTS)
        opts.update(kw)
        stream = opts.pop("stream", None)
        prm = _params(lmin, lmax, m0, opts["nc"], opts["q"], opts["p"], opts["tol_eig"],
                      opts["tol_solve"], opts["max_iter"], opts["max_cocg"], opts["precision"],
                      opts["ws_op"], opts["rhs_form"], opts["engine"], opts["seed"], stream,
                      opts["tol_solve_relaxed"], opts["precond"])
        h = C.c_void_p()
        st = make(C.byref(prm), C.byref(h))
        if st != 0:
            raise RafeastError(st, lib().rafeast_last_error(None).decode())
        self = cls.__new__(cls)
        self._setup(h, int(n), m0, opts["nc"], lmin, lmax, opts["precision"], opts["p"],
                    owned=True, own_stream=stream is None)
        return self

    @classmethod
    def from_dense(cls, K, lmin, lmax, m0, **kw):
        """rafeast_plan_dense: A = K, a dense symmetric matrix (kernel PCA).
        Keyword arguments as Plan()."""
        K = np.asfortranarray(K, dtype=np.float64)
        n = K.shape[0]
        if K.shape != (n, n):
            raise ValueError("K must be square")
        return cls._from_dense(lambda prm, h: lib().rafeast_plan_dense(n, _dptr(K), n, prm, h),
                               n, lmin, lmax, m0, kw)

    @classmethod
    def from_covariance(cls, X, lmin, lmax, m0, scale=None, **kw):
        """rafeast_plan_gram: A = scale X^T X (default scale 1/(rows - 1), the
        sample covariance of the rows of X).  Keyword arguments as Plan()."""
        X = np.asfortranarray(X, dtype=np.float64)
        rows, n = X.shape
        sc = 1.0 / (rows - 1) if scale is None else float(scale)
        return cls._from_dense(
            lambda prm, h: lib().rafeast_plan_gram(rows, n, _dptr(X), rows, sc, prm, h),
            n, lmin, lmax, m0, kw)

    def _setup(self, h, n, m0, nc, lmin, lmax, precision, p, owned, own_stream=True):
        self._h = h
        self._owned = owned
        self._own_stream = own_stream
        self.n = n
        self.m0 = m0
        self.nc = nc
        self.lmin, self.lmax = lmin, lmax
        self.precision = precision
        self.w = min(m0 + (p if p >= 0 else (10 if m0 <= 50 else min(20, -(-m0 // 2)))), self.n)

    # ------------------------------------------------------------------ life
    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                lib().rafeast_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _ready(self):
        # A plan made without a stream runs on a stream of its own: device
        # tensors that torch is still writing on its current stream (a fill,
        # a copy) must be complete before the plan reads them.
        if self._own_stream:
            import torch

            torch.cuda.current_stream().synchronize()

    def _check(self, st):
        if st != 0:
            raise RafeastError(st, lib().rafeast_last_error(self._h).decode())

    @property
    def handle(self):
        return self._h

    @property
    def tuning(self):
        """rafeast_plan_tuning: the chosen resident slots per thread (0 for the
        streaming engine) and the timed candidates as (slots, ms) pairs."""
        ch, cnt = C.c_int32(), C.c_int32()
        cand = (C.c_int32 * 8)()
        ms = (C.c_float * 8)()
        self._check(lib().rafeast_plan_tuning(self._h, C.byref(ch), C.byref(cnt), cand, ms, 8))
        return dict(chosen=ch.value, candidates=[(cand[i], ms[i]) for i in range(min(cnt.value, 8))])

    @property
    def engine(self):
        """COCG engine the plan resolved: "resident" or "stream"."""
        e = lib().rafeast_plan_engine(self._h)
        return {v: k for k, v in ENGINE.items()}[e]

    # ------------------------------------------- learned preconditioner
    def pc_samples(self, z, R, theta_lo, theta_hi):
        """(X, G, h, rr) device tensors for real residuals R (device n x k FP64)."""
        self._ready()
        import torch

        z = np.asarray(z, dtype=np.complex128)
        zz = np.empty(2 * len(z))
        zz[0::2], zz[1::2] = z.real, z.imag
        k = R.shape[1]
        ns = len(z) * k
        X = torch.empty((ns, 4), dtype=torch.float64, device="cuda")
        G = torch.empty((ns, 8, 8, 2), dtype=torch.float64, device="cuda")
        h = torch.empty((ns, 8, 2), dtype=torch.float64, device="cuda")
        rr = torch.empty(ns, dtype=torch.float64, device="cuda")
        self._check(lib().rafeast_pc_samples(self._h, len(z), _dptr(zz), k,
                                             _tptr(R, torch.float64), k, theta_lo, theta_hi,
                                             _tptr(X), _tptr(G), _tptr(h), _tptr(rr)))
        return X, G, h, rr

    def pc_harvest(self, steps=(0, 32, 128)):
        """rafeast_pc_harvest: (X, G, h, rr) device tensors of the training
        samples from the COCG residuals of the plan's own shifted systems
        after each count of plain COCG iterations in steps (right-hand sides:
        the residual block of the plan's last Rayleigh-Ritz step)."""
        self._ready()
        import torch

        st = np.ascontiguousarray(steps, dtype=np.int32)
        cap = int(sum(1 if s == 0 else 2 for s in st)) * self.nc * self.m0
        X = torch.empty((cap, 4), dtype=torch.float64, device="cuda")
        G = torch.empty((cap, 8, 8, 2), dtype=torch.float64, device="cuda")
        h = torch.empty((cap, 8, 2), dtype=torch.float64, device="cuda")
        rr = torch.empty(cap, dtype=torch.float64, device="cuda")
        cnt = C.c_int32()
        self._check(lib().rafeast_pc_harvest(self._h, len(st),
                                             st.ctypes.data_as(C.POINTER(C.c_int32)), _tptr(X),
                                             _tptr(G), _tptr(h), _tptr(rr), C.byref(cnt)))
        k = cnt.value
        return X[:k], G[:k], h[:k], rr[:k]

    def pc_normalize(self, X, W):
        """rafeast_pc_normalize: W's input standardization from features X."""
        self._ready()
        import torch

        self._check(lib().rafeast_pc_normalize(self._h, X.shape[0], _tptr(X, torch.float64),
                                               _tptr(W, torch.float32)))

    def pc_attach(self, W):
        """rafeast_pc_attach: the plan copies the FP32 network parameters W."""
        self._ready()
        import torch

        self._check(lib().rafeast_pc_attach(self._h, _tptr(W, torch.float32)))

    def pc_forward(self, X, W):
        self._ready()
        import torch

        Y = torch.empty((X.shape[0], 16), dtype=torch.float32, device="cuda")
        self._check(lib().rafeast_pc_forward(self._h, X.shape[0], _tptr(X, torch.float64),
                                             _tptr(W, torch.float32), _tptr(Y)))
        return Y

    def pc_gradient(self, X, G, h, rr, W):
        self._ready()
        import torch

        g = torch.empty(lib().rafeast_pc_param_count(), dtype=torch.float32, device="cuda")
        loss = C.c_double()
        self._check(lib().rafeast_pc_gradient(self._h, X.shape[0], _tptr(X), _tptr(G), _tptr(h),
                                              _tptr(rr), _tptr(W, torch.float32), _tptr(g),
                                              C.byref(loss)))
        return g, loss.value

    def pc_train(self, X, G, h, rr, W, order, batch, lr):
        """Adam on W (device FP32, in place); order: host int32 [steps * batch]."""
        self._ready()
        import torch

        order = np.ascontiguousarray(order, dtype=np.int32)
        steps = len(order) // batch
        loss = np.zeros(steps)
        self._check(lib().rafeast_pc_train(self._h, X.shape[0], _tptr(X), _tptr(G), _tptr(h),
                                           _tptr(rr), _tptr(W, torch.float32), steps, batch,
                                           order.ctypes.data_as(C.POINTER(C.c_int32)), lr,
                                           _dptr(loss)))
        return loss

    def pc_solve(self, z, B, X, tol, coef=None):
        """Preconditioned (coef: [nz][8] complex) or plain FP64 COCG; X device
        complex128 n x (nz*k).  Returns (iters, resid)."""
        self._ready()
        import torch

        z = np.asarray(z, dtype=np.complex128)
        zz = np.empty(2 * len(z))
        zz[0::2], zz[1::2] = z.real, z.imag
        k = B.shape[1]
        cf = None
        if coef is not None:
            c = np.asarray(coef, dtype=np.complex128).reshape(len(z), 8)
            cf = np.empty(16 * len(z))
            cf[0::2], cf[1::2] = c.real.ravel(), c.imag.ravel()
        its = np.zeros(len(z) * k, dtype=np.int32)
        rs = np.zeros(len(z) * k)
        self._check(lib().rafeast_pc_solve(self._h, len(z), _dptr(zz), k, _tptr(B, torch.float64),
                                           k, _dptr(cf), _tptr(X, torch.complex128), tol,
                                           its.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(rs)))
        return its, rs

    # ----------------------------------------------------------------- calls
    def info(self):
        lo, hi, an = C.c_double(), C.c_double(), C.c_double()
        nnz = C.c_int64()
        z = np.zeros(2 * self.nc)
        w = np.zeros(2 * self.nc)
        self._check(lib().rafeast_plan_info(self._h, C.byref(lo), C.byref(hi), C.byref(an),
                                            C.byref(nnz), _dptr(z), _dptr(w)))
        return dict(sig_lo=lo.value, sig_hi=hi.value, anorm_inf=an.value, nnz=nnz.value,
                    z=z[0::2] + 1j * z[1::2], w=w[0::2] + 1j * w[1::2])

    def warmstart(self, omega=None, want_q0=False):
        om = None
        if omega is not None:
            om = np.asfortranarray(omega, dtype=np.float64)
            if om.shape != (self.n, self.w):
                raise ValueError(f"omega must be {self.n} x {self.w}")
        q0 = np.zeros((self.n, self.m0), order="F") if want_q0 else None
        inf = WsInfo()
        self._check(lib().rafeast_warmstart(self._h, _dptr(om), _dptr(q0), C.byref(inf)))
        out = dict(beta_m0=inf.beta_m0, beta_m0p1=inf.beta_m0p1, ratio=inf.ratio,
                   op={v: k for k, v in WS_OP.items()}[inf.op], t_ms=inf.t_ms,
                   r_halko=inf.r_halko, gap=inf.gap, proj_bound=inf.proj_bound)
        if want_q0:
            out["Q0"] = q0
        return out

    def solve(self, Q_init=None, want_vectors=True):
        qi = None
        if Q_init is not None:
            qi = np.asfortranarray(Q_init, dtype=np.float64)
            if qi.shape != (self.n, self.m0):
                raise ValueError("Q_init must be n x m0")
        lam = np.zeros(self.m0)
        res = np.zeros(self.m0)
        X = np.zeros((self.n, self.m0), order="F") if want_vectors else None
        r = Result()
        r.flags = 0
        r.lam = lam.ctypes.data
        r.resid = res.ctypes.data
        r.X = X.ctypes.data if X is not None else None
        st = lib().rafeast_solve(self._h, _dptr(qi), C.byref(r))
        if st not in RESULT_STATUSES:
            self._check(st)
        M = r.M
        return dict(status=STATUS[st], lam=lam[:M].copy(), resid=res[:M].copy(),
                    X=X[:, :M].copy() if X is not None else None, M=M, iters=r.iters,
                    cocg_iters=r.cocg_iters, cocg_max=r.cocg_max, refinements=r.refinements,
                    max_resid=r.max_resid, tol_solve_last=r.tol_solve_last,
                    cocg_node=list(r.cocg_node[: self.nc]), pc_fallbacks=r.pc_fallbacks,
                    t_ms={k: r.t_ms[i] for i, k in enumerate(PHASES)})

    def solve_device(self, lam, resid, X=None, Q_init=None):
        """rafeast_solve with RAFEAST_PTR_DEVICE outputs into torch tensors."""
        self._ready()
        import torch

        qi = None
        if Q_init is not None:
            qi = np.asfortranarray(Q_init, dtype=np.float64)
        r = Result()
        r.flags = 1
        r.lam = _tptr(lam, torch.float64).value
        r.resid = _tptr(resid, torch.float64).value
        r.X = _tptr(X, torch.float64).value if X is not None else None
        st = lib().rafeast_solve(self._h, _dptr(qi), C.byref(r))
        if st not in RESULT_STATUSES:
            self._check(st)
        return dict(status=STATUS[st], M=r.M, iters=r.iters, cocg_iters=r.cocg_iters,
                    cocg_max=r.cocg_max, refinements=r.refinements, max_resid=r.max_resid,
                    tol_solve_last=r.tol_solve_last,
                    cocg_node=list(r.cocg_node[: self.nc]), pc_fallbacks=r.pc_fallbacks,
                    t_ms={k: r.t_ms[i] for i, k in enumerate(PHASES)})

    # ------------------------------------------------ step-level (device) ---
    def spmm(self, X, Y, alpha=1.0, beta=0.0):
        self._ready()
        import torch

        k = X.shape[1]
        self._check(lib().rafeast_spmm(self._h, k, _tptr(X, torch.float64), X.stride(0),
                                       _tptr(Y, torch.float64), Y.stride(0), alpha, beta))

    def gram(self, X, Y, G):
        self._ready()
        import torch

        self._check(lib().rafeast_gram(self._h, X.shape[0], X.shape[1], Y.shape[1],
                                       _tptr(X, torch.float64), X.stride(0),
                                       _tptr(Y, torch.float64), Y.stride(0),
                                       _tptr(G, torch.float64), G.stride(0)))

    def cholqr2(self, Y):
        self._ready()
        import torch

        info = C.c_int32()
        self._check(lib().rafeast_cholqr2(self._h, Y.shape[0], Y.shape[1],
                                          _tptr(Y, torch.float64), Y.stride(0), C.byref(info)))
        return info.value

    def syev(self, H, theta, S):
        self._ready()
        import torch

        self._check(lib().rafeast_syev(self._h, H.shape[0], _tptr(H, torch.float64),
                                       _tptr(theta, torch.float64), _tptr(S, torch.float64)))

    def shifted_solve(self, z, B, X, tol):
        """X[:, j*k + c] = (z_j I - A)^{-1} B[:, c]; X complex64 (fp32 plan) or complex128."""
        self._ready()
        import torch

        z = np.asarray(z, dtype=np.complex128)
        zz = np.empty(2 * len(z))
        zz[0::2], zz[1::2] = z.real, z.imag
        k = B.shape[1]
        want = torch.complex64 if self.precision == "fp32" else torch.complex128
        it = (C.c_int32 * (len(z) * k))()
        rs = np.zeros(len(z) * k)
        self._check(lib().rafeast_shifted_solve(self._h, len(z), _dptr(zz), k,
                                                _tptr(B, torch.float64), B.stride(0),
                                                _tptr(X, want), tol, it, _dptr(rs)))
        return np.array(it[:], dtype=np.int64), rs

    def gaussian(self, Omega, seed):
        self._ready()
        import torch

        self._check(lib().rafeast_gaussian(self._h, Omega.shape[1], seed,
                                           _tptr(Omega, torch.float64), Omega.stride(0)))


_PLAN_DEFAULTS = dict(nc=8, q=2, p=-1, tol_eig=1e-10, tol_solve=1e-6, max_iter=20,
                      max_cocg=20000, precision="fp32", ws_op="auto", rhs_form="residual",
                      engine="auto", seed=0, tol_solve_relaxed=0.0, precond="none")


class Batch:
    """The batching form (rafeast_plan_batch): problems is a list of dicts with
    csr, lmin, lmax, m0 and any Plan keyword; common keywords apply to all."""

    def __init__(self, problems, stream=None, **common):
        L = lib()
        count = len(problems)
        As = (Csr * count)()
        prms = (Params * count)()
        self._keep = []
        self._spec = []
        for g, pr in enumerate(problems):
            kw = dict(_PLAN_DEFAULTS)
            kw.update(common)
            kw.update({k: v for k, v in pr.items() if k not in ("csr", "lmin", "lmax", "m0")})
            A, keep = _csr_struct(pr["csr"])
            self._keep.append(keep)
            As[g] = A
            prms[g] = _params(pr["lmin"], pr["lmax"], pr["m0"], kw["nc"], kw["q"], kw["p"],
                              kw["tol_eig"], kw["tol_solve"], kw["max_iter"], kw["max_cocg"],
                              kw["precision"], kw["ws_op"], kw["rhs_form"], kw["engine"],
                              kw["seed"], stream, kw["tol_solve_relaxed"])
            self._spec.append((int(pr["csr"].n), pr["m0"], kw["nc"], pr["lmin"], pr["lmax"],
                               kw["precision"], kw["p"]))
        h = C.c_void_p()
        st = L.rafeast_plan_batch(count, As, prms, C.byref(h))
        if st != 0:
            raise RafeastError(st, L.rafeast_batch_last_error(None).decode())
        self._h = h
        self.members = []
        for g in range(count):
            n, m0, nc, lmin, lmax, prec, p = self._spec[g]
            m = Plan.__new__(Plan)
            m._setup(C.c_void_p(L.rafeast_batch_plan(h, g)), n, m0, nc, lmin, lmax, prec, p,
                     owned=False)
            self.members.append(m)

    @property
    def resident_count(self):
        return lib().rafeast_batch_resident_count(self._h)

    def solve(self, Q_init=None, want_vectors=True):
        """Lock-step Phase 2 of all members: (result dicts, batch t_ms, batch status)."""
        count = len(self.members)
        outs, keep = [], []
        res = (Result * count)()
        for g, m in enumerate(self.members):
            lam = np.zeros(m.m0)
            rs = np.zeros(m.m0)
            X = np.zeros((m.n, m.m0), order="F") if want_vectors else None
            res[g].flags = 0
            res[g].lam = lam.ctypes.data
            res[g].resid = rs.ctypes.data
            res[g].X = X.ctypes.data if X is not None else None
            outs.append((lam, rs, X))
        qi = None
        if Q_init is not None:
            qi = (C.POINTER(C.c_double) * count)()
            for g, q in enumerate(Q_init):
                if q is not None:
                    a = np.asfortranarray(q, dtype=np.float64)
                    keep.append(a)
                    qi[g] = _dptr(a)
        tb = np.zeros(NPHASE)
        sts = (C.c_int * count)()
        st = lib().rafeast_batch_solve(self._h, qi, res, sts, _dptr(tb))
        if st not in RESULT_STATUSES:
            raise RafeastError(st, lib().rafeast_batch_last_error(self._h).decode())
        results = []
        for g, (lam, rs, X) in enumerate(outs):
            r = res[g]
            M = r.M
            results.append(dict(status=STATUS[sts[g]], lam=lam[:M].copy(), resid=rs[:M].copy(),
                                X=X[:, :M].copy() if X is not None else None, M=M,
                                iters=r.iters, cocg_iters=r.cocg_iters, cocg_max=r.cocg_max,
                                refinements=r.refinements, max_resid=r.max_resid,
                                tol_solve_last=r.tol_solve_last))
        return results, {k: float(tb[i]) for i, k in enumerate(PHASES)}, STATUS[st]

    def close(self):
        if getattr(self, "_h", None):
            for m in self.members:
                m._h = None
            lib().rafeast_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
