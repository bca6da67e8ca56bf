#!/usr/bin/env python
"""RA-FEAST throughput on one MI355X (eigenpairs/s at relative residual 1e-10).

Workload: union-symmetrised 10-NN graph Laplacian of 8000 uniform points in
the unit square (Gaussian weights, sigma = median kNN distance) + 1e-3 I,
window holding its 50 smallest eigenvalues, subspace m0 = 64.  One step is
the whole method on the resident matrix: Phase 1 (device Philox sketch,
power iterations with CholQR2, Rayleigh-Ritz truncation) and Phase 2 (FEAST
iterations with COCG shifted solves) until every in-window Ritz pair has
residual <= 1e-10; results stay in device memory.  RA-FEAST runs with
N_c = 4, q = 2, p = 20, complex-FP32 COCG (tolerance 1e-6) with FP64
reliable updates; plain FEAST (N_c = 16, random start) runs beside it on the same
matrix and kernels.

Prints one JSON line.  --gpus N with N > 1 is refused (single-GPU build).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(name="knn8000", n=8000, dim=2, k=10, seed=1, shift=1e-3, m0=64, p=20, q=2,
                nc_ra=4, nc_plain=16, tol_eig=1e-10, tol_solve=1e-6)
HBM_PEAK_GBS = 8000.0
# L2 -> CU (vL1D) bandwidth: 256 CUs x 64 B/clk x 2.4 GHz
L2_PEAK_GBS = 256 * 64 * 2.4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_workload():
    from workloads import knn_laplacian

    w = WORKLOAD
    csr = knn_laplacian(w["n"], w["dim"], w["k"], seed=w["seed"], weighted=True, shift=w["shift"])
    with open(os.path.join(ROOT, "tests", "golden", "windows.json")) as f:
        win = json.load(f)["knn8000"]
    if csr.nnz != win["nnz"]:
        raise RuntimeError("workload generator does not reproduce the stored window fixture")
    return csr, win


def run_steps(plan, steps, lam, res, X, warmstart):
    """Runs `steps` full solves; returns (seconds, list of per-step records)."""
    import torch

    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ws = plan.warmstart() if warmstart else None
        out = plan.solve_device(lam, res, X)
        recs.append((ws, out))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, recs


def spmm_rate(reps=20):
    """The FP64 CSR SpMM kernel (Rayleigh-Ritz W = A Q and the Phase-1 power
    steps) on a matrix large enough for HBM to matter: the 7-point Laplacian
    of a 100^3 grid (n = 1e6, 6.9M nonzeros) times a 64-column block.
    Compulsory bytes per call: 12 per nonzero (value, column), 4 (n+1) row
    pointers, one read of X and one write of Y (16 n k).  Timed with events on
    the stream the plan launches on."""
    import torch

    from paper_2512_01257_amd import native
    from workloads import grid_laplacian

    csr = grid_laplacian((100, 100, 100), 0.01)
    k = 64
    st = torch.cuda.current_stream()
    plan = native.Plan(csr, 0.5, 0.6, 1, nc=1, q=0, p=4, engine="stream", stream=st.cuda_stream)
    X = torch.randn((csr.n, k), dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    plan.spmm(X, Y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        plan.spmm(X, Y)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    plan.close()
    nbytes = 12.0 * csr.nnz + 4.0 * (csr.n + 1) + 16.0 * csr.n * k
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": "k_spmm_f64", "matrix": "7-point Laplacian of a 100^3 grid, n=1e6",
            "nnz": int(csr.nnz), "k": k, "avg_ms": round(ms, 4), "bytes_per_call": nbytes,
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def gram_shapes(reps=5):
    """The FP64 MFMA kernels of Rayleigh-Ritz and CholQR2 (k_gram_partial /
    k_gram_reduce, k_tsmm, k_chol_inv) on tall-skinny blocks of a large
    problem: Gram products X^T X of n = 1e6 rows and k = 84 (the warm start's
    m0 + p of the headline) or 192 (the largest block) columns, and CholQR2 of
    the 84-column block.  Wall-clock per call (each call allocates its partial
    sums); the kernels' own durations and MFMA utilisation come from rocprofv3."""
    import torch

    from paper_2512_01257_amd import native
    from workloads import grid_laplacian

    csr = grid_laplacian((100, 100, 100), 0.01)
    plan = native.Plan(csr, 0.5, 0.6, 1, nc=1, q=0, p=4, engine="stream")
    out = {}
    for k in (84, 192):
        X = torch.randn((csr.n, k), dtype=torch.float64, device="cuda")
        G = torch.empty((k, k), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()  # the plan runs on a stream of its own
        plan.gram(X, X, G)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.gram(X, X, G)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        ref = (X.T @ X)
        err = float((G - ref).abs().max() / ref.abs().max())
        out[f"gram_k{k}"] = dict(n=csr.n, k=k, wall_ms=round(ms, 3),
                                 flops=2.0 * csr.n * k * k, rel_diff_vs_torch=err)
        del X, G
    Y = torch.randn((csr.n, 84), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    plan.cholqr2(Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.cholqr2(Y)
    torch.cuda.synchronize()
    out["cholqr2_k84"] = dict(n=csr.n, k=84, wall_ms=round((time.perf_counter() - t0) / reps * 1e3, 3))
    plan.close()
    return out


def gemm_shapes(reps=6):
    """The matrix-core GEMM behind the dense operators of the statistical
    workloads (rafeast_gemm), on the products of the stats workload at their
    full width: the kernel matrix's K P (8192 x 8192 times 1024 columns) and
    the covariance's X V (1024 x 65536 data, 512 columns; the inner dimension
    split in chunks) and X^T T, in FP32 and FP64.  Wall-clock per call
    (includes the call's workspace allocation and its synchronisation); the
    kernels' own durations come from rocprofv3."""
    import torch

    from paper_2512_01257_amd import native

    peak = {"fp32": 157.3, "fp64": 78.6}
    out = {}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        for name, acol, M, N, K in (("kernel_KP", True, 8192, 1024, 8192),
                                    ("cov_XV", True, 1024, 512, 65536),
                                    ("cov_XtT", False, 65536, 512, 1024)):
            A = torch.randn((K, M) if acol else (M, K), dtype=dt, device="cuda")
            B = torch.randn((K, N), dtype=dt, device="cuda")
            Cm = torch.zeros((M, N), dtype=dt, device="cuda")
            native.gemm(A, B, Cm, a_cols=acol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                native.gemm(A, B, Cm, a_cols=acol)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            ref = (A.T if acol else A).double() @ B.double()
            err = float((Cm.double() - ref).abs().max() / ref.abs().max())
            tf = 2.0 * M * N * K / ms / 1e9
            out[f"{name}_{prec}"] = dict(M=M, N=N, K=K, wall_ms=round(ms, 3),
                                         tflops_wall=round(tf, 1),
                                         frac_of_peak_wall=round(tf / peak[prec], 3),
                                         rel_diff_vs_fp64=err)
            print(f"gemm {name} {prec}: {ms:.3f} ms", flush=True)
            del A, B, Cm, ref
            torch.cuda.empty_cache()
    return out


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or platform.machine()


def cpu_baseline(csr, win, runs):
    """The oracle (FP64, sparse LU shifted solves) on the same workload, timed
    twice: with one thread (the paper's single-threaded setting) and with the
    BLAS thread pool at its default size.  The sparse LU factorizations and
    solves are single-threaded in both; the dense Rayleigh-Ritz and
    orthonormalisation steps use the pool."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import feast as F
    from oracle.philox import gaussian_sketch

    w = WORKLOAD
    A = csr.to_scipy()
    om = gaussian_sketch(csr.n, w["m0"] + w["p"], 0)

    def timed():
        t, M = 0.0, 0
        for _ in range(runs):
            t0 = time.perf_counter()
            out = F.ra_feast(A, win["lmin"], win["lmax"], w["m0"], w["nc_ra"], om, q=w["q"],
                             tol=w["tol_eig"])
            t += time.perf_counter() - t0
            M += out["M"]
        return M / t, t

    cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    v_all, t_all = timed()
    with threadpool_limits(limits=1):
        v_one, t_one = timed()
    return dict(value=v_all, unit="eigenpairs/s", cores=int(cores), kind="oracle",
                cpu_model=cpu_model(), host_cpus=os.cpu_count(),
                single_thread=dict(value=v_one, cores=1, seconds=round(t_one, 2)),
                sample=f"{runs} full RA-FEAST solve(s) of the same workload (N_c=4, q=2, "
                       f"p=20, FP64, sparse-LU shifted solves) per setting: {t_all:.1f} s with "
                       f"{cores} BLAS threads, {t_one:.1f} s with one thread")


def main_batch(args):
    """The batching workload: 32 unweighted kNN Laplacians (2D/3D, k in
    {8, 12, 16}, n log-uniform in [2000, 60000]), each with its own window
    of 10-40 smallest eigenvalues and m0 = ceil(1.5 count), N_c = 4, q = 2.
    One step: warm start and lock-step Phase 2 of all 32 (rafeast_batch_solve);
    compared with the 32 problems solved one after another (rafeast_solve)."""
    import numpy as np
    import torch

    from paper_2512_01257_amd import native
    from workloads import knn_laplacian

    with open(os.path.join(ROOT, "tests", "golden", "windows.json")) as f:
        wins = json.load(f)["batch32"]
    probs = []
    for wn in wins:
        csr = knn_laplacian(wn["n"], wn["dim"], wn["k"], seed=wn["seed"], weighted=False)
        if csr.nnz != wn["nnz"]:
            raise RuntimeError("workload generator does not reproduce the stored window fixture")
        probs.append(dict(csr=csr, lmin=wn["lmin"], lmax=wn["lmax"], m0=wn["m0"]))
    kw = dict(nc=4, q=2, tol_eig=1e-10, tol_solve=1e-6, precision="fp32", seed=0,
              tol_solve_relaxed=args.relaxed if args.relaxed_phase2 else 0.0)

    def check(outs):
        err = 0.0
        for wn, o in zip(wins, outs):
            if o["status"] != "OK" or o["M"] != wn["count"]:
                raise RuntimeError(f"member did not converge: {o['status']} M={o['M']}")
            ev = np.array(wn["eigenvalues"][: wn["count"]])
            err = max(err, float(np.abs(o["lam"] - ev).max()) / max(abs(wn["lmin"]), wn["lmax"]))
        if err > 1e-10:
            raise RuntimeError(f"eigenvalue error {err:.3e} (relative to s_win) above 1e-10")
        return err

    t0 = time.perf_counter()
    B = native.Batch(probs, **kw)
    plan_ms = (time.perf_counter() - t0) * 1e3

    def batch_step():
        for m in B.members:
            m.warmstart()
        return B.solve(want_vectors=False)

    for _ in range(args.warmup):
        batch_step()
    log(f"timing {args.steps} batch step(s), {len(probs)} problems, "
        f"{B.resident_count} in the shared resident launch")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for _ in range(args.steps):
        steps.append(batch_step())
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    err = check(steps[-1][0])
    M_step = sum(o["M"] for o in steps[-1][0])
    value = M_step * args.steps / secs
    t_ms = {k: round(sum(s[1][k] for s in steps) / args.steps, 2) for k in steps[0][1]}
    B.close()

    # the same problems one after another
    seq = None
    if args.plain_steps != 0:
        # each problem on the engine the batch gives it (members the resident
        # engine cannot hold: the multi-shift engine in FP64)
        def member_plan(p):
            if p["csr"].n > 8192:
                return native.Plan(p["csr"], p["lmin"], p["lmax"], p["m0"],
                                   **dict(kw, precision="fp64", engine="multishift"))
            return native.Plan(p["csr"], p["lmin"], p["lmax"], p["m0"], **kw)

        plans = [member_plan(p) for p in probs]
        for pl in plans:  # warm up
            pl.warmstart()
            pl.solve(want_vectors=False)
        log("timing the problems one after another")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = []
        for pl in plans:
            pl.warmstart()
            outs.append(pl.solve(want_vectors=False))
        torch.cuda.synchronize()
        s1 = time.perf_counter() - t0
        check(outs)
        seq = {"value": round(sum(o["M"] for o in outs) / s1, 3), "unit": "eigenpairs/s",
               "ms": round(s1 * 1e3, 2)}
        for pl in plans:
            pl.close()
    line = {
        "metric": "eigenpairs/s at rel. residual 1e-10, batch of 32 graph Laplacians",
        "value": round(value, 3),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {
            "workload": "batch of 32 unweighted kNN Laplacians (2D/3D points, k in {8,12,16}, "
                        "n log-uniform in [2000, 60000]), windows of 10-40 smallest "
                        "eigenvalues, m0 = ceil(1.5 count), N_c=4, q=2, COCG tol 1e-6",
            "problems": len(probs), "resident_members": int(sum(p["csr"].n <= 8192 for p in probs)),
            "eigenpairs_per_step": M_step, "n_total": int(sum(p["csr"].n for p in probs)),
            "tol_solve_relaxed": kw["tol_solve_relaxed"],
        },
        "batch_phase_ms_per_step": t_ms,
        "one_after_another": seq,
        "speedup_vs_one_after_another": None if seq is None else round(value / seq["value"], 3),
        "plan_ms": round(plan_ms, 2),
        "max_eig_error_vs_reference": err,
    }
    print(json.dumps(line), flush=True)


def main_learned(args):
    """The learned-preconditioner workload: 16-NN graph Laplacian of 10^6
    uniform points in the unit cube (Gaussian weights, + 1e-3 I), the N_c = 4
    shifts of the window of its 100 smallest eigenvalues, 64 right-hand sides.
    The coefficient network is trained on samples from a 20000-point graph of
    the same family; COCG preconditioned by the network's polynomials is
    timed against the same COCG without it, both to true residual 1e-10."""
    import numpy as np
    import torch

    from paper_2512_01257_amd import native
    from workloads import knn_laplacian
    from workloads.learned import flatten, init_weights, minibatch_order, residual_samples

    with open(os.path.join(ROOT, "tests", "golden", "windows.json")) as f:
        fx = json.load(f)["learned"]

    def features(plan, z, th_lo, th_hi):
        inf = plan.info()
        a = 2.0 / (inf["sig_hi"] - inf["sig_lo"])
        b = -(inf["sig_hi"] + inf["sig_lo"]) / (inf["sig_hi"] - inf["sig_lo"])
        return np.array([[a * zj.real + b, a * zj.imag, a * th_lo + b, a * th_hi + b] for zj in z])

    # training data: shifts of windows [0, s u] (s = 1, 1/2, ..., 1/32) on the small graph
    tr = fx["train"]
    csr_t = knn_laplacian(tr["n"], 3, 16, seed=tr["seed"], weighted=True, shift=1e-3)
    t0 = time.perf_counter()
    with native.Plan(csr_t, 0.0, tr["u"], 8, nc=4, q=1, p=4, precision="fp64") as pt:
        Xs, Gs, hs, rrs = [], [], [], []
        R = torch.from_numpy(np.ascontiguousarray(residual_samples(tr["n"], 64, 17))).cuda()
        for e in range(6):
            u = tr["u"] / 2.0 ** e
            with native.Plan(csr_t, 0.0, u, 8, nc=4, q=1, p=4, precision="fp64") as pw:
                z = pw.info()["z"]
            X, G, h, rr = pt.pc_samples(z, R, 1e-3, u)
            Xs.append(X), Gs.append(G), hs.append(h), rrs.append(rr)
        X, G, h, rr = (torch.cat(t) for t in (Xs, Gs, hs, rrs))
        ns = X.shape[0]
        W = torch.from_numpy(flatten(init_weights(1, out_scale=0.0))).cuda()
        pt.pc_normalize(X, W)
        _, loss0 = pt.pc_gradient(X, G, h, rr, W)
        order = minibatch_order(ns, 200, 2)
        pt.pc_train(X, G, h, rr, W, order, batch=64, lr=2e-3)
        _, loss1 = pt.pc_gradient(X, G, h, rr, W)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"trained on {ns} samples: mean loss {loss0:.4f} -> {loss1:.4f} ({train_s:.1f} s)")

    # the large graph
    te = fx["test"]
    t0 = time.perf_counter()
    csr = knn_laplacian(te["n"], 3, 16, seed=te["seed"], weighted=True, shift=1e-3)
    log(f"graph n={csr.n} nnz={csr.nnz} built in {time.perf_counter() - t0:.1f} s")
    nrhs = 64
    with native.Plan(csr, 0.0, te["u"], 8, nc=4, q=1, p=4, precision="fp64",
                     max_cocg=20000) as plan:
        z = plan.info()["z"]
        Xf = torch.from_numpy(features(plan, z, 1e-3, te["u"])).cuda()
        Y = plan.pc_forward(Xf, W).cpu().numpy().astype(np.float64)
        coef = (Y[:, 0::2] + 1j * Y[:, 1::2]) / Xf.cpu().numpy()[:, 1:2]  # c = y / Im z^
        B = torch.from_numpy(np.ascontiguousarray(residual_samples(csr.n, nrhs, 23))).cuda()
        out = {}
        for name, cf in (("plain", None), ("learned", coef)):
            Xs = torch.zeros((csr.n, len(z) * nrhs), dtype=torch.complex128, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its, rs = plan.pc_solve(z, B, Xs, 1e-10, coef=cf)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            if rs.max() > 1e-10:
                raise RuntimeError(f"{name}: residual {rs.max():.3e} above 1e-10")
            out[name] = dict(seconds=round(secs, 3), iters_max=int(its.max()),
                             iters_mean=round(float(its.mean()), 1),
                             spmm_per_iter=1 if cf is None else 8,
                             max_resid=float(rs.max()))
            log(f"{name}: {secs:.2f} s, iterations max {its.max()} mean {its.mean():.1f}")
            del Xs
    speed = out["plain"]["seconds"] / out["learned"]["seconds"]
    line = {
        "metric": "COCG time to true residual 1e-10, learned polynomial preconditioner vs none",
        "value": round(speed, 3),
        "unit": "x (plain time / preconditioned time)",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(out["learned"]["seconds"] * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {
            "workload": "16-NN graph Laplacian of 1e6 uniform points in [0,1]^3, Gaussian "
                        "weights, +1e-3 I; N_c=4 shifts of the window [0, u] holding about "
                        "its 100 smallest eigenvalues; 64 random right-hand sides; FP64 COCG",
            "n": csr.n, "nnz": csr.nnz, "u": te["u"], "u_method": te["method"],
            "train": {"n": tr["n"], "samples": int(ns), "steps": len(order) // 64,
                      "loss_before": loss0, "loss_after": loss1, "seconds": round(train_s, 2)},
        },
        "plain": out["plain"],
        "learned": out["learned"],
        "iteration_ratio": round(out["plain"]["iters_max"] / out["learned"]["iters_max"], 3),
    }
    print(json.dumps(line), flush=True)


def main_knn1e6(args):
    """The n = 10^6 configuration as an eigensolve: 16-NN graph Laplacian of
    10^6 uniform points in the unit cube (Gaussian weights, sigma = median
    neighbour distance, + 1e-3 I), window [0, u] meant to hold its 100
    smallest eigenvalues, m0 = 128, N_c = 4, q = 1, p = 20; RA-FEAST with the
    FP64 multi-shift engine (COCG tolerance 1e-6) until every in-window Ritz
    pair has scaled residual <= 1e-10.  The edge u is the power law fitted to
    mid-gaps at n = 1e4, 2e4, 5e4 (no spectrum of this matrix is computable
    on the host), so the count M and completeness are unpinned; the
    residuals are recomputed with torch's sparse product and the
    orthonormality of the returned vectors is checked on the device."""
    import numpy as np
    import torch

    from paper_2512_01257_amd import native
    from workloads import knn_laplacian

    with open(os.path.join(ROOT, "tests", "golden", "windows.json")) as f:
        te = json.load(f)["learned"]["test"]
    t0 = time.perf_counter()
    csr = knn_laplacian(te["n"], 3, 16, seed=te["seed"], weighted=True, shift=1e-3)
    log(f"graph n={csr.n} nnz={csr.nnz} built in {time.perf_counter() - t0:.1f} s")
    m0, lmin, lmax = 128, 0.0, te["u"]
    t0 = time.perf_counter()
    plan = native.Plan(csr, lmin, lmax, m0, nc=4, q=1, p=20, precision="fp64",
                       engine="multishift", tol_solve=1e-6, tol_eig=1e-10,
                       max_iter=args.max_iter)
    plan_ms = (time.perf_counter() - t0) * 1e3
    lam = torch.zeros(m0, dtype=torch.float64, device="cuda")
    res = torch.zeros(m0, dtype=torch.float64, device="cuda")
    X = torch.zeros((m0, csr.n), dtype=torch.float64, device="cuda")
    log("solving")
    secs, recs = run_steps(plan, 1, lam, res, X, warmstart=True)
    ws, out = recs[0]
    plan.close()
    M = out["M"]
    # checks outside the timed region: residuals by torch's sparse product
    A = torch.sparse_csr_tensor(torch.from_numpy(csr.rowptr.astype(np.int64)),
                                torch.from_numpy(csr.colind.astype(np.int64)),
                                torch.from_numpy(csr.values), size=(csr.n, csr.n)).cuda()
    V = X[:M].T.contiguous()  # n x M, the unit eigenvectors (column-major output)
    lv = lam[:M]
    R = (A @ V) - V * lv[None, :]
    s_win = max(abs(lmin), abs(lmax))
    resid = (R.norm(dim=0) / s_win).cpu().numpy()
    orth = float((V.T @ V - torch.eye(M, dtype=torch.float64, device="cuda")).abs().max())
    line = {
        "metric": "eigenpairs/s at rel. residual 1e-10, kNN n=1e6 (3D, k=16) bottom window",
        "value": round(M / secs, 4), "unit": "eigenpairs/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": round(secs * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+c128", "data": "synthetic",
        "config": {"workload": "16-NN graph Laplacian of 1e6 uniform points in [0,1]^3, "
                               "Gaussian weights, +1e-3 I; window [0, u], u from a power-law "
                               "fit to mid-gaps at n=1e4..5e4 (about 100 eigenvalues); m0=128, "
                               "N_c=4, q=1, p=20; FP64 multi-shift COCG, tol 1e-6",
                   "n": int(csr.n), "nnz": int(csr.nnz), "u": lmax, "m0": m0},
        "status": out["status"], "M": M, "feast_iters": out["iters"],
        "cocg_iters": int(out["cocg_iters"]), "cocg_max": out["cocg_max"],
        "cocg_node": out["cocg_node"], "phase_ms": out["t_ms"],
        "warmstart_ms": ws["t_ms"], "plan_ms": round(plan_ms, 1),
        "warmstart_bound": {k: ws[k] for k in ("beta_m0", "beta_m0p1", "r_halko", "proj_bound")},
        "max_resid_library": out["max_resid"],
        "max_resid_recomputed": float(resid.max()) if M else None,
        "orthonormality": orth,
        "eigenvalues": [float(v) for v in lv.cpu().numpy()[:5]] + ["..."] +
                       [float(v) for v in lv.cpu().numpy()[-3:]],
        "parity": "unpinned: no independent spectrum at this size; residuals, orthonormality "
                  "and the in-window count are reported",
    }
    print(json.dumps(line), flush=True)


def main_grid64(args):
    """The precision form at scale: Dirichlet 7-point 64^3 grid + 0.01 I
    (n = 262144), interior window of 39 eigenvalues around 0.5, m0 = 64,
    N_c = 8, p = 20, complex-FP32 COCG (streaming engine) with FP64 reliable
    updates; eigenvalues checked against the closed form.  --max-iter and
    --max-cocg cut the run short (for profiling; then no check)."""
    import numpy as np

    from paper_2512_01257_amd import native
    from workloads import gaussian, grid_laplacian

    csr = grid_laplacian((64, 64, 64), 0.01)
    lmin, lmax = 0.493673151133, 0.506687779116
    ms = args.engine == "multishift"
    prec = "fp64" if ms else args.precision
    if args.copy_probe:
        import torch

        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
    t0 = time.perf_counter()
    with native.Plan(csr, lmin, lmax, 64, nc=8, q=2, p=20, precision=prec, tol_solve=1e-6,
                     tol_solve_relaxed=args.relaxed if args.relaxed_phase2 else 0.0,
                     tol_eig=1e-10, max_iter=args.max_iter, max_cocg=args.max_cocg,
                     engine="multishift" if ms else "auto") as plan:
        plan_ms = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        ws = plan.warmstart(omega=gaussian(csr.n, 84, 0))
        out = plan.solve(want_vectors=False)
        secs = time.perf_counter() - t0
    err = None
    full = args.max_iter >= 20 and args.max_cocg >= 20000
    if full:
        from tests.closed_forms import grid_eigs

        vals, _ = grid_eigs((64, 64, 64), 0.01)
        ref = vals[(vals >= lmin) & (vals <= lmax)]
        if out["status"] != "OK" or out["M"] != len(ref):
            raise RuntimeError(f"64^3 solve: {out['status']} M={out['M']}")
        err = float(np.abs(out["lam"] - ref).max()) / lmax
    line = {
        "metric": "eigenpairs/s at rel. residual 1e-10, 64^3 interior window (precision form)",
        "value": round(out["M"] / secs, 4),
        "unit": "eigenpairs/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(secs * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+c128" if ms else ("c64+f64" if prec == "fp32" else "c128"),
        "data": "synthetic",
        "config": {"workload": "Dirichlet 7-point 64^3 grid + 0.01 I, window [0.493673151133, "
                               "0.506687779116] (39 eigenvalues), m0=64, N_c=8, q=2, p=20, "
                               + ("multi-shift FP64 COCG (one real seed CG per right-hand side)"
                                  if ms else "complex-FP32 COCG + FP64 reliable updates"
                                  if prec == "fp32" else "complex-FP64 COCG") + ", tol 1e-6",
                   "engine": "multishift" if ms else "stream", "precision": prec,
                   "max_iter": args.max_iter, "max_cocg": args.max_cocg,
                   "tol_solve_relaxed": args.relaxed if args.relaxed_phase2 else 0.0},
        "status": out["status"], "M": out["M"], "feast_iters": out["iters"],
        "cocg_iters": out["cocg_iters"], "cocg_max": out["cocg_max"],
        "phase_ms": out["t_ms"], "warmstart_ms": ws["t_ms"], "plan_ms": round(plan_ms, 1),
        "max_eig_error_vs_closed_form": err,
    }
    print(json.dumps(line), flush=True)


def main_stats(args):
    """The statistical applications of Section 4 at scale: a top window of the
    sample covariance of a 1024 x 65536 spiked data matrix (A = X^T X / 1023,
    never formed) and of an 8192 x 8192 Gaussian kernel matrix (kernel PCA),
    each window holding the eigenvalues that explain 95% of the trace (13 and
    15), m0 = 2 count, N_c = 8 (covariance) and 16 (kernel), q = 2, literal
    warmstart operator, complex-FP32 COCG with FP64 reliable updates on the
    streaming engine, products on rocBLAS GEMMs.  One step: warm start + solve
    of both; eigenvalues checked against the stored spectra.  The solve's
    operator flops (4 n^2 or 8 rows n per COCG column-iteration) over its time
    are reported as a lower bound on the GEMM rate."""
    import numpy as np
    import torch

    from paper_2512_01257_amd import native
    from workloads import gaussian
    from workloads.stats import rbf_kernel, spiked_data

    with open(os.path.join(ROOT, "tests", "golden", "windows.json")) as f:
        fix = json.load(f)["stats"]
    rel = args.relaxed if args.relaxed_phase2 else 0.0
    rows = {}
    tot_m, tot_s = 0, 0.0
    for name in ("cov_bench", "kpca_bench"):
        fx = fix[name]
        t0 = time.perf_counter()
        if fx["kind"] == "covariance":
            data = spiked_data(fx["rows"], fx["p"], seed=1)
            n = fx["p"]
            make = native.Plan.from_covariance
            flops_per_col = 8.0 * fx["rows"] * n
        else:
            data = rbf_kernel(fx["n"], bandwidth=0.4, seed=2)
            n = fx["n"]
            make = native.Plan.from_dense
            flops_per_col = 4.0 * n * n
        gen_ms = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        plan = make(data, fx["lmin"], fx["lmax"], fx["m0"], nc=fx["nc"], q=2, ws_op="literal",
                    tol_solve_relaxed=rel, precision=args.precision)
        plan_ms = (time.perf_counter() - t0) * 1e3
        del data
        lam = torch.zeros(fx["m0"], dtype=torch.float64, device="cuda")
        res = torch.zeros_like(lam)
        for _ in range(args.warmup):
            run_steps(plan, 1, lam, res, None, warmstart=True)
        secs, recs = run_steps(plan, args.steps, lam, res, None, warmstart=True)
        out = recs[-1][1]
        k = fx["count"]
        if out["status"] != "OK" or out["M"] != k:
            raise RuntimeError(f"{name}: {out['status']} M={out['M']}")
        got = np.sort(lam.cpu().numpy()[:k])[::-1]
        err = float(np.abs(got - np.array(fx["eigenvalues"][:k])).max()) / abs(fx["lmax"])
        if err > 1e-10:
            raise RuntimeError(f"{name}: eigenvalue error {err:.3e} relative to s_win")
        # the FP64 operator product alone (warm start / Rayleigh-Ritz form),
        # 192 columns, wall clock over 10 calls (each ends with a sync)
        V = torch.randn((n, 192), dtype=torch.float64, device="cuda")
        Yv = torch.empty_like(V)
        plan.spmm(V, Yv)
        t1 = time.perf_counter()
        for _ in range(10):
            plan.spmm(V, Yv)
        prod_s = (time.perf_counter() - t1) / 10
        del V, Yv
        plan.close()
        solve_ms = sum(o["t_ms"]["solve"] for _, o in recs) / args.steps
        coliters = sum(o["cocg_iters"] for _, o in recs) / args.steps
        rows[name] = dict(
            n=n, count=k, m0=fx["m0"], nc=fx["nc"], ms_per_step=round(secs / args.steps * 1e3, 2),
            eigenpairs_per_s=round(k * args.steps / secs, 3), feast_iters=out["iters"],
            cocg_iters=int(coliters), solve_ms=round(solve_ms, 2),
            warmstart_ms=round(sum(w["t_ms"] for w, _ in recs) / args.steps, 2),
            solve_operator_tflops=round(flops_per_col * coliters / (solve_ms * 1e-3) / 1e12, 2),
            fp64_product_192_ms=round(prod_s * 1e3, 3),
            fp64_product_192_tflops=round(flops_per_col / 2 * 192 / prod_s / 1e12, 2),
            max_eig_error_rel=err, plan_ms=round(plan_ms, 1), generate_ms=round(gen_ms, 1))
        tot_m += k * args.steps
        tot_s += secs
        log(f"{name}: {rows[name]}")
    line = {
        "metric": "eigenpairs/s at rel. residual 1e-10, top windows of a sample covariance and "
                  "a kernel matrix (Section 4)",
        "value": round(tot_m / tot_s, 3), "unit": "eigenpairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(tot_s / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
        "config": {"workload": "sample covariance of a 1024 x 65536 spiked data matrix and an "
                               "8192 x 8192 Gaussian kernel matrix; top windows by the 95% "
                               "variance rule; COCG tol 1e-6", "tol_solve_relaxed": rel,
                   "precision": args.precision},
        "table": rows,
    }
    print(json.dumps(line), flush=True)


def main_rgg(args):
    """The paper's sweep (Section 5.1, Table 1, Figure 1): random geometric
    graph Laplacians L = D - A (unit square, radius 1.5 sqrt(ln n / n)),
    window [0.001, 5.0], m0 = 40 (ceil(1.5 count) where the window holds 40
    or more eigenvalues).  Standard FEAST
    (N_c = 8, random start, run to residual 1e-10) against RA-FEAST with
    N_c in {2, 4, 8} and max_iter in {2, 4}; per configuration the mean
    time of warm start + solve over the seeds, the speedup over standard
    FEAST and the Max Error max_i |lambda_i - lambda_i^ref| against the
    stored reference spectra (oracle shift-invert Lanczos).  value = speedup
    of RA-FEAST (N_c = 2, max_iter = 4) at the largest n."""
    import numpy as np
    import torch

    from paper_2512_01257_amd import native
    from workloads import rgg_laplacian

    with open(os.path.join(ROOT, "tests", "golden", "windows.json")) as f:
        fix = json.load(f)["rgg"]
    ns = [int(v) for v in args.rgg_n.split(",")]
    configs = [("standard", 8, 20, "none")] + [
        (f"ra_nc{nc}_it{it}", nc, it, "auto") for nc in (8, 4, 2) for it in (4, 2)]
    direct = args.rgg_solver == "direct"
    table = {}
    for n in ns:
        rows = {name: dict(ms=[], err=[], ws_ms=[], found=0, feast_iters=[]) for name, *_ in configs}
        trials = [w for w in fix if w["n"] == n][: args.seeds]
        for w in trials:
            csr = rgg_laplacian(n, w["seed"])
            if csr.nnz != w["nnz"]:
                raise RuntimeError("workload generator does not reproduce the stored fixture")
            ref = np.array(w["eigenvalues"])
            for name, nc, it, ws_op in configs:
                rel = args.relaxed if args.relaxed_phase2 and ws_op != "none" else 0.0
                solver = dict(precision="fp32")
                if direct:  # exact solves: both methods factorize their shifted matrices
                    solver = dict(precision="fp64", engine="direct")

                def make():
                    return native.Plan(csr, w["lmin"], w["lmax"], w["m0"], nc=nc, q=2, p=-1,
                                       tol_solve_relaxed=rel, tol_eig=1e-10, tol_solve=1e-6,
                                       max_iter=it, ws_op=ws_op, seed=w["seed"], **solver)

                lam = torch.zeros(w["m0"], dtype=torch.float64, device="cuda")
                res = torch.zeros(w["m0"], dtype=torch.float64, device="cuda")
                if w is trials[0]:  # first-use costs (kernel loading)
                    plan = make()
                    run_steps(plan, 1, lam, res, None, warmstart=True)
                    plan.close()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan = make()
                plan_s = time.perf_counter() - t0
                secs, recs = run_steps(plan, 1, lam, res, None, warmstart=True)
                if direct:  # the factorizations are part of the method's time
                    secs += plan_s
                ws, out = recs[0]
                plan.close()
                r = rows[name]
                r["ms"].append(secs * 1e3)
                r["ws_ms"].append(ws["t_ms"])
                r["feast_iters"].append(out["iters"])
                got = lam.cpu().numpy()[: out["M"]]
                if out["M"] == len(ref):
                    r["found"] += 1
                    r["err"].append(float(np.abs(got - ref).max()) if len(ref) else 0.0)
            log(f"rgg n={n} seed={w['seed']} count={w['count']} m0={w['m0']}: " + ", ".join(
                f"{nm} {rows[nm]['ms'][-1]:.0f} ms" for nm, *_ in configs))
        base = float(np.mean(rows["standard"]["ms"]))
        table[str(n)] = {
            name: dict(mean_ms=round(float(np.mean(r["ms"])), 2),
                       speedup=round(base / float(np.mean(r["ms"])), 2),
                       max_error_mean=float(np.mean(r["err"])) if r["err"] else None,
                       max_error_max=float(np.max(r["err"])) if r["err"] else None,
                       all_found=f"{r['found']}/{len(r['ms'])}",
                       phase1_ms=round(float(np.mean(r["ws_ms"])), 3),
                       feast_iters=round(float(np.mean(r["feast_iters"])), 2))
            for name, r in rows.items()}
    top = table[str(ns[-1])]["ra_nc2_it4"]
    line = {
        "metric": "speedup of RA-FEAST over standard FEAST (N_c=8), RGG Laplacians, window [0.001, 5]",
        "value": top["speedup"],
        "unit": "x (standard FEAST time / RA-FEAST N_c=2, max_iter=4 time)",
        "n_gpus": 1, "steps": args.seeds, "warmup": 1,
        "ms_per_step": top["mean_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128+f64" if direct else "c64+f64", "data": "synthetic",
        "config": {"workload": "random geometric graph Laplacians L = D - A, n points in the unit "
                               "square, radius 1.5 sqrt(ln n / n); window [0.001, 5.0]; "
                               "m0 = 40, or ceil(1.5 count) if count >= 40; " + (
                                   "exact solves (band LDL^T, factorization timed)" if direct
                                   else "COCG tol 1e-6"),
                   "solver": args.rgg_solver,
                   "n": ns, "seeds": args.seeds,
                   "ra_tol_solve_relaxed": args.relaxed if args.relaxed_phase2 else 0.0},
        "table": table,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--cpu-runs", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 256 MiB device-to-device (a dispatch of known traffic "
                         "for scaling memory counters)")
    ap.add_argument("--workload",
                    choices=("knn8000", "batch32", "learned", "grid64", "rgg", "stats",
                             "knn1e6"),
                    default="knn8000",
                    help="knn8000: the headline workload (default); batch32: the batching "
                         "form over 32 graphs; learned: the learned preconditioner at n=1e6; "
                         "grid64: the precision form on the 64^3 grid; rgg: the paper's "
                         "random-geometric-graph sweep; stats: the statistical applications "
                         "(covariance and kernel PCA top windows); knn1e6: the n=1e6 kNN "
                         "window as an eigensolve (multi-shift engine)")
    ap.add_argument("--relaxed", type=float, default=1e-2,
                    help="starting COCG tolerance of the relaxed Phase-2 figures (0: skip)")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32",
                    help="stats: COCG precision (complex FP32 with FP64 reliable updates, or FP64)")
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="headline: RA-FEAST steps timed with FP64 solves on the streaming and "
                         "the multi-shift engine (0: skip)")
    ap.add_argument("--relaxed-phase2", action="store_true",
                    help="grid64, batch32, rgg (RA configurations only): relaxed Phase-2 solves "
                         "starting at --relaxed")
    ap.add_argument("--engine", choices=("auto", "multishift"), default="auto",
                    help="grid64: COCG engine (multishift: FP64 multi-shift engine)")
    ap.add_argument("--max-iter", type=int, default=20, help="grid64: FEAST iteration cap")
    ap.add_argument("--max-cocg", type=int, default=20000, help="grid64: COCG iteration cap")
    ap.add_argument("--gram-only", action="store_true",
                    help="only the tall-skinny FP64 MFMA kernels (Gram, CholQR2) at n = 1e6")
    ap.add_argument("--gemm-only", action="store_true",
                    help="only the matrix-core GEMM of the statistical workloads' operators")
    ap.add_argument("--spmm-only", action="store_true",
                    help="only the FP64 SpMM rate measurement (for profiling)")
    ap.add_argument("--rgg-n", default="2000,4000,8000,16000", help="rgg: graph sizes")
    ap.add_argument("--seeds", type=int, default=3, help="rgg: seeds per size (at most 40)")
    ap.add_argument("--rgg-solver", choices=("cocg", "direct"), default="cocg",
                    help="rgg: shifted solves by COCG, or exact (the direct engine; the "
                         "factorizations are timed with each method, as in the paper)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); the multi-GPU path is not part of it.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch32":
        return main_batch(args)
    if args.workload == "learned":
        return main_learned(args)
    if args.workload == "grid64":
        return main_grid64(args)
    if args.workload == "knn1e6":
        return main_knn1e6(args)
    if args.workload == "rgg":
        return main_rgg(args)
    if args.workload == "stats":
        return main_stats(args)
    if args.gram_only:
        import torch

        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps({"gram": gram_shapes()}), flush=True)
        return
    if args.gemm_only:
        import torch

        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps({"gemm": gemm_shapes()}), flush=True)
        return
    if args.spmm_only:
        import torch

        assert torch.cuda.is_available(), "bench.py needs a GPU"
        if args.copy_probe:
            src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            del src
        print(json.dumps({"spmm": spmm_rate()}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2512_01257_amd import native

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = WORKLOAD
    csr, win = load_workload()
    lmin, lmax = win["lmin"], win["lmax"]
    m0 = w["m0"]

    t0 = time.perf_counter()
    ra = native.Plan(csr, lmin, lmax, m0, nc=w["nc_ra"], q=w["q"], p=w["p"],
                     tol_eig=w["tol_eig"], tol_solve=w["tol_solve"], precision="fp32", seed=0)
    plan_ms = (time.perf_counter() - t0) * 1e3
    plain = native.Plan(csr, lmin, lmax, m0, nc=w["nc_plain"], q=0, p=w["p"],
                        tol_eig=w["tol_eig"], tol_solve=w["tol_solve"], precision="fp32",
                        ws_op="none", seed=0)
    lam = torch.zeros(m0, dtype=torch.float64, device="cuda")
    res = torch.zeros(m0, dtype=torch.float64, device="cuda")
    X = torch.zeros((m0, csr.n), dtype=torch.float64, device="cuda")

    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"warmup {args.warmup} step(s)")
    run_steps(ra, args.warmup, lam, res, X, warmstart=True)
    log(f"timing {args.steps} RA-FEAST step(s)")
    secs, recs = run_steps(ra, args.steps, lam, res, X, warmstart=True)
    for ws, out in recs:
        if out["status"] != "OK" or out["M"] != win["count"]:
            raise RuntimeError(f"RA-FEAST step did not converge: {out}")
    # results of the last step checked against the stored reference spectrum
    ev = np.array(win["eigenvalues"][: win["count"]])
    err = float(np.abs(lam.cpu().numpy()[: win["count"]] - ev).max())
    if err > 1e-10 * lmax:
        raise RuntimeError(f"eigenvalue error {err:.3e} above 1e-10 * s_win")
    M_total = sum(out["M"] for _, out in recs)
    value = M_total / secs

    # plain FEAST on the same kernels
    pk = args.plain_steps if args.plain_steps is not None else max(1, args.steps // 2)
    plain_value = psecs = None
    if pk > 0:
        run_steps(plain, 1, lam, res, X, warmstart=True)
        log(f"timing {pk} plain-FEAST step(s)")
        psecs, precs = run_steps(plain, pk, lam, res, X, warmstart=True)
        for _, out in precs:
            if out["status"] != "OK":
                raise RuntimeError(f"plain FEAST did not converge: {out}")
        plain_value = sum(out["M"] for _, out in precs) / psecs

    # standard FEAST as the paper runs it (Section 5.1): exact solves from
    # factorizations of the N_c shifted matrices (the direct engine: band
    # LDL^T in FP64, factorized once when the plan is made), random start
    exact = None
    if pk > 0:
        t0 = time.perf_counter()
        dplan = native.Plan(csr, lmin, lmax, m0, nc=w["nc_plain"], q=0, p=w["p"],
                            tol_eig=w["tol_eig"], precision="fp64", ws_op="none", seed=0,
                            engine="direct")
        dplan_ms = (time.perf_counter() - t0) * 1e3
        run_steps(dplan, 1, lam, res, X, warmstart=True)
        log(f"timing {pk} standard-FEAST step(s) with exact factorizations")
        dsecs, drecs = run_steps(dplan, pk, lam, res, X, warmstart=True)
        for _, out in drecs:
            if out["status"] != "OK" or out["M"] != win["count"]:
                raise RuntimeError(f"standard FEAST (exact solves) did not converge: {out}")
        e_ = float(np.abs(lam.cpu().numpy()[: win["count"]] - np.array(
            win["eigenvalues"][: win["count"]])).max())
        if e_ > 1e-10 * lmax:
            raise RuntimeError(f"exact-solve eigenvalue error {e_:.3e} above 1e-10 * s_win")
        dval = sum(out["M"] for _, out in drecs) / dsecs
        dstep = dsecs / pk
        exact = {"value": round(dval, 3), "unit": "eigenpairs/s",
                 "ms_per_step": round(dstep * 1e3, 4), "nc": w["nc_plain"],
                 "feast_iters_per_step": [o["iters"] for _, o in drecs],
                 "plan_ms_with_factorization": round(dplan_ms, 2),
                 "value_with_factorization": round(win["count"] / (dstep + dplan_ms * 1e-3), 3),
                 "max_eig_error_vs_reference": e_,
                 "solver": "band LDL^T of each z_j I - A (reverse Cuthill-McKee order), FP64"}
        dplan.close()
        # RA-FEAST on the same exact solves (the paper's setting: both methods
        # factorize their shifted matrices)
        t0 = time.perf_counter()
        rplan = native.Plan(csr, lmin, lmax, m0, nc=w["nc_ra"], q=w["q"], p=w["p"],
                            tol_eig=w["tol_eig"], precision="fp64", seed=0, engine="direct")
        rplan_ms = (time.perf_counter() - t0) * 1e3
        run_steps(rplan, 1, lam, res, X, warmstart=True)
        log(f"timing {pk} RA-FEAST step(s) with exact factorizations")
        rsecs, rrecs = run_steps(rplan, pk, lam, res, X, warmstart=True)
        for _, out in rrecs:
            if out["status"] != "OK" or out["M"] != win["count"]:
                raise RuntimeError(f"RA-FEAST (exact solves) did not converge: {out}")
        e_ = float(np.abs(lam.cpu().numpy()[: win["count"]] - np.array(
            win["eigenvalues"][: win["count"]])).max())
        if e_ > 1e-10 * lmax:
            raise RuntimeError(f"exact-solve RA-FEAST eigenvalue error {e_:.3e} above 1e-10 * s_win")
        rstep = rsecs / pk
        exact["ra"] = {"value": round(sum(o["M"] for _, o in rrecs) / rsecs, 3),
                       "ms_per_step": round(rstep * 1e3, 4), "nc": w["nc_ra"],
                       "feast_iters_per_step": [o["iters"] for _, o in rrecs],
                       "plan_ms_with_factorization": round(rplan_ms, 2),
                       "value_with_factorization": round(
                           win["count"] / (rstep + rplan_ms * 1e-3), 3),
                       "max_eig_error_vs_reference": e_}
        rplan.close()

    # Phase 2 with relaxed solves (Section 3.3: k_inexact from relaxed
    # tolerances): the solves start at tol_solve_relaxed and tighten only when
    # a FEAST iteration stops contracting; same eigenpair target.  Plain FEAST
    # given the same control for comparison.
    relaxed = None
    if args.relaxed > 0.0:
        def relaxed_run(nc, q, ws_op, steps):
            pl = native.Plan(csr, lmin, lmax, m0, nc=nc, q=q, p=w["p"], tol_eig=w["tol_eig"],
                             tol_solve=w["tol_solve"], precision="fp32", ws_op=ws_op, seed=0,
                             tol_solve_relaxed=args.relaxed)
            run_steps(pl, 1, lam, res, X, warmstart=True)
            s_, r_ = run_steps(pl, steps, lam, res, X, warmstart=True)
            pl.close()
            for _, o in r_:
                if o["status"] != "OK" or o["M"] != win["count"]:
                    raise RuntimeError(f"relaxed-solve step did not converge: {o}")
            e_ = float(np.abs(lam.cpu().numpy()[: win["count"]] - ev).max())
            if e_ > 1e-10 * lmax:
                raise RuntimeError(f"relaxed-solve eigenvalue error {e_:.3e} above 1e-10 * s_win")
            o = r_[-1][1]
            return dict(value=round(sum(x["M"] for _, x in r_) / s_, 3),
                        ms_per_step=round(s_ / steps * 1e3, 4), feast_iters=o["iters"],
                        cocg_iters=int(o["cocg_iters"]), max_resid=o["max_resid"],
                        tol_solve_last=o["tol_solve_last"], max_eig_error_vs_reference=e_)
        log(f"timing {args.steps} RA-FEAST step(s) with relaxed Phase-2 solves")
        relaxed = dict(tol_solve_relaxed=args.relaxed,
                       ra=relaxed_run(w["nc_ra"], w["q"], "auto", args.steps))
        if plain_value is not None:
            relaxed["plain"] = relaxed_run(w["nc_plain"], 0, "none", pk)
            relaxed["speedup_vs_plain_same_control"] = round(
                relaxed["ra"]["value"] / relaxed["plain"]["value"], 3)
            relaxed["speedup_vs_plain_fixed_tol"] = round(relaxed["ra"]["value"] / plain_value, 3)

    # The same RA-FEAST steps with FP64 solves.  The FP64 resident engine
    # holds at most 4096 rows, so at n = 8000 FP64 runs on the streaming or
    # the multi-shift engine: what the complex-FP32 form with FP64 reliable
    # updates gains over the faster of them, at the same eigenpair target.
    fp64 = None
    if args.fp64_steps > 0:
        def fp64_run(engine, steps):
            pl = native.Plan(csr, lmin, lmax, m0, nc=w["nc_ra"], q=w["q"], p=w["p"],
                             tol_eig=w["tol_eig"], tol_solve=w["tol_solve"], precision="fp64",
                             ws_op="auto", seed=0, engine=engine)
            run_steps(pl, 1, lam, res, X, warmstart=True)
            s_, r_ = run_steps(pl, steps, lam, res, X, warmstart=True)
            eng = pl.engine
            pl.close()
            for _, o in r_:
                if o["status"] != "OK" or o["M"] != win["count"]:
                    raise RuntimeError(f"FP64-solve step ({engine}) did not converge: {o}")
            e_ = float(np.abs(lam.cpu().numpy()[: win["count"]] - ev).max())
            if e_ > 1e-10 * lmax:
                raise RuntimeError(f"FP64-solve eigenvalue error {e_:.3e} above 1e-10 * s_win")
            o = r_[-1][1]
            return dict(engine=eng, value=round(sum(x["M"] for _, x in r_) / s_, 3),
                        ms_per_step=round(s_ / steps * 1e3, 4), feast_iters=o["iters"],
                        cocg_iters=int(o["cocg_iters"]), max_eig_error_vs_reference=e_)
        log(f"timing {args.fp64_steps} RA-FEAST step(s) with FP64 solves on each FP64 engine")
        fp64 = dict(stream=fp64_run("stream", args.fp64_steps),
                    multishift=fp64_run("multishift", args.fp64_steps))
        best = max(fp64["stream"]["value"], fp64["multishift"]["value"])
        fp64["fp32_speedup_over_best_fp64"] = round(value / best, 3)

    # dominant kernel: the resident COCG engine (one launch per FEAST
    # iteration), timed by the library with HIP events on its own stream.  It
    # keeps every vector of a system in one CU's LDS and registers, so what
    # bounds it is on chip: each COCG iteration of a system streams the whole
    # matrix (FP32 value + 16-bit LDS offset per nonzero) from L2 into the CU.
    # Roof: 256 CUs x 64 B/clk L2->vL1D x 2.4 GHz.  The HBM-equivalent figure
    # (bytes a streaming engine would move for the same column-iterations) and
    # the measured HBM traffic are reported beside it.
    launches = sum(out["iters"] for _, out in recs)
    solve_ms = sum(out["t_ms"]["solve"] for _, out in recs)
    coliters = sum(out["cocg_iters"] for _, out in recs)
    ph_ra = {f"{k}_ms": sum(out["t_ms"][k] for _, out in recs) for k in recs[0][1]["t_ms"]}
    ph_ra["warmstart_ms"] = sum(ws["t_ms"] for ws, _ in recs)
    nnz, n = csr.nnz, csr.n
    B = w["nc_ra"] * m0
    avg_launch_s = solve_ms / launches * 1e-3
    coliters_per_launch = coliters / launches
    l2_bytes_per_launch = coliters_per_launch * 6.0 * nnz
    l2_achieved = l2_bytes_per_launch / avg_launch_s / 1e9
    hbm_model_bytes = coliters_per_launch * ((8.0 * nnz + 4.0 * (n + 1)) / B + 9.0 * n * 8.0)
    hbm_model_gbs = hbm_model_bytes / avg_launch_s / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "cocg_resident_knn8000_traffic.txt")
    if os.path.exists(tfile):
        with open(tfile) as f:
            tj = json.load(f)
        if tj.get("kernel_source_sha") == native.kernel_source_sha("k_cocg.hip"):
            traffic = tj.get("bytes_per_launch")

    onchip = None
    ofile = os.path.join(ROOT, "profiles", "cocg_resident_knn8000_onchip.txt")
    if os.path.exists(ofile):
        with open(ofile) as f:
            oj = json.load(f)
        if oj.get("kernel_source_sha") == native.kernel_source_sha("k_cocg.hip"):
            onchip = {k: oj[k] for k in ("cu_busy_frac_over_step", "l2_read_bytes_per_launch_128B",
                                         "l2_port_frac_while_busy", "l2_port_frac_over_launch")}

    phases = {k: round(v / args.steps, 3) for k, v in ph_ra.items() if k.endswith("_ms")}
    line = {
        "metric": "eigenpairs/s at rel. residual 1e-10, RA-FEAST vs plain FEAST; SpMM HBM GB/s",
        "value": round(value, 3),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {
            "workload": "knn-laplacian n=8000 (2D points, k=10, Gaussian weights, +1e-3 I), "
                        "50 smallest eigenvalues, m0=64; RA-FEAST N_c=4 q=2 p=20 vs plain "
                        "FEAST N_c=16; COCG tol 1e-6 (complex FP32 with FP64 reliable updates)",
            "n": n, "nnz": nnz, "m0": m0, "M": win["count"], "nc": w["nc_ra"], "q": w["q"],
            "p": w["p"], "tol_eig": w["tol_eig"], "tol_solve": w["tol_solve"],
        },
        "plain_feast": None if plain_value is None else {
            "value": round(plain_value, 3), "unit": "eigenpairs/s",
            "ms_per_step": round(psecs / pk * 1e3, 4), "nc": w["nc_plain"],
            # every step starts from the same device sketch (Philox key 0), so
            # the steps repeat identical work
            "feast_iters_per_step": [o["iters"] for _, o in precs],
            "cocg_iters_per_step": int(sum(o["cocg_iters"] for _, o in precs) / pk)},
        "speedup_vs_plain": None if plain_value is None else round(value / plain_value, 3),
        "plain_feast_exact_solves": exact,
        "speedup_vs_plain_exact_solves": None if exact is None else round(
            value / exact["value"], 3),
        "relaxed_phase2": relaxed,
        "fp64_solves": fp64,
        "plan_ms": round(plan_ms, 2),
        "ra_phase_ms_per_step": phases,
        "feast_iters_per_step": round(sum(o["iters"] for _, o in recs) / args.steps, 2),
        "cocg_iters_per_step": int(coliters / args.steps),
        "max_eig_error_vs_reference": err,
        "roofline": {
            "kernel": "k_cocg_resident<float>",
            "bound": "l2",
            "achieved": round(l2_achieved, 1),
            "peak": L2_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(l2_achieved / L2_PEAK_GBS, 4),
            "traffic": traffic,
            "basis": "achieved = 6 B per nonzero (FP32 value, 16-bit LDS offset) per COCG "
                     "column-iteration, streamed from L2 by the CU that owns the system, over "
                     "the mean launch; peak = 256 CUs x 64 B/clk x 2.4 GHz; traffic = HBM "
                     "bytes per launch (FETCH_SIZE + WRITE_SIZE)",
            "avg_launch_ms": round(avg_launch_s * 1e3, 4),
            "column_iterations_per_launch": round(coliters_per_launch, 1),
            "l2_bytes_per_launch": l2_bytes_per_launch,
            "onchip_counters": onchip,
            "hbm_measured_frac": None if traffic is None else round(
                traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4),
            "hbm_streaming_equivalent": {
                "achieved": round(hbm_model_gbs, 1), "peak": HBM_PEAK_GBS,
                "frac": round(hbm_model_gbs / HBM_PEAK_GBS, 4),
                "bytes_per_launch": hbm_model_bytes,
                "basis": "bytes a streaming engine would move for the same column-iterations: "
                         "(8 nnz + 4 (n+1)) / B + 9 passes of 8 n bytes each"},
        },
    }
    log("SpMM rate (FP64 CSR SpMM, 100^3 grid, 64 columns)")
    line["spmm"] = spmm_rate()
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_runs} run(s)")
        line["cpu_baseline"] = cpu_baseline(csr, win, args.cpu_runs)
    ra.close()
    plain.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
