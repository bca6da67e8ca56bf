/*
 * rafeast.h -- RA-FEAST partial symmetric eigensolver on one AMD MI355X (gfx950).
 *
 * Computes the eigenpairs (lambda_i, v_i) of a real symmetric sparse matrix A
 * whose eigenvalues lie in a closed interval [lmin, lmax] (the partial
 * eigenproblem of eq. partial-eig, Section 1), by
 *   Phase 1  randomized warmstart: Gaussian sketch, power iterations with
 *            orthonormalisation, Rayleigh-Ritz truncation (Algorithm 2,
 *            eq. rand-range, eq. B-def);
 *   Phase 2  FEAST iterations: shifted solves (z_j I - A) X_j = RHS at the
 *            N_c quadrature nodes (eq. projector-quad), combination,
 *            orthonormalisation, Rayleigh-Ritz (Algorithm 1).
 * The shifted systems are solved matrix-free by COCG (conjugate orthogonal CG
 * for complex-symmetric matrices) on CSR sparse-matrix products.
 *
 * Conventions
 *  - Every call returns a rafeast_status; no exception crosses this ABI.
 *  - Host arrays in the high-level calls (rafeast_plan/warmstart/solve) are
 *    column-major n x k (element (i, c) at [c*n + i]) unless stated.
 *  - Device arrays in the step-level calls (rafeast_spmm ... rafeast_gaussian)
 *    are row-major n x k (element (i, c) at [i*ld + c]), allocated and owned
 *    by the caller, and must be valid on the current HIP device.
 *  - The caller owns every buffer it passes; the plan owns its own copies of
 *    A and all workspace.  A plan is not thread-safe; distinct plans are
 *    independent.  All work is enqueued on the plan's stream
 *    (rafeast_params.hip_stream, or a stream the plan creates when NULL);
 *    every call returns after its work on that stream has completed.  Device
 *    inputs must be complete when that stream reaches the call: work of the
 *    caller's on another stream that writes them is the caller's to finish
 *    (or order) first.
 */
#ifndef RAFEAST_H
#define RAFEAST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rafeast_status {
  RAFEAST_OK = 0,
  RAFEAST_INVALID_ARG = 1,        /* null pointer, n <= 0, lmin >= lmax, m0 < 1 or m0 > n,
                                     nc < 1 or nc > 64, q < 0, 0 <= p < 4 (Assumption 1.5),
                                     tolerances <= 0, unknown enum value */
  RAFEAST_BAD_CSR = 2,            /* rowptr not monotone, rowptr[0] != base, column out of
                                     range, columns unsorted or duplicated, non-finite value */
  RAFEAST_NOT_SYMMETRIC = 3,      /* pattern or values not symmetric:
                                     |a_ij - a_ji| > 1e-14 * ||A||_inf */
  RAFEAST_OOM = 4,                /* device allocation failed */
  RAFEAST_DEVICE = 5,             /* HIP runtime error or no usable device; see last_error */
  RAFEAST_NO_CONVERGENCE = 6,     /* max_iter reached; results are still written */
  RAFEAST_SUBSPACE_TOO_SMALL = 7, /* M >= m0: the window may hold more eigenvalues than the
                                     subspace; results are still written */
  RAFEAST_BREAKDOWN = 8,          /* COCG or orthonormalisation broke down and was not
                                     recovered; results are still written */
  RAFEAST_EMPTY_WINDOW = 9,       /* no Ritz value in the window (M = 0); a warning */
  RAFEAST_UNSUPPORTED = 10        /* valid request this build does not serve (reason in
                                     last_error) */
} rafeast_status;

/* rafeast_params.precision: arithmetic of the shifted solves. */
enum { RAFEAST_FP64 = 0,          /* complex FP64 COCG */
       RAFEAST_FP32_REFINED = 1 };/* complex FP32 COCG with FP64 true-residual updates */

/* rafeast_params.ws_op: Phase-1 operator (eq. B-def and Assumption 1.2). */
enum { RAFEAST_WS_AUTO = 0,       /* FLIP for a bottom window, LITERAL for a top window,
                                     FOLD for an interior window (Gershgorin bounds) */
       RAFEAST_WS_LITERAL = 1,    /* B = (A - lmin I)/(lmax - lmin) */
       RAFEAST_WS_FLIP = 2,       /* C = (s_hi I - A)/(s_hi - lmin) */
       RAFEAST_WS_FOLD = 3,       /* F = I - ((A - cI)/R)^2, c = window centre,
                                     R = max(c - s_lo, s_hi - c) */
       RAFEAST_WS_NONE = 4 };     /* plain FEAST start: orthonormalised sketch, no power steps */

/* rafeast_params.rhs_form: right-hand sides of the shifted solves. */
enum { RAFEAST_RHS_RESIDUAL = 0,  /* solve against Ritz residuals r_i and use
                                     (zI-A)^{-1} q = (q + (zI-A)^{-1} r)/(z - theta) */
       RAFEAST_RHS_LITERAL = 1 }; /* solve against the Ritz vectors q_i (Algorithm 1) */

/* rafeast_params.engine: COCG engine.  AUTO takes RESIDENT when n fits on
 * chip (n <= 8192 at FP32_REFINED, n <= 4096 at FP64, row lengths permitting)
 * and STREAM otherwise.  Both run the same method (COCG with reliable updates:
 * FP64 true-residual checks that keep the search direction) to the same
 * stopping test. */
enum { RAFEAST_ENGINE_AUTO = 0,
       RAFEAST_ENGINE_RESIDENT = 1,  /* one workgroup per system, vectors in LDS/registers */
       RAFEAST_ENGINE_STREAM = 2,    /* all systems in lock step, vectors in HBM, rows
                                        reordered by reverse Cuthill-McKee */
       RAFEAST_ENGINE_MULTISHIFT = 3 };/* precision FP64 and CSR plans only: the nc shifted
                                        systems of each right-hand side share one Krylov
                                        space, K(z_j I - A, b) = K(A, b); one real CG on
                                        the positive definite seed A - s I (s below the
                                        Gershgorin interval) drives them all, each with its
                                        own complex search direction and iterate, stopped
                                        at its own residual (|r_k| / |pi_k|, the shifted
                                        residual collinear with the seed's).  One real
                                        SpMV of the m0 columns per iteration instead of
                                        nc complex ones; vectors in HBM in the streaming
                                        engine's row order.  Never chosen by AUTO */
enum { RAFEAST_ENGINE_DIRECT = 4 };  /* precision FP64 and CSR plans only: standard FEAST
                                        with exact solves (Section 5.1's baseline): the plan
                                        factorizes each z_j I - A once as L D L^T
                                        (complex symmetric, no pivoting: Im z_j != 0 makes
                                        every pivot exist) in the band of the reverse
                                        Cuthill-McKee order, and every filter application
                                        solves by substitution.  Memory nc n (b + 1) complex
                                        doubles for bandwidth b (OOM when the device cannot
                                        hold it; BREAKDOWN if a pivot vanishes).  Reports
                                        zero COCG iterations.  Never chosen by AUTO */

/* rafeast_params.precond: preconditioner of the shifted solves. */
enum { RAFEAST_PC_NONE = 0,       /* unpreconditioned COCG on the plan's engine */
       RAFEAST_PC_LEARNED = 1 };  /* FP64 COCG preconditioned by the learned polynomial
                                     p_j(A) ~ (z_j I - A)^{-1} (weights from
                                     rafeast_pc_attach); plain COCG is the fallback */

/* rafeast_result.flags */
enum { RAFEAST_PTR_DEVICE = 1 };  /* lambda/resid/X are device pointers */

/* rafeast_result.t_ms phases */
enum { RAFEAST_PH_RR = 0, RAFEAST_PH_SOLVE = 1, RAFEAST_PH_COMBINE = 2, RAFEAST_PH_ORTH = 3,
       RAFEAST_PH_TOTAL = 4, RAFEAST_NPHASE = 5 };

typedef struct rafeast_plan_s* rafeast_plan_t;
typedef struct rafeast_batch_s* rafeast_batch_t;

/* Symmetric matrix in CSR, host memory.  The full symmetric pattern is
 * required (a triangle-only input fails the symmetry check).  Within a row,
 * column indices must be strictly increasing. */
typedef struct rafeast_csr {
  int64_t n;               /* order, 1 <= n < 2^31 */
  const int32_t* rowptr;   /* [n+1], rowptr[0] == index_base */
  const int32_t* colind;   /* [nnz], index_base-based */
  const double* values;    /* [nnz] */
  int32_t index_base;      /* 0 or 1 */
} rafeast_csr;

typedef struct rafeast_params {
  double lmin, lmax;       /* search interval (closed) */
  int32_t m0;              /* subspace size (>= number of eigenvalues in the window) */
  int32_t nc;              /* quadrature nodes on the upper half circle, 1..64 */
  int32_t q;               /* power iterations of Phase 1 (op applied 2q+1 times) */
  int32_t p;               /* oversampling; < 0 selects Remark 1's rule:
                              p = 10 if m0 <= 50 else min(20, ceil(m0/2)) */
  double tol_eig;          /* stop when every in-window Ritz pair has
                              ||A q - theta q|| / (max(|lmin|,|lmax|) ||q||) <= tol_eig */
  double tol_solve;        /* relative residual of each COCG solve */
  int32_t max_iter;        /* FEAST iterations (filter applications) */
  int32_t max_cocg;        /* COCG iterations per system, over all residual checks */
  int32_t precision;       /* RAFEAST_FP64 | RAFEAST_FP32_REFINED */
  int32_t ws_op;           /* RAFEAST_WS_* */
  int32_t rhs_form;        /* RAFEAST_RHS_* */
  int32_t engine;          /* RAFEAST_ENGINE_* */
  uint64_t seed;           /* Philox key of the device-generated sketch */
  void* hip_stream;        /* hipStream_t to run on; NULL: the plan creates its own */
  double tol_solve_relaxed; /* Phase 2 with relaxed solves (Section 3.3: k_inexact, from
                              relaxed tolerances; Theorem 2).  0, or a value <= tol_solve:
                              every solve uses tol_solve.  A value in (tol_solve, 1):
                              the solves of each rafeast_solve start at this relative
                              tolerance, and whenever a filter application fails to halve
                              the largest counted residual the tolerance drops 100-fold,
                              not below tol_solve.  Needs rhs_form RESIDUAL, whose solve
                              error scales with the Ritz residual (a literal-form solve
                              error sets a floor near the tolerance) */
  int32_t precond;         /* RAFEAST_PC_NONE | RAFEAST_PC_LEARNED.  LEARNED (CSR plans
                              only): in every FEAST iteration the library forms each node's
                              features (Re z^_j, Im z^_j, theta^_lo, theta^_hi) from the
                              current Ritz values, evaluates the attached network for the
                              coefficients of p_j, and solves all (node, column) systems by
                              FP64 COCG preconditioned with p_j(A), to the true residual
                              ||b - (z_j I - A) x|| <= tol ||b||.  A system that does not
                              reach it (iteration budget, breakdown) is solved again by
                              plain FP64 COCG (counted in rafeast_result.pc_fallbacks) */
} rafeast_params;

/* Phase-1 diagnostics (Remark 1's post-hoc check of the power-count condition,
 * eq. power-cond): op-Ritz estimates of beta_{m0}, beta_{m0+1}, and the
 * warmstart error bound of Theorem 1 evaluated with them. */
typedef struct rafeast_ws_info {
  double beta_m0;
  double beta_m0p1;        /* NaN when p == 0 */
  double ratio;            /* (beta_m0p1 / beta_m0)^(2q+1) */
  int32_t op;              /* the RAFEAST_WS_* operator actually used */
  double t_ms;             /* device time of Phase 1 */
  double r_halko;          /* eq. R-Halko at failure probability delta = 0.01:
                              C1 sqrt(1 + m0/(p-1)) beta_m0p1 (beta_m0p1/beta_m0)^(2q),
                              C1 = 1 + (p/2) ln(2 m0 / delta); NaN when p < 2 */
  double gap;              /* delta_gap = beta_m0 - beta_m0p1 (eq. gap-def) */
  double proj_bound;       /* r_halko / gap, the bound on ||P - P~||_2 of Theorem 1
                              (eq. warmstart-error); Remark 1 asks for <= 1/2 */
} rafeast_ws_info;

typedef struct rafeast_result {
  int32_t flags;           /* in: RAFEAST_PTR_DEVICE or 0 */
  double* lambda;          /* in: [m0] buffer; out: first M entries, ascending */
  double* resid;           /* in: [m0] buffer; out: scaled residuals of those pairs */
  double* X;               /* in: nullable [n*m0] buffer; out: n x M column-major unit
                              eigenvectors, largest-magnitude entry positive */
  int32_t M;               /* out: eigenvalues found in [lmin, lmax] */
  int32_t iters;           /* out: FEAST filter applications performed */
  int64_t cocg_iters;      /* out: COCG iterations summed over all systems */
  int32_t cocg_max;        /* out: largest COCG iteration count of one system */
  int32_t refinements;     /* out: FP64 true-residual checks that continued the
                              iteration, summed over all systems */
  double max_resid;        /* out: max scaled residual over the M pairs */
  double t_ms[RAFEAST_NPHASE]; /* out: device time per phase (HIP events) */
  double tol_solve_last;   /* out: COCG tolerance of the last filter application
                              (the starting one when none ran) */
  int64_t cocg_node[64];   /* out: COCG iterations per quadrature node (first nc entries,
                              in the node order of rafeast_plan_info), summed over columns
                              and FEAST iterations; preconditioned iterations count once */
  int32_t pc_fallbacks;    /* out: systems re-solved by plain COCG after the learned
                              preconditioner missed the tolerance (precond LEARNED) */
} rafeast_result;

/* Fills *p with defaults: m0 = 0 (must be set), nc = 8, q = 2, p = -1,
 * tol_eig = 1e-10, tol_solve = 1e-6, max_iter = 20, max_cocg = 20000,
 * precision FP32_REFINED, ws_op AUTO, rhs_form RESIDUAL, engine AUTO, seed 0,
 * tol_solve_relaxed 0 (fixed tolerance), precond NONE. */
void rafeast_params_default(rafeast_params* p);

/* Validates A and the parameters, copies A to the device (FP64 values plus an
 * FP32 shadow), computes the Gershgorin interval and the quadrature table
 * (Gauss-Legendre on the upper half circle over [lmin, lmax]; eq. projector-quad),
 * and allocates all workspace.  On success *out owns everything; release it
 * with rafeast_destroy.  On failure *out is NULL and the status says why
 * (rafeast_last_error(NULL) holds the text). */
rafeast_status rafeast_plan(const rafeast_csr* A, const rafeast_params* prm, rafeast_plan_t* out);

/* Plans for the statistical applications of Section 4, whose operators are
 * dense: the same Phase 1 / Phase 2 calls (rafeast_warmstart, rafeast_solve,
 * rafeast_destroy, ...) then run with A applied as a matrix product (two for
 * the covariance form) instead of a sparse one, on the streaming COCG engine
 * (prm->engine AUTO or STREAM; RESIDENT is UNSUPPORTED).  Top windows suit
 * the literal warmstart operator (Assumption 1.3); ws_op AUTO picks it when
 * lmax reaches the upper spectral bound.  The learned-preconditioner calls and
 * the batching form take CSR plans only (UNSUPPORTED otherwise).
 *
 * rafeast_plan_dense: A = K, the kernel matrix of kernel PCA (eq.
 * kernel-eig).  K: host, n x n, column-major with leading dimension ldk >= n,
 * symmetric to 1e-14 relative (NOT_SYMMETRIC otherwise) and finite (BAD_CSR
 * otherwise, the status of malformed input); 1 <= n < 2^31.  The plan copies
 * K to the device (FP64, plus an FP32 copy for the FP32 engine).  Spectral
 * bounds: Gershgorin discs of K.  rafeast_plan_info reports nnz = n^2. */
rafeast_status rafeast_plan_dense(int64_t n, const double* K, int64_t ldk,
                                  const rafeast_params* prm, rafeast_plan_t* out);

/* rafeast_plan_gram: A = scale X^T X, the sample covariance of eq.
 * sample-cov with scale = 1/(rows - 1) (any scale > 0 is accepted).  X: host,
 * rows x n data matrix (rows samples of n features), column-major with
 * leading dimension ldx >= rows, finite; A (order n) is never formed: each
 * application is X^T (X V).  Spectral bounds: [0, scale ||X||_F^2] (A is
 * positive semidefinite and its largest eigenvalue is at most its trace).
 * rafeast_plan_info reports nnz = rows * n. */
rafeast_status rafeast_plan_gram(int64_t rows, int64_t n, const double* X, int64_t ldx,
                                 double scale, const rafeast_params* prm, rafeast_plan_t* out);

/* Phase 1 of Algorithm 2.  omega: nullable host array, column-major
 * n x (m0+p), the Gaussian sketch; NULL draws it on the device from
 * Philox4x32-10 keyed by prm.seed (rafeast_gaussian).  The op (chosen by
 * ws_op) is applied 2q+1 times with CholQR2 after each application; then
 * Rayleigh-Ritz of A on the result keeps the m0 Ritz vectors with the largest
 * |op| values.  With ws_op NONE the start is the orthonormalised first m0
 * sketch columns.  The start block stays in the plan for rafeast_solve.
 * Q0: nullable host n x m0 column-major output copy.  info: nullable. */
rafeast_status rafeast_warmstart(rafeast_plan_t plan, const double* omega, double* Q0,
                                 rafeast_ws_info* info);

/* Phase 2 (Algorithms 1/2).  Q_init: nullable host n x m0 column-major start
 * block (orthonormalised on entry; a checkpointed subspace resumes the
 * iteration).  NULL uses the block of the last rafeast_warmstart if no solve
 * has consumed it, otherwise the orthonormalised first m0 columns of the
 * device sketch (the ws_op NONE start).  Each iteration: Rayleigh-Ritz and residuals;
 * stop test; shifted COCG solves for all (node, column) pairs; combination
 * Q~ = sum_j Re[w_j (z_j I - A)^{-1} Q]; CholQR2.  Writes *res as documented
 * in rafeast_result.  Returns OK, NO_CONVERGENCE, SUBSPACE_TOO_SMALL,
 * EMPTY_WINDOW or BREAKDOWN with results written, or an error.  With the
 * environment variable RAFEAST_VERBOSE set (not "0"), one progress line per
 * iteration goes to stderr. */
rafeast_status rafeast_solve(rafeast_plan_t plan, const double* Q_init, rafeast_result* res);

/* Releases the plan and all its device memory.  NULL is a no-op. */
void rafeast_destroy(rafeast_plan_t plan);

/* Text of the last error on this plan (or of the last failed rafeast_plan when
 * plan is NULL).  Valid until the next call on the same plan. */
const char* rafeast_last_error(rafeast_plan_t plan);

/* Static name of a status code.  Takes any int: a value that is not one of
 * the rafeast_status codes gives "UNKNOWN". */
const char* rafeast_status_string(int s);

/* Gershgorin interval, ||A||_inf, nnz and the quadrature table of a plan.
 * z and w: nullable host arrays of 2*nc doubles (re, im interleaved), the
 * nodes in order of increasing |Im z| (the order the solves use; the filter
 * sum does not depend on it).  Dense plans: nnz = n^2 (rafeast_plan_dense)
 * or rows * n (rafeast_plan_gram), and for the covariance form the bound
 * scale ||X||_F^2 in place of ||A||_inf. */
rafeast_status rafeast_plan_info(rafeast_plan_t plan, double* sig_lo, double* sig_hi,
                                 double* anorm_inf, int64_t* nnz, double* z, double* w);

/* The COCG engine the plan resolved (RAFEAST_ENGINE_RESIDENT, _STREAM or
 * _MULTISHIFT); 0 for a NULL plan. */
int32_t rafeast_plan_engine(rafeast_plan_t plan);

/* The launch shape rafeast_plan chose by measurement (autotuning; the
 * batching form's tuned SpMM tiles).  Resident engine: the SELL slices each
 * thread holds (1, 2, 4 or 8; it fixes the slice-to-wave table), every count
 * from the smallest that fits up to the maximum timed on the plan's own
 * matrix (64 COCG iterations of the first min(systems, CUs) systems on
 * Gaussian right-hand sides); the fastest is used.  RAFEAST_TUNE=0 in the
 * environment keeps the smallest; RAFEAST_RESIDENT_SLOTS=r takes candidate r
 * untimed (rafeast_plan fails with INVALID_ARG if r is not a candidate).  The
 * count sets the order of the SpMV's row sums, so plans with equal counts
 * give bitwise equal results.  Out: *chosen (0 for the streaming engine,
 * which is not tuned), *count candidates, and up to max of them in cand[]
 * with their measured milliseconds in ms[] (0 when untimed: a single
 * candidate or tuning off).  Host pointers owned by the caller.  Errors:
 * INVALID_ARG for a NULL plan, chosen or count, max < 0, or NULL cand/ms
 * with max > 0. */
rafeast_status rafeast_plan_tuning(rafeast_plan_t plan, int32_t* chosen, int32_t* count,
                                   int32_t* cand, float* ms, int32_t max);

/* Reverse Cuthill-McKee order of the graph of A (host only, needs no
 * device): per connected component, breadth-first search from a
 * pseudo-peripheral vertex (George-Liu), neighbours by increasing degree, the
 * whole sequence reversed.  perm: caller-allocated host [n], perm[new] = old,
 * 0-based.  The streaming engine renumbers rows with it.  A is validated as
 * in rafeast_plan (BAD_CSR, NOT_SYMMETRIC, INVALID_ARG). */
rafeast_status rafeast_rcm_order(const rafeast_csr* A, int32_t* perm);

/* ---------------------------------------------------------------------------
 * Step-level calls on caller-owned device buffers (row-major, see top).  They
 * use the plan's matrix, stream and workspace and serve the tests of each
 * stage of the method.
 * ------------------------------------------------------------------------- */

/* Y = alpha * A X + beta * X for an n x k block (FP64).  X != Y. */
rafeast_status rafeast_spmm(rafeast_plan_t plan, int32_t k, const double* X, int32_t ldx,
                            double* Y, int32_t ldy, double alpha, double beta);

/* G = X^T Y (k1 x k2 row-major, ldg >= k2) for n x k1 X and n x k2 Y (FP64,
 * MFMA f64 split over row chunks, fixed-order final sum).  n is arbitrary. */
rafeast_status rafeast_gram(rafeast_plan_t plan, int64_t n, int32_t k1, int32_t k2,
                            const double* X, int32_t ldx, const double* Y, int32_t ldy,
                            double* G, int32_t ldg);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the Gram
 * product of rafeast_gram without a plan and without any allocation.
 * G = X^T Y (k1 x k2 row-major, ldg >= k2) for device arrays X (n x k1, ldx)
 * and Y (n x k2, ldy), FP64, enqueued on hip_stream (NULL: the null stream)
 * of the current device; the call returns after enqueueing and does not
 * wait.  The row-chunk partial sums go to a fixed scratch array of 2^21
 * doubles (16 MiB) that the library holds on each device it runs on until
 * the process ends: k1 * k2 must not exceed 2^21 (INVALID_ARG otherwise,
 * text in rafeast_last_error(NULL)); it uses as many row chunks as
 * rafeast_gram when they fit (then the results are identical), fewer
 * otherwise.  Every call on a device shares that device's scratch, so calls
 * that overlap on one device (concurrent streams or threads) race; serialise
 * them.  Errors: INVALID_ARG for null pointers, n < 1, k1 < 1, k2 < 1 or
 * ld < k; DEVICE for a HIP error. */
rafeast_status rafeast_gram_noalloc(void* hip_stream, int64_t n, int32_t k1, int32_t k2,
                                    const double* X, int32_t ldx, const double* Y, int32_t ldy,
                                    double* G, int32_t ldg);

/* C = alpha op(A) B + beta C on the matrix cores: the product form of the
 * dense operators of Section 4 (kernel matrix, eq. kernel-eig: K X; sample
 * covariance, eq. sample-cov: Xd^T (Xd X) / (rows - 1)).  C (M x N, ldc >= N)
 * and B (K x N, ldb >= N) row-major; op(A) M x K stored by rows (a_cols = 0:
 * op(A)(i, k) = A[i lda + k], lda >= K) or by columns (a_cols = 1:
 * A[k lda + i], lda >= M).  precision RAFEAST_FP64 (double buffers,
 * v_mfma_f64_16x16x4f64) or RAFEAST_FP32_REFINED (float buffers,
 * v_mfma_f32_16x16x4f32); alpha and beta are rounded to the buffers' type.
 * All pointers device, caller-owned (A and B may be null when K == 0, C when
 * M N == 0); beta == 0 does not read C.  A long inner
 * dimension with few output tiles is split into chunks summed in a fixed
 * order in a workspace this call allocates and frees.  Runs on hip_stream
 * (nullable: the null stream) and waits for it.  Errors: INVALID_ARG for null
 * pointers, negative sizes, short leading dimensions or another precision;
 * OOM; DEVICE. */
rafeast_status rafeast_gemm(void* hip_stream, int32_t precision, int32_t a_cols, int32_t M,
                            int32_t N, int32_t K, const void* A, int64_t lda, const void* B,
                            int64_t ldb, void* C, int64_t ldc, double alpha, double beta);

/* CholQR2 of an n x k block in place (Y <- Y R^{-1}, twice), k <= 192, with
 * column scaling; when the first Cholesky fails, the shifted variant is used
 * and a third pass added.  *info (host, nullable): 0 plain, 1 shifted,
 * 2 failed (Y unchanged from the last good pass). */
rafeast_status rafeast_cholqr2(rafeast_plan_t plan, int64_t n, int32_t k, double* Y, int32_t ldy,
                               int32_t* info);

/* Symmetric eigendecomposition of a k x k matrix H (k <= 192, read-only;
 * the symmetric part is used) by parallel cyclic Jacobi in FP64: theta[k]
 * ascending, S k x k row-major with column c the unit eigenvector of theta[c]. */
rafeast_status rafeast_syev(rafeast_plan_t plan, int32_t k, const double* H, double* theta,
                            double* S);

/* Shifted solves (z_j I - A) X_{j,c} = B_c for nz shifts and k right-hand
 * sides by COCG at the plan's precision and engine.  z: host [2*nz] (re, im).
 * B: device n x k FP64.  X: device n x (nz*k) complex (re, im interleaved),
 * FP64 when the plan's precision is FP64, FP32 otherwise; column j*k + c.
 * The solution is accumulated in FP64 and rounded to X's precision on output.
 * iters: nullable host [nz*k] COCG iterations per system.  resid: nullable
 * host [nz*k], ||B_c - (z_j I - A) x|| / ||B_c|| of the FP64 solution (the
 * stopping test is resid <= tol, tol relative).  Zero right-hand sides give
 * zero solutions.  A system whose COCG breaks down (p^T (z_j I - A) p = 0, or
 * a non-finite step) restarts from its true residual; after the fourth
 * breakdown it stops with its last FP64 solution and residual (resid > tol
 * tells the caller; the status stays OK).  The multi-shift engine takes
 * shifts off the real axis only (INVALID_ARG for Im z_j == 0): it divides by
 * the seed's residual polynomial at z_j, which has real roots. */
rafeast_status rafeast_shifted_solve(rafeast_plan_t plan, int32_t nz, const double* z, int32_t k,
                                     const double* B, int32_t ldb, void* X, double tol,
                                     int32_t* iters, double* resid);

/* Gaussian sketch Omega (n x w, FP64) from Philox4x32-10 and Box-Muller:
 * entry (i, c) uses counter (i lo, i hi, c/2, 0) and key (seed lo, seed hi);
 * u1, u2 are the two 64-bit output halves mapped to (0, 1) with 53 bits;
 * even c takes sqrt(-2 ln u1) cos(2 pi u2), odd c the sin. */
rafeast_status rafeast_gaussian(rafeast_plan_t plan, int32_t w, uint64_t seed, double* Omega,
                                int32_t ld);

/* ---------------------------------------------------------------------------
 * Batching form: many independent problems (matrix, window, parameters) run
 * their FEAST iterations in lock step.  In each iteration the shifted
 * systems of every member that fits on chip (the resident engine) are solved
 * in one persistent launch, replayed from a captured HIP graph: its work
 * items are (member, node, column) triples, longest first across members.
 * Members too large for the resident engine whose engine is AUTO run the
 * multi-shift engine in FP64 (others the engine they name), after that
 * launch, concurrently with each other.  The Rayleigh-Ritz,
 * combination and CholQR2 steps run per member.  Each member computes
 * exactly what rafeast_solve computes for it.
 * ------------------------------------------------------------------------- */

/* Plans count >= 1 problems: A[g] with prm[g] (host arrays of count).  All
 * members must share precision, tol_solve and max_cocg (INVALID_ARG
 * otherwise).  prm[0].hip_stream (or a stream the batch creates) carries the
 * shared launch; every member gets a stream of its own (owned by the batch;
 * the members' hip_stream fields are ignored), and the members outside the
 * shared launch solve concurrently from host worker threads.  Errors as rafeast_plan, for the first member
 * that fails (the text names it). */
rafeast_status rafeast_plan_batch(int32_t count, const rafeast_csr* A, const rafeast_params* prm,
                                  rafeast_batch_t* out);

/* The plan of member g (0 <= g < count; NULL otherwise), owned by the batch:
 * use it for rafeast_warmstart, rafeast_plan_info or rafeast_plan_engine;
 * do not destroy it or call rafeast_solve on it while the batch is in use. */
rafeast_plan_t rafeast_batch_plan(rafeast_batch_t batch, int32_t g);

/* Phase 2 for all members.  Q_init: nullable host array of count nullable
 * start blocks (as rafeast_solve).  res: host array of count results, each
 * set up as for rafeast_solve.  status: nullable host [count], each member's
 * rafeast_solve status.  t_ms: nullable host [RAFEAST_NPHASE], the batch's
 * device time per phase: RR summed over members, SOLVE the shared launch
 * plus the streaming-engine solves, COMBINE the members' combination and
 * CholQR2 together (ORTH is 0), TOTAL.  Returns OK when every member returned OK, else
 * the first non-OK member status (all members' results are written);
 * failures of the device or arguments return at once. */
rafeast_status rafeast_batch_solve(rafeast_batch_t batch, const double* const* Q_init,
                                   rafeast_result* res, rafeast_status* status, double* t_ms);

/* Members that ran on the resident engine in the shared launch. */
int32_t rafeast_batch_resident_count(rafeast_batch_t batch);

/* Releases the batch and its member plans.  NULL is a no-op. */
void rafeast_batch_destroy(rafeast_batch_t batch);

/* Text of the last error on the batch (NULL: the last failed
 * rafeast_plan_batch). */
const char* rafeast_batch_last_error(rafeast_batch_t batch);

/* ---------------------------------------------------------------------------
 * Learned polynomial preconditioner for the shifted solves (an addition to
 * the paper's method, which solves (z_j I - A) d = r unpreconditioned;
 * Section 2.1).  p(A) = sum_{k<8} c_k T_k(A^), A^ = a A + b I mapping the
 * plan's Gershgorin interval [lo, hi] onto [-1, 1] (a = 2/(hi - lo),
 * b = -(hi + lo)/(hi - lo)), T_k the Chebyshev polynomials, c_k complex.
 * The coefficients come from a network 4 -> 64 -> 64 -> 64 -> 16 (exact
 * GELU on the hidden layers) of the features (Re z^, Im z^, theta^_lo,
 * theta^_hi): the shift and the smallest and largest current Ritz values,
 * mapped like A.  The 16 outputs y are the coefficients scaled by the
 * shift's distance from the real axis: c_k = (y_2k + i y_2k+1) / Im z^ (the
 * coefficients of a good p grow like 1 / Im z^; scaled they are O(1)).
 * Parameters: rafeast_pc_param_count() floats, per layer W (out x in,
 * row-major) then b; used in BF16 (round to nearest even) with FP32 sums,
 * trained in FP32.  All arrays below are device pointers unless marked host.
 * ------------------------------------------------------------------------- */

/* Number of network parameters (9688): the 9680 weights and biases, then
 * the input standardization mu[4], sd[4]: each feature x_f enters the network
 * as (x_f - mu_f) / sd_f, in FP64 before the BF16 rounding of the inputs
 * (the mapped features of a window at the end of a wide spectrum differ by
 * less than a BF16 ulp); mu = 0, sd = 1 is the identity. */
int32_t rafeast_pc_param_count(void);

/* Sets the input standardization of W (device, rafeast_pc_param_count()
 * FP32) to the mean and standard deviation of each feature over the ns rows
 * X (device, ns x 4 FP64); sd = 1 for a feature whose standard deviation is
 * at most 1e-9 max(1, |mean|) (constant up to rounding).  Call before
 * rafeast_pc_train, which leaves it unchanged.  Errors: INVALID_ARG. */
rafeast_status rafeast_pc_normalize(rafeast_plan_t plan, int32_t ns, const double* X, float* W);

/* Training samples from k real residual vectors R (n x k FP64, row-major,
 * ldr) at nz shifts z (host, 2*nz): sample s = j*k + i has features X[s][4],
 * G[s] (8 x 8 complex, re/im interleaved, row-major), h[s] (8 complex) and
 * rr[s] with v_l = (z_j I - A) T_l(A^) R[:, i], G_lm = v_l^H v_m,
 * h_l = v_l^H R[:, i], rr = ||R[:, i]||^2.  The loss of coefficients c is
 * ||(zI - A) p(A) r - r||^2 / ||r||^2 = (c^H G c - 2 Re(c^H h) + rr) / rr. */
rafeast_status rafeast_pc_samples(rafeast_plan_t plan, int32_t nz, const double* z, int32_t k,
                                  const double* R, int32_t ldr, double theta_lo, double theta_hi,
                                  double* X, double* G, double* h, double* rr);

/* Network outputs Y[s][16] (FP32, the scaled coefficients y; c = y / X[s][1]
 * as above) of features X[s][4] for s < ns; W: FP32 parameters (used in BF16). */
rafeast_status rafeast_pc_forward(rafeast_plan_t plan, int32_t ns, const double* X, const float* W,
                                  float* Y);

/* Gradient grad[rafeast_pc_param_count()] (FP32) of the mean loss over the
 * ns samples at parameters W (zero for the standardization); loss: nullable
 * host, the mean loss. */
rafeast_status rafeast_pc_gradient(rafeast_plan_t plan, int32_t ns, const double* X,
                                   const double* G, const double* h, const double* rr,
                                   const float* W, float* grad, double* loss);

/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) on the weights of W
 * (not the standardization) in place for
 * `steps` minibatches of `batch` samples; order: host [steps * batch]
 * sample indices (< ns).  loss: nullable host [steps], each minibatch's mean
 * loss before its step. */
rafeast_status rafeast_pc_train(rafeast_plan_t plan, int32_t ns, const double* X, const double* G,
                                const double* h, const double* rr, float* W, int32_t steps,
                                int32_t batch, const int32_t* order, float lr, double* loss);

/* Training samples from the solver's own residuals: the COCG residual
 * vectors of the plan's shifted systems.  The right-hand sides are the Ritz
 * residual block R = A Q - Q Theta of the plan's last Rayleigh-Ritz step
 * (k = m0 columns: the end of the last rafeast_solve, e.g. one run with
 * max_iter 0 or 1), at the plan's quadrature nodes (in the order of
 * rafeast_plan_info).  For each of the nsteps counts s = steps[t] >= 0, plain
 * FP64 COCG runs exactly s iterations on all nc * m0 systems, and every
 * residual vector r of node j gives samples at that node's shift z_j (as
 * rafeast_pc_samples, features with theta_lo, theta_hi the smallest and
 * largest Ritz values of that step): s = 0 gives the m0 real right-hand
 * sides per node, s > 0 the real and the imaginary part of each complex
 * residual (2 m0 per node).  X[4], G[8][8] complex, h[8] complex, rr per
 * sample: caller-owned device buffers with room for
 * sum_t (steps[t] == 0 ? 1 : 2) * nc * m0 samples; *count (host) receives
 * the number written.  Errors: INVALID_ARG (null pointers, nsteps < 1, a
 * negative step, or no Rayleigh-Ritz step yet), UNSUPPORTED for dense plans. */
rafeast_status rafeast_pc_harvest(rafeast_plan_t plan, int32_t nsteps, const int32_t* steps,
                                  double* X, double* G, double* h, double* rr, int32_t* count);

/* Attaches network parameters W (device, rafeast_pc_param_count() FP32
 * values, as trained by rafeast_pc_train) to the plan: the plan copies them
 * and keeps a BF16 copy for the solves with precond LEARNED.  Errors:
 * INVALID_ARG for null pointers, UNSUPPORTED for dense plans. */
rafeast_status rafeast_pc_attach(rafeast_plan_t plan, const float* W);

/* COCG in FP64 for (z_j I - A) X_{j,c} = B_c (nz shifts, k right-hand
 * sides, B n x k FP64 row-major, ldb), preconditioned by p(A) with coef
 * (host [nz][8] complex, re/im interleaved; NULL: no preconditioner), all
 * systems in lock step, to true residual ||b - (zI - A) x|| <= tol ||b||
 * or max_cocg iterations.  X: n x (nz*k) complex FP64, column j*k + c.
 * iters, resid: nullable host [nz*k]. */
rafeast_status rafeast_pc_solve(rafeast_plan_t plan, int32_t nz, const double* z, int32_t k,
                                const double* B, int32_t ldb, const double* coef, void* X,
                                double tol, int32_t* iters, double* resid);

#ifdef __cplusplus
}
#endif

#endif /* RAFEAST_H */
