// Host-side launchers of the RA-FEAST kernels.  Every launcher enqueues on
// `st` and returns the launch status; none synchronises.  Blocks are
// row-major (element (i, c) at [i * ld + c]).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "device.h"  // cpx<T>

namespace rafeast {

// ---- sparse x dense (FP64, real) ------------------------------------------
// Y = alpha * A X + beta * X + gamma * X2 (X2 may be null), CSR A (FP64).
// span: max |i - j| over the nonzeros a_ij (0: unknown); it sets how many
// columns one sweep over the rows gathers (spmm_group_cols).
hipError_t launch_spmm_f64(hipStream_t st, int n, int k, const int* rowptr, const int* col,
                           const double* val, int64_t nnz, const double* X, int ldx, double* Y,
                           int ldy, double alpha, double beta, const double* X2, int ldx2,
                           double gamma, int64_t span);
int spmm_group_cols(int k, int64_t span);

// ---- tall-skinny products (FP64 MFMA) ----------------------------------------
// Number of row chunks the Gram splits n into, and the partial buffer it needs.
int gram_chunks(int64_t n);
size_t gram_partial_doubles(int64_t n, int k1, int k2);
// G = X^T Y; `part` holds gram_partial_doubles(n, k1, k2) doubles.
hipError_t launch_gram(hipStream_t st, int64_t n, int k1, int k2, const double* X, int ldx,
                       const double* Y, int ldy, double* G, int ldg, double* part);
// The same with an explicit number of row chunks (clamped to [1, gram_chunks(n)]);
// `part` holds chunks * k1 * k2 doubles.
hipError_t launch_gram_chunks(hipStream_t st, int64_t n, int k1, int k2, const double* X,
                              int ldx, const double* Y, int ldy, double* G, int ldg, double* part,
                              int chunks);
// Y = X S, X n x k, S k x k2 (row-major, lds), Y n x k2.  Y must not alias X.
hipError_t launch_tsmm(hipStream_t st, int64_t n, int k, int k2, const double* X, int ldx,
                       const double* S, int lds, double* Y, int ldy);

// ---- Rayleigh-Ritz residual ---------------------------------------------------
// R = W - Q diag(theta); res[c] = ||R_c|| / (s_win ||Q_c||); qn[c] = ||Q_c||.
// `part` holds 2 * k * gram_chunks(n) doubles.
hipError_t launch_residual(hipStream_t st, int64_t n, int k, const double* W, const double* Q,
                           int ld, const double* theta, double s_win, double* R, double* res,
                           double* qn, double* part);

// ---- filter combination ------------------------------------------------------
// gamma[j*k + i] = w_j / (z_j - theta_i) (complex, re/im interleaved).
hipError_t launch_gamma(hipStream_t st, int nc, int k, const double* zw /*[4*nc]: z, w*/,
                        const double* theta, double* gamma);
// Residual form:  Qt[r][i] = sum_j Re[gamma_ji (Q[r][i] + D[r][j*k+i])]
// Literal form:   Qt[r][i] = sum_j Re[w_j D[r][j*k+i]]
// D is complex (FP32 if d32 else FP64), row-major with ldd complex entries.
hipError_t launch_combine(hipStream_t st, int64_t n, int nc, int k, const double* gamma,
                          const double* zw, bool residual_form, const double* Q, int ldq,
                          const void* D, int ldd, bool d32, double* Qt, int ldt);

// ---- Gaussian sketch (Philox4x32-10 + Box-Muller) ---------------------------
hipError_t launch_gaussian(hipStream_t st, int64_t n, int w, uint64_t seed, double* O, int ld);

// ---- layout helpers -----------------------------------------------------------
// dst (row-major, ldd) <- src (column-major n x k, ld n) and back.
hipError_t launch_colmajor_to_rowmajor(hipStream_t st, int64_t n, int k, const double* src,
                                       double* dst, int ldd);
// dst (column-major n x cnt) <- columns sel[0..cnt) of src, each scaled to unit
// norm with its largest-magnitude entry positive (lowest index on ties).
// `part` holds 3 * cnt * gram_chunks(n) doubles + cnt ints of scratch.
hipError_t launch_export_vectors(hipStream_t st, int64_t n, int cnt, const int* sel,
                                 const double* src, int lds, double* dst, double* part);
// dst[:, 0..k) = src[:, 0..k); with status, nothing is written when *status
// is 2 (the failed Cholesky of a CholQR pass).
hipError_t launch_copy_cols(hipStream_t st, int64_t n, int k, const double* src, int lds,
                            double* dst, int ldd, const int* status = nullptr);
// p[0..n) = v by a kernel (usable inside a captured graph, unlike a memset).
hipError_t launch_fill_int(hipStream_t st, int* p, int v, int n);

// ---- small dense (one workgroup) ------------------------------------------------
// M such that Y M has orthonormal columns for G = Y^T Y (k x k): column
// scaling, Cholesky (shifted when it fails), triangular inverse.  flag: 0 ok,
// 1 shifted, 2 failed (M = diagonal scaling).
hipError_t launch_chol_inv(hipStream_t st, int k, int64_t nrows, const double* G, int ldg,
                           double* M, int ldm, int* flag);
// Parallel cyclic Jacobi: theta ascending, S row-major (column c = vector c).
// `work` holds 2 * k * k doubles.
hipError_t launch_jacobi(hipStream_t st, int k, const double* H, int ldh, double* theta,
                         double* S, int lds, double* work);
// Keep the m0 of k Ritz values with the largest |phi(theta)|,
// phi(t) = a + b t + c t^2; Ssel (k x m0) <- the kept columns of S in
// ascending-theta order; info[0] = m0-th largest |phi|, info[1] = (m0+1)-th.
hipError_t launch_select(hipStream_t st, int k, int m0, const double* theta, const double* S,
                         int lds, double a, double b, double c, double* Ssel, double* info);

// ---- COCG ---------------------------------------------------------------------
// SELL-64 copy of A for the resident COCG engine.  Rows are reordered by
// decreasing length (slot s holds row perm[s]; slots >= n are empty) and cut
// into slices of 64 slots.  FP64 entries are stored entry-major within a
// slice (the k-th entries of the 64 rows contiguous, 16 B per lane); FP32
// entries are stored pair-major (entries 2j and 2j+1 of a row adjacent, then
// the next row's pair), so one 16-byte lane load fetches two entries: the
// per-CU load rate from L2 is set by load instructions, not bytes.  An entry's column is
// stored as the byte offset of its slot in a complex vector of the entry's
// precision (slot * 8 for FP32 complex, slot * 16 for FP64 complex), so a
// gather needs no address arithmetic.  Slice widths are padded to a multiple
// of 4 with (own slot, 0).
struct SellEntry64 {
  int c;    // slot * 16
  int pad;
  double v;
};
struct SellMatrix {
  int n = 0;
  int nslices = 0;
  const int* sbase = nullptr;           // [nslices+1] entry offsets (multiples of 256)
  const int* perm = nullptr;            // [nslices*64] slot -> row (-1: empty slot)
  // FP32 entries: n32 values, then n32 uint16 LDS byte offsets (slot * 8).
  // A slice of width w holds w / 8 octs of 512 entries (values: two halves
  // of 64 lanes x 4; offsets: 64 lanes x 8), then a quad of 256 entries
  // (64 lanes x 4) if w % 8 == 4.
  const float* v32 = nullptr;
  int n32 = 0;
  const SellEntry64* e64 = nullptr;     // FP64 entries
  int zero_base = 0;                    // 256 entries (slot 0, value 0) start here
  const int* wave_slices = nullptr;     // [waves * wave_rpt] slice of each wave slot, -1 none
  int wave_rpt = 0;                     // slots per wave (1, 2, 4 or 8)
};

// One matrix (graph) of a resident launch, with the right-hand sides and
// outputs of its systems.  An item (g, j, i) solves (z_j I - A_g) d = B_g[:, i]
// into column j * kcols + i of D_g.
struct ResGraph {
  int nslices = 0;
  int zero_base = 0;
  int ldb = 0;
  int kcols = 0;                        // RHS columns of this graph
  int ldd = 0;
  int n32 = 0;                          // FP32 entry count (offsets follow the values)
  const int* sbase = nullptr;           // SellMatrix fields of A_g
  const int* perm = nullptr;
  const void* ent = nullptr;            // FP32 values (+ offsets) or SellEntry64
  const SellEntry64* ent64 = nullptr;
  const int* wave_slices = nullptr;     // table built for the launch's slots per wave
  const double* B = nullptr;            // n_g x kcols RHS (FP64), ldb
  void* D = nullptr;                    // n_g x (nz kcols) complex outputs, ldd
  const double* zs = nullptr;           // shifts (re, im)
  int* iters = nullptr;                 // [nz kcols] iterations per system
  double* resid = nullptr;              // nullable [nz kcols] final relative true residual
  int* stats = nullptr;                 // [2]: continued checks, breakdowns (accumulated)
  double tol = 0.0;                     // relative residual tolerance of this graph's systems
};

struct CocgLaunch {
  int nitems = 0;
  const int* items = nullptr;   // [3*nitems] (graph g, shift j, column i), longest first
  double tol = 1e-6;
  int maxit = 20000;
  int max_refine = 64;          // FP64 residual checks per system
  int* counter = nullptr;       // zeroed work counter
  void* xhi = nullptr;          // FP64 complex solution scratch, xhi_slots entries
  size_t xhi_slots = 0;         // >= blocks * (max_n rounded up to 64)
};

// FP64 scratch entries (complex) the resident engine needs for `blocks` workgroups.
size_t cocg_resident_xhi_slots(int n, int blocks);
// Largest n the resident engine takes at this precision.
int cocg_resident_max_n(bool fp32);
// Waves per resident workgroup, and the slice-to-wave table for slice widths
// (entries per row, in slice order, non-increasing) with at most rpt slots
// per wave; empty when the slices do not fit.
int cocg_resident_waves();
std::vector<int> cocg_resident_wave_table(const std::vector<int>& widths, int rpt);
// Dynamic LDS bytes the resident engine needs for n.
size_t cocg_resident_lds(int n, bool fp32);
// Sets the kernel attributes a resident launch for max_n and rpt needs (the
// launch sets them too; call this before capturing one into a graph).
hipError_t prepare_cocg_resident(int max_n, int rpt, bool fp32);
// One persistent launch over all items of L.  Either g0 (host pointer; all
// items name graph 0, passed by value) or graphs (device array of the graphs
// the items name) is given.  max_n: the largest n among them; rpt: the slots
// per wave every graph's wave table was built for.
hipError_t launch_cocg_resident(hipStream_t st, const ResGraph* g0, const ResGraph* graphs,
                                int max_n, int rpt, const CocgLaunch& L, bool fp32,
                                int num_blocks);


// ---- streaming COCG engine (any n) ------------------------------------------
// All columns c < ncols solve (zc[c] I - A) d_c = b_{c mod k} in lock step;
// vectors are n x Bp complex blocks, row-major, in the engine's row order
// (engine row r is caller row perm[r]).  Columns are handled in groups of
// 64 * stream_cpl(k, ncols, fp32) (CPL complex columns per lane); at most
// kStreamMaxGroups groups.
constexpr int kStreamMaxGroups = 128;
struct StreamGroups {
  int count;
  int g[kStreamMaxGroups];    // group of blockIdx.y
  int par[kStreamMaxGroups];  // which of the two p buffers holds the group's current p
};
// Dense symmetric operator of the statistical workloads: A = K (kind 1,
// n x n) or A = scale X^T X (kind 2, X rows x n).  Device matrices are
// column-major (leading dimension n for K, rows for X); the products run on
// rocBLAS (MFMA GEMMs), the handle bound to the caller's stream per call.
struct DenseOp {
  int kind = 0;
  int64_t n = 0, rows = 0;
  double scale = 1.0;
  const double* a64 = nullptr;     // K or Xd (column-major, ld rows), FP64
  const float* a32 = nullptr;      // the same, FP32
  double* t64 = nullptr;           // workspace of wslabs slabs of rows x tcols: kind 2,
  float* t32 = nullptr;            // Xd X in the first and the inner-dimension chunks of
                                   // its product after it; kind 1, the chunks of K X
  int64_t tcols = 0;               // most columns a product takes
  int wslabs = 0;
};
// Y = alpha A X + beta Y for row-major n x k blocks X (ldx) and Y (ldy),
// FP64; k <= tcols.
hipError_t dense_apply_f64(const DenseOp& A, hipStream_t st, int k, const double* X, int ldx,
                           double* Y, int ldy, double alpha, double beta);
// Y = A X in FP32, same layout.
hipError_t dense_apply_f32(const DenseOp& A, hipStream_t st, int k, const float* X, int ldx,
                           float* Y, int ldy);
// y += a x over count contiguous doubles.
hipError_t dense_axpy(hipStream_t st, int64_t count, double a, const double* x, double* y);
// C (M x N, row-major, ldc) = alpha op(A) B + beta C on the matrix cores;
// op(A)(i, k) = A[k lda + i] when acol, else A[i lda + k]; B (K x N) by rows.
// work (nullable): room for inner-dimension chunk slabs (work_elems elements).
hipError_t launch_gemm_f64(hipStream_t st, bool acol, int M, int N, int K, const double* A,
                           int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                           double alpha, double beta, double* work, size_t work_elems);
hipError_t launch_gemm_f32(hipStream_t st, bool acol, int M, int N, int K, const float* A,
                           int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                           float alpha, float beta, float* work, size_t work_elems);

// Band LDL^T of the shifted matrices (standard FEAST with exact solves).
// W: nz blocks of n x (b + 1) complex, row r of block j holding
// (z_j I - A)(r, r - d) in column d, A in engine (reverse Cuthill-McKee)
// order; factorized in place (D on d = 0, L below).  info: device [nz],
// 0 or 1 + the row of a vanishing pivot.
int band_panel_width(int b);
size_t band_lds_bytes(int b);
int band_solve_ring_rows(int b);
// whether bandwidth b fits the factorization's panel and the solve's LDS ring
bool band_supported(int b);
hipError_t band_assemble(hipStream_t st, int n, int b, const int* rowptr, const int* col,
                         const double* val, int nz, const double* z, cpx<double>* W);
hipError_t band_factor(hipStream_t st, int n, int b, int nz, cpx<double>* W, int* info);
// X[:, j k + c] = (z_j I - A)^{-1} B[:, c] (caller order through perm).
hipError_t band_solve(hipStream_t st, int n, int b, int nz, const cpx<double>* W, const int* perm,
                      const double* B, int ldb, int k, cpx<double>* X, int64_t ldx);
// resid[j k + c] = ||B_c - (z_j I - A) X_{j,c}|| / ||B_c||, caller-order CSR.
hipError_t band_resid(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                      int nz, const double* z, const double* B, int ldb, int k,
                      const cpx<double>* X, int64_t ldx, double* resid);

struct StreamMatrix {
  int n = 0;
  const DenseOp* dense = nullptr;  // set: A is this dense operator (no CSR; perm identity)
  const int* rowptr = nullptr;     // CSR in engine row order, columns renumbered
  const int* col = nullptr;
  const float* val32 = nullptr;
  const double* val64 = nullptr;
  const int* perm = nullptr;       // engine row -> caller row
};
struct StreamCols {                // per-column state, Bp entries (complex: 2 Bp)
  int* state = nullptr;
  int* it = nullptr;
  int* nref = nullptr;
  int* nbd = nullptr;
  double* rho = nullptr;
  double* alpha = nullptr;
  double* beta = nullptr;
  double* ctol2 = nullptr;
  double* res = nullptr;
  double* bn = nullptr;
  int* lastit = nullptr;           // iteration count at the last check
  int* span = nullptr;             // iterations between the last two checks (0: none yet)
  int* span0 = nullptr;            // length of the first check interval after a (re)start
  int* rstart = nullptr;           // iteration count at the last (re)start
  double* sprev = nullptr;         // ||s||^2 at the last check (1 at the start)
};
struct StreamWork {
  int Bp = 0;                      // stream_padded_columns(k, ncols, fp32)
  int num_cu = 0;
  void* x = nullptr;               // n x Bp complex (engine precision) each
  void* r = nullptr;
  void* p0 = nullptr;
  void* p1 = nullptr;
  void* w = nullptr;
  void* xh = nullptr;              // n x Bp complex FP64
  void* axh = nullptr;             // dense operator only: n x Bp complex FP64, A x_hi
  void* pc = nullptr;              // dense only: n x Bp complex, the iterating columns of p
  void* apc = nullptr;             //   packed side by side, and A times them
  int* cidx = nullptr;             // dense only: [Bp] packed column -> column (+ parity bit 30)
  int* cmap = nullptr;             // dense only: [Bp] column -> packed column (-1: none)
  double* part = nullptr;          // stream_partial_doubles(n, Bp, num_cu)
  double* zc = nullptr;            // [2 Bp] shift of each column (padding: any finite value)
  double* scale = nullptr;         // [Bp]
  int* cnt = nullptr;              // [2 * kStreamMaxGroups]
  StreamCols cols;
};
struct StreamLaunch {
  const double* B = nullptr;       // n x k RHS (FP64, caller row order), ldb
  int ldb = 0;
  int k = 0;
  int ncols = 0;
  void* D = nullptr;               // n x ncols complex outputs (caller row order), ldd
  int ldd = 0;
  double tol = 1e-6;
  int maxit = 20000;
  int max_updates = 64;            // FP64 residual checks that may continue a column
  int chunk = 8;                   // iterations between host census reads
  int* iters = nullptr;            // nullable [ncols]
  double* resid = nullptr;         // nullable [ncols]
  int* stats = nullptr;            // nullable [2]: refinements, breakdowns (accumulated)
};
int stream_cpl(int k, int ncols, bool fp32);
int stream_padded_columns(int k, int ncols, bool fp32);
int stream_blocks(int n, int num_cu);
size_t stream_partial_doubles(int n, int Bp, int num_cu);
// Runs to completion; synchronises `st` once per census (every `chunk` iterations).
hipError_t run_stream_cocg(hipStream_t st, const StreamMatrix& A, const StreamWork& W,
                           const StreamLaunch& L, bool fp32);

// ---- multi-shift COCG engine (FP64) ------------------------------------------
// The nz shifted systems of each column c < k share the right-hand side
// b_c: (z_j I - A) d_{j,c} = b_c.  One CG on the real SPD seed A - s I
// (s below the spectrum) drives all of them; every shifted system keeps its
// own search direction and iterate (complex FP64) and stops at its own
// residual.  Blocks are n x kp (kp = 64 ceil(k / 64)) in the streaming
// engine's row order (A: its StreamMatrix, FP64 values).
struct MsCols {                  // per column kp entries; per (j, c) nz x kp entries
  double* rr = nullptr;          // seed r^T r
  double* bn = nullptr;          // |b|
  double* alpha = nullptr;
  double* alpha_prev = nullptr;
  double* beta_prev = nullptr;
  double* scale = nullptr;       // pending rescale of the seed's r and p (1: none)
  int* colive = nullptr;         // some shift of the column still iterates
  cpx<double>* pi = nullptr;     // pi_k of each shift
  cpx<double>* pi_prev = nullptr;
  cpx<double>* pi_next = nullptr;
  cpx<double>* ipi = nullptr;    // 1 / pi_k
  cpx<double>* as = nullptr;     // alpha^s_k
  cpx<double>* bs = nullptr;     // beta^s_{k-1}
  int* live = nullptr;           // the shifted system still iterates
  int* its = nullptr;            // its iterations
  double* est = nullptr;         // its estimated relative residual |r_k| / (|pi_k| |b|)
  cpx<double>* gas = nullptr;    // combining mode: g_{j,c} alpha^s_k
};
struct MsWork {
  int kp = 0, nz = 0, nb = 0, num_cu = 0;  // nz: the most shifts this workspace holds
  double* r = nullptr;           // n x kp seed blocks
  double* p = nullptr;
  double* w = nullptr;
  cpx<double>* X = nullptr;      // nz blocks n x kp: shifted iterates
  cpx<double>* P = nullptr;      // nz blocks n x kp: shifted search directions
  double* part = nullptr;        // nb x kp partial sums
  double* y = nullptr;           // nullable n x kp: the filtered block accumulated in the
                                 //   combining mode (then X is not used)
  cpx<double>* sig = nullptr;    // [nz] sigma_j = s - z_j
  int* count = nullptr;          // [1] live systems
  MsCols cols;
};
struct MsLaunch {
  const double* B = nullptr;     // n x k right-hand sides (FP64, caller row order), ldb
  int ldb = 0;
  int k = 0;
  int nz = 0;
  const double* z = nullptr;     // host [2 nz] shifts (re, im)
  double seed = 0.0;             // s: A - s I is positive definite
  void* D = nullptr;             // n x (nz k) complex FP64 outputs (caller row order), ldd;
  int ldd = 0;                   //   column j k + c is d_{j,c}
  double tol = 1e-6;
  int maxit = 20000;
  int chunk = 8;                 // iterations between host reads of the live count
  int* iters = nullptr;          // nullable device [nz k]
  double* resid = nullptr;       // nullable device [nz k]: true relative residuals
                                 //   |b_c - (z_j I - A) d| / |b_c| in FP64
  // Combining mode (g non-null): the solutions are not stored; the engine
  // accumulates Qt[:, c] = gq_c Qin[:, c] + sum_j Re(g_{j,c} d_{j,c}) with
  // gq_c = sum_j Re(g_{j,c}) (0 when Qin is null) into Qt (caller row order,
  // ldq), the filter combination of one FEAST iteration; D, resid unused.
  const double* g = nullptr;     // device [2 nz k]: complex g_{j,c} at j k + c
  const double* Qin = nullptr;   // nullable device n x k (ldqin)
  int ldqin = 0;
  double* Qt = nullptr;
  int ldq = 0;
};
int ms_cpl(int k);
int ms_padded(int k);
int ms_blocks(int n, int num_cu);
// Runs to completion; synchronises st once per chunk of iterations.
hipError_t run_mshift(hipStream_t st, const StreamMatrix& A, const MsWork& W, const MsLaunch& L);

}  // namespace rafeast

namespace rafeast {
// dst (column-major n x k) <- src (row-major, lds).
hipError_t launch_rowmajor_to_colmajor(hipStream_t st, int64_t n, int k, const double* src,
                                       int lds, double* dst);
}  // namespace rafeast

namespace rafeast {
// ---- learned polynomial preconditioner ---------------------------------------
// T: 9 blocks T_0..T_8 (n x kc row-major, block stride n * kc) of T_k(A^) R;
// part: nchunks * kc * 136 doubles.  Per sample s = j * kc + i: X[s][4],
// G[s][8][8] and h[s][8] complex (re, im), rr[s].
hipError_t launch_pc_gram_assemble(hipStream_t st, int64_t n, int kc, const double* T, int nz,
                                   const double* zs, double a, double b, double th_lo,
                                   double th_hi, double* part, int nchunks, double* X, double* G,
                                   double* h, double* rr);
// dst (n x 2k real, row-major) <- Re, then Im, of columns c0..c0+k of the
// complex FP64 block src (n x ld).
hipError_t launch_split_complex(hipStream_t st, int64_t n, int ld, int c0, int k,
                                const cpx<double>* src, double* dst);
int mlp_param_count();
int mlp_backward_waves(int nb);
// wb <- BF16 values (held in FP32) of the FP32 parameters w
hipError_t launch_mlp_bf16(hipStream_t st, const float* w, float* wb);
// Y[s][16] = network(X[s]) for s < ns, with BF16 parameters wb
hipError_t launch_mlp_forward(hipStream_t st, int ns, const double* X, const float* wb, float* Y);
// grad = gradient of the mean loss over samples idx[0..nb); part holds
// mlp_backward_waves(nb) * mlp_param_count() floats, lpart as many doubles;
// loss (nullable) the mean loss
hipError_t launch_mlp_grad(hipStream_t st, int nb, const int* idx, const double* X,
                           const double* G, const double* h, const double* rr, const float* wb,
                           float* part, double* lpart, float* grad, double* loss);
hipError_t launch_adam(hipStream_t st, float* w, float* m, float* v, const float* g, float lr,
                       int step, float* wb);

struct PcCols {  // per column, Bc entries (complex: 2 Bc)
  int* active = nullptr;
  int* it = nullptr;
  int* pending = nullptr;
  double* bn2 = nullptr;
  double* res = nullptr;
  double* rho = nullptr;
  double* rhon = nullptr;
  double* alpha = nullptr;
  double* beta = nullptr;
};
struct PcSolve {
  int64_t n = 0;
  const int* rowptr = nullptr;     // CSR, FP64 values
  const int* col = nullptr;
  const double* val = nullptr;
  double a = 1, b = 0;             // A^ = a A + b I
  int Bc = 0;                      // columns (systems)
  const double* zc = nullptr;      // [2 Bc] shift of each column
  const double* coef = nullptr;    // nullable [8][Bc] complex Chebyshev coefficients
  const double* B = nullptr;       // n x kb RHS (FP64), column c takes B[:, c % kb]
  int ldb = 0, kb = 0;
  cpx<double>* x = nullptr;        // n x Bc complex FP64 blocks
  cpx<double>* r = nullptr;
  cpx<double>* u = nullptr;
  cpx<double>* p0 = nullptr;
  cpx<double>* p1 = nullptr;
  cpx<double>* w = nullptr;
  cpx<double>* t0 = nullptr;       // Clenshaw work blocks (unused without coef)
  cpx<double>* t1 = nullptr;
  cpx<double>* t2 = nullptr;
  double* part = nullptr;          // pc_blocks(n, num_cu) * Bc * 3 doubles
  int* counts = nullptr;           // [2]
  PcCols cols;
  double tol = 1e-10;
  int maxit = 20000;
  int num_cu = 256;
  bool progress = false;           // a line on stderr every 500 iterations
};
int pc_blocks(int64_t n, int num_cu);
// Preconditioned COCG (coef) or plain COCG (coef null) in FP64 on all Bc
// columns in lock step, to true residual ||b - (zI - A) x|| <= tol ||b||.
// Synchronises st once or twice per iteration.
hipError_t run_pc_cocg(hipStream_t st, const PcSolve& S);

}  // namespace rafeast
