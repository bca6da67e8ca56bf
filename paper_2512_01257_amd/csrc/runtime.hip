// RA-FEAST host runtime and C ABI: validation, plan (device copies of A,
// quadrature table, workspace), Phase 1 (randomized warmstart) and Phase 2
// (FEAST iterations) drivers.  All arithmetic of the method runs in the
// kernels declared in kernels.h; the host only sequences launches and reads
// back the small per-iteration scalars (Ritz values and residual norms).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rafeast.h"
#include "kernels.h"

using namespace rafeast;

namespace {

thread_local std::string g_plan_error;

constexpr int kMaxSmallK = 192;
#ifndef RAFEAST_SELL_BANK_GROUPS
#define RAFEAST_SELL_BANK_GROUPS 32  // lanes per LDS cycle of 8-byte gathers
#endif

// Ritz pairs with a smaller filter gain are spurious (not counted in M).
constexpr double kSpuriousGain = 0.25;

// Host workers driving streaming-engine members of a batch concurrently.
constexpr size_t kBatchWorkers = 8;

}  // namespace

struct rafeast_plan_s {
  rafeast_params prm{};
  int64_t n = 0, nnz = 0;
  int m0 = 0, w = 0, nc = 0, pov = 0;
  double sig_lo = 0, sig_hi = 0, anorm = 0;
  std::vector<double> zw;  // z_j (re, im) then w_j (re, im)
  hipStream_t st = nullptr;
  bool own_stream = false;
  int dev = 0, num_cu = 0;
  bool fp32 = true;
  int engine = RAFEAST_ENGINE_RESIDENT;
  // matrix
  int* d_rowptr = nullptr;
  int* d_col = nullptr;
  double* d_val = nullptr;
  int64_t span = 0;  // max |i - j| over the nonzeros (sets the SpMM's column groups)
  SellMatrix sell;
  int* d_sbase = nullptr;
  int* d_perm = nullptr;
  int* d_wtab = nullptr;
  float* d_v32 = nullptr;  // FP32 SELL values followed by their 16-bit offsets
  SellEntry64* d_e64 = nullptr;
  size_t sell_entries = 0;
  // n x w blocks (row-major, ld = w)
  double* d_Q = nullptr;
  double* d_W = nullptr;
  double* d_R = nullptr;
  double* d_T = nullptr;
  double* d_Y = nullptr;
  int ld = 0;
  // small matrices
  double* d_G = nullptr;     // kmax^2
  double* d_M = nullptr;     // kmax^2
  double* d_S = nullptr;     // kmax^2
  double* d_Ssel = nullptr;  // kmax * m0
  double* d_jw = nullptr;    // 2 kmax^2
  double* d_theta = nullptr; // kmax
  double* d_res = nullptr;   // kmax
  double* d_qn = nullptr;    // kmax
  // Q = Q~ mtot for the filtered block Q~ of the last iteration: CholQR2's
  // transforms (m0 x m0 row-major), valid while have_filter; d_mtmp the
  // buffer of their next product
  double* d_mtot = nullptr;  // m0^2
  double* d_mtmp = nullptr;  // m0^2
  double* d_gamma = nullptr; // 2 nc m0
  double* d_info = nullptr;  // 4
  double* d_zw = nullptr;    // 4 nc
  double* d_part = nullptr;
  size_t part_doubles = 0;
  void* d_D = nullptr;       // n x (nc m0) complex
  int* d_items = nullptr;    // 2 nc m0
  int* d_counter = nullptr;  // 1
  int* d_iters = nullptr;    // nc m0
  int* d_stats = nullptr;    // 2
  int* d_flag = nullptr;     // 3: one Cholesky status per CholQR pass
  int* d_sel = nullptr;      // m0
  void* d_xhi = nullptr;     // FP64 solution scratch of the resident COCG engine
  size_t xhi_slots = 0;
  std::vector<int> sell_widths; // slice widths, for wave tables of other slot counts
  // autotuned launch shape (resident engine: slots per thread), candidates
  // and their measured times
  int tune_choice = 0;
  std::vector<int> tune_cand;
  std::vector<float> tune_ms;
  // streaming engine: A in reverse Cuthill-McKee order, FP64 and FP32 values
  int* d_srow = nullptr;
  int* d_scol = nullptr;
  float* d_sv32 = nullptr;
  double* d_sv64 = nullptr;
  int* d_sperm = nullptr;
  StreamMatrix smat;
  StreamWork swork;               // sized for the nc * m0 systems of a solve
  MsWork mswork;                  // multi-shift engine: sized for nc shifts x m0 columns
  double* d_wrep = nullptr;       // its literal-form weights: w_j for every column (2 nc m0)
  // direct engine: band LDL^T factors of the nc shifted matrices (engine
  // order), the lower bandwidth, and the factorization's pivot report
  cpx<double>* d_band = nullptr;
  int band_b = 0;
  int* d_binfo = nullptr;
  float factor_ms = 0.0f;
  DenseOp dop;                    // dense operator (kind 0: A is the CSR matrix)
  double* d_k64 = nullptr;        // its device matrices and scratch
  float* d_k32 = nullptr;
  double* d_t64 = nullptr;
  float* d_t32 = nullptr;
  std::vector<void*> sbufs;       // device buffers behind swork
  int nitems = 0;
  bool have_start = false;
  bool have_filter = false;  // d_mtot holds the last filter step's transforms
  // COCG tolerance of the next filter application (tol_solve, or the relaxed
  // tolerance of Phase 2 while it still contracts)
  double tau = 0.0;
  int ws_used = RAFEAST_WS_NONE;
  // learned preconditioner inside the solve (precond LEARNED): network
  // parameters (FP32 and their BF16 values), per-node features and outputs,
  // and the FP64 solution block the preconditioned solves write
  float* d_pcW = nullptr;
  float* d_pcWb = nullptr;
  double* d_pcX = nullptr;   // nc x 4
  float* d_pcY = nullptr;    // nc x 16
  void* d_D64 = nullptr;     // n x (nc m0) complex FP64
  bool pc_ready = false;
  // Ritz values of the last Rayleigh-Ritz step (training-sample harvest)
  std::vector<double> last_theta;
  std::string err;
  hipEvent_t ev[8] = {};
};

// A batch: member plans sharing one stream, and the state of the shared
// resident launch.
struct rafeast_batch_s {
  std::vector<rafeast_plan_s*> plans;
  std::vector<int> res_idx;          // member -> slot in the descriptor array (-1: streaming)
  std::vector<int*> wtab;            // member -> wave table for the common slot count
  std::vector<int*> own_wtab;        // tables the batch allocated
  hipStream_t st = nullptr;
  bool own_stream = false;
  bool fp32 = true;
  int rpt = 0, max_n = 0, num_cu = 0, nres = 0;
  ResGraph* d_graphs = nullptr;
  std::vector<ResGraph> h_graphs;
  int* d_items = nullptr;
  std::vector<int> h_items;
  int* d_counter = nullptr;
  void* d_xhi = nullptr;
  size_t xhi_slots = 0;
  hipGraph_t graph = nullptr;        // captured counter reset + resident launch
  hipGraphExec_t gexec = nullptr;
  int graph_nitems = -1;             // the item count the capture was made for
  hipEvent_t ev[6] = {};              // total, solve phase, combine phase
  std::vector<hipStream_t> mst;       // member streams (owned)
  std::vector<hipEvent_t> mev;        // member events (owned)
  std::string err;
};

// ============================================================================
// helpers
// ============================================================================
namespace {

// Progress lines on stderr, one per FEAST iteration, when RAFEAST_VERBOSE is
// set to a non-empty value other than "0".
bool verbose_log() {
  static const bool on = [] {
    const char* v = std::getenv("RAFEAST_VERBOSE");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

rafeast_status fail(rafeast_plan_s* P, rafeast_status s, const std::string& msg) {
  if (P)
    P->err = msg;
  else
    g_plan_error = msg;
  return s;
}

rafeast_status hip_fail(rafeast_plan_s* P, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  return fail(P, e == hipErrorOutOfMemory ? RAFEAST_OOM : RAFEAST_DEVICE, msg);
}

#define HIPCHK(P, expr)                                   \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return hip_fail((P), _e, #expr); \
  } while (0)

#define RCHK(expr)                            \
  do {                                        \
    rafeast_status _s = (expr);               \
    if (_s != RAFEAST_OK) return _s;          \
  } while (0)

// Gauss-Legendre nodes (ascending) and weights on [-1, 1] by Newton's method
// on the Legendre three-term recurrence, starting from the Chebyshev-like
// estimate cos(pi (i + 3/4) / (N + 1/2)).
void gauss_legendre_newton(int N, std::vector<double>& x, std::vector<double>& wt) {
  x.assign(N, 0.0);
  wt.assign(N, 0.0);
  for (int i = 0; i < N; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (N + 0.5));
    double dp = 1.0;
    for (int itn = 0; itn < 100; ++itn) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= N; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = (N == 1) ? 1.0 : N * (t * p1 - p0) / (t * t - 1.0);
      const double dx = p1 / dp;
      t -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    // final derivative at the converged node
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= N; ++k) {
      const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = (N == 1) ? 1.0 : N * (t * p1 - p0) / (t * t - 1.0);
    x[i] = t;
    wt[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  std::vector<int> idx(N);
  for (int i = 0; i < N; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(N), ws(N);
  for (int i = 0; i < N; ++i) {
    xs[i] = x[idx[i]];
    ws[i] = wt[idx[i]];
  }
  x = xs;
  wt = ws;
}

rafeast_status validate_params(const rafeast_params* p, int64_t n, std::string& msg) {
  if (!(std::isfinite(p->lmin) && std::isfinite(p->lmax) && p->lmin < p->lmax)) {
    msg = "need finite lmin < lmax";
    return RAFEAST_INVALID_ARG;
  }
  if (p->m0 < 1 || p->m0 > n) {
    msg = "m0 must be in [1, n]";
    return RAFEAST_INVALID_ARG;
  }
  if (p->nc < 1 || p->nc > 64) {
    msg = "nc must be in [1, 64]";
    return RAFEAST_INVALID_ARG;
  }
  if (p->q < 0 || p->q > 64) {
    msg = "q must be in [0, 64]";
    return RAFEAST_INVALID_ARG;
  }
  if (p->p >= 0 && p->p < 4) {
    msg = "oversampling p must be >= 4 (Assumption 1.5) or < 0 for the default rule";
    return RAFEAST_INVALID_ARG;
  }
  if (!(p->tol_eig > 0.0) || !(p->tol_solve > 0.0) || !(p->tol_solve < 1.0)) {
    msg = "tolerances must satisfy tol_eig > 0 and 0 < tol_solve < 1";
    return RAFEAST_INVALID_ARG;
  }
  if (!(p->tol_solve_relaxed >= 0.0) || !(p->tol_solve_relaxed < 1.0)) {
    msg = "tol_solve_relaxed must satisfy 0 <= tol_solve_relaxed < 1";
    return RAFEAST_INVALID_ARG;
  }
  if (p->max_iter < 0 || p->max_cocg < 1) {
    msg = "need max_iter >= 0 and max_cocg >= 1";
    return RAFEAST_INVALID_ARG;
  }
  if (p->precision != RAFEAST_FP64 && p->precision != RAFEAST_FP32_REFINED) {
    msg = "unknown precision";
    return RAFEAST_INVALID_ARG;
  }
  if (p->ws_op < RAFEAST_WS_AUTO || p->ws_op > RAFEAST_WS_NONE) {
    msg = "unknown ws_op";
    return RAFEAST_INVALID_ARG;
  }
  if (p->rhs_form != RAFEAST_RHS_RESIDUAL && p->rhs_form != RAFEAST_RHS_LITERAL) {
    msg = "unknown rhs_form";
    return RAFEAST_INVALID_ARG;
  }
  if (p->engine < RAFEAST_ENGINE_AUTO || p->engine > RAFEAST_ENGINE_DIRECT) {
    msg = "unknown engine";
    return RAFEAST_INVALID_ARG;
  }
  if (p->engine == RAFEAST_ENGINE_MULTISHIFT && p->precision != RAFEAST_FP64) {
    msg = "the multi-shift engine runs in FP64 (precision RAFEAST_FP64)";
    return RAFEAST_INVALID_ARG;
  }
  if (p->engine == RAFEAST_ENGINE_DIRECT && p->precision != RAFEAST_FP64) {
    msg = "the direct engine runs in FP64 (precision RAFEAST_FP64)";
    return RAFEAST_INVALID_ARG;
  }
  if (p->precond != RAFEAST_PC_NONE && p->precond != RAFEAST_PC_LEARNED) {
    msg = "unknown precond";
    return RAFEAST_INVALID_ARG;
  }
  return RAFEAST_OK;
}

rafeast_status validate_csr(const rafeast_csr* A, int64_t& nnz, double& anorm, double& lo,
                            double& hi, std::string& msg) {
  if (A->n < 1 || A->n >= (int64_t(1) << 31)) {
    msg = "n must be in [1, 2^31)";
    return RAFEAST_INVALID_ARG;
  }
  if (A->index_base != 0 && A->index_base != 1) {
    msg = "index_base must be 0 or 1";
    return RAFEAST_INVALID_ARG;
  }
  if (!A->rowptr) {
    msg = "rowptr is NULL";
    return RAFEAST_INVALID_ARG;
  }
  const int64_t n = A->n;
    const int base = A->index_base;
  if (A->rowptr[0] != base) {
    msg = "rowptr[0] != index_base";
    return RAFEAST_BAD_CSR;
  }
  for (int64_t i = 0; i < n; ++i)
    if (A->rowptr[i + 1] < A->rowptr[i]) {
      msg = "rowptr not monotone at row " + std::to_string(i);
      return RAFEAST_BAD_CSR;
    }
  nnz = (int64_t)A->rowptr[n] - base;
  if (nnz > 0 && (!A->colind || !A->values)) {
    msg = "colind or values is NULL";
    return RAFEAST_INVALID_ARG;
  }
  anorm = 0.0;
  lo = INFINITY;
  hi = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t s = A->rowptr[i] - base, e = A->rowptr[i + 1] - base;
    double rs = 0.0, d = 0.0, off = 0.0;
    int64_t prev = -1;
    for (int64_t t = s; t < e; ++t) {
      const int64_t j = (int64_t)A->colind[t] - base;
      const double v = A->values[t];
      if (j < 0 || j >= n) {
        msg = "column out of range in row " + std::to_string(i);
        return RAFEAST_BAD_CSR;
      }
      if (j <= prev) {
        msg = "columns not strictly increasing in row " + std::to_string(i);
        return RAFEAST_BAD_CSR;
      }
      if (!std::isfinite(v)) {
        msg = "non-finite value in row " + std::to_string(i);
        return RAFEAST_BAD_CSR;
      }
      prev = j;
      rs += std::fabs(v);
      if (j == i)
        d = v;
      else
        off += std::fabs(v);
    }
    anorm = std::max(anorm, rs);
    lo = std::min(lo, d - off);
    hi = std::max(hi, d + off);
  }
  const double stol = 1e-14 * anorm;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t s = A->rowptr[i] - base, e = A->rowptr[i + 1] - base;
    for (int64_t t = s; t < e; ++t) {
      const int64_t j = (int64_t)A->colind[t] - base;
      if (j == i) continue;
      const int64_t sj = A->rowptr[j] - base, ej = A->rowptr[j + 1] - base;
      const int32_t* b = A->colind + sj;
      const int32_t* f = std::lower_bound(b, A->colind + ej, (int32_t)(i + base));
      if (f == A->colind + ej || *f != (int32_t)(i + base)) {
        msg = "pattern not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")";
        return RAFEAST_NOT_SYMMETRIC;
      }
      const double aji = A->values[sj + (f - b)];
      if (std::fabs(aji - A->values[t]) > stol) {
        msg = "values not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")";
        return RAFEAST_NOT_SYMMETRIC;
      }
    }
  }
  return RAFEAST_OK;
}

template <typename T>
rafeast_status dalloc(rafeast_plan_s* P, T** p, size_t count, const char* what) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(P, e, what);
  }
  return RAFEAST_OK;
}

void free_plan(rafeast_plan_s* P) {
  if (!P) return;
  if (P->d_D64 == P->d_D) P->d_D64 = nullptr;  // the FP64 plan's own solve block
  void* ptrs[] = {P->d_rowptr, P->d_col,  P->d_val,   P->d_sbase, P->d_perm, P->d_wtab, P->d_v32,
                  P->d_e64,   P->d_Q,    P->d_W,     P->d_R,     P->d_T,    P->d_Y,
                  P->d_G,      P->d_M,    P->d_S,     P->d_Ssel,  P->d_jw,   P->d_theta,
                  P->d_res,    P->d_qn,   P->d_gamma, P->d_info,  P->d_zw,   P->d_part,
                  P->d_D,      P->d_items, P->d_counter, P->d_iters, P->d_stats, P->d_flag,
                  P->d_sel, P->d_xhi, P->d_srow, P->d_scol, P->d_sv32, P->d_sv64, P->d_sperm,
                  P->d_k64, P->d_k32, P->d_t64, P->d_t32,
                  P->d_mtot, P->d_mtmp, P->d_pcW, P->d_pcWb, P->d_pcX, P->d_pcY, P->d_D64,
                  P->d_wrep, P->d_band, P->d_binfo};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (void* p : P->sbufs)
    if (p) (void)hipFree(p);
  for (auto& e : P->ev)
    if (e) (void)hipEventDestroy(e);
  if (P->own_stream && P->st) (void)hipStreamDestroy(P->st);
  delete P;
}

// A dense operator handed to rafeast_plan_dense (kind 1: K, n x n) or
// rafeast_plan_gram (kind 2: scale X^T X, X rows x n), host, column-major.
struct DenseSpec {
  int kind = 0;
  int64_t n = 0, rows = 0, ld = 0;
  const double* M = nullptr;
  double scale = 1.0;
};

// Checks a dense operator and returns nnz, ||A||_inf (kind 2: the trace
// bound scale ||X||_F^2) and the spectral bounds [lo, hi].
rafeast_status validate_dense(const DenseSpec& D, int64_t& nnz, double& anorm, double& lo,
                              double& hi, std::string& msg) {
  const int64_t lim = (int64_t)1 << 31;
  if (!D.M) {
    msg = "matrix is NULL";
    return RAFEAST_INVALID_ARG;
  }
  if (D.n < 1 || D.n >= lim) {
    msg = "need 1 <= n < 2^31";
    return RAFEAST_INVALID_ARG;
  }
  if (D.kind == 1) {
    const int64_t n = D.n;
    if (D.ld < n) {
      msg = "ldk < n";
      return RAFEAST_INVALID_ARG;
    }
    anorm = 0.0;
    lo = std::numeric_limits<double>::infinity();
    hi = -lo;
    for (int64_t i = 0; i < n; ++i) {
      double rs = 0.0;
      for (int64_t j = 0; j < n; ++j) {
        const double v = D.M[i + j * D.ld];
        if (!std::isfinite(v)) {
          msg = "K has a non-finite entry";
          return RAFEAST_BAD_CSR;
        }
        rs += std::fabs(v);
      }
      const double d = D.M[i + i * D.ld], off = rs - std::fabs(d);
      lo = std::min(lo, d - off);
      hi = std::max(hi, d + off);
      anorm = std::max(anorm, rs);
    }
    const double stol = 1e-14 * anorm;
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < j; ++i)
        if (std::fabs(D.M[i + j * D.ld] - D.M[j + i * D.ld]) > stol) {
          msg = "K is not symmetric";
          return RAFEAST_NOT_SYMMETRIC;
        }
    if (!(hi > lo)) hi = lo + std::max(1.0, std::fabs(lo));  // K = c I: any interval holding c
    nnz = n * n;
    return RAFEAST_OK;
  }
  if (D.kind != 2 || D.rows < 1 || D.rows >= lim || D.ld < D.rows) {
    msg = "need 1 <= rows < 2^31 and ldx >= rows";
    return RAFEAST_INVALID_ARG;
  }
  if (!(D.scale > 0.0) || !std::isfinite(D.scale)) {
    msg = "scale must be positive and finite";
    return RAFEAST_INVALID_ARG;
  }
  double fro2 = 0.0;
  for (int64_t j = 0; j < D.n; ++j)
    for (int64_t i = 0; i < D.rows; ++i) {
      const double v = D.M[i + j * D.ld];
      if (!std::isfinite(v)) {
        msg = "X has a non-finite entry";
        return RAFEAST_BAD_CSR;
      }
      fro2 += v * v;
    }
  if (!(fro2 > 0.0) || !std::isfinite(D.scale * fro2)) {
    msg = "X must be nonzero with a finite covariance";
    return RAFEAST_INVALID_ARG;
  }
  lo = 0.0;
  hi = D.scale * fro2;
  anorm = hi;
  nnz = D.rows * D.n;
  return RAFEAST_OK;
}

// Reverse Cuthill-McKee order of the graph of A (diagonal ignored): per
// connected component, breadth-first search from a pseudo-peripheral vertex
// (George-Liu: restart from a lowest-degree vertex of the last level while
// the eccentricity grows), neighbours taken by increasing degree, and the
// whole sequence reversed.  Returns perm with perm[new] = old.
std::vector<int> rcm_order(int64_t n, const std::vector<int>& rp, const std::vector<int>& cl) {
  std::vector<int> deg(n);
  for (int64_t i = 0; i < n; ++i) {
    int d = 0;
    for (int t = rp[i]; t < rp[i + 1]; ++t) d += cl[t] != i;
    deg[i] = d;
  }
  std::vector<int> by_deg(n);
  for (int64_t i = 0; i < n; ++i) by_deg[i] = (int)i;
  std::stable_sort(by_deg.begin(), by_deg.end(), [&](int a, int b) { return deg[a] < deg[b]; });
  std::vector<char> done(n, 0);
  std::vector<int> stamp(n, -1), level(n, 0), order;
  order.reserve(n);
  int stamp_id = 0;
  std::vector<int> q;
  q.reserve(n);
  // BFS over undone vertices from s; returns the eccentricity and a
  // lowest-degree vertex of the last level.
  auto bfs_levels = [&](int s, int& far) {
    ++stamp_id;
    q.clear();
    q.push_back(s);
    stamp[s] = stamp_id;
    level[s] = 0;
    int ecc = 0;
    for (size_t h = 0; h < q.size(); ++h) {
      const int u = q[h];
      for (int t = rp[u]; t < rp[u + 1]; ++t) {
        const int v = cl[t];
        if (v == u || done[v] || stamp[v] == stamp_id) continue;
        stamp[v] = stamp_id;
        level[v] = level[u] + 1;
        ecc = std::max(ecc, level[v]);
        q.push_back(v);
      }
    }
    far = s;
    for (int v : q)
      if (level[v] == ecc && (far == s || deg[v] < deg[far])) far = v;
    return ecc;
  };
  std::vector<int> nb;
  for (int s0 : by_deg) {
    if (done[s0]) continue;
    int s = s0, far = s0;
    int ecc = bfs_levels(s, far);
    for (int rep = 0; rep < 16 && far != s; ++rep) {
      int far2 = far;
      const int e2 = bfs_levels(far, far2);
      if (e2 <= ecc) break;
      s = far;
      ecc = e2;
      far = far2;
    }
    // Cuthill-McKee sweep of this component
    const size_t first = order.size();
    order.push_back(s);
    done[s] = 1;
    for (size_t h = first; h < order.size(); ++h) {
      const int u = order[h];
      nb.clear();
      for (int t = rp[u]; t < rp[u + 1]; ++t) {
        const int v = cl[t];
        if (v != u && !done[v]) {
          done[v] = 1;
          nb.push_back(v);
        }
      }
      std::sort(nb.begin(), nb.end(),
                [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// Device buffers of a streaming-engine workspace for Bp columns.
rafeast_status alloc_stream_work(rafeast_plan_s* P, int Bp, StreamWork& W,
                                 std::vector<void*>& bufs) {
  const int64_t n = P->n;
  const size_t cs = P->fp32 ? 2 * sizeof(float) : 2 * sizeof(double);
  auto get = [&](void** ptr, size_t bytes, const char* what) -> rafeast_status {
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 1);
    if (e != hipSuccess) {
      *ptr = nullptr;
      return hip_fail(P, e, what);
    }
    bufs.push_back(*ptr);
    return RAFEAST_OK;
  };
  W = StreamWork{};
  W.Bp = Bp;
  W.num_cu = P->num_cu;
  const size_t blk = (size_t)n * Bp;
  RCHK(get(&W.x, blk * cs, "stream x"));
  RCHK(get(&W.r, blk * cs, "stream r"));
  RCHK(get(&W.p0, blk * cs, "stream p"));
  RCHK(get(&W.p1, blk * cs, "stream p'"));
  RCHK(get(&W.w, blk * cs, "stream w"));
  RCHK(get(&W.xh, blk * 2 * sizeof(double), "stream x_hi"));
  if (P->dop.kind != 0) {
    if (P->dop.kind == 2 && 2 * (int64_t)Bp > P->dop.tcols)
      return fail(P, RAFEAST_UNSUPPORTED, "more columns than the covariance scratch holds");
    RCHK(get(&W.axh, blk * 2 * sizeof(double), "stream A x_hi"));
    RCHK(get(&W.pc, blk * cs, "stream packed p"));
    RCHK(get(&W.apc, blk * cs, "stream packed A p"));
    RCHK(get((void**)&W.cidx, (size_t)Bp * sizeof(int), "stream packed index"));
    RCHK(get((void**)&W.cmap, (size_t)Bp * sizeof(int), "stream packed map"));
  }
  RCHK(get((void**)&W.part, stream_partial_doubles((int)n, Bp, P->num_cu) * sizeof(double),
           "stream partials"));
  RCHK(get((void**)&W.zc, 2 * (size_t)Bp * sizeof(double), "stream shifts"));
  RCHK(get((void**)&W.scale, (size_t)Bp * sizeof(double), "stream scale"));
  RCHK(get((void**)&W.cnt, 2 * kStreamMaxGroups * sizeof(int), "stream census"));
  RCHK(get((void**)&W.cols.state, (size_t)Bp * sizeof(int), "stream state"));
  RCHK(get((void**)&W.cols.it, (size_t)Bp * sizeof(int), "stream it"));
  RCHK(get((void**)&W.cols.nref, (size_t)Bp * sizeof(int), "stream nref"));
  RCHK(get((void**)&W.cols.nbd, (size_t)Bp * sizeof(int), "stream nbd"));
  RCHK(get((void**)&W.cols.rho, 2 * (size_t)Bp * sizeof(double), "stream rho"));
  RCHK(get((void**)&W.cols.alpha, 2 * (size_t)Bp * sizeof(double), "stream alpha"));
  RCHK(get((void**)&W.cols.beta, 2 * (size_t)Bp * sizeof(double), "stream beta"));
  RCHK(get((void**)&W.cols.ctol2, (size_t)Bp * sizeof(double), "stream ctol"));
  RCHK(get((void**)&W.cols.res, (size_t)Bp * sizeof(double), "stream res"));
  RCHK(get((void**)&W.cols.bn, (size_t)Bp * sizeof(double), "stream bn"));
  RCHK(get((void**)&W.cols.lastit, (size_t)Bp * sizeof(int), "stream lastit"));
  RCHK(get((void**)&W.cols.span, (size_t)Bp * sizeof(int), "stream span"));
  RCHK(get((void**)&W.cols.span0, (size_t)Bp * sizeof(int), "stream span0"));
  RCHK(get((void**)&W.cols.rstart, (size_t)Bp * sizeof(int), "stream rstart"));
  RCHK(get((void**)&W.cols.sprev, (size_t)Bp * sizeof(double), "stream sprev"));
  return RAFEAST_OK;
}

// Device buffers of a multi-shift workspace for nz shifts and k columns: the
// shifted iterates, or (combining mode, the FEAST filter step) the block they
// are accumulated into.
rafeast_status alloc_ms_work(rafeast_plan_s* P, int nz, int k, MsWork& W,
                             std::vector<void*>& bufs, bool combining = false) {
  const int64_t n = P->n;
  auto get = [&](void** ptr, size_t bytes, const char* what) -> rafeast_status {
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 1);
    if (e != hipSuccess) {
      *ptr = nullptr;
      return hip_fail(P, e, what);
    }
    bufs.push_back(*ptr);
    return RAFEAST_OK;
  };
  W = MsWork{};
  W.kp = ms_padded(k);
  W.nz = nz;
  W.num_cu = P->num_cu;
  W.nb = ms_blocks((int)n, P->num_cu);
  const size_t blk = (size_t)n * W.kp, cs = (size_t)nz * W.kp;
  RCHK(get((void**)&W.r, blk * sizeof(double), "multi-shift r"));
  RCHK(get((void**)&W.p, blk * sizeof(double), "multi-shift p"));
  RCHK(get((void**)&W.w, blk * sizeof(double), "multi-shift w"));
  if (combining)
    RCHK(get((void**)&W.y, blk * sizeof(double), "multi-shift filtered block"));
  else
    RCHK(get((void**)&W.X, nz * blk * sizeof(cpx<double>), "multi-shift x"));
  RCHK(get((void**)&W.P, nz * blk * sizeof(cpx<double>), "multi-shift p^s"));
  RCHK(get((void**)&W.part, (size_t)W.nb * W.kp * sizeof(double), "multi-shift partials"));
  RCHK(get((void**)&W.sig, nz * sizeof(cpx<double>), "multi-shift sigma"));
  RCHK(get((void**)&W.count, sizeof(int), "multi-shift count"));
  MsCols& c = W.cols;
  RCHK(get((void**)&c.rr, W.kp * sizeof(double), "ms rr"));
  RCHK(get((void**)&c.bn, W.kp * sizeof(double), "ms bn"));
  RCHK(get((void**)&c.alpha, W.kp * sizeof(double), "ms alpha"));
  RCHK(get((void**)&c.alpha_prev, W.kp * sizeof(double), "ms alpha_prev"));
  RCHK(get((void**)&c.beta_prev, W.kp * sizeof(double), "ms beta_prev"));
  RCHK(get((void**)&c.scale, W.kp * sizeof(double), "ms scale"));
  RCHK(get((void**)&c.colive, W.kp * sizeof(int), "ms colive"));
  RCHK(get((void**)&c.pi, cs * sizeof(cpx<double>), "ms pi"));
  RCHK(get((void**)&c.pi_prev, cs * sizeof(cpx<double>), "ms pi_prev"));
  RCHK(get((void**)&c.pi_next, cs * sizeof(cpx<double>), "ms pi_next"));
  RCHK(get((void**)&c.ipi, cs * sizeof(cpx<double>), "ms 1/pi"));
  RCHK(get((void**)&c.as, cs * sizeof(cpx<double>), "ms alpha^s"));
  RCHK(get((void**)&c.bs, cs * sizeof(cpx<double>), "ms beta^s"));
  RCHK(get((void**)&c.live, cs * sizeof(int), "ms live"));
  RCHK(get((void**)&c.its, cs * sizeof(int), "ms its"));
  RCHK(get((void**)&c.est, cs * sizeof(double), "ms est"));
  if (combining) RCHK(get((void**)&c.gas, cs * sizeof(cpx<double>), "ms g alpha^s"));
  return RAFEAST_OK;
}

// The multi-shift seed: A - s I is positive definite for s below the
// Gershgorin interval.
double ms_seed(const rafeast_plan_s* P) {
  return P->sig_lo - 1e-3 * std::max(P->sig_hi - P->sig_lo, 1e-300);
}

// Shift of each streaming column: column c = j * k + i takes z_j; padding
// columns repeat z_0.
std::vector<double> stream_shifts(int nz, const double* z, int k, int Bp) {
  std::vector<double> zc(2 * (size_t)Bp);
  for (int c = 0; c < Bp; ++c) {
    const int j = c < nz * k ? c / k : 0;
    zc[2 * c] = z[2 * j];
    zc[2 * c + 1] = z[2 * j + 1];
  }
  return zc;
}

// ----------------------------------------------------------------------------
// building blocks on the plan
// ----------------------------------------------------------------------------
rafeast_status spmm(rafeast_plan_s* P, int k, const double* X, int ldx, double* Y, int ldy,
                    double alpha, double beta, const double* X2 = nullptr, int ldx2 = 0,
                    double gamma = 0.0) {
  if (P->dop.kind != 0) {
    // the GEMM forms alpha A X; the beta X and gamma X2 terms are added to it
    HIPCHK(P, dense_apply_f64(P->dop, P->st, k, X, ldx, Y, ldy, alpha, 0.0));
    if (beta != 0.0) {
      if (ldx != k || ldy != k) return fail(P, RAFEAST_UNSUPPORTED, "strided dense update");
      HIPCHK(P, dense_axpy(P->st, P->n * (int64_t)k, beta, X, Y));
    }
    if (X2) {
      if (ldx2 != k || ldy != k) return fail(P, RAFEAST_UNSUPPORTED, "strided dense update");
      HIPCHK(P, dense_axpy(P->st, P->n * (int64_t)k, gamma, X2, Y));
    }
    return RAFEAST_OK;
  }
  HIPCHK(P, launch_spmm_f64(P->st, (int)P->n, k, P->d_rowptr, P->d_col, P->d_val, P->nnz, X, ldx,
                            Y, ldy, alpha, beta, X2, ldx2, gamma, P->span));
  return RAFEAST_OK;
}

// CholQR2 on Y (n x k, ld) in place through P->d_T; *info as in rafeast_cholqr2.
// With track (k = m0), the product of the passes' transforms is formed on the
// device in d_mtot (pass 0 copies M, later passes multiply it on the right).
// A pass whose factorization failed writes nothing back to Y (the copy reads
// the pass's status on the device), so Y keeps the last good pass; the passes
// therefore run back to back and their statuses are read once at the end (a
// third pass follows when the first needed the shift).  d_mtot is not kept
// across a failure; the callers stop, or stop using it, on one.
rafeast_status cholqr2(rafeast_plan_s* P, int64_t n, int k, double* Y, int ldy, int* info,
                       double* tmp, int ldt, bool track = false) {
  int worst = 0;
  int passes = 2, read = 0;
  int flags[3] = {0, 0, 0};
  for (int pass = 0; pass < passes; ++pass) {
    HIPCHK(P, launch_gram(P->st, n, k, k, Y, ldy, Y, ldy, P->d_G, k, P->d_part));
    HIPCHK(P, launch_chol_inv(P->st, k, n, P->d_G, k, P->d_M, k, P->d_flag + pass));
    if (track) {
      if (pass == 0) {
        HIPCHK(P, hipMemcpyAsync(P->d_mtot, P->d_M, (size_t)k * k * sizeof(double),
                                 hipMemcpyDeviceToDevice, P->st));
      } else {
        HIPCHK(P, launch_tsmm(P->st, k, k, k, P->d_mtot, k, P->d_M, k, P->d_mtmp, k));
        std::swap(P->d_mtot, P->d_mtmp);
      }
    }
    HIPCHK(P, launch_tsmm(P->st, n, k, k, Y, ldy, P->d_M, k, tmp, ldt));
    HIPCHK(P, launch_copy_cols(P->st, n, k, tmp, ldt, Y, ldy, P->d_flag + pass));
    if (pass == passes - 1) {
      HIPCHK(P, hipMemcpyAsync(flags + read, P->d_flag + read, (pass + 1 - read) * sizeof(int),
                               hipMemcpyDeviceToHost, P->st));
      HIPCHK(P, hipStreamSynchronize(P->st));
      for (int q = read; q <= pass; ++q) {
        if (flags[q] == 2) {
          if (info) *info = 2;
          return RAFEAST_OK;  // Y keeps the last good pass
        }
        worst = std::max(worst, flags[q]);
      }
      read = pass + 1;
      if (flags[0] == 1 && passes == 2) passes = 3;
    }
  }
  if (info) *info = worst;
  return RAFEAST_OK;
}

// Rayleigh-Ritz on Q (n x m0): theta, rotated Q and W = A Q, residual block R,
// scaled residual norms; theta and res copied to the host arrays.
rafeast_status rayleigh_ritz(rafeast_plan_s* P, std::vector<double>& theta,
                             std::vector<double>& res, std::vector<double>& mu) {
  const int m0 = P->m0, ld = P->ld;
  const int64_t n = P->n;
  RCHK(spmm(P, m0, P->d_Q, ld, P->d_W, ld, 1.0, 0.0));
  HIPCHK(P, launch_gram(P->st, n, m0, m0, P->d_Q, ld, P->d_W, ld, P->d_G, m0, P->d_part));
  HIPCHK(P, launch_jacobi(P->st, m0, P->d_G, m0, P->d_theta, P->d_S, m0, P->d_jw));
  HIPCHK(P, launch_tsmm(P->st, n, m0, m0, P->d_Q, ld, P->d_S, m0, P->d_T, ld));
  std::swap(P->d_Q, P->d_T);
  HIPCHK(P, launch_tsmm(P->st, n, m0, m0, P->d_W, ld, P->d_S, m0, P->d_T, ld));
  std::swap(P->d_W, P->d_T);
  const double s_win = std::max(std::fabs(P->prm.lmin), std::fabs(P->prm.lmax));
  HIPCHK(P, launch_residual(P->st, n, m0, P->d_W, P->d_Q, ld, P->d_theta, s_win, P->d_R,
                            P->d_res, P->d_qn, P->d_part));
  theta.resize(m0);
  res.resize(m0);
  HIPCHK(P, hipMemcpyAsync(theta.data(), P->d_theta, m0 * sizeof(double), hipMemcpyDeviceToHost,
                           P->st));
  HIPCHK(P, hipMemcpyAsync(res.data(), P->d_res, m0 * sizeof(double), hipMemcpyDeviceToHost,
                           P->st));
  // filter gain of each Ritz vector q_i = Q~ y_i, y_i = mtot S e_i, of the
  // orthonormal block Q_prev that Q~ filtered: mu_i = 1 / ||y_i|| =
  // ||rho(A) Q_prev y_i|| / ||Q_prev y_i||; 1 before the first filter step.
  // Y = mtot S on the device; its column norms on the host.
  std::vector<double> Yh;
  if (P->have_filter) {
    HIPCHK(P, launch_tsmm(P->st, m0, m0, m0, P->d_mtot, m0, P->d_S, m0, P->d_mtmp, m0));
    Yh.resize((size_t)m0 * m0);
    HIPCHK(P, hipMemcpyAsync(Yh.data(), P->d_mtmp, Yh.size() * sizeof(double),
                             hipMemcpyDeviceToHost, P->st));
  }
  HIPCHK(P, hipStreamSynchronize(P->st));
  mu.assign(m0, 1.0);
  if (P->have_filter) {
    std::vector<double> ss(m0, 0.0);
    for (int r = 0; r < m0; ++r)
      for (int i = 0; i < m0; ++i) ss[i] += Yh[(size_t)r * m0 + i] * Yh[(size_t)r * m0 + i];
    for (int i = 0; i < m0; ++i) mu[i] = ss[i] > 0.0 ? 1.0 / std::sqrt(ss[i]) : 0.0;
  }
  return RAFEAST_OK;
}

// The resident-launch descriptor of the plan's matrix with the given RHS,
// outputs and shift table.
ResGraph resident_graph(const rafeast_plan_s* P, const double* d_zs, int k, const double* B,
                        int ldb, void* D, int ldd, int* d_iters, double* d_resid,
                        const int* wave_slices) {
  ResGraph gd;
  gd.nslices = P->sell.nslices;
  gd.zero_base = P->sell.zero_base;
  gd.ldb = ldb;
  gd.kcols = k;
  gd.ldd = ldd;
  gd.sbase = P->sell.sbase;
  gd.perm = P->sell.perm;
  gd.ent = P->fp32 ? (const void*)P->sell.v32 : (const void*)P->sell.e64;
  gd.n32 = P->sell.n32;
  gd.ent64 = P->sell.e64;
  gd.wave_slices = wave_slices;
  gd.B = B;
  gd.D = D;
  gd.zs = d_zs;
  gd.iters = d_iters;
  gd.resid = d_resid;
  gd.stats = P->d_stats;
  gd.tol = P->tau;
  return gd;
}

// COCG over items (0, j, i) of the given shift table; outputs into D.
rafeast_status run_cocg(rafeast_plan_s* P, int nitems, const int* d_items, const double* d_zs,
                        int k, const double* B, int ldb, void* D, int ldd, double tol,
                        int* d_iters, double* d_resid = nullptr) {
  // 32-bit indexing of the RHS and output blocks inside the kernel
  if (P->n * (int64_t)ldb >= (int64_t(1) << 31) || P->n * (int64_t)ldd >= (int64_t(1) << 31))
    return fail(P, RAFEAST_UNSUPPORTED, "blocks too large for the resident engine");
  const ResGraph gd =
      resident_graph(P, d_zs, k, B, ldb, D, ldd, d_iters, d_resid, P->sell.wave_slices);
  CocgLaunch L;
  L.nitems = nitems;
  L.items = d_items;
  L.tol = tol;
  L.maxit = P->prm.max_cocg;
  L.max_refine = 64;
  L.counter = P->d_counter;
  L.xhi = P->d_xhi;
  L.xhi_slots = P->xhi_slots;
  HIPCHK(P, hipMemsetAsync(P->d_counter, 0, sizeof(int), P->st));
  HIPCHK(P, launch_cocg_resident(P->st, &gd, nullptr, (int)P->n, P->sell.wave_rpt, L, P->fp32,
                                 P->num_cu));
  return RAFEAST_OK;
}

// Streaming engine: all nz * k systems of one solve in lock step.  W must be
// sized for stream_padded_columns(k, nz * k) columns, with W.zc filled by
// stream_shifts.
rafeast_status run_stream(rafeast_plan_s* P, const StreamWork& W, int nz, int k, const double* B,
                          int ldb, void* D, int ldd, double tol, int* d_iters,
                          double* d_resid = nullptr) {
  StreamLaunch L;
  L.B = B;
  L.ldb = ldb;
  L.k = k;
  L.ncols = nz * k;
  L.D = D;
  L.ldd = ldd;
  L.tol = tol;
  L.maxit = P->prm.max_cocg;
  L.iters = d_iters;
  L.resid = d_resid;
  L.stats = P->d_stats;
  HIPCHK(P, run_stream_cocg(P->st, P->smat, W, L, P->fp32));
  return RAFEAST_OK;
}

// Multi-shift engine in combining mode for one FEAST filter step: the
// weights g (gamma_{j,i} of the residual form, w_j of the literal form) on
// the device, the filtered block written to P->d_Y.
rafeast_status run_ms_combine(rafeast_plan_s* P, const double* B, const double* g,
                              const double* Qin) {
  MsLaunch L;
  L.B = B;
  L.ldb = P->ld;
  L.k = P->m0;
  L.nz = P->nc;
  L.z = P->zw.data();
  L.seed = ms_seed(P);
  L.tol = P->tau;
  L.maxit = P->prm.max_cocg;
  L.iters = P->d_iters;
  L.g = g;
  L.Qin = Qin;
  L.ldqin = P->ld;
  L.Qt = P->d_Y;
  L.ldq = P->ld;
  HIPCHK(P, run_mshift(P->st, P->smat, P->mswork, L));
  return RAFEAST_OK;
}

// Multi-shift engine: the nz shifts of every column c < k in one seed CG.
rafeast_status run_ms(rafeast_plan_s* P, const MsWork& W, int nz, const double* z, int k,
                      const double* B, int ldb, void* D, int ldd, double tol, int* d_iters,
                      double* d_resid = nullptr) {
  MsLaunch L;
  L.B = B;
  L.ldb = ldb;
  L.k = k;
  L.nz = nz;
  L.z = z;
  L.seed = ms_seed(P);
  L.D = D;
  L.ldd = ldd;
  L.tol = tol;
  L.maxit = P->prm.max_cocg;
  L.iters = d_iters;
  L.resid = d_resid;
  HIPCHK(P, run_mshift(P->st, P->smat, W, L));
  return RAFEAST_OK;
}

// Direct engine: assemble and factorize z_j I - A for the plan's nc nodes
// (once per plan: the shifts are fixed).  A vanishing pivot is BREAKDOWN.
rafeast_status band_factor_shifts(rafeast_plan_s* P) {
  const int n = (int)P->n, b = P->band_b;
  hipEvent_t t0 = P->ev[0], t1 = P->ev[1];
  HIPCHK(P, hipEventRecord(t0, P->st));
  HIPCHK(P, band_assemble(P->st, n, b, P->d_srow, P->d_scol, P->d_sv64, P->nc, P->d_zw,
                          P->d_band));
  HIPCHK(P, band_factor(P->st, n, b, P->nc, P->d_band, P->d_binfo));
  HIPCHK(P, hipEventRecord(t1, P->st));
  std::vector<int> info(P->nc);
  HIPCHK(P, hipMemcpyAsync(info.data(), P->d_binfo, P->nc * sizeof(int), hipMemcpyDeviceToHost,
                           P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  HIPCHK(P, hipEventElapsedTime(&P->factor_ms, t0, t1));
  for (int j = 0; j < P->nc; ++j)
    if (info[j] != 0)
      return fail(P, RAFEAST_BREAKDOWN,
                  "LDL^T of z_" + std::to_string(j) + " I - A: pivot " +
                      std::to_string(info[j] - 1) + " vanished");
  if (verbose_log())
    std::fprintf(stderr, "rafeast: direct engine: bandwidth %d, %d shifts factorized in %.2f ms\n",
                 b, P->nc, P->factor_ms);
  return RAFEAST_OK;
}

// Orders (shift, column) pairs longest-first: the smaller Im z, the more COCG
// iterations a system needs.
std::vector<int> make_items(int nz, const double* zs, int k, int g = 0) {
  std::vector<int> js(nz);
  for (int j = 0; j < nz; ++j) js[j] = j;
  std::stable_sort(js.begin(), js.end(),
                   [&](int a, int b) { return std::fabs(zs[2 * a + 1]) < std::fabs(zs[2 * b + 1]); });
  std::vector<int> items;
  items.reserve(3 * (size_t)nz * k);
  for (int j : js)
    for (int i = 0; i < k; ++i) {
      items.push_back(g);
      items.push_back(j);
      items.push_back(i);
    }
  return items;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0f;
  return ms;
}

int resolve_ws_op(const rafeast_plan_s* P) {
  const int op = P->prm.ws_op;
  if (op != RAFEAST_WS_AUTO) return op;
  if (P->prm.lmin <= P->sig_lo) return RAFEAST_WS_FLIP;
  if (P->prm.lmax >= P->sig_hi) return RAFEAST_WS_LITERAL;
  return RAFEAST_WS_FOLD;
}

// ----------------------------------------------------------------------------
// learned polynomial preconditioner: device buffers, spectral map, solver
// ----------------------------------------------------------------------------
namespace {
struct DevBuf {  // device allocations released together
  std::vector<void*> ptrs;
  ~DevBuf() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  template <typename T>
  hipError_t get(T** p, size_t count) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, (count ? count : 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(q);
    *p = (T*)q;
    return e;
  }
};

void spectral_map(const rafeast_plan_s* P, double& a, double& b) {
  a = 2.0 / (P->sig_hi - P->sig_lo);
  b = -(P->sig_hi + P->sig_lo) / (P->sig_hi - P->sig_lo);
}

// FP64 COCG on the nz * k systems (z_j I - A) X[:, j k + i] = B[:, i] in lock
// step (X n x nz k complex, row-major), preconditioned by p_j(A) with
// coefficients coef (host [nz][8] complex) or plain (coef null).  iters,
// resid: nullable host [nz k].
rafeast_status pc_solve_run(rafeast_plan_s* P, int nz, const double* z, int k, const double* B,
                            int ldb, const double* coef, void* Xout, double tol, int* iters,
                            double* resid, int maxit = -1, void* r_out = nullptr) {
  const int64_t n = P->n;
  const int Bc = nz * k;
  DevBuf buf;
  PcSolve S;
  S.n = n;
  S.rowptr = P->d_rowptr;
  S.col = P->d_col;
  S.val = P->d_val;
  spectral_map(P, S.a, S.b);
  S.Bc = Bc;
  S.B = B;
  S.ldb = ldb;
  S.kb = k;
  S.tol = tol;
  S.maxit = maxit >= 0 ? maxit : P->prm.max_cocg;
  S.num_cu = P->num_cu;
  S.progress = verbose_log();
  const size_t blk = (size_t)n * Bc;
  S.x = (cpx<double>*)Xout;
  HIPCHK(P, buf.get(&S.r, blk));
  HIPCHK(P, buf.get(&S.p0, blk));
  HIPCHK(P, buf.get(&S.p1, blk));
  HIPCHK(P, buf.get(&S.w, blk));
  if (coef) {
    HIPCHK(P, buf.get(&S.u, blk));
    HIPCHK(P, buf.get(&S.t0, blk));
    HIPCHK(P, buf.get(&S.t1, blk));
    HIPCHK(P, buf.get(&S.t2, blk));
  }
  double *zc = nullptr, *cf = nullptr;
  HIPCHK(P, buf.get(&S.part, (size_t)pc_blocks(n, P->num_cu) * Bc * 3));
  HIPCHK(P, buf.get(&S.counts, 2));
  HIPCHK(P, buf.get(&zc, 2 * (size_t)Bc));
  HIPCHK(P, buf.get(&S.cols.active, Bc));
  HIPCHK(P, buf.get(&S.cols.it, Bc));
  HIPCHK(P, buf.get(&S.cols.pending, Bc));
  HIPCHK(P, buf.get(&S.cols.bn2, Bc));
  HIPCHK(P, buf.get(&S.cols.res, Bc));
  HIPCHK(P, buf.get(&S.cols.rho, 2 * (size_t)Bc));
  HIPCHK(P, buf.get(&S.cols.rhon, 2 * (size_t)Bc));
  HIPCHK(P, buf.get(&S.cols.alpha, 2 * (size_t)Bc));
  HIPCHK(P, buf.get(&S.cols.beta, 2 * (size_t)Bc));
  std::vector<double> hz(2 * (size_t)Bc), hc;
  for (int c = 0; c < Bc; ++c) {
    hz[2 * c] = z[2 * (c / k)];
    hz[2 * c + 1] = z[2 * (c / k) + 1];
  }
  HIPCHK(P, hipMemcpyAsync(zc, hz.data(), hz.size() * sizeof(double), hipMemcpyHostToDevice,
                           P->st));
  S.zc = zc;
  if (coef) {  // [8][Bc] complex from the per-shift [nz][8] complex
    hc.resize(16 * (size_t)Bc);
    for (int t = 0; t < 8; ++t)
      for (int c = 0; c < Bc; ++c) {
        hc[(size_t)t * 2 * Bc + 2 * c] = coef[(c / k) * 16 + 2 * t];
        hc[(size_t)t * 2 * Bc + 2 * c + 1] = coef[(c / k) * 16 + 2 * t + 1];
      }
    HIPCHK(P, buf.get(&cf, hc.size()));
    HIPCHK(P, hipMemcpyAsync(cf, hc.data(), hc.size() * sizeof(double), hipMemcpyHostToDevice,
                             P->st));
    S.coef = cf;
  }
  HIPCHK(P, run_pc_cocg(P->st, S));
  if (r_out)
    HIPCHK(P, hipMemcpyAsync(r_out, S.r, blk * sizeof(cpx<double>), hipMemcpyDeviceToDevice,
                             P->st));
  std::vector<int> hit(Bc);
  std::vector<double> hres(Bc);
  HIPCHK(P, hipMemcpyAsync(hit.data(), S.cols.it, Bc * sizeof(int), hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipMemcpyAsync(hres.data(), S.cols.res, Bc * sizeof(double), hipMemcpyDeviceToHost,
                           P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  if (iters) std::memcpy(iters, hit.data(), Bc * sizeof(int));
  if (resid) std::memcpy(resid, hres.data(), Bc * sizeof(double));
  return RAFEAST_OK;
}
}  // namespace

// ----------------------------------------------------------------------------
// Phase 2 in steps (one plan, or several in lock step for the batching form)
// ----------------------------------------------------------------------------
struct SolveRun {
  std::vector<double> theta, rs, mu;
  std::vector<int> iters;
  rafeast_status status = RAFEAST_NO_CONVERGENCE;
  int it = 0, M = 0;
  double maxres = 0.0;
  double prev_maxres = 0.0;  // largest counted residual of the previous test (0: none)
  int64_t cocg_sum = 0;
  int cocg_max = 0;
  std::vector<int64_t> cocg_node;  // per quadrature node, summed over columns and iterations
  int pc_fallbacks = 0;
  bool pc_solved = false;          // the last solves ran preconditioned (iters filled on host)
  bool combined = false;           // the solves wrote the filtered block themselves (d_Y)
  bool breakdown = false, done = false;
  double t_ph[RAFEAST_NPHASE] = {0, 0, 0, 0, 0};
};

// Counted pairs: theta in the closed window and filter gain >= 1/4 (an
// eigenvector in the window has gain |rho| >= 1/2; a mixture of outside
// eigenvectors whose Ritz value falls in the window has a small gain).
bool counted(const rafeast_plan_s* P, const SolveRun& S, int i) {
  return S.theta[i] >= P->prm.lmin && S.theta[i] <= P->prm.lmax && S.mu[i] >= kSpuriousGain;
}

// Start block: Q_init, else the last warm start, else the orthonormalised
// device sketch.
rafeast_status solve_begin(rafeast_plan_s* P, const double* Q_init, SolveRun& S) {
  P->err.clear();
  const int64_t n = P->n;
  const int m0 = P->m0, ld = P->ld;
  HIPCHK(P, hipEventRecord(P->ev[6], P->st));
  if (Q_init) {
    HIPCHK(P, hipMemcpyAsync(P->d_T, Q_init, (size_t)n * m0 * sizeof(double),
                             hipMemcpyHostToDevice, P->st));
    HIPCHK(P, launch_colmajor_to_rowmajor(P->st, n, m0, P->d_T, P->d_Q, ld));
    int ci = 0;
    RCHK(cholqr2(P, n, m0, P->d_Q, ld, &ci, P->d_T, ld));
    if (ci == 2) return fail(P, RAFEAST_BREAKDOWN, "Q_init is rank deficient");
  } else if (!P->have_start) {
    HIPCHK(P, launch_gaussian(P->st, n, m0, P->prm.seed, P->d_Q, ld));
    int ci = 0;
    RCHK(cholqr2(P, n, m0, P->d_Q, ld, &ci, P->d_T, ld));
    if (ci == 2) return fail(P, RAFEAST_BREAKDOWN, "random start is rank deficient");
  }
  HIPCHK(P, hipMemsetAsync(P->d_stats, 0, 2 * sizeof(int), P->st));
  P->have_filter = false;
  P->tau = std::max(P->prm.tol_solve, P->prm.tol_solve_relaxed);
  if (P->prm.precond == RAFEAST_PC_LEARNED && !P->pc_ready)
    return fail(P, RAFEAST_INVALID_ARG, "precond LEARNED needs rafeast_pc_attach first");
  S = SolveRun();
  S.iters.assign(P->nitems, 0);
  S.cocg_node.assign(P->nc, 0);
  return RAFEAST_OK;
}

// Rayleigh-Ritz and the stopping tests; S.done when the iteration ends here.
rafeast_status solve_test(rafeast_plan_s* P, SolveRun& S) {
  const int m0 = P->m0;
  HIPCHK(P, hipEventRecord(P->ev[0], P->st));
  RCHK(rayleigh_ritz(P, S.theta, S.rs, S.mu));
  P->last_theta = S.theta;
  HIPCHK(P, hipEventRecord(P->ev[1], P->st));
  HIPCHK(P, hipEventSynchronize(P->ev[1]));
  S.t_ph[RAFEAST_PH_RR] += elapsed(P->ev[0], P->ev[1]);
  S.M = 0;
  S.maxres = 0.0;
  int in_window = 0;  // Ritz values in the window, spurious or not
  for (int i = 0; i < m0; ++i) in_window += S.theta[i] >= P->prm.lmin && S.theta[i] <= P->prm.lmax;
  for (int i = 0; i < m0; ++i)
    if (counted(P, S, i)) {
      ++S.M;
      S.maxres = std::max(S.maxres, S.rs[i]);
    }
  if (S.M > 0 && S.maxres <= P->prm.tol_eig) {
    S.status = RAFEAST_OK;
    S.done = true;
  } else if (in_window == 0 && S.it >= 2) {
    S.status = RAFEAST_EMPTY_WINDOW;
    S.done = true;
  } else if (S.it >= P->prm.max_iter) {
    S.done = true;
  }
  // Relaxed solves (Theorem 2): e_{m+1} <= rho e_m + eps^(m), and in the
  // residual-correction form a solve of relative accuracy tau contributes
  // eps^(m) of order tau e_m.  While the iteration keeps contracting, tau
  // stays; a filter application that fails to halve the largest counted
  // residual means the solve error has caught up with the contraction, and
  // tau drops 100-fold, not below tol_solve.
  if (!S.done && S.it >= 1 && S.prev_maxres > 0.0 && S.M > 0 && P->tau > P->prm.tol_solve &&
      S.maxres > 0.5 * S.prev_maxres)
    P->tau = std::max(P->prm.tol_solve, 1e-2 * P->tau);
  if (S.M > 0) S.prev_maxres = S.maxres;
  return RAFEAST_OK;
}

// The shifted solves with the learned preconditioner (precond LEARNED): the
// features of each node from the current Ritz values, the network's
// coefficients, FP64 preconditioned COCG on all (node, column) systems into
// d_D64, and plain FP64 COCG for every system that missed the tolerance by
// true residual.  Fills S.iters (preconditioned plus fallback iterations).
rafeast_status solve_learned(rafeast_plan_s* P, SolveRun& S) {
  const int m0 = P->m0, nc = P->nc, ld = P->ld;
  const int64_t n = P->n;
  const bool residual_form = P->prm.rhs_form == RAFEAST_RHS_RESIDUAL;
  const double* B = residual_form ? P->d_R : P->d_Q;
  double a = 0.0, b = 0.0;
  spectral_map(P, a, b);
  const double th_lo = a * S.theta.front() + b, th_hi = a * S.theta.back() + b;
  std::vector<double> feat(4 * (size_t)nc);
  for (int j = 0; j < nc; ++j) {
    feat[4 * j + 0] = a * P->zw[2 * j] + b;
    feat[4 * j + 1] = a * P->zw[2 * j + 1];
    feat[4 * j + 2] = th_lo;
    feat[4 * j + 3] = th_hi;
  }
  std::vector<float> out(16 * (size_t)nc);
  HIPCHK(P, hipMemcpyAsync(P->d_pcX, feat.data(), feat.size() * sizeof(double),
                           hipMemcpyHostToDevice, P->st));
  HIPCHK(P, launch_mlp_forward(P->st, nc, P->d_pcX, P->d_pcWb, P->d_pcY));
  HIPCHK(P, hipMemcpyAsync(out.data(), P->d_pcY, out.size() * sizeof(float),
                           hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  // the network predicts the coefficients scaled by Im z^: c = y / Im z^
  std::vector<double> coef(16 * (size_t)nc);
  for (size_t t = 0; t < coef.size(); ++t) coef[t] = (double)out[t] / feat[4 * (t / 16) + 1];
  const int Bc = nc * m0;
  std::vector<double> res(Bc);
  RCHK(pc_solve_run(P, nc, P->zw.data(), m0, B, ld, coef.data(), P->d_D64, P->tau, S.iters.data(),
                    res.data()));
  // judge by true residual; the systems that missed the tolerance are solved
  // again by plain FP64 COCG, all misses of one node in one lock-step solve
  DevBuf fb;
  for (int j = 0; j < nc; ++j) {
    std::vector<int> miss;
    for (int i = 0; i < m0; ++i)
      if (!(res[(size_t)j * m0 + i] <= P->tau)) miss.push_back(i);
    if (miss.empty()) continue;
    const int kf = (int)miss.size();
    double* Bf = nullptr;
    cpx<double>* Xf = nullptr;
    HIPCHK(P, fb.get(&Bf, (size_t)n * kf));
    HIPCHK(P, fb.get(&Xf, (size_t)n * kf));
    for (int t = 0; t < kf; ++t)
      HIPCHK(P, hipMemcpy2DAsync(Bf + t, (size_t)kf * sizeof(double), B + miss[t],
                                 (size_t)ld * sizeof(double), sizeof(double), (size_t)n,
                                 hipMemcpyDeviceToDevice, P->st));
    std::vector<int> it(kf);
    std::vector<double> r1(kf);
    RCHK(pc_solve_run(P, 1, P->zw.data() + 2 * j, kf, Bf, kf, nullptr, Xf, P->tau, it.data(),
                      r1.data()));
    for (int t = 0; t < kf; ++t) {
      const int c = j * m0 + miss[t];
      HIPCHK(P, hipMemcpy2DAsync((cpx<double>*)P->d_D64 + c, (size_t)Bc * sizeof(cpx<double>),
                                 Xf + t, (size_t)kf * sizeof(cpx<double>), sizeof(cpx<double>),
                                 (size_t)n, hipMemcpyDeviceToDevice, P->st));
      S.iters[c] += it[t];
    }
    HIPCHK(P, hipStreamSynchronize(P->st));
    S.pc_fallbacks += kf;
    if (verbose_log())
      std::fprintf(stderr, "rafeast: node %d: %d systems solved again without the preconditioner\n",
                   j, kf);
  }
  S.pc_solved = true;
  return RAFEAST_OK;
}

// The shifted solves of one plan, for all (node, column) pairs.
rafeast_status solve_shifted_systems(rafeast_plan_s* P, SolveRun& S) {
  const int m0 = P->m0, nc = P->nc, ld = P->ld;
  const bool residual_form = P->prm.rhs_form == RAFEAST_RHS_RESIDUAL;
  S.pc_solved = false;
  S.combined = false;
  if (P->prm.precond == RAFEAST_PC_LEARNED) return solve_learned(P, S);
  if (P->engine == RAFEAST_ENGINE_MULTISHIFT) {
    // the filter combination happens inside the engine: weights first
    if (residual_form)
      HIPCHK(P, launch_gamma(P->st, nc, m0, P->d_zw, P->d_theta, P->d_gamma));
    RCHK(run_ms_combine(P, residual_form ? P->d_R : P->d_Q,
                        residual_form ? P->d_gamma : P->d_wrep, residual_form ? P->d_Q : nullptr));
    S.combined = true;
    return RAFEAST_OK;
  }
  if (P->engine == RAFEAST_ENGINE_DIRECT) {
    // exact solves by the factors; no Krylov iterations to report
    HIPCHK(P, hipMemsetAsync(P->d_iters, 0, P->nitems * sizeof(int), P->st));
    HIPCHK(P, band_solve(P->st, (int)P->n, P->band_b, nc, P->d_band, P->d_sperm,
                         residual_form ? P->d_R : P->d_Q, ld, m0,
                         static_cast<cpx<double>*>(P->d_D), (int64_t)nc * m0));
    return RAFEAST_OK;
  }
  if (P->engine == RAFEAST_ENGINE_STREAM)
    return run_stream(P, P->swork, nc, m0, residual_form ? P->d_R : P->d_Q, ld, P->d_D, nc * m0,
                      P->tau, P->d_iters);
  return run_cocg(P, P->nitems, P->d_items, P->d_zw, m0, residual_form ? P->d_R : P->d_Q, ld,
                  P->d_D, nc * m0, P->tau, P->d_iters);
}

// After the solves (between events ev[2] and ev[3]): combination
// Q~ = sum_j Re[w_j (z_j I - A)^{-1} Q], CholQR2, timings, counters.
rafeast_status solve_combine(rafeast_plan_s* P, SolveRun& S) {
  const int64_t n = P->n;
  const int m0 = P->m0, nc = P->nc, ld = P->ld;
  const bool residual_form = P->prm.rhs_form == RAFEAST_RHS_RESIDUAL;
  if (!S.pc_solved)
    HIPCHK(P, hipMemcpyAsync(S.iters.data(), P->d_iters, P->nitems * sizeof(int),
                             hipMemcpyDeviceToHost, P->st));
  if (!S.combined) {
    HIPCHK(P, launch_gamma(P->st, nc, m0, P->d_zw, P->d_theta, P->d_gamma));
    HIPCHK(P, launch_combine(P->st, n, nc, m0, P->d_gamma, P->d_zw, residual_form, P->d_Q, ld,
                             S.pc_solved ? P->d_D64 : P->d_D, nc * m0,
                             S.pc_solved ? false : P->fp32, P->d_Y, ld));
  }
  HIPCHK(P, hipEventRecord(P->ev[4], P->st));
  std::swap(P->d_Q, P->d_Y);
  int ci = 0;
  RCHK(cholqr2(P, n, m0, P->d_Q, ld, &ci, P->d_T, ld, true));
  P->have_filter = ci != 2;
  HIPCHK(P, hipEventRecord(P->ev[5], P->st));
  HIPCHK(P, hipEventSynchronize(P->ev[5]));
  if (ci == 2) S.breakdown = true;
  S.t_ph[RAFEAST_PH_SOLVE] += elapsed(P->ev[2], P->ev[3]);
  S.t_ph[RAFEAST_PH_COMBINE] += elapsed(P->ev[3], P->ev[4]);
  S.t_ph[RAFEAST_PH_ORTH] += elapsed(P->ev[4], P->ev[5]);
  int64_t it_sum = 0;
  int it_max = 0;
  for (size_t c = 0; c < S.iters.size(); ++c) {
    const int v = S.iters[c];
    it_sum += v;
    it_max = std::max(it_max, v);
    S.cocg_node[c / m0] += v;
  }
  S.cocg_sum += it_sum;
  S.cocg_max = std::max(S.cocg_max, it_max);
  if (verbose_log())
    std::fprintf(stderr,
                 "rafeast: iteration %d: M %d, max residual %.3e, COCG %lld (max %d), "
                 "solve %.1f ms\n",
                 S.it + 1, S.M, S.maxres, (long long)it_sum, it_max, elapsed(P->ev[2], P->ev[3]));
  ++S.it;
  return RAFEAST_OK;
}

// Status and outputs of a finished iteration.
rafeast_status solve_finish(rafeast_plan_s* P, SolveRun& S, rafeast_result* res) {
  const int64_t n = P->n;
  const int m0 = P->m0, ld = P->ld;
  rafeast_status status = S.status;
  if (status == RAFEAST_OK && S.M >= m0) status = RAFEAST_SUBSPACE_TOO_SMALL;
  if (S.breakdown && status != RAFEAST_OK) status = RAFEAST_BREAKDOWN;
  // outputs: counted pairs, ascending (theta is sorted)
  std::vector<int> sel;
  for (int i = 0; i < m0; ++i)
    if (counted(P, S, i)) sel.push_back(i);
  std::vector<double> lam(sel.size()), rsel(sel.size());
  for (size_t a = 0; a < sel.size(); ++a) {
    lam[a] = S.theta[sel[a]];
    rsel[a] = S.rs[sel[a]];
  }
  const bool dev_out = (res->flags & RAFEAST_PTR_DEVICE) != 0;
  if (!sel.empty()) {
    if (dev_out) {
      HIPCHK(P, hipMemcpyAsync(res->lambda, lam.data(), lam.size() * sizeof(double),
                               hipMemcpyHostToDevice, P->st));
      HIPCHK(P, hipMemcpyAsync(res->resid, rsel.data(), rsel.size() * sizeof(double),
                               hipMemcpyHostToDevice, P->st));
    } else {
      std::memcpy(res->lambda, lam.data(), lam.size() * sizeof(double));
      std::memcpy(res->resid, rsel.data(), rsel.size() * sizeof(double));
    }
  }
  if (res->X && !sel.empty()) {
    HIPCHK(P, hipMemcpyAsync(P->d_sel, sel.data(), sel.size() * sizeof(int), hipMemcpyHostToDevice,
                             P->st));
    double* dst = dev_out ? res->X : P->d_T;
    HIPCHK(P, launch_export_vectors(P->st, n, (int)sel.size(), P->d_sel, P->d_Q, ld, dst, nullptr));
    if (!dev_out)
      HIPCHK(P, hipMemcpyAsync(res->X, P->d_T, (size_t)n * sel.size() * sizeof(double),
                               hipMemcpyDeviceToHost, P->st));
  }
  int stats[2] = {0, 0};
  HIPCHK(P, hipMemcpyAsync(stats, P->d_stats, 2 * sizeof(int), hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipEventRecord(P->ev[7], P->st));
  HIPCHK(P, hipEventSynchronize(P->ev[7]));
  S.t_ph[RAFEAST_PH_TOTAL] = elapsed(P->ev[6], P->ev[7]);
  P->have_start = false;  // the next solve without Q_init starts afresh
  res->M = S.M;
  res->iters = S.it;
  res->cocg_iters = S.cocg_sum;
  res->cocg_max = S.cocg_max;
  res->refinements = stats[0];
  res->max_resid = S.maxres;
  res->tol_solve_last = P->tau;
  for (int i = 0; i < RAFEAST_NPHASE; ++i) res->t_ms[i] = S.t_ph[i];
  for (int j = 0; j < 64; ++j) res->cocg_node[j] = j < (int)S.cocg_node.size() ? S.cocg_node[j] : 0;
  res->pc_fallbacks = S.pc_fallbacks;
  if (stats[1] > 0 && status != RAFEAST_OK)
    P->err = std::to_string(stats[1]) + " COCG systems broke down";
  return status;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

void rafeast_params_default(rafeast_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->lmin = 0.0;
  p->lmax = 0.0;
  p->m0 = 0;
  p->nc = 8;
  p->q = 2;
  p->p = -1;
  p->tol_eig = 1e-10;
  p->tol_solve = 1e-6;
  p->max_iter = 20;
  p->max_cocg = 20000;
  p->precision = RAFEAST_FP32_REFINED;
  p->ws_op = RAFEAST_WS_AUTO;
  p->rhs_form = RAFEAST_RHS_RESIDUAL;
  p->engine = RAFEAST_ENGINE_AUTO;
  p->seed = 0;
  p->hip_stream = nullptr;
}

const char* rafeast_status_string(int s) {
  // switched on as int: a C caller may pass any value, and an enum object
  // holding one outside the enumerators is undefined in C++
  switch (s) {
    case RAFEAST_OK: return "OK";
    case RAFEAST_INVALID_ARG: return "INVALID_ARG";
    case RAFEAST_BAD_CSR: return "BAD_CSR";
    case RAFEAST_NOT_SYMMETRIC: return "NOT_SYMMETRIC";
    case RAFEAST_OOM: return "OOM";
    case RAFEAST_DEVICE: return "DEVICE";
    case RAFEAST_NO_CONVERGENCE: return "NO_CONVERGENCE";
    case RAFEAST_SUBSPACE_TOO_SMALL: return "SUBSPACE_TOO_SMALL";
    case RAFEAST_BREAKDOWN: return "BREAKDOWN";
    case RAFEAST_EMPTY_WINDOW: return "EMPTY_WINDOW";
    case RAFEAST_UNSUPPORTED: return "UNSUPPORTED";
  }
  return "UNKNOWN";
}

const char* rafeast_last_error(rafeast_plan_t plan) {
  return plan ? plan->err.c_str() : g_plan_error.c_str();
}

void rafeast_destroy(rafeast_plan_t plan) { free_plan(plan); }

// Autotuned launch shape of the resident engine: how many SELL slices
// (slots) each thread holds, which fixes the wave table and the kernel
// instance.  Every slot count from the smallest that fits up to the engine's
// maximum is timed on the plan's own matrix: the first min(systems, CUs)
// systems of the solve order (the hardest shift first) on Gaussian
// right-hand sides, run for a fixed 64 iterations (tolerance 0), one untimed
// launch and then the best of two timed ones; the fastest count wins (ties
// to fewer slots).  RAFEAST_TUNE=0 keeps the smallest count;
// RAFEAST_RESIDENT_SLOTS=r takes candidate r untimed (plan creation fails if
// r is not a candidate), so that two plans can be given the same layout and
// hence the same summation order.
rafeast_status tune_resident(rafeast_plan_s* P) {
  const int maxr = P->fp32 ? 8 : 4;
  std::vector<std::vector<int>> tabs;
  P->tune_cand.clear();
  for (int r = P->sell.wave_rpt; r <= maxr; r *= 2) {
    std::vector<int> t = cocg_resident_wave_table(P->sell_widths, r);
    if (t.empty()) continue;
    P->tune_cand.push_back(r);
    tabs.push_back(std::move(t));
  }
  P->tune_ms.assign(P->tune_cand.size(), 0.0f);
  P->tune_choice = P->sell.wave_rpt;
  if (const char* forced = std::getenv("RAFEAST_RESIDENT_SLOTS")) {
    size_t c = 0;
    while (c < P->tune_cand.size() && std::to_string(P->tune_cand[c]) != forced) ++c;
    if (c == P->tune_cand.size())
      return fail(P, RAFEAST_INVALID_ARG,
                  std::string("RAFEAST_RESIDENT_SLOTS=") + forced +
                      " is not a slot count this matrix can use");
    HIPCHK(P, hipMemcpyAsync(P->d_wtab, tabs[c].data(), tabs[c].size() * sizeof(int),
                             hipMemcpyHostToDevice, P->st));
    HIPCHK(P, hipStreamSynchronize(P->st));
    P->tune_choice = P->tune_cand[c];
    P->sell.wave_rpt = P->tune_choice;
    return RAFEAST_OK;
  }
  const char* env = std::getenv("RAFEAST_TUNE");
  if (P->tune_cand.size() < 2 || (env && std::strcmp(env, "0") == 0)) return RAFEAST_OK;
  const int m0 = P->m0, ld = P->ld;
  HIPCHK(P, launch_gaussian(P->st, P->n, m0, 0x7u, P->d_R, ld));
  CocgLaunch L;
  L.nitems = std::min(P->nitems, std::max(P->num_cu, 1));
  L.items = P->d_items;
  L.tol = 0.0;
  L.maxit = 64;
  L.max_refine = 64;
  L.counter = P->d_counter;
  L.xhi = P->d_xhi;
  L.xhi_slots = P->xhi_slots;
  int* d_tab = nullptr;
  HIPCHK(P, hipMalloc(&d_tab, (size_t)cocg_resident_waves() * maxr * sizeof(int)));
  hipError_t e = hipSuccess;
  size_t best = 0;
  for (size_t c = 0; c < P->tune_cand.size() && e == hipSuccess; ++c) {
    e = hipMemcpyAsync(d_tab, tabs[c].data(), tabs[c].size() * sizeof(int),
                       hipMemcpyHostToDevice, P->st);
    const ResGraph gd = resident_graph(P, P->d_zw, m0, P->d_R, ld, P->d_D, P->nc * m0,
                                       P->d_iters, nullptr, d_tab);
    float tbest = 0.0f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = launch_fill_int(P->st, P->d_counter, 0, 1);
      if (e == hipSuccess) e = hipEventRecord(P->ev[0], P->st);
      if (e == hipSuccess)
        e = launch_cocg_resident(P->st, &gd, nullptr, (int)P->n, P->tune_cand[c], L, P->fp32,
                                 P->num_cu);
      if (e == hipSuccess) e = hipEventRecord(P->ev[1], P->st);
      if (e == hipSuccess) e = hipEventSynchronize(P->ev[1]);
      const float t = elapsed(P->ev[0], P->ev[1]);
      if (rep == 1 || (rep == 2 && t < tbest)) tbest = t;
    }
    P->tune_ms[c] = tbest;
    if (tbest < P->tune_ms[best]) best = c;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->d_wtab, tabs[best].data(), tabs[best].size() * sizeof(int),
                       hipMemcpyHostToDevice, P->st);
  if (e == hipSuccess) e = hipStreamSynchronize(P->st);
  (void)hipFree(d_tab);
  HIPCHK(P, e);
  P->tune_choice = P->tune_cand[best];
  P->sell.wave_rpt = P->tune_choice;
  if (verbose_log()) {
    std::fprintf(stderr, "rafeast: resident slots per thread:");
    for (size_t c = 0; c < P->tune_cand.size(); ++c)
      std::fprintf(stderr, " %d: %.3f ms%s", P->tune_cand[c], P->tune_ms[c],
                   c == best ? " (chosen)" : "");
    std::fprintf(stderr, "\n");
  }
  return RAFEAST_OK;
}

// rafeast_plan, rafeast_plan_dense and rafeast_plan_gram: exactly one of A
// (CSR) and D (dense operator) is set.
static rafeast_status plan_create(const rafeast_csr* A, const DenseSpec* D,
                                  const rafeast_params* prm, rafeast_plan_t* out) {
  g_plan_error.clear();
  if (!out) return fail(nullptr, RAFEAST_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if ((!A && !D) || !prm) return fail(nullptr, RAFEAST_INVALID_ARG, "A or prm is NULL");
  std::string msg;
  int64_t nnz = 0;
  double anorm = 0, lo = 0, hi = 0;
  rafeast_status s = A ? validate_csr(A, nnz, anorm, lo, hi, msg)
                       : validate_dense(*D, nnz, anorm, lo, hi, msg);
  if (s != RAFEAST_OK) return fail(nullptr, s, msg);
  const int64_t n = A ? A->n : D->n;
  s = validate_params(prm, n, msg);
  if (s != RAFEAST_OK) return fail(nullptr, s, msg);
  if (D && prm->precond == RAFEAST_PC_LEARNED)
    return fail(nullptr, RAFEAST_UNSUPPORTED, "the learned preconditioner takes CSR plans");
  int pov = prm->p;
  if (pov < 0) pov = prm->m0 <= 50 ? 10 : std::min(20, (prm->m0 + 1) / 2);
  int w = (int)std::min<int64_t>((int64_t)prm->m0 + pov, n);
  if (w > kMaxSmallK)
    return fail(nullptr, RAFEAST_UNSUPPORTED,
                "m0 + p = " + std::to_string(w) + " exceeds the small-matrix limit 192");
  const bool fp32 = prm->precision == RAFEAST_FP32_REFINED;
  int engine = prm->engine;
  if (D && (engine == RAFEAST_ENGINE_RESIDENT || engine == RAFEAST_ENGINE_MULTISHIFT ||
            engine == RAFEAST_ENGINE_DIRECT))
    return fail(nullptr, RAFEAST_UNSUPPORTED, "dense operators run on the streaming engine");
  if (engine == RAFEAST_ENGINE_DIRECT && prm->precond != RAFEAST_PC_NONE)
    return fail(nullptr, RAFEAST_UNSUPPORTED, "the direct engine solves exactly (precond NONE)");
  if (engine == RAFEAST_ENGINE_MULTISHIFT && prm->m0 > 192)
    return fail(nullptr, RAFEAST_UNSUPPORTED, "the multi-shift engine takes m0 <= 192");
  if (D) engine = RAFEAST_ENGINE_STREAM;
  if (engine == RAFEAST_ENGINE_RESIDENT && n > cocg_resident_max_n(fp32))
    return fail(nullptr, RAFEAST_UNSUPPORTED,
                "n too large for the resident COCG engine at this precision");
  if (engine == RAFEAST_ENGINE_AUTO && n > cocg_resident_max_n(fp32))
    engine = RAFEAST_ENGINE_STREAM;
  if ((int64_t)prm->nc * prm->m0 > (int64_t)1 << 20)
    return fail(nullptr, RAFEAST_UNSUPPORTED, "nc * m0 too large");
  {
    // the streaming engine is the fallback of AUTO, so its limits apply to both
    const int ncols = prm->nc * prm->m0;
    const int gw = 64 * stream_cpl(prm->m0, ncols, fp32);
    if ((engine == RAFEAST_ENGINE_AUTO || engine == RAFEAST_ENGINE_STREAM) &&
        (ncols + gw - 1) / gw > kStreamMaxGroups)
      return fail(nullptr, RAFEAST_UNSUPPORTED,
                  "nc * m0 exceeds the streaming engine's column limit");
  }

  int ndev = 0;
  hipError_t he = hipGetDeviceCount(&ndev);
  if (he != hipSuccess || ndev < 1)
    return fail(nullptr, RAFEAST_DEVICE, "no HIP device available");

  rafeast_plan_s* P = new rafeast_plan_s();
  P->prm = *prm;
  P->n = n;
  P->nnz = nnz;
  P->m0 = prm->m0;
  P->pov = pov;
  P->w = w;
  P->nc = prm->nc;
  P->sig_lo = lo;
  P->sig_hi = hi;
  P->anorm = anorm;
  P->fp32 = fp32;
  P->engine = engine;
  P->ld = w;

  auto bail = [&](rafeast_status st) {
    g_plan_error = P->err;
    free_plan(P);
    return st;
  };
#define PCHK(expr)                                    \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return bail(hip_fail(P, _e, #expr)); \
  } while (0)
#define PRCHK(expr)                       \
  do {                                    \
    rafeast_status _s = (expr);           \
    if (_s != RAFEAST_OK) return bail(_s); \
  } while (0)

  PCHK(hipGetDevice(&P->dev));
  hipDeviceProp_t props;
  PCHK(hipGetDeviceProperties(&props, P->dev));
  P->num_cu = props.multiProcessorCount;
  if (prm->hip_stream) {
    P->st = (hipStream_t)prm->hip_stream;
  } else {
    PCHK(hipStreamCreateWithFlags(&P->st, hipStreamNonBlocking));
    P->own_stream = true;
  }
  for (auto& e : P->ev) PCHK(hipEventCreate(&e));

  // quadrature table (eq. projector-quad, upper half circle)
  {
    std::vector<double> x, om;
    gauss_legendre_newton(P->nc, x, om);
    const double c = 0.5 * (prm->lmin + prm->lmax), r = 0.5 * (prm->lmax - prm->lmin);
    P->zw.assign(4 * P->nc, 0.0);
    for (int j = 0; j < P->nc; ++j) {
      const double ph = 0.5 * M_PI * (1.0 - x[j]);
      const double er = std::cos(ph), ei = std::sin(ph);
      P->zw[2 * j] = c + r * er;
      P->zw[2 * j + 1] = r * ei;
      P->zw[2 * P->nc + 2 * j] = 0.5 * om[j] * r * er;
      P->zw[2 * P->nc + 2 * j + 1] = 0.5 * om[j] * r * ei;
    }
    // nodes ordered by increasing |Im z| (the sum does not depend on the
    // order): the systems nearest the real axis take the most COCG
    // iterations, and the streaming engine's column groups (consecutive
    // shifts) then keep the slow ones together, so groups of easy shifts
    // stop costing bandwidth or flops early
    std::vector<int> ord(P->nc);
    for (int j = 0; j < P->nc; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
      return std::fabs(P->zw[2 * a + 1]) < std::fabs(P->zw[2 * b + 1]);
    });
    std::vector<double> zw2(P->zw.size());
    for (int j = 0; j < P->nc; ++j)
      for (int h = 0; h < 2; ++h) {
        zw2[2 * j + h] = P->zw[2 * ord[j] + h];
        zw2[2 * P->nc + 2 * j + h] = P->zw[2 * P->nc + 2 * ord[j] + h];
      }
    P->zw.swap(zw2);
  }

  if (D) {
    // dense operator: device copies (FP64, FP32) compacted to leading
    // dimension rows, scratch for the covariance form's X V, the BLAS handle,
    // and the identity row order of the streaming engine
    DenseOp& op = P->dop;
    op.kind = D->kind;
    op.n = n;
    op.rows = D->kind == 2 ? D->rows : n;
    op.scale = D->kind == 2 ? D->scale : 1.0;
    const size_t cnt = (size_t)op.rows * n;
    {
      std::vector<double> h64(cnt);
      std::vector<float> h32(cnt);
      for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < op.rows; ++i) {
          const double v = D->M[i + j * D->ld];
          h64[(size_t)j * op.rows + i] = v;
          h32[(size_t)j * op.rows + i] = (float)v;
        }
      PRCHK(dalloc(P, &P->d_k64, cnt, "dense operator"));
      PRCHK(dalloc(P, &P->d_k32, cnt, "dense operator fp32"));
      PCHK(hipMemcpy(P->d_k64, h64.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
      PCHK(hipMemcpy(P->d_k32, h32.data(), cnt * sizeof(float), hipMemcpyHostToDevice));
    }
    op.a64 = P->d_k64;
    op.a32 = P->d_k32;
    // workspace: the widest product is the streaming engine's packed
    // complex block (2 Bp real columns) or a small dense step
    const int Bp = stream_padded_columns(P->m0, P->nc * P->m0, fp32);
    op.tcols = std::max<int64_t>(2 * (int64_t)Bp, kMaxSmallK);
    // covariance: X V (rows x tcols) and chunk slabs of its long inner
    // dimension n (chunks of at least 512, at most 32); kernel: up to four
    // chunk slabs of K X (n x tcols) for products with few output tiles
    op.wslabs = op.kind == 2 ? 1 + (int)std::min<int64_t>(32, std::max<int64_t>(1, n / 512)) : 4;
    const size_t wrows = op.kind == 2 ? (size_t)op.rows : (size_t)n;
    PRCHK(dalloc(P, &P->d_t64, (size_t)op.wslabs * wrows * op.tcols, "dense workspace"));
    PRCHK(dalloc(P, &P->d_t32, (size_t)op.wslabs * wrows * op.tcols, "dense workspace fp32"));
    op.t64 = P->d_t64;
    op.t32 = P->d_t32;
    std::vector<int> ident(n);
    for (int64_t r = 0; r < n; ++r) ident[r] = (int)r;
    PRCHK(dalloc(P, &P->d_sperm, n, "stream perm"));
    PCHK(hipMemcpy(P->d_sperm, ident.data(), n * sizeof(int), hipMemcpyHostToDevice));
    P->smat.n = (int)n;
    P->smat.dense = &P->dop;
    P->smat.perm = P->d_sperm;
    P->engine = engine;
  }
  // CSR (FP64) and SELL-64 copies of A
  if (A) {
    const int base = A->index_base;
    std::vector<int> rp(n + 1), cl(nnz);
    for (int64_t i = 0; i <= n; ++i) rp[i] = A->rowptr[i] - base;
    for (int64_t t = 0; t < nnz; ++t) cl[t] = A->colind[t] - base;
    for (int64_t i = 0; i < n; ++i)
      for (int t = rp[i]; t < rp[i + 1]; ++t)
        P->span = std::max<int64_t>(P->span, std::abs((int64_t)cl[t] - i));
    PRCHK(dalloc(P, &P->d_rowptr, n + 1, "rowptr"));
    PRCHK(dalloc(P, &P->d_col, nnz, "colind"));
    PRCHK(dalloc(P, &P->d_val, nnz, "values"));
    PCHK(hipMemcpy(P->d_rowptr, rp.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice));
    if (nnz) {
      PCHK(hipMemcpy(P->d_col, cl.data(), nnz * sizeof(int), hipMemcpyHostToDevice));
      PCHK(hipMemcpy(P->d_val, A->values, nnz * sizeof(double), hipMemcpyHostToDevice));
    }
    if (engine != RAFEAST_ENGINE_STREAM && engine != RAFEAST_ENGINE_MULTISHIFT &&
        engine != RAFEAST_ENGINE_DIRECT) {
    // SELL-64 of the resident engine: rows sorted by decreasing length (ties
    // by index), slices of 64 slots, widths padded to a multiple of 4
    const int nsl = (int)((n + 63) / 64);
    std::vector<int> order(n), slot_of(n);
    for (int64_t i = 0; i < n; ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return (rp[a + 1] - rp[a]) > (rp[b + 1] - rp[b]);
    });
    for (int64_t sl = 0; sl < n; ++sl) slot_of[order[sl]] = (int)sl;
    std::vector<int> perm((size_t)nsl * 64, -1);
    for (int64_t sl = 0; sl < n; ++sl) perm[sl] = order[sl];
    std::vector<int> sb(nsl + 1, 0);
    for (int s = 0; s < nsl; ++s) {
      int wd = 0;
      for (int l = 0; l < 64; ++l) {
        const int64_t sl = (int64_t)s * 64 + l;
        if (sl < n) wd = std::max(wd, rp[order[sl] + 1] - rp[order[sl]]);
      }
      wd = (wd + 3) & ~3;
      sb[s + 1] = sb[s] + wd * 64;
    }
    const size_t tot = (size_t)sb[nsl] + 256;  // + a block of zero entries
    // FP32: values then 16-bit LDS byte offsets (slot * 8 < 65536 since the
    // FP32 resident engine holds at most 8192 slots)
    std::vector<float> v32(tot, 0.0f);
    std::vector<uint16_t> o32(tot, 0);
    std::vector<SellEntry64> e64(tot, SellEntry64{0, 0, 0.0});
    // Order of each row's entries (free: it only changes the rounding of the
    // row's sum).  At entry position kk the 64 lanes of a slice gather p at
    // the slots of their kk-th entries in one LDS instruction, which the LDS
    // serves a group of lanes per cycle (taken as 32 lanes of 8-byte complex
    // FP32, 16 of 16-byte complex FP64, i.e. 64 banks of 4 bytes); lanes of a
    // group whose slots fall in the same bank group (slot mod 32, mod 16)
    // conflict.  Greedy per position:
    // each lane takes its remaining entry whose bank group its lane group
    // has used least; padding entries (value zero) point at a slot of the
    // least used group.
    const int bgrp = fp32 ? RAFEAST_SELL_BANK_GROUPS : RAFEAST_SELL_BANK_GROUPS / 2;
    std::vector<int> pick, padslot;
    auto order_slice = [&](int s, int wd) {
      pick.assign((size_t)wd * 64, -1);
      padslot.assign((size_t)wd * 64, 0);
      std::vector<std::vector<int>> rem(64);
      for (int l = 0; l < 64; ++l) {
        const int64_t sl = (int64_t)s * 64 + l;
        if (sl < n)
          for (int t = rp[order[sl]]; t < rp[order[sl] + 1]; ++t) rem[l].push_back(t);
      }
      std::vector<int> cnt((64 / bgrp) * bgrp);
      for (int kk = 0; kk < wd; ++kk) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int l = 0; l < 64; ++l) {
          int* c = cnt.data() + (l / bgrp) * bgrp;
          if (!rem[l].empty()) {
            size_t best = 0;
            for (size_t u = 1; u < rem[l].size(); ++u)
              if (c[slot_of[cl[rem[l][u]]] % bgrp] < c[slot_of[cl[rem[l][best]]] % bgrp]) best = u;
            const int t = rem[l][best];
            rem[l].erase(rem[l].begin() + best);
            pick[(size_t)kk * 64 + l] = t;
            ++c[slot_of[cl[t]] % bgrp];
          } else {
            int r = 0;
            for (int q = 1; q < bgrp; ++q)
              if (c[q] < c[r]) r = q;
            padslot[(size_t)kk * 64 + l] = r;
            ++c[r];
          }
        }
      }
    };
    for (int s = 0; s < nsl; ++s) {
      const int wd = (sb[s + 1] - sb[s]) / 64;
      order_slice(s, wd);
      for (int kk = 0; kk < wd; ++kk)
        for (int l = 0; l < 64; ++l) {
          const int64_t sl = (int64_t)s * 64 + l;
          const size_t e = (size_t)sb[s] + (size_t)kk * 64 + l;
          const int row = sl < n ? order[sl] : -1;
          // FP32 positions: octs of eight entries (values as two 16-byte
          // halves for all lanes, offsets 16 bytes per lane), then a quad
          size_t vi, oi;
          const int n8 = wd / 8;
          if (kk < 8 * n8) {
            const int o = kk / 8, j = kk % 8;
            vi = (size_t)sb[s] + (size_t)o * 512 + (size_t)(j / 4) * 256 + (size_t)l * 4 + j % 4;
            oi = (size_t)sb[s] + (size_t)o * 512 + (size_t)l * 8 + j;
          } else {
            vi = oi = (size_t)sb[s] + (size_t)n8 * 512 + (size_t)l * 4 + (kk - 8 * n8);
          }
          const int t = pick[(size_t)kk * 64 + l];
          if (row >= 0 && t >= 0) {
            v32[vi] = (float)A->values[t];
            o32[oi] = (uint16_t)(slot_of[cl[t]] * 8);
            e64[e] = SellEntry64{slot_of[cl[t]] * 16, 0, A->values[t]};
          } else {
            // padding: zero value at a slot of the least used bank group
            const int ps = padslot[(size_t)kk * 64 + l];
            o32[oi] = (uint16_t)(ps * 8);
            e64[e] = SellEntry64{ps * 16, 0, 0.0};
          }
        }
    }
    PRCHK(dalloc(P, &P->d_sbase, nsl + 1, "sell base"));
    PRCHK(dalloc(P, &P->d_perm, (size_t)nsl * 64, "sell perm"));
    if (fp32 && (size_t)nsl * 64 * 8 > 65536)
      return bail(fail(P, RAFEAST_UNSUPPORTED, "too many rows for 16-bit SELL offsets"));
    PRCHK(dalloc(P, &P->d_v32, tot + tot / 2, "sell v32"));
    PRCHK(dalloc(P, &P->d_e64, tot, "sell e64"));
    PCHK(hipMemcpy(P->d_sbase, sb.data(), (nsl + 1) * sizeof(int), hipMemcpyHostToDevice));
    PCHK(hipMemcpy(P->d_perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice));
    if (tot) {
      PCHK(hipMemcpy(P->d_v32, v32.data(), tot * sizeof(float), hipMemcpyHostToDevice));
      PCHK(hipMemcpy(P->d_v32 + tot, o32.data(), tot * sizeof(uint16_t), hipMemcpyHostToDevice));
      PCHK(hipMemcpy(P->d_e64, e64.data(), tot * sizeof(SellEntry64), hipMemcpyHostToDevice));
    }
    P->sell.n = (int)n;
    P->sell.nslices = nsl;
    P->sell.sbase = P->d_sbase;
    P->sell.perm = P->d_perm;
    P->sell.v32 = P->d_v32;
    P->sell.n32 = (int)tot;
    P->sell.e64 = P->d_e64;
    P->sell.zero_base = sb[nsl];
    P->sell_entries = tot;
    // slice-to-wave table for the smallest slot count per wave that fits
    std::vector<int> widths(nsl);
    for (int s2 = 0; s2 < nsl; ++s2) widths[s2] = (sb[s2 + 1] - sb[s2]) / 64;
    P->sell_widths = widths;
    std::vector<int> tab;
    int rpt = 0;
    for (int cand : {1, 2, 4, 8}) {
      if (!fp32 && cand > 4) break;
      tab = cocg_resident_wave_table(widths, cand);
      if (!tab.empty()) {
        rpt = cand;
        break;
      }
    }
    if (rpt == 0 && engine == RAFEAST_ENGINE_RESIDENT)
      return bail(fail(P, RAFEAST_UNSUPPORTED, "matrix does not fit the resident engine"));
    if (rpt == 0) {
      engine = RAFEAST_ENGINE_STREAM;  // AUTO: rows too long for the on-chip layout
    } else {
      engine = RAFEAST_ENGINE_RESIDENT;
      // room for the largest slot count the tuner may choose
      PRCHK(dalloc(P, &P->d_wtab, (size_t)cocg_resident_waves() * 8, "wave table"));
      PCHK(hipMemcpy(P->d_wtab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
      P->sell.wave_slices = P->d_wtab;
      P->sell.wave_rpt = rpt;
    }
    }
    if (engine == RAFEAST_ENGINE_STREAM || engine == RAFEAST_ENGINE_MULTISHIFT ||
        engine == RAFEAST_ENGINE_DIRECT) {
      // CSR of the streaming engine in reverse Cuthill-McKee order, so that
      // the rows a workgroup gathers sit close to its own (and, for the
      // direct engine, the order whose band holds the factors)
      const std::vector<int> perm = rcm_order(n, rp, cl);
      std::vector<int> inv(n);
      for (int64_t r = 0; r < n; ++r) inv[perm[r]] = (int)r;
      std::vector<int> srp(n + 1, 0), scl(nnz);
      std::vector<double> sv(nnz);
      std::vector<float> sv32(nnz);
      std::vector<std::pair<int, double>> row;
      for (int64_t r = 0; r < n; ++r) {
        const int o = perm[r];
        row.clear();
        for (int t = rp[o]; t < rp[o + 1]; ++t) row.emplace_back(inv[cl[t]], A->values[t]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
                    return a.first < b.first;
                  });
        srp[r + 1] = srp[r] + (int)row.size();
        for (size_t u = 0; u < row.size(); ++u) {
          scl[srp[r] + u] = row[u].first;
          sv[srp[r] + u] = row[u].second;
          sv32[srp[r] + u] = (float)row[u].second;
        }
      }
      PRCHK(dalloc(P, &P->d_srow, n + 1, "stream rowptr"));
      PRCHK(dalloc(P, &P->d_scol, nnz, "stream colind"));
      PRCHK(dalloc(P, &P->d_sv64, nnz, "stream values"));
      PRCHK(dalloc(P, &P->d_sv32, nnz, "stream values fp32"));
      PRCHK(dalloc(P, &P->d_sperm, n, "stream perm"));
      PCHK(hipMemcpy(P->d_srow, srp.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice));
      PCHK(hipMemcpy(P->d_sperm, perm.data(), n * sizeof(int), hipMemcpyHostToDevice));
      if (nnz) {
        PCHK(hipMemcpy(P->d_scol, scl.data(), nnz * sizeof(int), hipMemcpyHostToDevice));
        PCHK(hipMemcpy(P->d_sv64, sv.data(), nnz * sizeof(double), hipMemcpyHostToDevice));
        PCHK(hipMemcpy(P->d_sv32, sv32.data(), nnz * sizeof(float), hipMemcpyHostToDevice));
      }
      P->smat.n = (int)n;
      P->smat.rowptr = P->d_srow;
      P->smat.col = P->d_scol;
      P->smat.val32 = P->d_sv32;
      P->smat.val64 = P->d_sv64;
      P->smat.perm = P->d_sperm;
      if (engine == RAFEAST_ENGINE_DIRECT) {
        // lower bandwidth of the reordered matrix, and room for the factors
        int b = 0;
        for (int64_t r = 0; r < n; ++r)
          if (srp[r + 1] > srp[r]) b = std::max<int>(b, (int)r - scl[srp[r]]);
        P->band_b = b;
        if (!band_supported(b))
          return bail(fail(P, RAFEAST_UNSUPPORTED,
                           "bandwidth " + std::to_string(b) +
                               " of the reordered matrix exceeds the direct engine's LDS "
                               "(the factorization's panel, the solve's ring of b + 32 rows)"));
        const size_t bytes = (size_t)P->nc * (size_t)n * (size_t)(b + 1) * sizeof(cpx<double>);
        size_t fr = 0, tot = 0;
        PCHK(hipMemGetInfo(&fr, &tot));
        if (bytes > fr / 10 * 9)
          return bail(fail(P, RAFEAST_OOM,
                           "the band factors need " + std::to_string(bytes >> 20) +
                               " MiB (bandwidth " + std::to_string(b) + ", " +
                               std::to_string(P->nc) + " shifts); " +
                               std::to_string(fr >> 20) + " MiB free"));
        hipError_t e = hipMalloc(&P->d_band, bytes);
        if (e != hipSuccess) return bail(hip_fail(P, e, "band factors"));
        PRCHK(dalloc(P, &P->d_binfo, (size_t)P->nc, "band pivot report"));
      }
    }
    P->engine = engine;
  }

  // workspace
  const size_t blk = (size_t)n * w;
  PRCHK(dalloc(P, &P->d_Q, blk, "Q"));
  PRCHK(dalloc(P, &P->d_W, blk, "W"));
  PRCHK(dalloc(P, &P->d_R, blk, "R"));
  PRCHK(dalloc(P, &P->d_T, blk, "T"));
  PRCHK(dalloc(P, &P->d_Y, blk, "Y"));
  const size_t kk2 = (size_t)kMaxSmallK * kMaxSmallK;
  PRCHK(dalloc(P, &P->d_G, kk2, "G"));
  PRCHK(dalloc(P, &P->d_M, kk2, "M"));
  PRCHK(dalloc(P, &P->d_S, kk2, "S"));
  PRCHK(dalloc(P, &P->d_Ssel, (size_t)kMaxSmallK * P->m0, "Ssel"));
  PRCHK(dalloc(P, &P->d_jw, 2 * kk2, "jacobi work"));
  PRCHK(dalloc(P, &P->d_theta, kMaxSmallK, "theta"));
  PRCHK(dalloc(P, &P->d_res, kMaxSmallK, "res"));
  PRCHK(dalloc(P, &P->d_qn, kMaxSmallK, "qn"));
  PRCHK(dalloc(P, &P->d_mtot, (size_t)P->m0 * P->m0, "mtot"));
  PRCHK(dalloc(P, &P->d_mtmp, (size_t)P->m0 * P->m0, "mtot product"));
  PRCHK(dalloc(P, &P->d_gamma, 2 * (size_t)P->nc * P->m0, "gamma"));
  PRCHK(dalloc(P, &P->d_info, 4, "info"));
  PRCHK(dalloc(P, &P->d_zw, 4 * P->nc, "zw"));
  P->part_doubles = std::max(gram_partial_doubles(n, w, w), (size_t)2 * w * gram_chunks(n));
  PRCHK(dalloc(P, &P->d_part, P->part_doubles, "partials"));
  const size_t cs = fp32 ? 2 * sizeof(float) : 2 * sizeof(double);
  // the solutions of one filter step (the multi-shift engine combines them
  // as it goes and needs no such block unless the learned solver runs)
  if (P->engine != RAFEAST_ENGINE_MULTISHIFT || prm->precond == RAFEAST_PC_LEARNED) {
    hipError_t e = hipMalloc(&P->d_D, (size_t)n * P->nc * P->m0 * cs);
    if (e != hipSuccess) return bail(hip_fail(P, e, "solve block"));
  }
  if (prm->precond == RAFEAST_PC_LEARNED) {
    const int npar = mlp_param_count();
    PRCHK(dalloc(P, &P->d_pcW, (size_t)npar, "network parameters"));
    PRCHK(dalloc(P, &P->d_pcWb, (size_t)npar, "network BF16 parameters"));
    PRCHK(dalloc(P, &P->d_pcX, 4 * (size_t)P->nc, "network features"));
    PRCHK(dalloc(P, &P->d_pcY, 16 * (size_t)P->nc, "network outputs"));
    if (!fp32) {
      P->d_D64 = P->d_D;  // the plan's solve block is FP64 already
    } else {
      hipError_t e = hipMalloc(&P->d_D64, (size_t)n * P->nc * P->m0 * 2 * sizeof(double));
      if (e != hipSuccess) return bail(hip_fail(P, e, "FP64 solve block"));
    }
  }
  P->nitems = P->nc * P->m0;
  PRCHK(dalloc(P, &P->d_items, 3 * (size_t)P->nitems, "items"));
  PRCHK(dalloc(P, &P->d_counter, 1, "counter"));
  PRCHK(dalloc(P, &P->d_iters, (size_t)P->nitems, "iters"));
  PRCHK(dalloc(P, &P->d_stats, 2, "stats"));
  PRCHK(dalloc(P, &P->d_flag, 3, "flag"));
  PRCHK(dalloc(P, &P->d_sel, P->m0, "sel"));
  if (P->engine == RAFEAST_ENGINE_RESIDENT) {
    P->xhi_slots = cocg_resident_xhi_slots((int)n, P->num_cu);
    hipError_t e = hipMalloc(&P->d_xhi, P->xhi_slots * 2 * sizeof(double));
    if (e != hipSuccess) return bail(hip_fail(P, e, "solution scratch"));
  } else if (P->engine == RAFEAST_ENGINE_DIRECT) {
    // the factors are the whole workspace
  } else if (P->engine == RAFEAST_ENGINE_MULTISHIFT) {
    PRCHK(alloc_ms_work(P, P->nc, P->m0, P->mswork, P->sbufs, true));
    if (prm->rhs_form == RAFEAST_RHS_LITERAL) {  // literal form: g_{j,c} = w_j
      std::vector<double> wr(2 * (size_t)P->nc * P->m0);
      for (int j = 0; j < P->nc; ++j)
        for (int c = 0; c < P->m0; ++c) {
          wr[2 * ((size_t)j * P->m0 + c)] = P->zw[2 * P->nc + 2 * j];
          wr[2 * ((size_t)j * P->m0 + c) + 1] = P->zw[2 * P->nc + 2 * j + 1];
        }
      PRCHK(dalloc(P, &P->d_wrep, wr.size(), "repeated weights"));
      PCHK(hipMemcpy(P->d_wrep, wr.data(), wr.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  } else {
    const int Bp = stream_padded_columns(P->m0, P->nc * P->m0, fp32);
    PRCHK(alloc_stream_work(P, Bp, P->swork, P->sbufs));
    const std::vector<double> zc = stream_shifts(P->nc, P->zw.data(), P->m0, Bp);
    PCHK(hipMemcpy(P->swork.zc, zc.data(), zc.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  PCHK(hipMemcpy(P->d_zw, P->zw.data(), 4 * P->nc * sizeof(double), hipMemcpyHostToDevice));
  {
    std::vector<int> items = make_items(P->nc, P->zw.data(), P->m0);
    PCHK(hipMemcpy(P->d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  if (P->engine == RAFEAST_ENGINE_RESIDENT) PRCHK(tune_resident(P));
  if (P->engine == RAFEAST_ENGINE_DIRECT) PRCHK(band_factor_shifts(P));
  PCHK(hipMemset(P->d_stats, 0, 2 * sizeof(int)));
  PCHK(hipDeviceSynchronize());
#undef PCHK
#undef PRCHK
  *out = P;
  return RAFEAST_OK;
}

rafeast_status rafeast_plan(const rafeast_csr* A, const rafeast_params* prm,
                            rafeast_plan_t* out) {
  if (!A) {
    g_plan_error = "A or prm is NULL";
    if (out) *out = nullptr;
    return RAFEAST_INVALID_ARG;
  }
  return plan_create(A, nullptr, prm, out);
}

rafeast_status rafeast_plan_dense(int64_t n, const double* K, int64_t ldk,
                                  const rafeast_params* prm, rafeast_plan_t* out) {
  DenseSpec D;
  D.kind = 1;
  D.n = n;
  D.rows = n;
  D.ld = ldk;
  D.M = K;
  return plan_create(nullptr, &D, prm, out);
}

rafeast_status rafeast_plan_gram(int64_t rows, int64_t n, const double* X, int64_t ldx,
                                 double scale, const rafeast_params* prm, rafeast_plan_t* out) {
  DenseSpec D;
  D.kind = 2;
  D.n = n;
  D.rows = rows;
  D.ld = ldx;
  D.M = X;
  D.scale = scale;
  return plan_create(nullptr, &D, prm, out);
}

rafeast_status rafeast_plan_tuning(rafeast_plan_t P, int32_t* chosen, int32_t* count,
                                   int32_t* cand, float* ms, int32_t max) {
  if (!P || !chosen || !count || max < 0 || (max > 0 && (!cand || !ms)))
    return fail(P, RAFEAST_INVALID_ARG, "null argument");
  *chosen = P->engine == RAFEAST_ENGINE_RESIDENT ? P->tune_choice : 0;
  *count = (int32_t)P->tune_cand.size();
  for (int32_t i = 0; i < max && i < *count; ++i) {
    cand[i] = P->tune_cand[i];
    ms[i] = P->tune_ms[i];
  }
  return RAFEAST_OK;
}

int32_t rafeast_plan_engine(rafeast_plan_t P) { return P ? P->engine : 0; }

rafeast_status rafeast_rcm_order(const rafeast_csr* A, int32_t* perm) {
  if (!A || !perm || !A->rowptr || !A->colind || !A->values)
    return fail(nullptr, RAFEAST_INVALID_ARG, "null argument");
  std::string msg;
  int64_t nnz = 0;
  double anorm = 0, lo = 0, hi = 0;
  rafeast_status s = validate_csr(A, nnz, anorm, lo, hi, msg);
  if (s != RAFEAST_OK) return fail(nullptr, s, msg);
  const int64_t n = A->n;
    const int base = A->index_base;
  std::vector<int> rp(n + 1), cl(nnz);
  for (int64_t i = 0; i <= n; ++i) rp[i] = A->rowptr[i] - base;
  for (int64_t t = 0; t < nnz; ++t) cl[t] = A->colind[t] - base;
  const std::vector<int> ord = rcm_order(n, rp, cl);
  std::memcpy(perm, ord.data(), n * sizeof(int32_t));
  return RAFEAST_OK;
}

rafeast_status rafeast_plan_info(rafeast_plan_t P, double* sig_lo, double* sig_hi,
                                 double* anorm_inf, int64_t* nnz, double* z, double* w) {
  if (!P) return RAFEAST_INVALID_ARG;
  if (sig_lo) *sig_lo = P->sig_lo;
  if (sig_hi) *sig_hi = P->sig_hi;
  if (anorm_inf) *anorm_inf = P->anorm;
  if (nnz) *nnz = P->nnz;
  if (z) std::memcpy(z, P->zw.data(), 2 * P->nc * sizeof(double));
  if (w) std::memcpy(w, P->zw.data() + 2 * P->nc, 2 * P->nc * sizeof(double));
  return RAFEAST_OK;
}

rafeast_status rafeast_warmstart(rafeast_plan_t P, const double* omega, double* Q0,
                                 rafeast_ws_info* info) {
  if (!P) return RAFEAST_INVALID_ARG;
  P->err.clear();
  const int64_t n = P->n;
  const int m0 = P->m0, w = P->w, ld = P->ld;
  HIPCHK(P, hipEventRecord(P->ev[0], P->st));
  if (omega) {
    HIPCHK(P, hipMemcpyAsync(P->d_T, omega, (size_t)n * w * sizeof(double), hipMemcpyHostToDevice,
                             P->st));
    HIPCHK(P, launch_colmajor_to_rowmajor(P->st, n, w, P->d_T, P->d_Y, ld));
  } else {
    HIPCHK(P, launch_gaussian(P->st, n, w, P->prm.seed, P->d_Y, ld));
  }
  const int op = resolve_ws_op(P);
  double bm0 = NAN, bm1 = NAN;
  if (op == RAFEAST_WS_NONE) {
    HIPCHK(P, launch_copy_cols(P->st, n, m0, P->d_Y, ld, P->d_Q, ld));
    int ci = 0;
    RCHK(cholqr2(P, n, m0, P->d_Q, ld, &ci, P->d_T, ld));
    if (ci == 2) return fail(P, RAFEAST_BREAKDOWN, "orthonormalisation of the sketch failed");
  } else {
    const double lmin = P->prm.lmin, lmax = P->prm.lmax;
    const double c0 = 0.5 * (lmin + lmax);
    const double Rr = std::max(c0 - P->sig_lo, P->sig_hi - c0);
    double pa = 0, pb = 0, pc = 0;  // phi(t) = pa + pb t + pc t^2
    for (int t = 0; t < 2 * P->prm.q + 1; ++t) {
      if (op == RAFEAST_WS_LITERAL) {
        const double s = 1.0 / (lmax - lmin);
        RCHK(spmm(P, w, P->d_Y, ld, P->d_W, ld, s, -s * lmin));
      } else if (op == RAFEAST_WS_FLIP) {
        const double s = 1.0 / (P->sig_hi - lmin);
        RCHK(spmm(P, w, P->d_Y, ld, P->d_W, ld, -s, s * P->sig_hi));
      } else {
        RCHK(spmm(P, w, P->d_Y, ld, P->d_T, ld, 1.0 / Rr, -c0 / Rr));
        RCHK(spmm(P, w, P->d_T, ld, P->d_W, ld, -1.0 / Rr, c0 / Rr, P->d_Y, ld, 1.0));
      }
      int ci = 0;
      RCHK(cholqr2(P, n, w, P->d_W, ld, &ci, P->d_T, ld));
      if (ci == 2) return fail(P, RAFEAST_BREAKDOWN, "orthonormalisation in Phase 1 failed");
      std::swap(P->d_Y, P->d_W);
    }
    if (op == RAFEAST_WS_LITERAL) {
      const double s = 1.0 / (lmax - lmin);
      pa = -s * lmin;
      pb = s;
    } else if (op == RAFEAST_WS_FLIP) {
      const double s = 1.0 / (P->sig_hi - lmin);
      pa = s * P->sig_hi;
      pb = -s;
    } else {
      pa = 1.0 - c0 * c0 / (Rr * Rr);
      pb = 2.0 * c0 / (Rr * Rr);
      pc = -1.0 / (Rr * Rr);
    }
    // Rayleigh-Ritz truncation to m0 vectors
    RCHK(spmm(P, w, P->d_Y, ld, P->d_W, ld, 1.0, 0.0));
    HIPCHK(P, launch_gram(P->st, n, w, w, P->d_Y, ld, P->d_W, ld, P->d_G, w, P->d_part));
    HIPCHK(P, launch_jacobi(P->st, w, P->d_G, w, P->d_theta, P->d_S, w, P->d_jw));
    HIPCHK(P, launch_select(P->st, w, m0, P->d_theta, P->d_S, w, pa, pb, pc, P->d_Ssel,
                            P->d_info));
    HIPCHK(P, launch_tsmm(P->st, n, w, m0, P->d_Y, ld, P->d_Ssel, m0, P->d_Q, ld));
    double hinfo[2];
    HIPCHK(P, hipMemcpyAsync(hinfo, P->d_info, 2 * sizeof(double), hipMemcpyDeviceToHost, P->st));
    HIPCHK(P, hipStreamSynchronize(P->st));
    bm0 = hinfo[0];
    bm1 = hinfo[1];
  }
  HIPCHK(P, hipEventRecord(P->ev[1], P->st));
  HIPCHK(P, hipEventSynchronize(P->ev[1]));
  P->have_start = true;
  P->ws_used = op;
  if (Q0) {
    HIPCHK(P, launch_rowmajor_to_colmajor(P->st, n, m0, P->d_Q, ld, P->d_T));
    HIPCHK(P, hipMemcpyAsync(Q0, P->d_T, (size_t)n * m0 * sizeof(double), hipMemcpyDeviceToHost,
                             P->st));
    HIPCHK(P, hipStreamSynchronize(P->st));
  }
  if (info) {
    info->beta_m0 = bm0;
    info->beta_m0p1 = bm1;
    info->ratio = std::pow(bm1 / bm0, 2.0 * P->prm.q + 1.0);
    info->op = op;
    info->t_ms = elapsed(P->ev[0], P->ev[1]);
    // Theorem 1 with the Rayleigh-Ritz estimates of beta_m0 and beta_m0+1
    // (eq. R-Halko with C1(delta) = 1 + (p/2) ln(2 m0 / delta), delta = 0.01)
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const int q = P->prm.q, pov = P->w - m0;
    info->gap = bm0 - bm1;
    if (pov >= 2 && std::isfinite(bm1)) {
      const double delta = 0.01;
      const double c1 = 1.0 + 0.5 * pov * std::log(2.0 * m0 / delta);
      info->r_halko =
          c1 * std::sqrt(1.0 + (double)m0 / (pov - 1)) * bm1 * std::pow(bm1 / bm0, 2.0 * q);
      info->proj_bound = info->gap > 0.0 ? info->r_halko / info->gap : nan;
    } else {
      info->r_halko = nan;
      info->proj_bound = nan;
    }
  }
  return RAFEAST_OK;
}

rafeast_status rafeast_solve(rafeast_plan_t P, const double* Q_init, rafeast_result* res) {
  if (!P || !res || !res->lambda || !res->resid) return RAFEAST_INVALID_ARG;
  SolveRun S;
  RCHK(solve_begin(P, Q_init, S));
  for (;;) {
    RCHK(solve_test(P, S));
    if (S.done) break;
    HIPCHK(P, hipEventRecord(P->ev[2], P->st));
    RCHK(solve_shifted_systems(P, S));
    HIPCHK(P, hipEventRecord(P->ev[3], P->st));
    RCHK(solve_combine(P, S));
  }
  return solve_finish(P, S, res);
}

// ---------------------------------------------------------------------------
// step-level calls
// ---------------------------------------------------------------------------
rafeast_status rafeast_spmm(rafeast_plan_t P, int32_t k, const double* X, int32_t ldx, double* Y,
                            int32_t ldy, double alpha, double beta) {
  if (!P || !X || !Y || k < 1 || ldx < k || ldy < k || X == Y) return RAFEAST_INVALID_ARG;
  RCHK(spmm(P, k, X, ldx, Y, ldy, alpha, beta));
  HIPCHK(P, hipStreamSynchronize(P->st));
  return RAFEAST_OK;
}

rafeast_status rafeast_gram(rafeast_plan_t P, int64_t n, int32_t k1, int32_t k2, const double* X,
                            int32_t ldx, const double* Y, int32_t ldy, double* G, int32_t ldg) {
  if (!P || !X || !Y || !G || n < 1 || k1 < 1 || k2 < 1 || ldx < k1 || ldy < k2 || ldg < k2)
    return RAFEAST_INVALID_ARG;
  double* part = nullptr;
  HIPCHK(P, hipMalloc(&part, gram_partial_doubles(n, k1, k2) * sizeof(double)));
  hipError_t e = launch_gram(P->st, n, k1, k2, X, ldx, Y, ldy, G, ldg, part);
  if (e == hipSuccess) e = hipStreamSynchronize(P->st);
  (void)hipFree(part);
  HIPCHK(P, e);
  return RAFEAST_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Gram product without allocation.  The row-chunk partial sums live in a
// file-scope device array of fixed size; each device holds its own copy at
// its own address, which hipGetSymbolAddress returns once per device (in host
// code the array's name is not a device address).
// ----------------------------------------------------------------------------
constexpr size_t kGramScratchDoubles = size_t(1) << 21;  // 16 MiB per device
static __device__ __align__(256) double scratch[kGramScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device (resolved on the first
// call made with that device current).
hipError_t gram_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

rafeast_status rafeast_gram_noalloc(void* hip_stream, int64_t n, int32_t k1, int32_t k2,
                                    const double* X, int32_t ldx, const double* Y, int32_t ldy,
                                    double* G, int32_t ldg) {
  if (!X || !Y || !G || n < 1 || k1 < 1 || k2 < 1 || ldx < k1 || ldy < k2 || ldg < k2)
    return fail(nullptr, RAFEAST_INVALID_ARG, "rafeast_gram_noalloc: bad argument");
  const size_t tile = (size_t)k1 * (size_t)k2;
  if (tile > kGramScratchDoubles)
    return fail(nullptr, RAFEAST_INVALID_ARG,
                "rafeast_gram_noalloc: k1 * k2 = " + std::to_string(tile) +
                    " exceeds the scratch of " + std::to_string(kGramScratchDoubles) +
                    " doubles");
  double* part = nullptr;
  hipError_t e = gram_scratch(&part);
  if (e != hipSuccess) return hip_fail(nullptr, e, "rafeast_gram_noalloc: scratch address");
  // as many row chunks as rafeast_gram uses when they fit, fewer otherwise
  const int chunks = (int)std::min<size_t>((size_t)gram_chunks(n), kGramScratchDoubles / tile);
  e = launch_gram_chunks(static_cast<hipStream_t>(hip_stream), n, k1, k2, X, ldx, Y, ldy, G, ldg,
                         part, chunks);
  if (e != hipSuccess) return hip_fail(nullptr, e, "rafeast_gram_noalloc: launch");
  return RAFEAST_OK;
}

rafeast_status rafeast_gemm(void* hip_stream, int32_t precision, int32_t a_cols, int32_t M,
                            int32_t N, int32_t K, const void* A, int64_t lda, const void* B,
                            int64_t ldb, void* C, int64_t ldc, double alpha, double beta) {
  // A and B may be null when K == 0, C when M N == 0 (nothing is read there)
  if ((K > 0 && M > 0 && !A) || (K > 0 && N > 0 && !B) || ((int64_t)M * N > 0 && !C) || M < 0 ||
      N < 0 || K < 0 || ldb < N || ldc < N ||
      lda < (a_cols ? M : K) || lda < 1 || (a_cols != 0 && a_cols != 1) ||
      (precision != RAFEAST_FP64 && precision != RAFEAST_FP32_REFINED))
    return fail(nullptr, RAFEAST_INVALID_ARG, "rafeast_gemm: bad argument");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const bool f64 = precision == RAFEAST_FP64;
  const size_t es = f64 ? sizeof(double) : sizeof(float);
  // room for as many chunk slabs as the launcher may choose (at most 64)
  const size_t room = K >= 1024 ? std::min<size_t>(64, (size_t)K / 512) * M * N : 0;
  void* work = nullptr;
  if (room) {
    const hipError_t e = hipMalloc(&work, room * es);
    if (e != hipSuccess) return hip_fail(nullptr, e, "rafeast_gemm: workspace");
  }
  hipError_t e =
      f64 ? launch_gemm_f64(st, a_cols, M, N, K, (const double*)A, lda, (const double*)B, ldb,
                            (double*)C, ldc, alpha, beta, (double*)work, room)
          : launch_gemm_f32(st, a_cols, M, N, K, (const float*)A, lda, (const float*)B, ldb,
                            (float*)C, ldc, (float)alpha, (float)beta, (float*)work, room);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (work) (void)hipFree(work);
  if (e != hipSuccess) return hip_fail(nullptr, e, "rafeast_gemm");
  return RAFEAST_OK;
}

rafeast_status rafeast_cholqr2(rafeast_plan_t P, int64_t n, int32_t k, double* Y, int32_t ldy,
                               int32_t* info) {
  if (!P || !Y || n < 1 || k < 1 || k > kMaxSmallK || ldy < k || k > n) return RAFEAST_INVALID_ARG;
  double* tmp = nullptr;
  double* part = nullptr;
  hipError_t e = hipMalloc(&tmp, (size_t)n * k * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&part, gram_partial_doubles(n, k, k) * sizeof(double));
  rafeast_status s = RAFEAST_OK;
  int ci = 0;
  if (e != hipSuccess) {
    s = hip_fail(P, e, "cholqr2 workspace");
  } else {
    double* keep = P->d_part;
    P->d_part = part;
    s = cholqr2(P, n, k, Y, ldy, &ci, tmp, k);
    P->d_part = keep;
    if (s == RAFEAST_OK) {
      e = hipStreamSynchronize(P->st);
      if (e != hipSuccess) s = hip_fail(P, e, "cholqr2");
    }
  }
  if (tmp) (void)hipFree(tmp);
  if (part) (void)hipFree(part);
  if (info) *info = ci;
  return s;
}

rafeast_status rafeast_syev(rafeast_plan_t P, int32_t k, const double* H, double* theta,
                            double* S) {
  if (!P || !H || !theta || !S || k < 1 || k > kMaxSmallK) return RAFEAST_INVALID_ARG;
  HIPCHK(P, launch_jacobi(P->st, k, H, k, theta, S, k, P->d_jw));
  HIPCHK(P, hipStreamSynchronize(P->st));
  return RAFEAST_OK;
}

rafeast_status rafeast_shifted_solve(rafeast_plan_t P, int32_t nz, const double* z, int32_t k,
                                     const double* B, int32_t ldb, void* X, double tol,
                                     int32_t* iters, double* resid) {
  if (!P || !z || !B || !X || nz < 1 || k < 1 || ldb < k || !(tol > 0.0) || !(tol < 1.0))
    return RAFEAST_INVALID_ARG;
  double* d_z = nullptr;
  int* d_items = nullptr;
  int* d_it = nullptr;
  double* d_rs = nullptr;
  std::vector<int> items = make_items(nz, z, k);
  const int nitems = nz * k;
  rafeast_status s = RAFEAST_OK;
  hipError_t e = hipMalloc(&d_z, 2 * nz * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&d_items, items.size() * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&d_it, nitems * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&d_rs, nitems * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_z, z, 2 * nz * sizeof(double), hipMemcpyHostToDevice, P->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice,
                       P->st);
  if (e != hipSuccess) {
    s = hip_fail(P, e, "shifted_solve setup");
  } else {
    if (P->engine == RAFEAST_ENGINE_DIRECT) {
      // factorize the requested shifts into a band workspace of this call
      const int n = (int)P->n, b = P->band_b;
      cpx<double>* Wb = nullptr;
      int* d_info = nullptr;
      e = hipMalloc(&Wb, (size_t)nz * n * (b + 1) * sizeof(cpx<double>));
      if (e == hipSuccess) e = hipMalloc(&d_info, nz * sizeof(int));
      if (e != hipSuccess) s = hip_fail(P, e, "shifted_solve band workspace");
      if (s == RAFEAST_OK) {
        e = band_assemble(P->st, n, b, P->d_srow, P->d_scol, P->d_sv64, nz, d_z, Wb);
        if (e == hipSuccess) e = band_factor(P->st, n, b, nz, Wb, d_info);
        std::vector<int> info(nz);
        if (e == hipSuccess)
          e = hipMemcpyAsync(info.data(), d_info, nz * sizeof(int), hipMemcpyDeviceToHost, P->st);
        if (e == hipSuccess) e = hipStreamSynchronize(P->st);
        if (e != hipSuccess) s = hip_fail(P, e, "shifted_solve factorization");
        for (int j = 0; s == RAFEAST_OK && j < nz; ++j)
          if (info[j] != 0)
            s = fail(P, RAFEAST_BREAKDOWN,
                     "LDL^T of z_" + std::to_string(j) + " I - A: pivot " +
                         std::to_string(info[j] - 1) + " vanished");
      }
      if (s == RAFEAST_OK) {
        e = hipMemsetAsync(d_it, 0, nitems * sizeof(int), P->st);
        if (e == hipSuccess)
          e = band_solve(P->st, n, b, nz, Wb, P->d_sperm, B, ldb, k,
                         static_cast<cpx<double>*>(X), (int64_t)nz * k);
        if (e == hipSuccess)
          e = band_resid(P->st, n, P->d_rowptr, P->d_col, P->d_val, nz, d_z, B, ldb, k,
                         static_cast<const cpx<double>*>(X), (int64_t)nz * k, d_rs);
        if (e == hipSuccess) e = hipStreamSynchronize(P->st);
        if (e != hipSuccess) s = hip_fail(P, e, "shifted_solve");
      }
      if (Wb) (void)hipFree(Wb);
      if (d_info) (void)hipFree(d_info);
    } else if (P->engine == RAFEAST_ENGINE_MULTISHIFT) {
      std::vector<void*> bufs;
      MsWork W;
      // pi_k = R_k(z_j - s) can vanish for a real z_j inside the seed's
      // spectrum: the engine takes shifts off the real axis only
      bool real_shift = false;
      for (int j = 0; j < nz; ++j) real_shift = real_shift || !(z[2 * j + 1] != 0.0);
      if (real_shift)
        s = fail(P, RAFEAST_INVALID_ARG, "the multi-shift engine takes shifts with Im z != 0");
      else if (k > 192)
        s = fail(P, RAFEAST_UNSUPPORTED, "the multi-shift engine takes k <= 192");
      else
        s = alloc_ms_work(P, nz, k, W, bufs);
      if (s == RAFEAST_OK) s = run_ms(P, W, nz, z, k, B, ldb, X, nz * k, tol, d_it, d_rs);
      if (s == RAFEAST_OK) {
        e = hipStreamSynchronize(P->st);
        if (e != hipSuccess) s = hip_fail(P, e, "shifted_solve");
      }
      for (void* b : bufs) (void)hipFree(b);
    } else if (P->engine == RAFEAST_ENGINE_STREAM) {
      // a workspace of this call's width, released below
      const int gw = 64 * stream_cpl(k, nitems, P->fp32);
      const int Bp = stream_padded_columns(k, nitems, P->fp32);
      std::vector<void*> bufs;
      StreamWork W;
      if (Bp / gw > kStreamMaxGroups)
        s = fail(P, RAFEAST_UNSUPPORTED, "nz * k exceeds the streaming engine's column limit");
      else
        s = alloc_stream_work(P, Bp, W, bufs);
      if (s == RAFEAST_OK) {
        const std::vector<double> zc = stream_shifts(nz, z, k, Bp);
        e = hipMemcpyAsync(W.zc, zc.data(), zc.size() * sizeof(double), hipMemcpyHostToDevice,
                           P->st);
        if (e != hipSuccess) s = hip_fail(P, e, "shifted_solve shifts");
      }
      if (s == RAFEAST_OK) s = run_stream(P, W, nz, k, B, ldb, X, nz * k, tol, d_it, d_rs);
      if (s == RAFEAST_OK) {
        e = hipStreamSynchronize(P->st);
        if (e != hipSuccess) s = hip_fail(P, e, "shifted_solve");
      }
      for (void* b : bufs) (void)hipFree(b);
    } else {
      s = run_cocg(P, nitems, d_items, d_z, k, B, ldb, X, nz * k, tol, d_it, d_rs);
    }
    if (s == RAFEAST_OK && iters) {
      e = hipMemcpyAsync(iters, d_it, nitems * sizeof(int), hipMemcpyDeviceToHost, P->st);
      if (e != hipSuccess) s = hip_fail(P, e, "copy iterations");
    }
    if (s == RAFEAST_OK && resid) {
      e = hipMemcpyAsync(resid, d_rs, nitems * sizeof(double), hipMemcpyDeviceToHost, P->st);
      if (e != hipSuccess) s = hip_fail(P, e, "copy residuals");
    }
    if (s == RAFEAST_OK) {
      e = hipStreamSynchronize(P->st);
      if (e != hipSuccess) s = hip_fail(P, e, "shifted_solve");
    }
  }
  if (d_z) (void)hipFree(d_z);
  if (d_items) (void)hipFree(d_items);
  if (d_it) (void)hipFree(d_it);
  if (d_rs) (void)hipFree(d_rs);
  return s;
}

rafeast_status rafeast_gaussian(rafeast_plan_t P, int32_t w, uint64_t seed, double* Omega,
                                int32_t ld) {
  if (!P || !Omega || w < 1 || ld < w) return RAFEAST_INVALID_ARG;
  HIPCHK(P, launch_gaussian(P->st, P->n, w, seed, Omega, ld));
  HIPCHK(P, hipStreamSynchronize(P->st));
  return RAFEAST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batching form
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_batch_error;

rafeast_status batch_fail(rafeast_batch_s* B, rafeast_status st, const std::string& msg) {
  if (B)
    B->err = msg;
  else
    g_batch_error = msg;
  return st;
}

void free_batch(rafeast_batch_s* B) {
  if (!B) return;
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  for (int* t : B->own_wtab) (void)hipFree(t);
  void* ptrs[] = {B->d_graphs, B->d_items, B->d_counter, B->d_xhi};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (auto& e : B->ev)
    if (e) (void)hipEventDestroy(e);
  for (rafeast_plan_s* P : B->plans) free_plan(P);
  for (hipEvent_t e : B->mev)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t q : B->mst)
    if (q) (void)hipStreamDestroy(q);
  if (B->own_stream && B->st) (void)hipStreamDestroy(B->st);
  delete B;
}

#define BCHK(B, expr)                                                          \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess)                                                      \
      return batch_fail((B), _e == hipErrorOutOfMemory ? RAFEAST_OOM : RAFEAST_DEVICE, \
                        std::string(#expr) + ": " + hipGetErrorString(_e));    \
  } while (0)

// One shared resident launch for the active resident members: descriptors
// and (member, node, column) items, longest first across members (the cost
// of a system is taken as nnz * sqrt(spectral width / |Im z|), the COCG
// iteration count growing as the shift nears the spectrum).  The counter
// reset and the launch are captured once per item count and replayed.
rafeast_status batch_resident_solves(rafeast_batch_s* B, const std::vector<char>& active) {
  struct Key {
    double cost;
    int k, j, i;
  };
  std::vector<Key> keys;
  for (size_t g = 0; g < B->plans.size(); ++g) {
    const int k = B->res_idx[g];
    if (k < 0 || !active[g]) continue;
    rafeast_plan_s* P = B->plans[g];
    const bool residual_form = P->prm.rhs_form == RAFEAST_RHS_RESIDUAL;
    B->h_graphs[k] = resident_graph(P, P->d_zw, P->m0, residual_form ? P->d_R : P->d_Q, P->ld,
                                    P->d_D, P->nc * P->m0, P->d_iters, nullptr, B->wtab[g]);
    B->h_graphs[k].tol = P->tau;  // each member's own Phase-2 tolerance
    const double width = std::max(P->sig_hi - P->sig_lo, 1e-300);
    for (int j = 0; j < P->nc; ++j) {
      const double im = std::max(std::fabs(P->zw[2 * j + 1]), 1e-300);
      const double cost = (double)P->nnz * std::sqrt(width / im);
      for (int i = 0; i < P->m0; ++i) keys.push_back(Key{cost, k, j, i});
    }
  }
  if (keys.empty()) return RAFEAST_OK;
  std::stable_sort(keys.begin(), keys.end(),
                   [](const Key& a, const Key& b) { return a.cost > b.cost; });
  const int nitems = (int)keys.size();
  B->h_items.resize(3 * (size_t)nitems);
  for (int t = 0; t < nitems; ++t) {
    B->h_items[3 * t] = keys[t].k;
    B->h_items[3 * t + 1] = keys[t].j;
    B->h_items[3 * t + 2] = keys[t].i;
  }
  BCHK(B, hipMemcpyAsync(B->d_graphs, B->h_graphs.data(), B->nres * sizeof(ResGraph),
                         hipMemcpyHostToDevice, B->st));
  BCHK(B, hipMemcpyAsync(B->d_items, B->h_items.data(), B->h_items.size() * sizeof(int),
                         hipMemcpyHostToDevice, B->st));
  if (B->graph_nitems != nitems) {
    if (B->gexec) BCHK(B, hipGraphExecDestroy(B->gexec));
    if (B->graph) BCHK(B, hipGraphDestroy(B->graph));
    B->gexec = nullptr;
    B->graph = nullptr;
    const rafeast_plan_s* P0 = B->plans[0];
    CocgLaunch L;
    L.nitems = nitems;
    L.items = B->d_items;
    L.tol = P0->prm.tol_solve;
    L.maxit = P0->prm.max_cocg;
    L.max_refine = 64;
    L.counter = B->d_counter;
    L.xhi = B->d_xhi;
    L.xhi_slots = B->xhi_slots;
    BCHK(B, prepare_cocg_resident(B->max_n, B->rpt, B->fp32));
    BCHK(B, hipStreamBeginCapture(B->st, hipStreamCaptureModeRelaxed));
    hipError_t e = launch_fill_int(B->st, B->d_counter, 0, 1);
    if (e == hipSuccess)
      e = launch_cocg_resident(B->st, nullptr, B->d_graphs, B->max_n, B->rpt, L, B->fp32,
                               B->num_cu);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(B->st, &g);
    BCHK(B, e);
    BCHK(B, e2);
    B->graph = g;
    BCHK(B, hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
    B->graph_nitems = nitems;
  }
  BCHK(B, hipGraphLaunch(B->gexec, B->st));
  return RAFEAST_OK;
}
}  // namespace

extern "C" {

rafeast_status rafeast_plan_batch(int32_t count, const rafeast_csr* A, const rafeast_params* prm,
                                  rafeast_batch_t* out) {
  if (!out) return batch_fail(nullptr, RAFEAST_INVALID_ARG, "null output");
  *out = nullptr;
  if (count < 1 || !A || !prm) return batch_fail(nullptr, RAFEAST_INVALID_ARG, "need count >= 1 and arrays");
  for (int g = 0; g < count; ++g) {
    if (prm[g].precond != RAFEAST_PC_NONE)
      return batch_fail(nullptr, RAFEAST_UNSUPPORTED,
                        "the batching form runs unpreconditioned COCG (member " +
                            std::to_string(g) + " asks for precond LEARNED)");
    if (prm[g].engine == RAFEAST_ENGINE_DIRECT)
      return batch_fail(nullptr, RAFEAST_UNSUPPORTED,
                        "the batching form runs COCG (member " + std::to_string(g) +
                            " asks for the direct engine)");
  }
  for (int g = 1; g < count; ++g)
    if (prm[g].precision != prm[0].precision || prm[g].tol_solve != prm[0].tol_solve ||
        prm[g].max_cocg != prm[0].max_cocg)
      return batch_fail(nullptr, RAFEAST_INVALID_ARG,
                        "batch members must share precision, tol_solve and max_cocg");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return batch_fail(nullptr, RAFEAST_DEVICE, "no HIP device available");
  rafeast_batch_s* B = new rafeast_batch_s();
  B->fp32 = prm[0].precision == RAFEAST_FP32_REFINED;
  auto bail = [&](rafeast_status st) {
    g_batch_error = B->err;
    free_batch(B);
    return st;
  };
#define BPCHK(expr)                                                   \
  do {                                                                \
    hipError_t _e = (expr);                                           \
    if (_e != hipSuccess)                                             \
      return bail(batch_fail(B, _e == hipErrorOutOfMemory ? RAFEAST_OOM : RAFEAST_DEVICE, \
                             std::string(#expr) + ": " + hipGetErrorString(_e)));         \
  } while (0)
  if (prm[0].hip_stream) {
    B->st = (hipStream_t)prm[0].hip_stream;
  } else {
    BPCHK(hipStreamCreateWithFlags(&B->st, hipStreamNonBlocking));
    B->own_stream = true;
  }
  for (auto& e : B->ev) BPCHK(hipEventCreate(&e));
  B->mst.assign(count, nullptr);
  B->mev.assign(count, nullptr);
  for (int g = 0; g < count; ++g) {
    BPCHK(hipStreamCreateWithFlags(&B->mst[g], hipStreamNonBlocking));
    BPCHK(hipEventCreateWithFlags(&B->mev[g], hipEventDisableTiming));
  }
  for (int g = 0; g < count; ++g) {
    rafeast_params q = prm[g];
    q.hip_stream = B->mst[g];
    // members left to the library's choice that the shared resident launch
    // cannot hold run the multi-shift engine (FP64; it needs nothing from
    // the shared launch and takes one real SpMV of m0 columns per iteration)
    if (q.engine == RAFEAST_ENGINE_AUTO && A[g].n > cocg_resident_max_n(B->fp32) &&
        q.m0 <= 192) {
      q.engine = RAFEAST_ENGINE_MULTISHIFT;
      q.precision = RAFEAST_FP64;
    }
    rafeast_plan_t P = nullptr;
    const rafeast_status st = rafeast_plan(&A[g], &q, &P);
    if (st != RAFEAST_OK) {
      B->err = "member " + std::to_string(g) + ": " + rafeast_last_error(nullptr);
      return bail(st);
    }
    B->plans.push_back(P);
  }
  // resident members share one launch: a common slot count per wave and
  // LDS sized for the largest of them
  B->res_idx.assign(count, -1);
  B->wtab.assign(count, nullptr);
  for (int g = 0; g < count; ++g) {
    rafeast_plan_s* P = B->plans[g];
    if (P->engine != RAFEAST_ENGINE_RESIDENT) continue;
    B->res_idx[g] = B->nres++;
    B->rpt = std::max(B->rpt, P->sell.wave_rpt);
    B->max_n = std::max<int>(B->max_n, (int)P->n);
  }
  B->num_cu = B->plans[0]->num_cu;
  if (B->nres > 0) {
    for (int g = 0; g < count; ++g) {
      rafeast_plan_s* P = B->plans[g];
      if (B->res_idx[g] < 0) continue;
      if (P->sell.wave_rpt == B->rpt) {
        B->wtab[g] = const_cast<int*>(P->sell.wave_slices);
        continue;
      }
      // more slots per wave than the member needs always fit
      const std::vector<int> tab = cocg_resident_wave_table(P->sell_widths, B->rpt);
      if (tab.empty())
        return bail(batch_fail(B, RAFEAST_UNSUPPORTED, "wave table of member " + std::to_string(g)));
      int* d = nullptr;
      BPCHK(hipMalloc(&d, tab.size() * sizeof(int)));
      B->own_wtab.push_back(d);
      BPCHK(hipMemcpy(d, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
      B->wtab[g] = d;
    }
    size_t items = 0;
    for (int g = 0; g < count; ++g)
      if (B->res_idx[g] >= 0) items += 3 * (size_t)B->plans[g]->nitems;
    B->h_graphs.resize(B->nres);
    BPCHK(hipMalloc(&B->d_graphs, B->nres * sizeof(ResGraph)));
    BPCHK(hipMalloc(&B->d_items, items * sizeof(int)));
    BPCHK(hipMalloc(&B->d_counter, sizeof(int)));
    B->xhi_slots = (size_t)B->num_cu * ((size_t)(B->max_n + 63) / 64 * 64);
    BPCHK(hipMalloc(&B->d_xhi, B->xhi_slots * 2 * sizeof(double)));
  }
#undef BPCHK
  *out = B;
  return RAFEAST_OK;
}

rafeast_plan_t rafeast_batch_plan(rafeast_batch_t B, int32_t g) {
  if (!B || g < 0 || g >= (int32_t)B->plans.size()) return nullptr;
  return B->plans[g];
}

int32_t rafeast_batch_resident_count(rafeast_batch_t B) { return B ? B->nres : 0; }

rafeast_status rafeast_batch_solve(rafeast_batch_t B, const double* const* Q_init,
                                   rafeast_result* res, rafeast_status* status, double* t_ms) {
  if (!B || !res) return RAFEAST_INVALID_ARG;
  const int count = (int)B->plans.size();
  for (int g = 0; g < count; ++g)
    if (!res[g].lambda || !res[g].resid) return batch_fail(B, RAFEAST_INVALID_ARG, "result arrays");
  B->err.clear();
  double tb[RAFEAST_NPHASE] = {0, 0, 0, 0, 0};
  auto member_fail = [&](int g, rafeast_status st) {
    return batch_fail(B, st, "member " + std::to_string(g) + ": " + B->plans[g]->err);
  };
  BCHK(B, hipEventRecord(B->ev[0], B->st));
  for (int g = 0; g < count; ++g)  // members start after the batch's start mark
    BCHK(B, hipStreamWaitEvent(B->plans[g]->st, B->ev[0], 0));
  std::vector<SolveRun> S(count);
  for (int g = 0; g < count; ++g) {
    const rafeast_status st = solve_begin(B->plans[g], Q_init ? Q_init[g] : nullptr, S[g]);
    if (st != RAFEAST_OK) return member_fail(g, st);
  }
  std::vector<char> active(count, 1);
  for (;;) {
    int nact = 0;
    for (int g = 0; g < count; ++g) {
      if (!active[g]) continue;
      const rafeast_status st = solve_test(B->plans[g], S[g]);
      if (st != RAFEAST_OK) return member_fail(g, st);
      if (S[g].done)
        active[g] = 0;
      else
        ++nact;
    }
    if (nact == 0) break;
    // every active member's solves: the shared resident launch on the batch
    // stream, and the streaming members concurrently, each on its own
    // stream from a host worker (their kernels are small, so several in
    // flight fill the device).  A member's own solve time is this phase.
    BCHK(B, hipEventRecord(B->ev[2], B->st));
    for (int g = 0; g < count; ++g) {
      if (!active[g]) continue;
      rafeast_plan_s* P = B->plans[g];
      BCHK(B, hipEventRecord(B->mev[g], P->st));     // its right-hand sides are ready
      BCHK(B, hipStreamWaitEvent(B->st, B->mev[g], 0));
      BCHK(B, hipEventRecord(P->ev[2], P->st));
    }
    RCHK(batch_resident_solves(B, active));
    std::vector<int> todo;
    for (int g = 0; g < count; ++g)
      if (active[g] && B->res_idx[g] < 0) todo.push_back(g);
    std::vector<rafeast_status> sst(count, RAFEAST_OK);
    {
      std::atomic<size_t> next{0};
      auto worker = [&]() {
        for (size_t t = next++; t < todo.size(); t = next++)
          sst[todo[t]] = solve_shifted_systems(B->plans[todo[t]], S[todo[t]]);
      };
      const size_t nthr = std::min<size_t>(todo.size(), kBatchWorkers);
      std::vector<std::thread> pool;
      for (size_t t = 1; t < nthr; ++t) pool.emplace_back(worker);
      if (nthr > 0) worker();
      for (auto& th : pool) th.join();
    }
    for (int g : todo)
      if (sst[g] != RAFEAST_OK) return member_fail(g, sst[g]);
    BCHK(B, hipEventRecord(B->ev[5], B->st));  // the shared launch is done
    for (int g = 0; g < count; ++g) {
      if (!active[g]) continue;
      rafeast_plan_s* P = B->plans[g];
      if (B->res_idx[g] >= 0) BCHK(B, hipStreamWaitEvent(P->st, B->ev[5], 0));
      BCHK(B, hipEventRecord(B->mev[g], P->st));
      BCHK(B, hipStreamWaitEvent(B->st, B->mev[g], 0));
    }
    BCHK(B, hipEventRecord(B->ev[3], B->st));
    for (int g = 0; g < count; ++g) {
      if (!active[g]) continue;
      rafeast_plan_s* P = B->plans[g];
      BCHK(B, hipStreamWaitEvent(P->st, B->ev[3], 0));
      BCHK(B, hipEventRecord(P->ev[3], P->st));
      const rafeast_status st = solve_combine(P, S[g]);
      if (st != RAFEAST_OK) return member_fail(g, st);
      BCHK(B, hipEventRecord(B->mev[g], P->st));
      BCHK(B, hipStreamWaitEvent(B->st, B->mev[g], 0));
    }
    BCHK(B, hipEventRecord(B->ev[4], B->st));
    BCHK(B, hipEventSynchronize(B->ev[4]));
    tb[RAFEAST_PH_SOLVE] += elapsed(B->ev[2], B->ev[3]);
    tb[RAFEAST_PH_COMBINE] += elapsed(B->ev[3], B->ev[4]);  // combination and CholQR2
  }
  rafeast_status first = RAFEAST_OK;
  for (int g = 0; g < count; ++g) {
    const rafeast_status st = solve_finish(B->plans[g], S[g], &res[g]);
    BCHK(B, hipEventRecord(B->mev[g], B->plans[g]->st));
    BCHK(B, hipStreamWaitEvent(B->st, B->mev[g], 0));
    if (st != RAFEAST_OK && st != RAFEAST_NO_CONVERGENCE && st != RAFEAST_SUBSPACE_TOO_SMALL &&
        st != RAFEAST_EMPTY_WINDOW && st != RAFEAST_BREAKDOWN)
      return member_fail(g, st);
    if (status) status[g] = st;
    if (st != RAFEAST_OK && first == RAFEAST_OK) first = st;
    tb[RAFEAST_PH_RR] += S[g].t_ph[RAFEAST_PH_RR];
  }
  BCHK(B, hipEventRecord(B->ev[1], B->st));
  BCHK(B, hipEventSynchronize(B->ev[1]));
  tb[RAFEAST_PH_TOTAL] = elapsed(B->ev[0], B->ev[1]);
  if (t_ms)
    for (int i = 0; i < RAFEAST_NPHASE; ++i) t_ms[i] = tb[i];
  return first;
}

void rafeast_batch_destroy(rafeast_batch_t B) { free_batch(B); }

const char* rafeast_batch_last_error(rafeast_batch_t B) {
  return B ? B->err.c_str() : g_batch_error.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned polynomial preconditioner
// ---------------------------------------------------------------------------

extern "C" {

int32_t rafeast_pc_param_count(void) { return mlp_param_count(); }

rafeast_status rafeast_pc_samples(rafeast_plan_t P, int32_t nz, const double* z, int32_t k,
                                  const double* R, int32_t ldr, double theta_lo, double theta_hi,
                                  double* X, double* G, double* h, double* rr) {
  if (P && P->dop.kind != 0)
    return fail(P, RAFEAST_UNSUPPORTED, "the learned preconditioner takes CSR plans");
  if (!P || !z || !R || !X || !G || !h || !rr || nz < 1 || k < 1 || ldr < k)
    return RAFEAST_INVALID_ARG;
  P->err.clear();
  const int64_t n = P->n;
  double a, b;
  spectral_map(P, a, b);
  DevBuf buf;
  double *T = nullptr, *part = nullptr, *dz = nullptr;
  const size_t bs = (size_t)n * k;
  const int nchunks = (int)std::max<int64_t>(1, std::min<int64_t>(256, (n + 2047) / 2048));
  HIPCHK(P, buf.get(&T, 9 * bs));
  HIPCHK(P, buf.get(&part, (size_t)nchunks * k * 136));
  HIPCHK(P, buf.get(&dz, 2 * (size_t)nz));
  HIPCHK(P, hipMemcpyAsync(dz, z, 2 * nz * sizeof(double), hipMemcpyHostToDevice, P->st));
  HIPCHK(P, launch_copy_cols(P->st, n, k, R, ldr, T, k));
  // T_1 = A^ T_0, T_{k+1} = 2 A^ T_k - T_{k-1}
  RCHK(spmm(P, k, T, k, T + bs, k, a, b));
  for (int t = 1; t < 8; ++t)
    RCHK(spmm(P, k, T + t * bs, k, T + (t + 1) * bs, k, 2.0 * a, 2.0 * b, T + (t - 1) * bs, k,
              -1.0));
  HIPCHK(P, launch_pc_gram_assemble(P->st, n, k, T, nz, dz, a, b, theta_lo, theta_hi, part,
                                    nchunks, X, G, h, rr));
  HIPCHK(P, hipStreamSynchronize(P->st));
  return RAFEAST_OK;
}

rafeast_status rafeast_pc_forward(rafeast_plan_t P, int32_t ns, const double* X, const float* W,
                                  float* Y) {
  if (!P || !X || !W || !Y || ns < 1) return RAFEAST_INVALID_ARG;
  DevBuf buf;
  float* wb = nullptr;
  HIPCHK(P, buf.get(&wb, mlp_param_count()));
  HIPCHK(P, launch_mlp_bf16(P->st, W, wb));
  HIPCHK(P, launch_mlp_forward(P->st, ns, X, wb, Y));
  HIPCHK(P, hipStreamSynchronize(P->st));
  return RAFEAST_OK;
}

rafeast_status rafeast_pc_gradient(rafeast_plan_t P, int32_t ns, const double* X, const double* G,
                                   const double* h, const double* rr, const float* W, float* grad,
                                   double* loss) {
  if (!P || !X || !G || !h || !rr || !W || !grad || ns < 1) return RAFEAST_INVALID_ARG;
  DevBuf buf;
  float *wb = nullptr, *part = nullptr;
  double *lpart = nullptr, *dl = nullptr;
  int* idx = nullptr;
  const int npar = mlp_param_count(), waves = mlp_backward_waves(ns);
  HIPCHK(P, buf.get(&wb, npar));
  HIPCHK(P, buf.get(&part, (size_t)waves * npar));
  HIPCHK(P, buf.get(&lpart, waves));
  HIPCHK(P, buf.get(&dl, 1));
  HIPCHK(P, buf.get(&idx, ns));
  std::vector<int> order(ns);
  for (int i = 0; i < ns; ++i) order[i] = i;
  HIPCHK(P, hipMemcpyAsync(idx, order.data(), ns * sizeof(int), hipMemcpyHostToDevice, P->st));
  HIPCHK(P, launch_mlp_bf16(P->st, W, wb));
  HIPCHK(P, launch_mlp_grad(P->st, ns, idx, X, G, h, rr, wb, part, lpart, grad, dl));
  double hl = 0.0;
  HIPCHK(P, hipMemcpyAsync(&hl, dl, sizeof(double), hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  if (loss) *loss = hl;
  return RAFEAST_OK;
}

rafeast_status rafeast_pc_train(rafeast_plan_t P, int32_t ns, const double* X, const double* G,
                                const double* h, const double* rr, float* W, int32_t steps,
                                int32_t batch, const int32_t* order, float lr, double* loss) {
  if (!P || !X || !G || !h || !rr || !W || !order || ns < 1 || steps < 1 || batch < 1 ||
      !(lr > 0.0f))
    return RAFEAST_INVALID_ARG;
  for (int64_t t = 0; t < (int64_t)steps * batch; ++t)
    if (order[t] < 0 || order[t] >= ns) return fail(P, RAFEAST_INVALID_ARG, "order out of range");
  DevBuf buf;
  float *wb = nullptr, *part = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  double *lpart = nullptr, *dl = nullptr;
  int* idx = nullptr;
  const int npar = mlp_param_count(), waves = mlp_backward_waves(batch);
  HIPCHK(P, buf.get(&wb, npar));
  HIPCHK(P, buf.get(&part, (size_t)waves * npar));
  HIPCHK(P, buf.get(&m, npar));
  HIPCHK(P, buf.get(&v, npar));
  HIPCHK(P, buf.get(&g, npar));
  HIPCHK(P, buf.get(&lpart, waves));
  HIPCHK(P, buf.get(&dl, steps));
  HIPCHK(P, buf.get(&idx, (size_t)steps * batch));
  HIPCHK(P, hipMemcpyAsync(idx, order, (size_t)steps * batch * sizeof(int),
                           hipMemcpyHostToDevice, P->st));
  HIPCHK(P, hipMemsetAsync(m, 0, npar * sizeof(float), P->st));
  HIPCHK(P, hipMemsetAsync(v, 0, npar * sizeof(float), P->st));
  HIPCHK(P, launch_mlp_bf16(P->st, W, wb));
  for (int t = 0; t < steps; ++t) {
    HIPCHK(P, launch_mlp_grad(P->st, batch, idx + (size_t)t * batch, X, G, h, rr, wb, part, lpart,
                              g, dl + t));
    HIPCHK(P, launch_adam(P->st, W, m, v, g, lr, t + 1, wb));
  }
  if (loss)
    HIPCHK(P, hipMemcpyAsync(loss, dl, steps * sizeof(double), hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  return RAFEAST_OK;
}

rafeast_status rafeast_pc_harvest(rafeast_plan_t P, int32_t nsteps, const int32_t* steps,
                                  double* X, double* G, double* h, double* rr, int32_t* count) {
  if (P && P->dop.kind != 0)
    return fail(P, RAFEAST_UNSUPPORTED, "the learned preconditioner takes CSR plans");
  if (!P || !X || !G || !h || !rr || !count || nsteps < 1 || !steps) return RAFEAST_INVALID_ARG;
  for (int t = 0; t < nsteps; ++t)
    if (steps[t] < 0) return fail(P, RAFEAST_INVALID_ARG, "negative COCG step count");
  if ((int)P->last_theta.size() != P->m0)
    return fail(P, RAFEAST_INVALID_ARG, "no Rayleigh-Ritz step yet (run rafeast_solve first)");
  P->err.clear();
  *count = 0;
  const int64_t n = P->n;
  const int m0 = P->m0, nc = P->nc, Bc = nc * m0;
  const double th_lo = P->last_theta.front(), th_hi = P->last_theta.back();
  DevBuf buf;
  cpx<double>* xs = nullptr;
  cpx<double>* rs = nullptr;
  double* split = nullptr;
  int64_t s0 = 0;  // samples written
  for (int t = 0; t < nsteps; ++t) {
    if (steps[t] == 0) {  // the right-hand sides themselves (real)
      for (int j = 0; j < nc; ++j) {
        RCHK(rafeast_pc_samples(P, 1, P->zw.data() + 2 * j, m0, P->d_R, P->ld, th_lo, th_hi,
                                X + 4 * s0, G + 128 * s0, h + 16 * s0, rr + s0));
        s0 += m0;
      }
      continue;
    }
    if (!xs) {
      HIPCHK(P, buf.get(&xs, (size_t)n * Bc));
      HIPCHK(P, buf.get(&rs, (size_t)n * Bc));
      HIPCHK(P, buf.get(&split, (size_t)n * 2 * m0));
    }
    // exactly steps[t] plain FP64 COCG iterations (a tolerance no residual meets)
    RCHK(pc_solve_run(P, nc, P->zw.data(), m0, P->d_R, P->ld, nullptr, xs, 1e-300, nullptr,
                      nullptr, steps[t], rs));
    for (int j = 0; j < nc; ++j) {
      HIPCHK(P, launch_split_complex(P->st, n, Bc, j * m0, m0, rs, split));
      RCHK(rafeast_pc_samples(P, 1, P->zw.data() + 2 * j, 2 * m0, split, 2 * m0, th_lo, th_hi,
                              X + 4 * s0, G + 128 * s0, h + 16 * s0, rr + s0));
      s0 += 2 * m0;
    }
  }
  *count = (int32_t)s0;
  return RAFEAST_OK;
}

rafeast_status rafeast_pc_normalize(rafeast_plan_t P, int32_t ns, const double* X, float* W) {
  if (!P || !X || !W || ns < 1) return RAFEAST_INVALID_ARG;
  P->err.clear();
  std::vector<double> hx(4 * (size_t)ns);
  HIPCHK(P, hipMemcpyAsync(hx.data(), X, hx.size() * sizeof(double), hipMemcpyDeviceToHost, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  float ms[8];
  for (int f = 0; f < 4; ++f) {
    double mean = 0.0;
    for (int s = 0; s < ns; ++s) mean += hx[4 * (size_t)s + f];
    mean /= ns;
    double var = 0.0;
    for (int s = 0; s < ns; ++s) {
      const double d = hx[4 * (size_t)s + f] - mean;
      var += d * d;
    }
    const double sd = std::sqrt(var / ns);
    ms[f] = (float)mean;
    // a spread at the rounding level of the feature is a constant feature
    const bool varies = std::isfinite(sd) && sd > 1e-9 * std::max(1.0, std::fabs(mean));
    ms[4 + f] = varies ? (float)sd : 1.0f;
  }
  const int npar = mlp_param_count();
  HIPCHK(P, hipMemcpyAsync(W + (npar - 8), ms, sizeof(ms), hipMemcpyHostToDevice, P->st));
  HIPCHK(P, hipStreamSynchronize(P->st));
  return RAFEAST_OK;
}

rafeast_status rafeast_pc_attach(rafeast_plan_t P, const float* W) {
  if (P && P->dop.kind != 0)
    return fail(P, RAFEAST_UNSUPPORTED, "the learned preconditioner takes CSR plans");
  if (!P || !W) return RAFEAST_INVALID_ARG;
  P->err.clear();
  const int npar = mlp_param_count();
  if (!P->d_pcW) {  // plans made with precond NONE get the buffers on first attach
    HIPCHK(P, hipMalloc(&P->d_pcW, npar * sizeof(float)));
    HIPCHK(P, hipMalloc(&P->d_pcWb, npar * sizeof(float)));
    HIPCHK(P, hipMalloc(&P->d_pcX, 4 * (size_t)P->nc * sizeof(double)));
    HIPCHK(P, hipMalloc(&P->d_pcY, 16 * (size_t)P->nc * sizeof(float)));
  }
  HIPCHK(P, hipMemcpyAsync(P->d_pcW, W, npar * sizeof(float), hipMemcpyDeviceToDevice, P->st));
  HIPCHK(P, launch_mlp_bf16(P->st, P->d_pcW, P->d_pcWb));
  HIPCHK(P, hipStreamSynchronize(P->st));
  P->pc_ready = true;
  return RAFEAST_OK;
}

rafeast_status rafeast_pc_solve(rafeast_plan_t P, int32_t nz, const double* z, int32_t k,
                                const double* B, int32_t ldb, const double* coef, void* Xout,
                                double tol, int32_t* iters, double* resid) {
  if (P && P->dop.kind != 0)
    return fail(P, RAFEAST_UNSUPPORTED, "the learned preconditioner takes CSR plans");
  if (!P || !z || !B || !Xout || nz < 1 || k < 1 || ldb < k || !(tol > 0.0) || !(tol < 1.0))
    return RAFEAST_INVALID_ARG;
  P->err.clear();
  return pc_solve_run(P, nz, z, k, B, ldb, coef, Xout, tol, iters, resid);
}

}  // extern "C"
