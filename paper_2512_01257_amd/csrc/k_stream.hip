// Streaming COCG engine for systems too large to keep in one workgroup's LDS.
// All shifted systems (z_c I - A) d_c = b_c advance in lock step, one kernel
// sequence per iteration, and every vector is an n x Bp complex block in HBM,
// row-major: row r of a block holds the Bp columns' values contiguously, so
// the gather of a neighbour row is one coalesced read of 64 * CPL columns.
//
// Method: COCG on the unconjugated bilinear form, in the engine precision,
// with reliable updates in FP64: whenever a column's recursive residual has
// dropped by the factor delta since its last check (or below the tolerance,
// or the column hit its iteration cap), the engine folds x into the FP64
// solution x_hi, recomputes the true residual s = b - (zI - A) x_hi in FP64,
// and continues the same Krylov recurrence from r = s (the search direction
// is kept; beta is recomputed from s).  This removes the drift between the
// recursive and the true residual that FP32 storage causes, without the
// restarts that would throw away the recurrence.  The iteration restarts from
// p = s only after a breakdown (p^T (zI - A) p = 0) or a stall: a column
// whose recursive residual has not dropped by delta within 4x the length of
// its previous check interval (and 2x the first interval after its last
// start, the initial plateau a restart has to cross again) is checked early,
// and if its true residual has not at least halved since the last check, the
// recurrence starts afresh.
// Each column has its own scalars and a state on the device:
//   1  iterating
//   0  waiting for the FP64 residual check (reliable update)
//   3  waiting for the FP64 residual check after a breakdown (restart)
//   2  solved (true residual <= tol) or given up (iteration or update
//      budget spent, repeated breakdown); frozen
// Columns that are not in state 1 keep their vectors unchanged while the
// others iterate (the p update copies them, alpha = 0).  Checks run between
// chunks of iterations.  The columns are cut into groups of
// 64 * CPL; a group with no iterating column is skipped by the row kernels
// (the host passes the list of live groups by value), so shifts that
// converge early stop costing bandwidth.  Group order follows the column
// order c = j * k + i.
//
// An iteration: K1 forms p = r + beta p on the rows each wave owns, K2 the
// SpMV w = (zI - A) p gathering only p (a fused form that gathered r and the
// old p and formed p on the fly read twice the neighbour bytes, 20% slower),
// the finalisers turn partials into alpha, K3 updates x and r.
// Row kernels: 256 threads (4 waves).  Each XCD sweeps one contiguous eighth
// of the rows with all its waves side by side (see wave_rows), keeping the
// neighbour gathers in that XCD's L2.  A wave takes one row at a time; its 64
// lanes hold CPL consecutive complex columns each.  The
// matrix row (column indices and values) is wave-uniform and comes through
// the scalar cache.  Reductions are per-workgroup partials, summed in a fixed
// order by one-column-per-lane finaliser kernels, so results are
// deterministic.
#include <utility>

#include "device.h"
#include "kernels.h"

namespace rafeast {

namespace {

constexpr int kST = 256;             // threads of a row kernel
constexpr int kSW = kST / 64;        // waves of a row kernel
constexpr int kFinThreads = 1024;    // finaliser: 16 columns x 64 partial groups
constexpr int kFinCols = 16;
constexpr int kFinGroups = kFinThreads / kFinCols;

// Rows of a wave.  The rows are cut into 8 contiguous stripes, one per XCD
// (dispatch round-robins workgroup ids over the 8 XCDs, so workgroup b runs
// on XCD b mod 8); inside a stripe the XCD's waves take consecutive rows and
// sweep the stripe together, so the rows in flight on an XCD form a window of
// about (waves per XCD) rows and the neighbour rows a gather needs were
// loaded recently into the same L2.  Row k of this wave is
// first + k * stride, k < count.
struct WaveRows {
  int first, stride, count;
};

__device__ __forceinline__ WaveRows wave_rows(int n) {
  const int nb = gridDim.x;
  int x = 0, i = (int)blockIdx.x, per_x = nb, lo = 0, hi = n;
  if (nb % 8 == 0) {
    x = (int)(blockIdx.x % 8);
    i = (int)(blockIdx.x / 8);
    per_x = nb / 8;
    const int stripe = (n + 7) / 8;
    lo = min(n, x * stripe);
    hi = min(n, lo + stripe);
  }
  const int stride = per_x * kSW;
  const int first = lo + i * kSW + wave_id();
  return {first, stride, first < hi ? (hi - first + stride - 1) / stride : 0};
}

__device__ __forceinline__ bool waiting(int st) { return st == 0 || st == 3; }

__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_bcast(double v, int l) { return readlane_f64(v, l); }

template <typename T, int CPL>
struct Chunk {
  cpx<T> v[CPL];
};

template <typename T, int CPL>
__device__ __forceinline__ Chunk<T, CPL> ld(const cpx<T>* __restrict__ p) {
  Chunk<T, CPL> c;
#pragma unroll
  for (int q = 0; q < CPL; ++q) c.v[q] = p[q];
  return c;
}

template <typename T, int CPL>
__device__ __forceinline__ void st(cpx<T>* __restrict__ p, const Chunk<T, CPL>& c) {
#pragma unroll
  for (int q = 0; q < CPL; ++q) p[q] = c.v[q];
}

// The same as a non-temporal store: the value streams past L2 (written once,
// read by a later kernel), which keeps L2 for the rows a gather reuses.
template <typename T, int CPL>
__device__ __forceinline__ void st_nt(cpx<T>* __restrict__ p, const Chunk<T, CPL>& c) {
  T* f = reinterpret_cast<T*>(p);
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    __builtin_nontemporal_store(c.v[q].re, f + 2 * q);
    __builtin_nontemporal_store(c.v[q].im, f + 2 * q + 1);
  }
}

// Sum the 4 waves' per-lane partials and store the workgroup's partials at
// part[(blockIdx.x * Bp + c) * NQ + u].
template <int CPL, int NQ>
__device__ __forceinline__ void put_partials(const double (&acc)[CPL][NQ], double* __restrict__ part,
                                             int Bp, int c0, double* sh) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int kPer = 64 * CPL * NQ;
#pragma unroll
  for (int q = 0; q < CPL; ++q)
#pragma unroll
    for (int u = 0; u < NQ; ++u) sh[wv * kPer + (lane * CPL + q) * NQ + u] = acc[q][u];
  __syncthreads();
  for (int e = threadIdx.x; e < kPer; e += kST) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSW; ++w) s += sh[w * kPer + e];
    part[((size_t)blockIdx.x * Bp + c0) * NQ + e] = s;
  }
}

// Column of finaliser thread t (16 columns per block; thread t and t + 16k
// share a column).
__device__ __forceinline__ int fin_col() { return blockIdx.x * kFinCols + (threadIdx.x % kFinCols); }

// Fixed-order column sums of the partials of nb workgroups, for the 16
// columns of this finaliser block: 64 interleaved partial groups, then a
// fixed combination.  Result valid in threads 0..15 (column fin_col()).
// `want` must be the same in all threads of a column.
template <int NQ>
__device__ __forceinline__ void col_sums(const double* __restrict__ part, int nb, int Bp,
                                         bool want, double (&out)[NQ]) {
  __shared__ double sh[kFinThreads * NQ];
  const int t = threadIdx.x, g = t / kFinCols;
  const int c = fin_col();
  double s[NQ];
#pragma unroll
  for (int u = 0; u < NQ; ++u) s[u] = 0.0;
  if (want && c < Bp)
    for (int b = g; b < nb; b += kFinGroups)
#pragma unroll
      for (int u = 0; u < NQ; ++u) s[u] += part[((size_t)b * Bp + c) * NQ + u];
#pragma unroll
  for (int u = 0; u < NQ; ++u) sh[t * NQ + u] = s[u];
  __syncthreads();
  if (t < kFinCols) {
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      double a = 0.0;
      for (int gg = 0; gg < kFinGroups; ++gg) a += sh[(gg * kFinCols + t) * NQ + u];
      out[u] = a;
    }
  }
}

}  // namespace

// K1: the new search direction of the group's live columns, p = r + beta p
// (frozen columns keep p), written to the other p buffer; own rows only, so
// the SpMV after it gathers a single vector.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_pupd(int n, int Bp, StreamGroups grp,
                                                const double* __restrict__ beta,
                                                const int* __restrict__ state,
                                                const cpx<T>* __restrict__ r,
                                                cpx<T>* __restrict__ pa, cpx<T>* __restrict__ pb) {
  const int lane = threadIdx.x & 63;
  const int c0 = grp.g[blockIdx.y] * 64 * CPL;
  const cpx<T>* __restrict__ pold = grp.par[blockIdx.y] ? pb : pa;
  cpx<T>* __restrict__ pnew = grp.par[blockIdx.y] ? pa : pb;
  const int cl = c0 + lane * CPL;
  T bre[CPL], bim[CPL];
  bool live[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    bre[q] = T(beta[2 * (cl + q)]);
    bim[q] = T(beta[2 * (cl + q) + 1]);
    live[q] = state[cl + q] == 1;
  }
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const size_t ro = (size_t)(wr.first + wr.stride * k) * Bp + cl;
    const Chunk<T, CPL> r0 = ld<T, CPL>(r + ro);
    const Chunk<T, CPL> p0 = ld<T, CPL>(pold + ro);
    Chunk<T, CPL> pn;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (live[q]) {
        pn.v[q].re = r0.v[q].re + bre[q] * p0.v[q].re - bim[q] * p0.v[q].im;
        pn.v[q].im = r0.v[q].im + bre[q] * p0.v[q].im + bim[q] * p0.v[q].re;
      } else {
        pn.v[q] = p0.v[q];
      }
    }
    st<T, CPL>(pnew + ro, pn);
  }
}

// K2: w = (z I - A) p over the group's columns (p the current buffer, frozen
// columns give w = 0) and the partials of mu = p^T w.  A wave takes one row
// at a time; the row's entries come lane-parallel (lane l holds entry l) and
// are broadcast with readlane, the next row's entries in flight during this
// row's gathers; each gather is one 16-byte load per lane.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_spmm(int n, const int* __restrict__ rowptr,
                                                const int* __restrict__ col,
                                                const T* __restrict__ val, int Bp,
                                                StreamGroups grp, const double* __restrict__ zc,
                                                const int* __restrict__ state,
                                                const cpx<T>* __restrict__ pa,
                                                const cpx<T>* __restrict__ pb,
                                                cpx<T>* __restrict__ w,
                                                double* __restrict__ part) {
  extern __shared__ double sh[];
  const int lane = threadIdx.x & 63;
  const int c0 = grp.g[blockIdx.y] * 64 * CPL;
  const cpx<T>* __restrict__ p = grp.par[blockIdx.y] ? pb : pa;
  const int cl = c0 + lane * CPL;
  T zre[CPL], zim[CPL];
  bool live[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    zre[q] = T(zc[2 * (cl + q)]);
    zim[q] = T(zc[2 * (cl + q) + 1]);
    live[q] = state[cl + q] == 1;
  }
  double acc[CPL][2];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q][0] = acc[q][1] = 0.0;
  const WaveRows wr = wave_rows(n);
  int win = -64, rs = 0, re = 0;  // row-pointer window: lane l holds row (win + l)
  auto span = [&](int k, int& s, int& e) {
    if (k - win >= 64) {
      win = k;
      const int kr = k + lane;
      const int rl = wr.first + wr.stride * kr;
      rs = kr < wr.count ? rowptr[rl] : 0;
      re = kr < wr.count ? rowptr[rl + 1] : 0;
    }
    s = __builtin_amdgcn_readlane(rs, k - win);
    e = __builtin_amdgcn_readlane(re, k - win);
  };
  // lane l <- entry l of a row (own row with value 0 beyond the row's end)
  auto entries = [&](int row, int s, int len, int& mc, T& mv) {
    mc = row;
    mv = T(0);
    if (lane < len) {
      mc = col[s + lane];
      mv = val[s + lane];
    }
  };
  int s = 0, e = 0, mc = 0;
  T mv = T(0);
  if (wr.count > 0) {
    span(0, s, e);
    entries(wr.first, s, e - s, mc, mv);
  }
  for (int k = 0; k < wr.count; ++k) {
    const int row = wr.first + wr.stride * k;
    const int len = e - s;
    const size_t ro = (size_t)row * Bp + cl;
    const Chunk<T, CPL> p0 = ld<T, CPL>(p + ro);
    // next row's entries, in flight during this row's gathers
    int s2 = 0, e2 = 0, mc2 = 0;
    T mv2 = T(0);
    if (k + 1 < wr.count) {
      span(k + 1, s2, e2);
      entries(row + wr.stride, s2, e2 - s2, mc2, mv2);
    }
    T ar[CPL], ai[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) ar[q] = ai[q] = T(0);
    for (int base = 0; base < len; base += 64) {
      int cc = mc;
      T cv = mv;
      if (base > 0) entries(row, s + base, len - base, cc, cv);  // rows longer than 64
      const int m = min(64, len - base);
      constexpr int NB = 8;  // entries per batch
      for (int t0 = 0; t0 < m; t0 += NB) {
        int j[NB];
        T a[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          j[u] = __builtin_amdgcn_readlane(cc, t0 + u);
          a[u] = lane_bcast(cv, t0 + u);
        }
        Chunk<T, CPL> pj[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) pj[u] = ld<T, CPL>(p + (size_t)j[u] * Bp + cl);
#pragma unroll
        for (int u = 0; u < NB; ++u)
#pragma unroll
          for (int q = 0; q < CPL; ++q) {
            ar[q] += a[u] * pj[u].v[q].re;
            ai[q] += a[u] * pj[u].v[q].im;
          }
      }
    }
    Chunk<T, CPL> ww;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (live[q]) {
        ww.v[q].re = zre[q] * p0.v[q].re - zim[q] * p0.v[q].im - ar[q];
        ww.v[q].im = zre[q] * p0.v[q].im + zim[q] * p0.v[q].re - ai[q];
      } else {
        ww.v[q] = cpx<T>{T(0), T(0)};
      }
      const double pr = p0.v[q].re, pi = p0.v[q].im, wr_ = ww.v[q].re, wi = ww.v[q].im;
      acc[q][0] += pr * wr_ - pi * wi;
      acc[q][1] += pr * wi + pi * wr_;
    }
    st_nt<T, CPL>(w + ro, ww);  // read by the update kernel, not by this sweep
    s = s2;
    e = e2;
    mc = mc2;
    mv = mv2;
  }
  put_partials<CPL, 2>(acc, part, Bp, c0, sh);
}

// K3: x += alpha p, r -= alpha w; partials of r^T r (complex) and ||r||^2.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_update(int n, int Bp, StreamGroups grp,
                                                  const double* __restrict__ alpha,
                                                  cpx<T>* __restrict__ x, cpx<T>* __restrict__ r,
                                                  const cpx<T>* __restrict__ pa,
                                                  const cpx<T>* __restrict__ pb,
                                                  const cpx<T>* __restrict__ w,
                                                  double* __restrict__ part) {
  extern __shared__ double sh[];
  const int c0 = grp.g[blockIdx.y] * 64 * CPL;
  const cpx<T>* __restrict__ p = grp.par[blockIdx.y] ? pb : pa;
  const int cl = c0 + (threadIdx.x & 63) * CPL;
  T are[CPL], aim[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    are[q] = T(alpha[2 * (cl + q)]);
    aim[q] = T(alpha[2 * (cl + q) + 1]);
  }
  double acc[CPL][3];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const int row = wr.first + k * wr.stride;
    const size_t ro = (size_t)row * Bp + cl;
    Chunk<T, CPL> xx = ld<T, CPL>(x + ro);
    Chunk<T, CPL> rr = ld<T, CPL>(r + ro);
    const Chunk<T, CPL> pp = ld<T, CPL>(p + ro);
    const Chunk<T, CPL> ww = ld<T, CPL>(w + ro);
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      xx.v[q].re += are[q] * pp.v[q].re - aim[q] * pp.v[q].im;
      xx.v[q].im += are[q] * pp.v[q].im + aim[q] * pp.v[q].re;
      rr.v[q].re -= are[q] * ww.v[q].re - aim[q] * ww.v[q].im;
      rr.v[q].im -= are[q] * ww.v[q].im + aim[q] * ww.v[q].re;
      const double a = rr.v[q].re, b = rr.v[q].im;
      acc[q][0] += a * a - b * b;
      acc[q][1] += 2.0 * a * b;
      acc[q][2] += a * a + b * b;
    }
    st<T, CPL>(x + ro, xx);
    st<T, CPL>(r + ro, rr);
  }
  put_partials<CPL, 3>(acc, part, Bp, c0, sh);
}

// alpha = rho / mu for iterating columns; a breakdown (mu = 0 or alpha not
// finite) sends the column to a restart check.
__global__ __launch_bounds__(kFinThreads) void k_s_fin_mu(int Bp, int nb,
                                                          const double* __restrict__ part,
                                                          StreamCols cols) {
  const int c = fin_col();
  const bool want = c < Bp && cols.state[c] == 1;
  double m[2];
  col_sums<2>(part, nb, Bp, want, m);
  if (threadIdx.x >= kFinCols || c >= Bp) return;
  double ar = 0.0, ai = 0.0;
  if (want) {
    const zd a = zdiv(zd{cols.rho[2 * c], cols.rho[2 * c + 1]}, zd{m[0], m[1]});
    if ((m[0] == 0.0 && m[1] == 0.0) || !isfinite(a.re) || !isfinite(a.im)) {
      cols.state[c] = 3;
      cols.nbd[c] += 1;
    } else {
      ar = a.re;
      ai = a.im;
    }
  }
  cols.alpha[2 * c] = ar;
  cols.alpha[2 * c + 1] = ai;
}

// beta = rho_new / rho; a column whose recursive residual reached its check
// threshold, or whose iteration count reached the cap, waits for a check
// (rho keeps the previous value, which the check's beta needs).
__global__ __launch_bounds__(kFinThreads) void k_s_fin_rho(int Bp, int nb,
                                                           const double* __restrict__ part,
                                                           StreamCols cols, int maxit) {
  const int c = fin_col();
  const bool want = c < Bp && cols.state[c] == 1;
  double s[3];
  col_sums<3>(part, nb, Bp, want, s);
  if (threadIdx.x >= kFinCols || c >= Bp) return;
  double br = 0.0, bi = 0.0;
  if (want) {
    const int it = cols.it[c] + 1;
    cols.it[c] = it;
    const int sp = cols.span[c];
    const bool stall = sp > 0 && it - cols.lastit[c] > max(max(4 * sp, 2 * cols.span0[c]), 256);
    if (s[2] <= cols.ctol2[c] || it >= maxit || !isfinite(s[2]) || stall) {
      cols.state[c] = 0;
    } else {
      const zd bt = zdiv(zd{s[0], s[1]}, zd{cols.rho[2 * c], cols.rho[2 * c + 1]});
      br = bt.re;
      bi = bt.im;
      cols.rho[2 * c] = s[0];
      cols.rho[2 * c + 1] = s[1];
    }
  }
  cols.beta[2 * c] = br;
  cols.beta[2 * c + 1] = bi;
}

// Group census (one wave per group): cnt[g] = columns of group g in state 1,
// cnt[gridDim.x + g] = columns waiting for a check (state 0 or 3).
__global__ __launch_bounds__(64) void k_s_count(int Bp, int gw, StreamCols cols,
                                                int* __restrict__ cnt) {
  const int g = blockIdx.x;
  double a = 0.0, wt = 0.0;
  for (int c = g * gw + (int)threadIdx.x; c < (g + 1) * gw && c < Bp; c += 64) {
    a += cols.state[c] == 1 ? 1.0 : 0.0;
    wt += waiting(cols.state[c]) ? 1.0 : 0.0;
  }
  a = wave_sum(a);
  wt = wave_sum(wt);
  if (threadIdx.x == 0) {
    cnt[g] = (int)a;
    cnt[gridDim.x + g] = (int)wt;
  }
}

// Check, step 1: x_hi += x (FP64) and x = 0 for waiting columns.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_xhi(int n, int Bp, StreamGroups grp,
                                               const int* __restrict__ state,
                                               cpx<T>* __restrict__ x,
                                               cpx<double>* __restrict__ xh) {
  const int cl = grp.g[blockIdx.y] * 64 * CPL + (threadIdx.x & 63) * CPL;
  bool on[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) on[q] = waiting(state[cl + q]);
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const int row = wr.first + k * wr.stride;
    const size_t ro = (size_t)row * Bp + cl;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const cpx<T> xv = x[ro + q];
      cpx<double> h = xh[ro + q];
      h.re += (double)xv.re;
      h.im += (double)xv.im;
      xh[ro + q] = h;
      x[ro + q] = cpx<T>{T(0), T(0)};
    }
  }
}

// Check, step 2: s = b/||b|| - (z x_hi - A x_hi) in FP64 with the FP64
// values of A; r = s (and p = s after a breakdown); partials of s^T s and
// ||s||^2.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_resid64(
    int n, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ val, int Bp, StreamGroups grp, const double* __restrict__ zc,
    const int* __restrict__ state, const double* __restrict__ B, int ldb, int kcols,
    const double* __restrict__ scale, const int* __restrict__ perm,
    const cpx<double>* __restrict__ xh, cpx<T>* __restrict__ r, cpx<T>* __restrict__ pa,
    cpx<T>* __restrict__ pb, double* __restrict__ part) {
  extern __shared__ double sh[];
  const int c0 = grp.g[blockIdx.y] * 64 * CPL;
  cpx<T>* __restrict__ p = grp.par[blockIdx.y] ? pb : pa;
  const int cl = c0 + (threadIdx.x & 63) * CPL;
  double zre[CPL], zim[CPL], scl[CPL];
  bool on[CPL], rst[CPL];
  int ci[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    zre[q] = zc[2 * (cl + q)];
    zim[q] = zc[2 * (cl + q) + 1];
    on[q] = waiting(state[cl + q]);
    rst[q] = state[cl + q] == 3;
    ci[q] = (cl + q) % kcols;
    scl[q] = scale[cl + q];
  }
  double acc[CPL][3];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const int row = wr.first + k * wr.stride;
    const size_t ro = (size_t)row * Bp + cl;
    double ar[CPL], ai[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) ar[q] = ai[q] = 0.0;
    const int s = rowptr[row], e = rowptr[row + 1];
    for (int t = s; t < e; ++t) {
      const int j = col[t];
      const double a = val[t];
      const size_t jo = (size_t)j * Bp + cl;
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        if (!on[q]) continue;
        const cpx<double> xj = xh[jo + q];
        ar[q] += a * xj.re;
        ai[q] += a * xj.im;
      }
    }
    const size_t orow = (size_t)perm[row];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const cpx<double> xr = xh[ro + q];
      const double b = scl[q] != 0.0 ? B[orow * ldb + ci[q]] * scl[q] : 0.0;
      const double sr = b - (zre[q] * xr.re - zim[q] * xr.im - ar[q]);
      const double si = -(zre[q] * xr.im + zim[q] * xr.re - ai[q]);
      r[ro + q] = cpx<T>{T(sr), T(si)};
      if (rst[q]) p[ro + q] = cpx<T>{T(sr), T(si)};
      acc[q][0] += sr * sr - si * si;
      acc[q][1] += 2.0 * sr * si;
      acc[q][2] += sr * sr + si * si;
    }
  }
  put_partials<CPL, 3>(acc, part, Bp, c0, sh);
}

// Dense operator: the iterating columns of the current p packed side by side
// (packed column u holds column cidx[u] & 0xfffffff, read from the p buffer
// of parity ((cidx[u] >> 30) & 1) ^ flip), so the GEMM multiplies only the
// columns that iterate, not whole column groups.
template <typename T>
__global__ __launch_bounds__(kST) void k_s_pack(int n, int Bp, int nl,
                                                const int* __restrict__ cidx, int flip,
                                                const cpx<T>* __restrict__ pa,
                                                const cpx<T>* __restrict__ pb,
                                                cpx<T>* __restrict__ pc) {
  const int u = blockIdx.y * 64 + (threadIdx.x & 63);
  if (u >= nl) return;
  const int code = cidx[u];
  const int c = code & 0xfffffff;
  const cpx<T>* __restrict__ src = (((code >> 30) & 1) ^ flip) ? pb : pa;
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const size_t r = (size_t)(wr.first + wr.stride * k) * Bp;
    pc[r + u] = src[r + c];
  }
}

// Dense operator, K2 after the packed product: w = z p - A p for iterating
// columns (A p of column c at packed column cmap[c] of apc), 0 for frozen
// ones, and the partials of mu = p^T w, as k_s_spmm.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_shiftw_packed(int n, int Bp, StreamGroups grp,
                                                         const double* __restrict__ zc,
                                                         const int* __restrict__ state,
                                                         const int* __restrict__ cmap,
                                                         const cpx<T>* __restrict__ pa,
                                                         const cpx<T>* __restrict__ pb,
                                                         const cpx<T>* __restrict__ apc,
                                                         cpx<T>* __restrict__ w,
                                                         double* __restrict__ part) {
  extern __shared__ double sh[];
  const int c0 = grp.g[blockIdx.y] * 64 * CPL;
  const cpx<T>* __restrict__ p = grp.par[blockIdx.y] ? pb : pa;
  const int cl = c0 + (threadIdx.x & 63) * CPL;
  T zre[CPL], zim[CPL];
  int pk[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    zre[q] = T(zc[2 * (cl + q)]);
    zim[q] = T(zc[2 * (cl + q) + 1]);
    pk[q] = state[cl + q] == 1 ? cmap[cl + q] : -1;
  }
  double acc[CPL][2];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q][0] = acc[q][1] = 0.0;
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const size_t rb = (size_t)(wr.first + wr.stride * k) * Bp;
    const Chunk<T, CPL> p0 = ld<T, CPL>(p + rb + cl);
    Chunk<T, CPL> ww;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (pk[q] >= 0) {
        const cpx<T> a = apc[rb + pk[q]];
        ww.v[q].re = zre[q] * p0.v[q].re - zim[q] * p0.v[q].im - a.re;
        ww.v[q].im = zre[q] * p0.v[q].im + zim[q] * p0.v[q].re - a.im;
      } else {
        ww.v[q] = cpx<T>{T(0), T(0)};
      }
      const double pr = p0.v[q].re, pi = p0.v[q].im, wr_ = ww.v[q].re, wi = ww.v[q].im;
      acc[q][0] += pr * wr_ - pi * wi;
      acc[q][1] += pr * wi + pi * wr_;
    }
    st<T, CPL>(w + rb + cl, ww);
  }
  put_partials<CPL, 2>(acc, part, Bp, c0, sh);
}

// Dense operator, check step 2 after the product: ax holds A x_hi (FP64,
// from a GEMM); the rest as k_s_resid64.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_resid64d(
    int n, int Bp, StreamGroups grp, const double* __restrict__ zc,
    const int* __restrict__ state, const double* __restrict__ B, int ldb, int kcols,
    const double* __restrict__ scale, const cpx<double>* __restrict__ xh,
    const cpx<double>* __restrict__ ax, cpx<T>* __restrict__ r, cpx<T>* __restrict__ pa,
    cpx<T>* __restrict__ pb, double* __restrict__ part) {
  extern __shared__ double sh[];
  const int c0 = grp.g[blockIdx.y] * 64 * CPL;
  cpx<T>* __restrict__ p = grp.par[blockIdx.y] ? pb : pa;
  const int cl = c0 + (threadIdx.x & 63) * CPL;
  double zre[CPL], zim[CPL], scl[CPL];
  bool on[CPL], rst[CPL];
  int ci[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    zre[q] = zc[2 * (cl + q)];
    zim[q] = zc[2 * (cl + q) + 1];
    on[q] = waiting(state[cl + q]);
    rst[q] = state[cl + q] == 3;
    ci[q] = (cl + q) % kcols;
    scl[q] = scale[cl + q];
  }
  double acc[CPL][3];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const int row = wr.first + k * wr.stride;
    const size_t ro = (size_t)row * Bp + cl;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const cpx<double> xr = xh[ro + q], a = ax[ro + q];
      const double b = scl[q] != 0.0 ? B[(size_t)row * ldb + ci[q]] * scl[q] : 0.0;
      const double sr = b - (zre[q] * xr.re - zim[q] * xr.im - a.re);
      const double si = -(zre[q] * xr.im + zim[q] * xr.re - a.im);
      r[ro + q] = cpx<T>{T(sr), T(si)};
      if (rst[q]) p[ro + q] = cpx<T>{T(sr), T(si)};
      acc[q][0] += sr * sr - si * si;
      acc[q][1] += 2.0 * sr * si;
      acc[q][2] += sr * sr + si * si;
    }
  }
  put_partials<CPL, 3>(acc, part, Bp, c0, sh);
}

// Check, step 3: accept (true residual <= tol), give up (update, iteration
// or breakdown budget spent), or continue: a reliable update keeps p and
// takes beta = s^T s / rho_prev; a restart takes beta = 0, so the next p is
// r = s (after a breakdown, or when ||s|| is not at most half the previous
// check's).  The next check comes when the recursive residual has dropped by
// delta from ||s|| (or reaches tol), or at a stall.
__global__ __launch_bounds__(kFinThreads) void k_s_fin_verify(int Bp, int nb,
                                                              const double* __restrict__ part,
                                                              StreamCols cols, double tol,
                                                              double delta, int maxit,
                                                              int max_updates) {
  const int c = fin_col();
  const int st0 = c < Bp ? cols.state[c] : 2;
  const bool want = waiting(st0);
  double s[3];
  col_sums<3>(part, nb, Bp, want, s);
  if (threadIdx.x >= kFinCols || !want) return;
  cols.res[c] = sqrt(s[2]);
  if (s[2] <= tol * tol || !isfinite(s[2]) || cols.nref[c] >= max_updates ||
      cols.it[c] >= maxit || cols.nbd[c] > 3) {
    cols.state[c] = 2;
    return;
  }
  cols.nref[c] += 1;
  double br = 0.0, bi = 0.0;  // beta = 0 restarts: the next p is r = s
  if (st0 == 0 && s[2] <= 0.25 * cols.sprev[c]) {
    const zd bt = zdiv(zd{s[0], s[1]}, zd{cols.rho[2 * c], cols.rho[2 * c + 1]});
    if (isfinite(bt.re) && isfinite(bt.im)) {
      br = bt.re;
      bi = bt.im;
    }
  }
  const int it = cols.it[c];
  cols.span[c] = it - cols.lastit[c];
  if (cols.lastit[c] == cols.rstart[c]) cols.span0[c] = max(cols.span0[c], it - cols.lastit[c]);
  cols.lastit[c] = it;
  if (br == 0.0 && bi == 0.0) cols.rstart[c] = it;
  cols.sprev[c] = s[2];
  cols.rho[2 * c] = s[0];
  cols.rho[2 * c + 1] = s[1];
  cols.beta[2 * c] = br;
  cols.beta[2 * c + 1] = bi;
  cols.ctol2[c] = fmax(tol * tol, delta * delta * s[2]);
  cols.state[c] = 1;
}

// Start, step 1: partials of ||b_c||^2 (column c takes RHS column c % kcols).
template <int CPL>
__global__ __launch_bounds__(kST) void k_s_bnorm(int n, int Bp, const double* __restrict__ B,
                                                 int ldb, int kcols, int ncols,
                                                 double* __restrict__ part) {
  extern __shared__ double sh[];
  const int c0 = blockIdx.y * 64 * CPL;
  const int cl = c0 + (threadIdx.x & 63) * CPL;
  double acc[CPL][1];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q][0] = 0.0;
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const int row = wr.first + k * wr.stride;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (cl + q >= ncols) continue;
      const double b = B[(size_t)row * ldb + (cl + q) % kcols];
      acc[q][0] += b * b;
    }
  }
  put_partials<CPL, 1>(acc, part, Bp, c0, sh);
}

// Start, step 2: per-column set-up; zero and padding columns are solved at once.
__global__ __launch_bounds__(kFinThreads) void k_s_fin_bnorm(int Bp, int nb,
                                                             const double* __restrict__ part,
                                                             int ncols, double* __restrict__ scale,
                                                             StreamCols cols, double tol,
                                                             double delta) {
  const int c = fin_col();
  double s[1];
  col_sums<1>(part, nb, Bp, c < ncols, s);
  if (threadIdx.x >= kFinCols || c >= Bp) return;
  cols.it[c] = 0;
  cols.nref[c] = 0;
  cols.nbd[c] = 0;
  cols.alpha[2 * c] = cols.alpha[2 * c + 1] = 0.0;
  cols.beta[2 * c] = cols.beta[2 * c + 1] = 0.0;
  cols.res[c] = 0.0;
  cols.rho[2 * c] = cols.rho[2 * c + 1] = 0.0;
  cols.lastit[c] = 0;
  cols.span[c] = 0;
  cols.span0[c] = 0;
  cols.rstart[c] = 0;
  cols.sprev[c] = 1.0;  // the start residual b / ||b||
  const double nrm = c < ncols ? sqrt(s[0]) : 0.0;
  cols.bn[c] = nrm;
  if (!(nrm > 0.0) || !isfinite(nrm)) {
    scale[c] = 0.0;
    cols.state[c] = 2;
    return;
  }
  scale[c] = 1.0 / nrm;
  cols.ctol2[c] = fmax(tol * tol, delta * delta);
  cols.state[c] = 1;
}

// Start, step 3: r = p = b / ||b|| (engine row order), x = x_hi = 0; partials of r^T r.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_start(int n, int Bp, const double* __restrict__ B,
                                                 int ldb, int kcols,
                                                 const double* __restrict__ scale,
                                                 const int* __restrict__ perm,
                                                 cpx<T>* __restrict__ x, cpx<T>* __restrict__ r,
                                                 cpx<T>* __restrict__ p,
                                                 cpx<double>* __restrict__ xh,
                                                 double* __restrict__ part) {
  extern __shared__ double sh[];
  const int c0 = blockIdx.y * 64 * CPL;
  const int cl = c0 + (threadIdx.x & 63) * CPL;
  double scl[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) scl[q] = scale[cl + q];
  double acc[CPL][1];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q][0] = 0.0;
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const int row = wr.first + k * wr.stride;
    const size_t ro = (size_t)row * Bp + cl;
    const size_t orow = (size_t)perm[row];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const double b = scl[q] != 0.0 ? B[orow * ldb + (cl + q) % kcols] * scl[q] : 0.0;
      const cpx<T> v{T(b), T(0)};
      r[ro + q] = v;
      p[ro + q] = v;
      x[ro + q] = cpx<T>{T(0), T(0)};
      xh[ro + q] = cpx<double>{0.0, 0.0};
      acc[q][0] += (double)v.re * (double)v.re;
    }
  }
  put_partials<CPL, 1>(acc, part, Bp, c0, sh);
}

__global__ __launch_bounds__(kFinThreads) void k_s_fin_start(int Bp, int nb,
                                                             const double* __restrict__ part,
                                                             StreamCols cols) {
  const int c = fin_col();
  const bool want = c < Bp && cols.state[c] == 1;
  double s[1];
  col_sums<1>(part, nb, Bp, want, s);
  if (threadIdx.x >= kFinCols || !want) return;
  cols.rho[2 * c] = s[0];
  cols.rho[2 * c + 1] = 0.0;
}

// Output: D[perm[row]][c] = ||b_c|| x_hi[row][c] for c < ncols.
template <typename T, int CPL>
__global__ __launch_bounds__(kST) void k_s_out(int n, int Bp, int ncols,
                                               const double* __restrict__ bn,
                                               const int* __restrict__ perm,
                                               const cpx<double>* __restrict__ xh,
                                               cpx<T>* __restrict__ D, int ldd) {
  const int cl = blockIdx.y * 64 * CPL + (threadIdx.x & 63) * CPL;
  const WaveRows wr = wave_rows(n);
  for (int k = 0; k < wr.count; ++k) {
    const int row = wr.first + k * wr.stride;
    const size_t ro = (size_t)row * Bp + cl;
    const size_t orow = (size_t)perm[row];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (cl + q >= ncols) continue;
      const cpx<double> h = xh[ro + q];
      const double s = bn[cl + q];
      D[orow * ldd + cl + q] = cpx<T>{T(h.re * s), T(h.im * s)};
    }
  }
}

// Per-column report: iterations, final relative true residual; stats[0] +=
// FP64 residual checks that continued the iteration, stats[1] += columns
// given up after repeated breakdowns.
__global__ void k_s_report(int ncols, StreamCols cols, int* __restrict__ iters,
                           double* __restrict__ resid, int* __restrict__ stats) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  if (iters) iters[c] = cols.it[c];
  if (resid) resid[c] = cols.res[c];
  if (stats) {
    if (cols.nref[c]) atomicAdd(&stats[0], cols.nref[c]);
    if (cols.nbd[c] > 3) atomicAdd(&stats[1], 1);
  }
}

// ---------------------------------------------------------------------------
// host side
int stream_cpl(int k, int ncols, bool fp32) {
  // A lane moves 16 bytes per load: two FP32 complex columns, or one FP64
  // complex column.  The per-CU rate from L2 is set by load instructions, so
  // 8-byte lanes would halve the gather bandwidth.  Narrow FP32 solves (under
  // 128 columns) use one column per lane.
  (void)k;
  return (fp32 && ncols >= 128) ? 2 : 1;
}

int stream_padded_columns(int k, int ncols, bool fp32) {
  const int gw = 64 * stream_cpl(k, ncols, fp32);
  return (ncols + gw - 1) / gw * gw;
}

int stream_blocks(int n, int num_cu) {
  // eight workgroups per CU for large n; four up to 2^17 rows, where the
  // finalisers' partial sums (one per workgroup and column) cost more than
  // the extra occupancy gives (measured 3-5% on n of 10^4 to 6 10^4)
  int nb = num_cu * (n <= (1 << 17) ? 4 : 8);
  const int need = (n + kSW - 1) / kSW;
  if (nb > need) nb = (need + 7) / 8 * 8;
  return nb < 8 ? 8 : nb;
}

size_t stream_partial_doubles(int n, int Bp, int num_cu) {
  return (size_t)stream_blocks(n, num_cu) * Bp * 3;
}

template <typename T, int CPL>
static hipError_t run_stream_t(hipStream_t stm, const StreamMatrix& A, const StreamWork& W,
                               const StreamLaunch& L) {
  const int n = A.n, Bp = W.Bp;
  const int gw = 64 * CPL, ng = Bp / gw;
  const int nb = stream_blocks(n, W.num_cu);
  const dim3 blk(kST), fgrid((Bp + kFinCols - 1) / kFinCols), fblk(kFinThreads);
  auto shm = [](int nq) { return (size_t)kSW * 64 * CPL * nq * sizeof(double); };
  // check spacing: FP32 storage drifts by about kappa * 6e-8 of the residual
  // per check interval, so checks come every decade; FP64 rarely needs one
  const double delta = sizeof(T) == 4 ? 0.1 : 1e-4;
  const T* val = sizeof(T) == 4 ? (const T*)(const void*)A.val32 : (const T*)(const void*)A.val64;
  cpx<T>* X = (cpx<T>*)W.x;
  cpx<T>* R = (cpx<T>*)W.r;
  cpx<T>* Pa = (cpx<T>*)W.p0;
  cpx<T>* Pb = (cpx<T>*)W.p1;
  std::vector<int> parity(ng, 0);  // current p of group g: parity[g] ? Pb : Pa
  cpx<T>* Wv = (cpx<T>*)W.w;
  cpx<double>* XH = (cpx<double>*)W.xh;
  hipError_t e = hipSuccess;
#define SLAUNCH(...)                      \
  do {                                    \
    hipLaunchKernelGGL(__VA_ARGS__);      \
    e = hipGetLastError();                \
    if (e != hipSuccess) return e;        \
  } while (0)
  // Dense operator: the check products over runs of consecutive waiting
  // groups, as real row-major blocks (a complex column is two real ones).
  auto dense_check_product = [&](const StreamGroups& grp) -> hipError_t {
    for (int a = 0; a < grp.count;) {
      int b = a + 1;
      while (b < grp.count && grp.g[b] == grp.g[b - 1] + 1) ++b;
      const size_t c0 = (size_t)grp.g[a] * gw;
      const hipError_t e2 =
          dense_apply_f64(*A.dense, stm, 2 * gw * (b - a), (const double*)(XH + c0), 2 * Bp,
                          (double*)((cpx<double>*)W.axh + c0), 2 * Bp, 1.0, 0.0);
      if (e2 != hipSuccess) return e2;
      a = b;
    }
    return hipSuccess;
  };
  const dim3 gall(nb, ng);
  SLAUNCH(k_s_bnorm<CPL>, gall, blk, shm(1), stm, n, Bp, L.B, L.ldb, L.k, L.ncols, W.part);
  SLAUNCH(k_s_fin_bnorm, fgrid, fblk, 0, stm, Bp, nb, W.part, L.ncols, W.scale, W.cols, L.tol,
          delta);
  SLAUNCH((k_s_start<T, CPL>), gall, blk, shm(1), stm, n, Bp, L.B, L.ldb, L.k, W.scale, A.perm, X,
          R, Pa, XH, W.part);
  SLAUNCH(k_s_fin_start, fgrid, fblk, 0, stm, Bp, nb, W.part, W.cols);
  std::vector<int> cnt(2 * ng);
  std::vector<int> hstate(A.dense ? Bp : 0), hidx, hmap;
  auto census = [&]() -> hipError_t {
    hipLaunchKernelGGL(k_s_count, dim3(ng), dim3(64), 0, stm, Bp, gw, W.cols, W.cnt);
    hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return e2;
    e2 = hipMemcpyAsync(cnt.data(), W.cnt, 2 * ng * sizeof(int), hipMemcpyDeviceToHost, stm);
    if (e2 != hipSuccess) return e2;
    if (A.dense) {
      e2 = hipMemcpyAsync(hstate.data(), W.cols.state, Bp * sizeof(int), hipMemcpyDeviceToHost,
                          stm);
      if (e2 != hipSuccess) return e2;
    }
    return hipStreamSynchronize(stm);
  };
  // Dense operator: the packed list of the iterating columns, each with its
  // group's p parity at the start of the chunk, and the column -> packed map.
  int nl = 0;
  auto pack_list = [&]() -> hipError_t {
    hidx.clear();
    hmap.assign(Bp, -1);
    for (int c = 0; c < Bp; ++c)
      if (hstate[c] == 1) {
        hmap[c] = (int)hidx.size();
        hidx.push_back(c | (parity[c / gw] << 30));
      }
    nl = (int)hidx.size();
    hipError_t e2 = hipSuccess;
    if (nl > 0)
      e2 = hipMemcpyAsync(W.cidx, hidx.data(), nl * sizeof(int), hipMemcpyHostToDevice, stm);
    if (e2 == hipSuccess)
      e2 = hipMemcpyAsync(W.cmap, hmap.data(), Bp * sizeof(int), hipMemcpyHostToDevice, stm);
    return e2;
  };
  e = census();
  if (e != hipSuccess) return e;
  const int chunk = L.chunk > 0 ? L.chunk : 8;
  // Every column stays live or waiting from the start until it is done, and
  // each pass gives each live column at least one iteration and checks each
  // waiting one, so no column outlasts maxit + 2 * max_updates + 2 passes.
  const long guard = (long)L.maxit + 2L * L.max_updates + 8;
  for (long pass = 0; pass < guard; ++pass) {
    // group lists with each group's current p buffer
    auto list = [&](int off) {
      StreamGroups gl;
      gl.count = 0;
      for (int g = 0; g < ng; ++g)
        if (cnt[off + g] > 0) {
          gl.par[gl.count] = parity[g];
          gl.g[gl.count++] = g;
        }
      return gl;
    };
    StreamGroups live = list(0), wait = list(ng);
    if (live.count == 0 && wait.count == 0) break;
    if (live.count > 0) {
      const dim3 gl(nb, live.count);
      if (A.dense) {
        e = pack_list();
        if (e != hipSuccess) return e;
      }
      for (int k = 0; k < chunk; ++k) {
        SLAUNCH((k_s_pupd<T, CPL>), gl, blk, 0, stm, n, Bp, live, W.cols.beta, W.cols.state, R,
                Pa, Pb);
        for (int i = 0; i < live.count; ++i) {  // the new p is now current
          live.par[i] ^= 1;
          parity[live.g[i]] ^= 1;
        }
        if (A.dense) {
          // the packed columns' p (parity flipped once per iteration so far),
          // their product, then the shift
          cpx<T>* Pc = (cpx<T>*)W.pc;
          cpx<T>* APc = (cpx<T>*)W.apc;
          if (nl > 0)
            SLAUNCH((k_s_pack<T>), dim3(nb, (nl + 63) / 64), blk, 0, stm, n, Bp, nl, W.cidx,
                    (k + 1) & 1, Pa, Pb, Pc);
          if constexpr (sizeof(T) == 4)
            e = dense_apply_f32(*A.dense, stm, 2 * nl, (const float*)Pc, 2 * Bp, (float*)APc,
                                2 * Bp);
          else
            e = dense_apply_f64(*A.dense, stm, 2 * nl, (const double*)Pc, 2 * Bp,
                                (double*)APc, 2 * Bp, 1.0, 0.0);
          if (e != hipSuccess) return e;
          SLAUNCH((k_s_shiftw_packed<T, CPL>), gl, blk, shm(2), stm, n, Bp, live, W.zc,
                  W.cols.state, W.cmap, Pa, Pb, APc, Wv, W.part);
        } else {
          SLAUNCH((k_s_spmm<T, CPL>), gl, blk, shm(2), stm, n, A.rowptr, A.col, val, Bp, live,
                  W.zc, W.cols.state, Pa, Pb, Wv, W.part);
        }
        SLAUNCH(k_s_fin_mu, fgrid, fblk, 0, stm, Bp, nb, W.part, W.cols);
        SLAUNCH((k_s_update<T, CPL>), gl, blk, shm(3), stm, n, Bp, live, W.cols.alpha, X, R, Pa,
                Pb, Wv, W.part);
        SLAUNCH(k_s_fin_rho, fgrid, fblk, 0, stm, Bp, nb, W.part, W.cols, L.maxit);
      }
      e = census();
      if (e != hipSuccess) return e;
      wait = list(ng);
    }
    if (wait.count > 0) {
      const dim3 gw2(nb, wait.count);
      SLAUNCH((k_s_xhi<T, CPL>), gw2, blk, 0, stm, n, Bp, wait, W.cols.state, X, XH);
      if (A.dense) {
        e = dense_check_product(wait);
        if (e != hipSuccess) return e;
        SLAUNCH((k_s_resid64d<T, CPL>), gw2, blk, shm(3), stm, n, Bp, wait, W.zc, W.cols.state,
                L.B, L.ldb, L.k, W.scale, XH, (const cpx<double>*)W.axh, R, Pa, Pb, W.part);
      } else {
        SLAUNCH((k_s_resid64<T, CPL>), gw2, blk, shm(3), stm, n, A.rowptr, A.col, A.val64, Bp,
                wait, W.zc, W.cols.state, L.B, L.ldb, L.k, W.scale, A.perm, XH, R, Pa, Pb, W.part);
      }
      SLAUNCH(k_s_fin_verify, fgrid, fblk, 0, stm, Bp, nb, W.part, W.cols, L.tol, delta,
              L.maxit, L.max_updates);
      e = census();
      if (e != hipSuccess) return e;
    }
  }
  SLAUNCH((k_s_out<T, CPL>), gall, blk, 0, stm, n, Bp, L.ncols, W.cols.bn, A.perm, XH,
          (cpx<T>*)L.D, L.ldd);
  SLAUNCH(k_s_report, dim3((L.ncols + 255) / 256), dim3(256), 0, stm, L.ncols, W.cols, L.iters,
          L.resid, L.stats);
#undef SLAUNCH
  return hipSuccess;
}

hipError_t run_stream_cocg(hipStream_t st, const StreamMatrix& A, const StreamWork& W,
                           const StreamLaunch& L, bool fp32) {
  const int cpl = stream_cpl(L.k, L.ncols, fp32);
  if (W.Bp % (64 * cpl) != 0 || W.Bp < L.ncols || W.Bp / (64 * cpl) > kStreamMaxGroups)
    return hipErrorInvalidValue;
  if (fp32) {
    switch (cpl) {
      case 1: return run_stream_t<float, 1>(st, A, W, L);
      case 2: return run_stream_t<float, 2>(st, A, W, L);
    }
  } else if (cpl == 1) {
    return run_stream_t<double, 1>(st, A, W, L);
  }
  return hipErrorInvalidValue;
}

}  // namespace rafeast
