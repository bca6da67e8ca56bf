// Multi-shift COCG engine (FP64) for the shifted systems of one filter
// application.  In the residual-correction form (and in the literal form) all
// N_c shifted systems of column i share the right-hand side b_i, so one Krylov
// space serves them: K(z_j I - A, b) = K(A, b) for every z_j.  The engine runs
// CG on a real symmetric positive definite seed M = A - s I (s below the
// spectrum) and obtains every shifted system's iterate from the seed's scalars.
//
// Seed CG (x0 = 0):  r_0 = b, p_k = r_k + beta_{k-1} p_{k-1},
//   alpha_k = r_k^T r_k / p_k^T M p_k,  r_{k+1} = r_k - alpha_k M p_k,
//   beta_k = r_{k+1}^T r_{k+1} / r_k^T r_k.
// With R_k the residual polynomial (r_k = R_k(M) b, R_k(0) = 1) and the
// system (M + sigma I) x = b, the shifted residual is collinear with the
// seed's: r^sigma_k = r_k / pi_k with pi_k = R_k(-sigma).  The three-term
// recurrence of R_k gives
//   pi_{k+1} = (1 + c_k + alpha_k sigma) pi_k - c_k pi_{k-1},
//   c_k = beta_{k-1} alpha_k / alpha_{k-1}  (pi_{-1} = pi_0 = 1, beta_{-1} = 0),
// and the shifted iterate follows
//   p^s_k = r_k / pi_k + beta^s_{k-1} p^s_{k-1},  x^s_{k+1} = x^s_k + alpha^s_k p^s_k,
//   alpha^s_k = alpha_k pi_k / pi_{k+1},  beta^s_k = beta_k (pi_k / pi_{k+1})^2.
// (z_j I - A) d = b is (M + sigma_j I) x = b with sigma_j = s - z_j and
// d = -x.  The seed's R_k has real roots (Ritz values of M) and sigma_j is
// off the real axis, so pi_k never vanishes: no breakdown.  A shifted
// system stops (its x and p are frozen) when its residual |r_k| / |pi_k|
// drops below tol |b|; the seed runs until every shift of its column has
// stopped.  The seed's r, p and the pi's are rescaled together when |r_k|
// falls below 1e-100 |b| (the shifted quantities depend on their ratios).
//
// Combining mode (the filter step of FEAST): only the weighted sum
// sum_j Re(g_j d_j) of the solutions is needed, so the engine accumulates it
// into one real block as the iterates advance and never stores them: per
// iteration a shift then moves its direction only (32 B per row and column
// instead of 64).
//
// Layout: engine rows in the streaming engine's reverse Cuthill-McKee order,
// blocks n x kp row-major (kp = 64 CPL, column c of lane c / CPL); the seed
// r, p, w are real, the shifted p^s and x^s complex, one n x kp block per
// shift.  Row kernels: 256 threads, a wave per row, the rows cut into eight
// contiguous stripes (one per XCD) swept by that XCD's waves side by side,
// so the SpMV's neighbour rows were read recently into the same L2.
// Reductions: per-workgroup partials summed in a fixed order per column.
#include "device.h"
#include "kernels.h"

namespace rafeast {

namespace {

constexpr int kMT = 256;          // threads of a row kernel
constexpr int kMW = kMT / 64;     // its waves

struct Rows {
  int first, stride, count;
};

// Rows of this wave: workgroup b runs on XCD b mod 8 and takes a share of
// that XCD's contiguous eighth of the rows.
__device__ __forceinline__ Rows my_rows(int n) {
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
  const int stride = per_x * kMW;
  const int first = lo + i * kMW + wave_id();
  return {first, stride, first < hi ? (hi - first + stride - 1) / stride : 0};
}

// Sum the four waves' per-lane values and store the workgroup's partial of
// each column at part[blockIdx.x * kp + c].
template <int CPL>
__device__ __forceinline__ void put_partial(const double (&acc)[CPL], double* __restrict__ part,
                                            int kp) {
  __shared__ double sh[kMW * 64 * CPL];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < CPL; ++q) sh[wv * 64 * CPL + lane * CPL + q] = acc[q];
  __syncthreads();
  for (int e = threadIdx.x; e < kp; e += kMT) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kMW; ++w) s += sh[w * 64 * CPL + e];
    part[(size_t)blockIdx.x * kp + e] = s;
  }
}

constexpr int kFT = 256;  // threads of a finaliser workgroup (one per column)

// Fixed-order sum of column c's partials over nb workgroups by the kFT
// threads of the calling workgroup (strided partial sums, then a tree); every
// thread must call it and receives the total.
__device__ __forceinline__ double col_total(const double* __restrict__ part, int nb, int kp,
                                            int c) {
  __shared__ double sh[kFT];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < nb; b += kFT) s += part[(size_t)b * kp + c];
  sh[t] = s;
  __syncthreads();
  for (int o = kFT / 2; o > 0; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  const double tot = sh[0];
  __syncthreads();
  return tot;
}

__device__ __forceinline__ zd zinv(zd a) { return zdiv(zd{1.0, 0.0}, a); }

}  // namespace

// r = b (rows gathered through perm), p = 0, every shift's p^s = x^s = 0;
// partials of b^T b.
template <int CPL>
__global__ __launch_bounds__(kMT) void k_ms_init(int n, int k, int kp, int nz,
                                                 const int* __restrict__ perm,
                                                 const double* __restrict__ B, int ldb,
                                                 double* __restrict__ r, double* __restrict__ p,
                                                 cpx<double>* __restrict__ X,
                                                 cpx<double>* __restrict__ Ps,
                                                 double* __restrict__ y,
                                                 double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  const Rows rw = my_rows(n);
  const size_t blk = (size_t)n * kp;
  for (int t = 0; t < rw.count; ++t) {
    const int row = rw.first + rw.stride * t;
    const int src = perm[row];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane * CPL + q;
      const double v = c < k ? B[(size_t)src * ldb + c] : 0.0;
      const size_t o = (size_t)row * kp + c;
      r[o] = v;
      p[o] = 0.0;
      if (y) y[o] = 0.0;
      for (int j = 0; j < nz; ++j) {
        if (!y) X[j * blk + o] = cpx<double>{0.0, 0.0};
        Ps[j * blk + o] = cpx<double>{0.0, 0.0};
      }
      acc[q] += v * v;
    }
  }
  put_partial<CPL>(acc, part, kp);
}

// Column state after the start: |b|, r^T r, the seed scalars and every
// shift's pi; a system with b = 0 is done at once (x = 0).
__global__ __launch_bounds__(kFT) void k_ms_fin0(int k, int kp, int nz, int nb,
                                                 const double* __restrict__ part, MsCols cols,
                                                 int* __restrict__ count) {
  const int c = blockIdx.x;
  const double tot = col_total(part, nb, kp, c);
  if (threadIdx.x != 0) return;
  const double rr = c < k ? tot : 0.0;
  cols.rr[c] = rr;
  cols.bn[c] = sqrt(rr);
  cols.alpha[c] = 0.0;
  cols.alpha_prev[c] = 1.0;
  cols.beta_prev[c] = 0.0;
  cols.scale[c] = 1.0;
  int nl = 0;
  for (int j = 0; j < nz; ++j) {
    const int e = j * kp + c;
    cols.pi[e] = cpx<double>{1.0, 0.0};
    cols.pi_prev[e] = cpx<double>{1.0, 0.0};
    cols.ipi[e] = cpx<double>{1.0, 0.0};
    cols.bs[e] = cpx<double>{0.0, 0.0};
    cols.as[e] = cpx<double>{0.0, 0.0};
    const int lv = rr > 0.0 ? 1 : 0;
    cols.live[e] = lv;
    cols.its[e] = 0;
    cols.est[e] = 0.0;
    nl += lv;
  }
  cols.colive[c] = nl > 0 ? 1 : 0;
  if (nl) atomicAdd(count, nl);
}

// Seed search direction p = s (r + beta p) for the live columns; with a
// rescale s != 1 the residual is scaled too.
template <int CPL>
__global__ __launch_bounds__(kMT) void k_ms_pupd(int n, int kp, MsCols cols,
                                                 double* __restrict__ r, double* __restrict__ p) {
  const int lane = threadIdx.x & 63;
  double beta[CPL], sc[CPL];
  bool on[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = lane * CPL + q;
    on[q] = cols.colive[c] != 0;
    beta[q] = cols.beta_prev[c];
    sc[q] = cols.scale[c];
  }
  const Rows rw = my_rows(n);
  for (int t = 0; t < rw.count; ++t) {
    const size_t o = (size_t)(rw.first + rw.stride * t) * kp + lane * CPL;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const double rv = r[o + q];
      p[o + q] = sc[q] * (rv + beta[q] * p[o + q]);
      if (sc[q] != 1.0) r[o + q] = sc[q] * rv;
    }
  }
}

// w = M p = A p - s p on the live columns (a wave per row, the row's entries
// broadcast from the lanes that loaded them, neighbour rows of p gathered
// eight at a time); partials of p^T w.
template <int CPL>
__global__ __launch_bounds__(kMT) void k_ms_spmv(int n, int kp, const int* __restrict__ rowptr,
                                                 const int* __restrict__ col,
                                                 const double* __restrict__ val, double shift,
                                                 const int* __restrict__ colive,
                                                 const double* __restrict__ p,
                                                 double* __restrict__ w,
                                                 double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int cl = lane * CPL;
  bool on[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) on[q] = colive[cl + q] != 0;
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  const Rows rw = my_rows(n);
  for (int t = 0; t < rw.count; ++t) {
    const int row = rw.first + rw.stride * t;
    const int s = rowptr[row], e = rowptr[row + 1];
    const size_t ro = (size_t)row * kp + cl;
    double a[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) a[q] = 0.0;
    for (int base = s; base < e; base += 64) {
      const int m = min(64, e - base);
      // lane l holds entry base + l (own row with value 0 past the end)
      int mc = row;
      double mv = 0.0;
      if (lane < m) {
        mc = col[base + lane];
        mv = val[base + lane];
      }
      for (int t0 = 0; t0 < m; t0 += 8) {
        int jj[8];
        double av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          jj[u] = __builtin_amdgcn_readlane(mc, t0 + u);
          av[u] = readlane_f64(mv, t0 + u);
        }
        double pv[8][CPL];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < CPL; ++q) pv[u][q] = p[(size_t)jj[u] * kp + cl + q];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < CPL; ++q) a[q] = fma(av[u], pv[u][q], a[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const double pr = p[ro + q];
      const double wv = a[q] - shift * pr;
      w[ro + q] = wv;
      acc[q] += pr * wv;
    }
  }
  put_partial<CPL>(acc, part, kp);
}

// alpha_k of every live column, then for each live shift pi_{k+1},
// alpha^s_k = alpha_k pi_k / pi_{k+1} and 1 / pi_k for the update kernel.
__global__ __launch_bounds__(kFT) void k_ms_fin_alpha(int kp, int k, int nz, int nb,
                                                      const double* __restrict__ part,
                                                      const cpx<double>* __restrict__ sig,
                                                      const double* __restrict__ g,
                                                      MsCols cols) {
  const int c = blockIdx.x;
  if (!cols.colive[c]) {  // uniform over the workgroup
    if (threadIdx.x == 0) cols.scale[c] = 1.0;
    return;
  }
  const double pw = col_total(part, nb, kp, c);
  if (threadIdx.x != 0) return;
  cols.scale[c] = 1.0;  // a rescale has been applied by the direction update
  const double alpha = pw != 0.0 ? cols.rr[c] / pw : 0.0;
  cols.alpha[c] = alpha;
  const double cc = cols.beta_prev[c] * alpha / cols.alpha_prev[c];
  for (int j = 0; j < nz; ++j) {
    const int e = j * kp + c;
    if (!cols.live[e]) continue;
    const zd pk{cols.pi[e].re, cols.pi[e].im}, pm{cols.pi_prev[e].re, cols.pi_prev[e].im};
    const zd f{1.0 + cc + alpha * sig[j].re, alpha * sig[j].im};
    const zd fp = zmul(f, pk);
    const zd pn{fp.re - cc * pm.re, fp.im - cc * pm.im};
    cols.pi_next[e] = cpx<double>{pn.re, pn.im};
    const zd q = zdiv(pk, pn);
    cols.as[e] = cpx<double>{alpha * q.re, alpha * q.im};
    const zd ip = zinv(pk);
    cols.ipi[e] = cpx<double>{ip.re, ip.im};
    if (g) {  // combining mode: the weight of this step's update of x^s
      const zd gw = zmul(zd{g[2 * (j * k + c)], g[2 * (j * k + c) + 1]},
                         zd{alpha * q.re, alpha * q.im});
      cols.gas[e] = cpx<double>{gw.re, gw.im};
    }
  }
}

// r <- r - alpha w (partials of the new r^T r); for every live shift, with
// the old r: p^s = r / pi_k + beta^s p^s, x^s += alpha^s p^s.
template <int CPL>
__global__ __launch_bounds__(kMT) void k_ms_update(int n, int kp, int nz, MsCols cols,
                                                   double* __restrict__ r,
                                                   const double* __restrict__ w,
                                                   cpx<double>* __restrict__ X,
                                                   cpx<double>* __restrict__ Ps,
                                                   double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int cl = lane * CPL;
  double alpha[CPL];
  bool on[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    on[q] = cols.colive[cl + q] != 0;
    alpha[q] = cols.alpha[cl + q];
  }
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  const Rows rw = my_rows(n);
  const size_t blk = (size_t)n * kp;
  for (int t = 0; t < rw.count; ++t) {
    const size_t o = (size_t)(rw.first + rw.stride * t) * kp + cl;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const double ro = r[o + q];
      const double rn = ro - alpha[q] * w[o + q];
      r[o + q] = rn;
      acc[q] += rn * rn;
      for (int j = 0; j < nz; ++j) {
        const int e = j * kp + cl + q;
        if (!cols.live[e]) continue;
        const cpx<double> ip = cols.ipi[e], b = cols.bs[e], a = cols.as[e];
        const cpx<double> po = Ps[j * blk + o + q];
        const double pr = ro * ip.re + (b.re * po.re - b.im * po.im);
        const double pi = ro * ip.im + (b.re * po.im + b.im * po.re);
        Ps[j * blk + o + q] = cpx<double>{pr, pi};
        cpx<double> x = X[j * blk + o + q];
        x.re += a.re * pr - a.im * pi;
        x.im += a.re * pi + a.im * pr;
        X[j * blk + o + q] = x;
      }
    }
  }
  put_partial<CPL>(acc, part, kp);
}

// The same update with the per-shift scalars of this lane's columns held in
// registers (NZ >= nz shifts, NZ * CPL <= 8) and every live shift's loads of
// a row issued before any of its arithmetic, so that a wave keeps 2 NZ CPL
// loads in flight instead of two.
template <int CPL, int NZ>
__global__ __launch_bounds__(kMT) void k_ms_update_r(int n, int kp, int nz, MsCols cols,
                                                     double* __restrict__ r,
                                                     const double* __restrict__ w,
                                                     cpx<double>* __restrict__ X,
                                                     cpx<double>* __restrict__ Ps,
                                                     double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int cl = lane * CPL;
  double alpha[CPL];
  bool on[CPL], lv[CPL][NZ];
  zd ip[CPL][NZ], bs[CPL][NZ], as[CPL][NZ];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    on[q] = cols.colive[cl + q] != 0;
    alpha[q] = cols.alpha[cl + q];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      const int e = j * kp + cl + q;
      lv[q][j] = j < nz && cols.live[e] != 0;
      ip[q][j] = lv[q][j] ? zd{cols.ipi[e].re, cols.ipi[e].im} : zd{0.0, 0.0};
      bs[q][j] = lv[q][j] ? zd{cols.bs[e].re, cols.bs[e].im} : zd{0.0, 0.0};
      as[q][j] = lv[q][j] ? zd{cols.as[e].re, cols.as[e].im} : zd{0.0, 0.0};
    }
  }
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  const Rows rw = my_rows(n);
  const size_t blk = (size_t)n * kp;
  for (int t = 0; t < rw.count; ++t) {
    const size_t o = (size_t)(rw.first + rw.stride * t) * kp + cl;
    double ro[CPL];
    cpx<double> po[CPL][NZ], xo[CPL][NZ];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      ro[q] = on[q] ? r[o + q] : 0.0;
#pragma unroll
      for (int j = 0; j < NZ; ++j)
        if (lv[q][j]) {
          po[q][j] = Ps[j * blk + o + q];
          xo[q][j] = X[j * blk + o + q];
        }
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const double rn = ro[q] - alpha[q] * w[o + q];
      r[o + q] = rn;
      acc[q] += rn * rn;
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        if (!lv[q][j]) continue;
        const zd b = bs[q][j], a = as[q][j];
        const double pr = ro[q] * ip[q][j].re + (b.re * po[q][j].re - b.im * po[q][j].im);
        const double pi = ro[q] * ip[q][j].im + (b.re * po[q][j].im + b.im * po[q][j].re);
        Ps[j * blk + o + q] = cpx<double>{pr, pi};
        X[j * blk + o + q] =
            cpx<double>{xo[q][j].re + (a.re * pr - a.im * pi), xo[q][j].im + (a.re * pi + a.im * pr)};
      }
    }
  }
  put_partial<CPL>(acc, part, kp);
}

// Combining mode of the update: the shifted directions as in k_ms_update_r,
// and instead of every shift's iterate the one real block
// y += sum_j Re(g_{j,c} alpha^s_k p^s_k) (the weighted sum of the iterates).
template <int CPL, int NZ>
__global__ __launch_bounds__(kMT) void k_ms_update_y(int n, int kp, int nz, MsCols cols,
                                                     double* __restrict__ r,
                                                     const double* __restrict__ w,
                                                     double* __restrict__ y,
                                                     cpx<double>* __restrict__ Ps,
                                                     double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int cl = lane * CPL;
  double alpha[CPL];
  bool on[CPL], lv[CPL][NZ];
  zd ip[CPL][NZ], bs[CPL][NZ], ga[CPL][NZ];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    on[q] = cols.colive[cl + q] != 0;
    alpha[q] = cols.alpha[cl + q];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      const int e = j * kp + cl + q;
      lv[q][j] = j < nz && cols.live[e] != 0;
      ip[q][j] = lv[q][j] ? zd{cols.ipi[e].re, cols.ipi[e].im} : zd{0.0, 0.0};
      bs[q][j] = lv[q][j] ? zd{cols.bs[e].re, cols.bs[e].im} : zd{0.0, 0.0};
      ga[q][j] = lv[q][j] ? zd{cols.gas[e].re, cols.gas[e].im} : zd{0.0, 0.0};
    }
  }
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  const Rows rw = my_rows(n);
  const size_t blk = (size_t)n * kp;
  for (int t = 0; t < rw.count; ++t) {
    const size_t o = (size_t)(rw.first + rw.stride * t) * kp + cl;
    double ro[CPL], yo[CPL];
    cpx<double> po[CPL][NZ];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      ro[q] = on[q] ? r[o + q] : 0.0;
      yo[q] = on[q] ? y[o + q] : 0.0;
#pragma unroll
      for (int j = 0; j < NZ; ++j)
        if (lv[q][j]) po[q][j] = Ps[j * blk + o + q];
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const double rn = ro[q] - alpha[q] * w[o + q];
      r[o + q] = rn;
      acc[q] += rn * rn;
      double yv = yo[q];
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        if (!lv[q][j]) continue;
        const zd b = bs[q][j];
        const double pr = ro[q] * ip[q][j].re + (b.re * po[q][j].re - b.im * po[q][j].im);
        const double pi = ro[q] * ip[q][j].im + (b.re * po[q][j].im + b.im * po[q][j].re);
        Ps[j * blk + o + q] = cpx<double>{pr, pi};
        yv += ga[q][j].re * pr - ga[q][j].im * pi;
      }
      y[o + q] = yv;
    }
  }
  put_partial<CPL>(acc, part, kp);
}

// Combining mode, generic shift count: as k_ms_update with y in place of the
// iterates.
template <int CPL>
__global__ __launch_bounds__(kMT) void k_ms_update_yg(int n, int kp, int nz, MsCols cols,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ y,
                                                      cpx<double>* __restrict__ Ps,
                                                      double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int cl = lane * CPL;
  double alpha[CPL];
  bool on[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    on[q] = cols.colive[cl + q] != 0;
    alpha[q] = cols.alpha[cl + q];
  }
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  const Rows rw = my_rows(n);
  const size_t blk = (size_t)n * kp;
  for (int t = 0; t < rw.count; ++t) {
    const size_t o = (size_t)(rw.first + rw.stride * t) * kp + cl;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      if (!on[q]) continue;
      const double ro = r[o + q];
      const double rn = ro - alpha[q] * w[o + q];
      r[o + q] = rn;
      acc[q] += rn * rn;
      double yv = y[o + q];
      for (int j = 0; j < nz; ++j) {
        const int e = j * kp + cl + q;
        if (!cols.live[e]) continue;
        const cpx<double> ip = cols.ipi[e], b = cols.bs[e], ga = cols.gas[e];
        const cpx<double> po = Ps[j * blk + o + q];
        const double pr = ro * ip.re + (b.re * po.re - b.im * po.im);
        const double pi = ro * ip.im + (b.re * po.im + b.im * po.re);
        Ps[j * blk + o + q] = cpx<double>{pr, pi};
        yv += ga.re * pr - ga.im * pi;
      }
      y[o + q] = yv;
    }
  }
  put_partial<CPL>(acc, part, kp);
}

// beta_k, beta^s_k = beta_k (pi_k / pi_{k+1})^2, the pi shift, the
// convergence test |r_{k+1}| / |pi_{k+1}| <= tol |b| (or the iteration cap),
// the live counts, and the rescale of a column whose seed residual has
// fallen below 1e-100 |b|.
__global__ __launch_bounds__(kFT) void k_ms_fin_beta(int kp, int nz, int nb,
                                                     const double* __restrict__ part, double tol,
                                                     int maxit, MsCols cols,
                                                     int* __restrict__ count) {
  const int c = blockIdx.x;
  if (!cols.colive[c]) return;  // uniform over the workgroup
  const double rn = col_total(part, nb, kp, c);
  if (threadIdx.x != 0) return;
  const double rr = cols.rr[c];
  const double beta = rr > 0.0 ? rn / rr : 0.0;
  const double bn = cols.bn[c];
  const double rnorm = sqrt(rn);
  int nl = 0;
  for (int j = 0; j < nz; ++j) {
    const int e = j * kp + c;
    if (!cols.live[e]) continue;
    const zd pk{cols.pi[e].re, cols.pi[e].im}, pn{cols.pi_next[e].re, cols.pi_next[e].im};
    const zd q = zdiv(pk, pn);
    const zd q2 = zmul(q, q);
    cols.bs[e] = cpx<double>{beta * q2.re, beta * q2.im};
    cols.pi_prev[e] = cols.pi[e];
    cols.pi[e] = cols.pi_next[e];
    const int it = cols.its[e] + 1;
    cols.its[e] = it;
    const double est = rnorm / sqrt(pn.re * pn.re + pn.im * pn.im);
    cols.est[e] = bn > 0.0 ? est / bn : 0.0;
    if (est <= tol * bn || it >= maxit) {
      cols.live[e] = 0;
    } else {
      ++nl;
    }
  }
  cols.alpha_prev[c] = cols.alpha[c];
  cols.beta_prev[c] = beta;
  cols.rr[c] = rn;
  cols.colive[c] = nl > 0 ? 1 : 0;
  if (nl > 0 && rn > 0.0 && rn < 1e-200 * bn * bn) {
    const double s = 1e100;
    cols.scale[c] = s;
    cols.rr[c] = rn * s * s;
    for (int j = 0; j < nz; ++j) {
      const int e = j * kp + c;
      cols.pi[e] = cpx<double>{cols.pi[e].re * s, cols.pi[e].im * s};
      cols.pi_prev[e] = cpx<double>{cols.pi_prev[e].re * s, cols.pi_prev[e].im * s};
    }
  }
  if (nl) atomicAdd(count, nl);
}

// True residual of shift j: partials of |b - (z_j I - A) d|^2 with d = -x^s_j,
// i.e. of |b + z_j x - A x|^2 (a complex SpMV over x^s_j).
template <int CPL>
__global__ __launch_bounds__(kMT) void k_ms_true(int n, int k, int kp,
                                                 const int* __restrict__ rowptr,
                                                 const int* __restrict__ col,
                                                 const double* __restrict__ val,
                                                 const int* __restrict__ perm,
                                                 const double* __restrict__ B, int ldb,
                                                 double zre, double zim,
                                                 const cpx<double>* __restrict__ x,
                                                 double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int cl = lane * CPL;
  double acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = 0.0;
  const Rows rw = my_rows(n);
  for (int t = 0; t < rw.count; ++t) {
    const int row = rw.first + rw.stride * t;
    const int s = rowptr[row], e = rowptr[row + 1];
    double ar[CPL], ai[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) ar[q] = ai[q] = 0.0;
    for (int base = s; base < e; base += 64) {
      const int m = min(64, e - base);
      int mc = row;
      double mv = 0.0;
      if (lane < m) {
        mc = col[base + lane];
        mv = val[base + lane];
      }
      for (int u = 0; u < m; ++u) {
        const int j = __builtin_amdgcn_readlane(mc, u);
        const double a = readlane_f64(mv, u);
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          const cpx<double> v = x[(size_t)j * kp + cl + q];
          ar[q] = fma(a, v.re, ar[q]);
          ai[q] = fma(a, v.im, ai[q]);
        }
      }
    }
    const size_t src = (size_t)perm[row] * ldb;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = cl + q;
      if (c >= k) continue;
      const cpx<double> v = x[(size_t)row * kp + c];
      const double sr = B[src + c] + (zre * v.re - zim * v.im) - ar[q];
      const double si = (zre * v.im + zim * v.re) - ai[q];
      acc[q] += sr * sr + si * si;
    }
  }
  put_partial<CPL>(acc, part, kp);
}

// resid[j k + c] = sqrt(sum of the partials) / |b_c| (0 for b_c = 0).
__global__ __launch_bounds__(kFT) void k_ms_fin_true(int k, int kp, int j, int nb,
                                                     const double* __restrict__ part,
                                                     const double* __restrict__ bn,
                                                     double* __restrict__ resid) {
  const int c = blockIdx.x;
  const double s2 = col_total(part, nb, kp, c);
  if (threadIdx.x != 0 || c >= k) return;
  resid[(size_t)j * k + c] = bn[c] > 0.0 ? sqrt(s2) / bn[c] : 0.0;
}

// D[perm[row]][j k + c] = -x^s_j (the solution of (z_j I - A) d = b).
template <int CPL>
__global__ __launch_bounds__(kMT) void k_ms_out(int n, int k, int kp, int nz,
                                                const int* __restrict__ perm,
                                                const cpx<double>* __restrict__ X,
                                                cpx<double>* __restrict__ D, int ldd) {
  const int lane = threadIdx.x & 63;
  const Rows rw = my_rows(n);
  const size_t blk = (size_t)n * kp;
  for (int t = 0; t < rw.count; ++t) {
    const int row = rw.first + rw.stride * t;
    const size_t dst = (size_t)perm[row] * ldd;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane * CPL + q;
      if (c >= k) continue;
      for (int j = 0; j < nz; ++j) {
        const cpx<double> x = X[j * blk + (size_t)row * kp + c];
        D[dst + (size_t)j * k + c] = cpx<double>{-x.re, -x.im};
      }
    }
  }
}

// Combining mode output: Qt[perm[row]][c] = gq_c Qin[perm[row]][c] - y[row][c]
// (d = -x, so the weighted sum of the solutions is -y) with
// gq_c = sum_j Re(g_{j,c}) (the residual form's q term; Qin null: 0).
template <int CPL>
__global__ __launch_bounds__(kMT) void k_ms_out_y(int n, int k, int kp, int nz,
                                                  const int* __restrict__ perm,
                                                  const double* __restrict__ y,
                                                  const double* __restrict__ g,
                                                  const double* __restrict__ Qin, int ldqin,
                                                  double* __restrict__ Qt, int ldq) {
  const int lane = threadIdx.x & 63;
  double gq[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int c = lane * CPL + q;
    double s = 0.0;
    if (c < k && Qin)
      for (int j = 0; j < nz; ++j) s += g[2 * (j * k + c)];
    gq[q] = s;
  }
  const Rows rw = my_rows(n);
  for (int t = 0; t < rw.count; ++t) {
    const int row = rw.first + rw.stride * t;
    const size_t dst = (size_t)perm[row];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = lane * CPL + q;
      if (c >= k) continue;
      const double qv = Qin ? gq[q] * Qin[dst * ldqin + c] : 0.0;
      Qt[dst * ldq + c] = qv - y[(size_t)row * kp + c];
    }
  }
}

// iters[j k + c] and resid[j k + c] (estimated relative residual) per system.
__global__ void k_ms_report(int k, int kp, int nz, MsCols cols, int* __restrict__ iters,
                            double* __restrict__ resid) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nz * k) return;
  const int j = e / k, c = e % k;
  if (iters) iters[e] = cols.its[j * kp + c];
  if (resid) resid[e] = cols.est[j * kp + c];
}

int ms_cpl(int k) { return (k + 63) / 64; }
int ms_padded(int k) { return 64 * ms_cpl(k); }
int ms_blocks(int n, int num_cu) {
  int nb = num_cu * 4;
  const int need = (n + kMW - 1) / kMW;
  if (nb > need) nb = (need + 7) / 8 * 8;
  return nb < 8 ? 8 : nb;
}

namespace {

template <int CPL>
hipError_t run_ms_t(hipStream_t st, const StreamMatrix& A, const MsWork& W, const MsLaunch& L) {
  const int n = A.n, k = L.k, kp = W.kp, nz = L.nz;
  const int nb = W.nb;
  const dim3 grid(nb), blk(kMT), fg(kp), fb(kFT);
#define MCHK(expr)                   \
  do {                               \
    hipError_t _e = (expr);          \
    if (_e != hipSuccess) return _e; \
  } while (0)
#define MLAUNCH(...)                 \
  do {                               \
    hipLaunchKernelGGL(__VA_ARGS__); \
    MCHK(hipGetLastError());         \
  } while (0)
  // shifts of the seed form: sigma_j = s - z_j
  std::vector<cpx<double>> sg(nz);
  for (int j = 0; j < nz; ++j) sg[j] = cpx<double>{L.seed - L.z[2 * j], -L.z[2 * j + 1]};
  MCHK(hipMemcpyAsync(W.sig, sg.data(), nz * sizeof(cpx<double>), hipMemcpyHostToDevice, st));
  MCHK(hipMemsetAsync(W.count, 0, sizeof(int), st));
  const bool comb = L.g != nullptr;
  double* yb = comb ? W.y : nullptr;
  MLAUNCH((k_ms_init<CPL>), grid, blk, 0, st, n, k, kp, nz, A.perm, L.B, L.ldb, W.r, W.p, W.X,
          W.P, yb, W.part);
  MLAUNCH(k_ms_fin0, fg, fb, 0, st, k, kp, nz, nb, W.part, W.cols, W.count);
  int live = 0;
  MCHK(hipMemcpyAsync(&live, W.count, sizeof(int), hipMemcpyDeviceToHost, st));
  MCHK(hipStreamSynchronize(st));
  for (int it = 0; it < L.maxit && live > 0; ++it) {
    MLAUNCH((k_ms_pupd<CPL>), grid, blk, 0, st, n, kp, W.cols, W.r, W.p);
    MLAUNCH((k_ms_spmv<CPL>), grid, blk, 0, st, n, kp, A.rowptr, A.col, A.val64, L.seed,
            W.cols.colive, W.p, W.w, W.part);
    MLAUNCH(k_ms_fin_alpha, fg, fb, 0, st, kp, k, nz, nb, W.part, W.sig, L.g, W.cols);
    if (comb) {
      if (nz * CPL <= 2)
        MLAUNCH((k_ms_update_y<CPL, (2 / CPL > 0 ? 2 / CPL : 1)>), grid, blk, 0, st, n, kp, nz,
                W.cols, W.r, W.w, yb, W.P, W.part);
      else if (nz * CPL <= 4)
        MLAUNCH((k_ms_update_y<CPL, (4 / CPL > 0 ? 4 / CPL : 1)>), grid, blk, 0, st, n, kp, nz,
                W.cols, W.r, W.w, yb, W.P, W.part);
      else if (nz * CPL <= 8)
        MLAUNCH((k_ms_update_y<CPL, (8 / CPL > 0 ? 8 / CPL : 1)>), grid, blk, 0, st, n, kp, nz,
                W.cols, W.r, W.w, yb, W.P, W.part);
      else
        MLAUNCH((k_ms_update_yg<CPL>), grid, blk, 0, st, n, kp, nz, W.cols, W.r, W.w, yb, W.P,
                W.part);
    } else if (nz * CPL <= 1)
      MLAUNCH((k_ms_update_r<CPL, 1>), grid, blk, 0, st, n, kp, nz, W.cols, W.r, W.w, W.X, W.P,
              W.part);
    else if (nz * CPL <= 2)
      MLAUNCH((k_ms_update_r<CPL, (2 / CPL > 0 ? 2 / CPL : 1)>), grid, blk, 0, st, n, kp, nz,
              W.cols, W.r, W.w, W.X, W.P, W.part);
    else if (nz * CPL <= 4)
      MLAUNCH((k_ms_update_r<CPL, (4 / CPL > 0 ? 4 / CPL : 1)>), grid, blk, 0, st, n, kp, nz,
              W.cols, W.r, W.w, W.X, W.P, W.part);
    else if (nz * CPL <= 8)
      MLAUNCH((k_ms_update_r<CPL, (8 / CPL > 0 ? 8 / CPL : 1)>), grid, blk, 0, st, n, kp, nz,
              W.cols, W.r, W.w, W.X, W.P, W.part);
    else
      MLAUNCH((k_ms_update<CPL>), grid, blk, 0, st, n, kp, nz, W.cols, W.r, W.w, W.X, W.P,
              W.part);
    MCHK(hipMemsetAsync(W.count, 0, sizeof(int), st));
    MLAUNCH(k_ms_fin_beta, fg, fb, 0, st, kp, nz, nb, W.part, L.tol, L.maxit, W.cols, W.count);
    if ((it + 1) % L.chunk == 0 || it + 1 == L.maxit) {
      MCHK(hipMemcpyAsync(&live, W.count, sizeof(int), hipMemcpyDeviceToHost, st));
      MCHK(hipStreamSynchronize(st));
    }
  }
  if (comb) {
    MLAUNCH((k_ms_out_y<CPL>), grid, blk, 0, st, n, k, kp, nz, A.perm, yb, L.g, L.Qin, L.ldqin,
            L.Qt, L.ldq);
    if (L.iters)
      MLAUNCH(k_ms_report, dim3((nz * k + 255) / 256), dim3(256), 0, st, k, kp, nz, W.cols,
              L.iters, (double*)nullptr);
    return hipSuccess;
  }
  MLAUNCH((k_ms_out<CPL>), grid, blk, 0, st, n, k, kp, nz, A.perm, W.X,
          static_cast<cpx<double>*>(L.D), L.ldd);
  if (L.iters)
    MLAUNCH(k_ms_report, dim3((nz * k + 255) / 256), dim3(256), 0, st, k, kp, nz, W.cols, L.iters,
            (double*)nullptr);
  if (L.resid) {
    const size_t bsz = (size_t)n * kp;
    for (int j = 0; j < nz; ++j) {
      MLAUNCH((k_ms_true<CPL>), grid, blk, 0, st, n, k, kp, A.rowptr, A.col, A.val64, A.perm,
              L.B, L.ldb, L.z[2 * j], L.z[2 * j + 1], W.X + j * bsz, W.part);
      MLAUNCH(k_ms_fin_true, fg, fb, 0, st, k, kp, j, nb, W.part, W.cols.bn, L.resid);
    }
  }
  return hipSuccess;
#undef MLAUNCH
#undef MCHK
}

}  // namespace

hipError_t run_mshift(hipStream_t st, const StreamMatrix& A, const MsWork& W, const MsLaunch& L) {
  if (L.k < 1 || L.nz < 1 || L.k > W.kp || W.kp != ms_padded(L.k) || L.nz > W.nz || !A.val64 ||
      W.nb != ms_blocks(A.n, W.num_cu) || L.chunk < 1)
    return hipErrorInvalidValue;
  if (L.g ? (!W.y || !W.cols.gas || !L.Qt || L.ldq < L.k || (L.Qin && L.ldqin < L.k))
          : (!W.X || !L.D || L.ldd < L.nz * L.k))
    return hipErrorInvalidValue;
  switch (ms_cpl(L.k)) {
    case 1: return run_ms_t<1>(st, A, W, L);
    case 2: return run_ms_t<2>(st, A, W, L);
    case 3: return run_ms_t<3>(st, A, W, L);
  }
  return hipErrorInvalidValue;
}

}  // namespace rafeast
