// Exact shifted solves for standard FEAST, the baseline of Section 5.1 (FEAST
// with sparse direct factorizations of the shifted matrices).  Each shifted
// matrix M_j = z_j I - A is factorized once as M_j = L_j D_j L_j^T (complex
// symmetric: the transpose, not the conjugate transpose; L unit lower
// triangular, D diagonal) and every filter application solves by substitution.
//
// Order: A in reverse Cuthill-McKee order (the streaming engine's), whose lower
// bandwidth b bounds the factors: LDL^T without pivoting creates no fill
// outside the band.  No pivoting is needed: the leading principal submatrices
// of z I - A are z I - A_k with A_k real symmetric, whose eigenvalues z - mu
// are nonzero for Im z != 0, so every pivot exists; and the imaginary part of
// M is Im z I, definite, for which elimination without pivoting has bounded
// element growth (N. J. Higham, Factorizing complex symmetric matrices with
// positive definite real and imaginary parts, Math. Comp. 1998).
//
// Storage: per shift an n x (b + 1) complex array W, row r holding M(r, r - d)
// in W[r][d], d = 0..b (d = 0 the diagonal).  After the factorization
// W[r][0] = D(r) and W[r][d] = L(r, r - d).
//
// Factorization: panels of nb = 32 columns, all shifts together, two
// launches per panel.  One workgroup per shift factorizes the panel's
// diagonal block in LDS and gives every row below it that the band reaches
// its multipliers (a product with the block's inverse triangle); the Schur
// complement of the b x b
// window below the panel, W(i, j) -= sum_k l_ik d_k l_jk, is spread over
// many workgroups per shift in 64 x 64 blocks of 4 x 4 register tiles, so a
// factorization's time grows with the number of shifts, not only with one
// CU's rate.  Solves: one workgroup per (shift, group of
// right-hand sides); blocks of 32 rows, each first reduced by the solved rows
// within the band, then solved within the block in LDS; forward with L, then
// D, then backward with L^T.
#include "device.h"
#include "kernels.h"

#include <algorithm>

namespace rafeast {

namespace {

typedef cpx<double> zc;

__device__ __forceinline__ zc cmul(zc a, zc b) {
  return zc{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ zc csub(zc a, zc b) { return zc{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ zc cinv(zc a) {
  // 1 / a with the larger component scaled out (Smith's method)
  if (fabs(a.re) >= fabs(a.im)) {
    const double r = a.im / a.re, den = a.re + a.im * r;
    return zc{1.0 / den, -r / den};
  }
  const double r = a.re / a.im, den = a.re * r + a.im;
  return zc{r / den, -1.0 / den};
}
__device__ __forceinline__ bool cfinite(zc a) { return isfinite(a.re) && isfinite(a.im); }

constexpr int kPanelThreads = 256;
constexpr int kPanelRows = kPanelThreads / 2;  // rows per staged chunk (two threads each)
constexpr int kBandMaxPanel = 32;  // panel width
constexpr size_t kBandSolveRingBytes = 128 * 1024;  // LDS ring of the solve
constexpr int kSolveThreads = 256;
constexpr int kSolveRows = 32;  // rows per solve block
constexpr int kSolveCols = 2;   // right-hand sides per workgroup
constexpr int kSolveSlices = kSolveThreads / kSolveRows;  // threads per block row

// W_j: every entry zero, then z_j on the diagonal and -A(r, c) at (r, r - c)
// for the lower entries c <= r of the reordered CSR.  Thread per row.
__global__ __launch_bounds__(256) void k_band_assemble(int n, int b, const int* __restrict__ rowptr,
                                                       const int* __restrict__ col,
                                                       const double* __restrict__ val,
                                                       const double* __restrict__ z,
                                                       zc* __restrict__ W, size_t stride) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const int j = blockIdx.y;
  zc* __restrict__ row = W + (size_t)j * stride + (size_t)r * (b + 1);
  for (int d = 0; d <= b; ++d) row[d] = zc{0.0, 0.0};
  row[0] = zc{z[2 * j], z[2 * j + 1]};
  for (int t = rowptr[r]; t < rowptr[r + 1]; ++t) {
    const int c = col[t];
    if (c > r || r - c > b) continue;
    row[r - c].re -= val[t];
  }
}

// Panel c of the band LDL^T of W_j (workgroup j).  The workgroup factorizes
// the panel's diagonal block (nb x nb, in LDS: multipliers l = m / d and the
// rank-one updates, column by column, each thread owning fixed entries) and
// forms the inverse of its unit lower triangle L11 (by elimination on the
// identity, likewise).  Every row i below the block that the band reaches then
// takes its multipliers as a product with that inverse:
//   l_ik = (sum_{q <= k} m_iq (L11^{-1})_kq) / d_k,
// i.e. L21 = M21 L11^{-T} D^{-1}: chunks of rows staged in LDS, two threads
// per row with nb / 2 independent sums each.
// info[j] = 1 + the row of a vanishing or non-finite pivot (that shift's
// factorization stops there: later panels and updates of it return at once).
__global__ __launch_bounds__(kPanelThreads) void k_band_panel(int n, int b, int nb, int c,
                                                              zc* __restrict__ Wall,
                                                              size_t stride,
                                                              int* __restrict__ info) {
  constexpr int L = kBandMaxPanel + 1;
  __shared__ zc Pd[kBandMaxPanel][L];  // the diagonal block, then its factors
  __shared__ zc Li[kBandMaxPanel][L];  // Li[k][q] = (L11^{-1})_kq, q <= k
  __shared__ zc Dinv[kBandMaxPanel];
  __shared__ int bad;
  const int j = blockIdx.x;
  if (info[j] != 0) return;
  zc* __restrict__ W = Wall + (size_t)j * stride;
  const int ldw = b + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int e = min(c + nb, n), w = e - c, rend = min(n, e + b);
  for (int idx = tid; idx < kBandMaxPanel * kBandMaxPanel; idx += nt) {
    const int ii = idx / kBandMaxPanel, kk = idx % kBandMaxPanel;
    const int i = c + ii, k = c + kk;
    Pd[ii][kk] = (ii < w && kk <= ii && i - k <= b) ? W[(size_t)i * ldw + (i - k)] : zc{0.0, 0.0};
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // the block's pivot steps: every thread owns fixed entries of the 32 x 32
  // block (entry t + 256 u: row (t + 256 u) / 32, column (t + 256 u) % 32)
  static_assert(kBandMaxPanel == 32, "entry indices by shifts");
  constexpr int kOwn = kBandMaxPanel * kBandMaxPanel / kPanelThreads;
  static_assert(kOwn * kPanelThreads == kBandMaxPanel * kBandMaxPanel, "entry ownership");
  int fail = 0;
  for (int kk = 0; kk < w; ++kk) {
    const zc d = Pd[kk][kk];
    if (!(cfinite(d) && (d.re != 0.0 || d.im != 0.0))) {
      fail = c + kk + 1;
      break;  // uniform: every thread read the same pivot
    }
    const zc inv = cinv(d);
    if (tid == 0) Dinv[kk] = inv;
    if (tid > kk && tid < w) Pd[tid][kk] = cmul(Pd[tid][kk], inv);  // column kk's multipliers
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kOwn; ++u) {
      const int en = tid + kPanelThreads * u, ii = en >> 5, jj = en & 31;
      if (jj > kk && jj <= ii && ii < w)
        Pd[ii][jj] = csub(Pd[ii][jj], cmul(cmul(Pd[ii][kk], d), Pd[jj][kk]));
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) {
      bad = 1;
      info[j] = fail;
    }
  } else {
    // L11^{-1} by elimination on the identity, column q at a time:
    // X[i][:q] -= l_iq X[q][:q] for i > q
#pragma unroll
    for (int u = 0; u < kOwn; ++u) {
      const int en = tid + kPanelThreads * u, i = en >> 5, q = en & 31;
      Li[i][q] = zc{i == q ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    for (int q = 0; q + 1 < w; ++q) {
#pragma unroll
      for (int u = 0; u < kOwn; ++u) {
        const int en = tid + kPanelThreads * u, i = en >> 5, jx = en & 31;
        if (i > q && i < w && jx <= q) Li[i][jx] = csub(Li[i][jx], cmul(Pd[i][q], Li[q][jx]));
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (bad) return;
  // the block back to W: multipliers below its diagonal, pivots on it
  for (int idx = tid; idx < w * w; idx += nt) {
    const int ii = idx / w, kk = idx % w, i = c + ii, k = c + kk;
    if (kk <= ii && i - k <= b) W[(size_t)i * ldw + (i - k)] = Pd[ii][kk];
  }
  // rows below the block, in chunks of kPanelRows staged in LDS by coalesced
  // loads; two threads per row, one per half of the nb sums (16 each)
  extern __shared__ zc Rs[];  // [kPanelRows][L]
  constexpr int H = kBandMaxPanel / 2;
  const int rr = tid % kPanelRows, h = tid / kPanelRows;
  for (int i0 = e; i0 < rend; i0 += kPanelRows) {
    for (int idx = tid; idx < kPanelRows * kBandMaxPanel; idx += nt) {
      const int r = idx / kBandMaxPanel, q = idx % kBandMaxPanel, i = i0 + r;
      Rs[r * L + q] = (i < rend && q < w && i - (c + q) <= b) ? W[(size_t)i * ldw + (i - c - q)]
                                                              : zc{0.0, 0.0};
    }
    __syncthreads();
    const int i = i0 + rr;
    if (i < rend) {
      zc acc[H];
#pragma unroll
      for (int k = 0; k < H; ++k) acc[k] = zc{0.0, 0.0};
      const int qend = min(w, H * (h + 1));
#pragma unroll 1
      for (int q = 0; q < qend; ++q) {
        const zc mq = Rs[rr * L + q];
#pragma unroll
        for (int k = 0; k < H; ++k) {
          if (H * h + k >= q) {
            const zc l = Li[H * h + k][q];
            acc[k].re += mq.re * l.re - mq.im * l.im;
            acc[k].im += mq.re * l.im + mq.im * l.re;
          }
        }
      }
      zc* __restrict__ row = W + (size_t)i * ldw;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int kk = H * h + k;
        if (kk < w && i - (c + kk) <= b) row[i - c - kk] = cmul(acc[k], Dinv[kk]);
      }
    }
    __syncthreads();
  }
}

// Schur complement of the window below panel c of W_j (shift blockIdx.y):
// W(i, jc) -= sum_{k in panel} l_ik d_k l_jc,k for e <= jc <= i < rend, in
// 64 x 64 blocks of the window's lower triangle (blockIdx.x enumerates the
// pairs bi >= bj), each thread a 4 x 4 tile.  The panel's multipliers of the
// block's rows and columns and the pivots are staged in LDS.
constexpr int kSchurBlock = 64;
__global__ __launch_bounds__(256) void k_band_schur(int n, int b, int nb, int c,
                                                    zc* __restrict__ Wall, size_t stride,
                                                    const int* __restrict__ info) {
  __shared__ zc Lr[kSchurBlock][kBandMaxPanel + 1];
  __shared__ zc Lc[kSchurBlock][kBandMaxPanel + 1];
  __shared__ zc Dp[kBandMaxPanel];
  const int j = blockIdx.y;
  if (info[j] != 0) return;
  zc* __restrict__ W = Wall + (size_t)j * stride;
  const int ldw = b + 1;
  const int e = min(c + nb, n), w = e - c, rend = min(n, e + b), m = rend - e;
  const int t = blockIdx.x;
  int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  while (bi * (bi + 1) / 2 > t) --bi;
  const int bj = t - bi * (bi + 1) / 2;
  const int i0 = e + bi * kSchurBlock, j0 = e + bj * kSchurBlock;
  const int tid = threadIdx.x;
  // multipliers l(r, k) = W[r][r - k] of the block's rows and columns
  for (int idx = tid; idx < kSchurBlock * w; idx += 256) {
    const int r = idx / w, kk = idx % w, k = c + kk;
    const int ri = i0 + r, rj = j0 + r;
    Lr[r][kk] = (ri < rend && ri - k <= b) ? W[(size_t)ri * ldw + (ri - k)] : zc{0.0, 0.0};
    Lc[r][kk] = (rj < rend && rj - k <= b) ? W[(size_t)rj * ldw + (rj - k)] : zc{0.0, 0.0};
  }
  if (tid < w) Dp[tid] = W[(size_t)(c + tid) * ldw];
  __syncthreads();
  const int ti = tid / 16, tj = tid % 16;
  if (i0 + 4 * ti >= rend || j0 + 4 * tj > i0 + 4 * ti + 3) return;  // tile outside the triangle
  zc acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = zc{0.0, 0.0};
  for (int kk = 0; kk < w; ++kk) {
    const zc dk = Dp[kk];
    zc a[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = cmul(Lr[4 * ti + u][kk], dk);
      bv[u] = Lc[4 * tj + u][kk];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[u][v].re += a[u].re * bv[v].re - a[u].im * bv[v].im;
        acc[u][v].im += a[u].re * bv[v].im + a[u].im * bv[v].re;
      }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 4 * ti + u, jc = j0 + 4 * tj + v;
      if (i < rend && jc <= i) {
        zc* p = W + (size_t)i * ldw + (i - jc);
        *p = csub(*p, acc[u][v]);
      }
    }
  (void)m;
}

// X[:, j k + c] = M_j^{-1} B[:, c] for the columns of group blockIdx.x and
// shift blockIdx.y, with the factors of W_j.  Rows of A in the engine order
// r map to caller rows perm[r]; B (n x k, ldb) and X (n x (nz k) complex,
// ldx) are in caller order.  The solve runs in place in X.
// LDS: a ring of the last ring_rows solved rows of the group's columns
// (ring_rows a power of two >= b + 32), so the band terms read solved values
// from LDS; per block the strict lower triangle and the pivots.  Band terms:
// eight threads per block row, the row's band streamed in order by each
// (forward), or consecutive rows of the block on consecutive threads, which
// makes each row's band entries contiguous across the threads (backward, L^T
// read by columns).
__global__ __launch_bounds__(kSolveThreads) void k_band_solve(int n, int b, const zc* __restrict__ Wall,
                                                              size_t stride,
                                                              const int* __restrict__ perm,
                                                              const double* __restrict__ B, int ldb,
                                                              int k, zc* __restrict__ X,
                                                              int64_t ldx, int ring_rows) {
  extern __shared__ zc ring[];  // [ring_rows][kSolveCols]
  __shared__ zc yb[kSolveRows][kSolveCols];
  __shared__ zc tri[kSolveRows][kSolveRows + 1];  // tri[r][q] = L(r0 + r, r0 + q), q < r
  __shared__ zc piv[kSolveRows];
  __shared__ zc part[kSolveSlices][kSolveRows][kSolveCols];
  const int j = blockIdx.y, g = blockIdx.x;
  const zc* __restrict__ W = Wall + (size_t)j * stride;
  const int ldw = b + 1, mask = ring_rows - 1;
  const int c0g = g * kSolveCols, ncol = min(kSolveCols, k - c0g);
  const int tid = threadIdx.x;
  auto xat = [&](int r, int cc) -> zc& {
    return X[(size_t)perm[r] * ldx + (size_t)j * k + c0g + cc];
  };
  auto stage = [&](int r0, int nr) {
    for (int idx = tid; idx < kSolveRows * kSolveRows; idx += kSolveThreads) {
      const int r = idx / kSolveRows, q = idx % kSolveRows;
      zc v{0.0, 0.0};
      if (r < nr && q < r && r - q <= b) v = W[(size_t)(r0 + r) * ldw + (r - q)];
      tri[r][q] = v;
    }
    if (tid < nr) piv[tid] = W[(size_t)(r0 + tid) * ldw];
  };
  // right-hand sides into X
  for (int idx = tid; idx < n * ncol; idx += kSolveThreads) {
    const int r = idx / ncol, cc = idx % ncol;
    xat(r, cc) = zc{B[(size_t)perm[r] * ldb + c0g + cc], 0.0};
  }
  __syncthreads();
  const int rr = tid % kSolveRows, h = tid / kSolveRows;  // block row, slice
  const bool lead = tid < kSolveRows * kSolveCols;        // one thread per (row, column)
  const int lr = tid / kSolveCols, lc = tid % kSolveCols;

  // forward: L y = b
  for (int r0 = 0; r0 < n; r0 += kSolveRows) {
    const int nr = min(kSolveRows, n - r0);
    stage(r0, nr);
    zc s[kSolveCols];
#pragma unroll
    for (int cc = 0; cc < kSolveCols; ++cc) s[cc] = zc{0.0, 0.0};
    if (rr < nr) {
      const int r = r0 + rr;
      const zc* __restrict__ wrow = W + (size_t)r * ldw;
#pragma unroll 4
      for (int q = r0 - 1 - h; q >= max(0, r - b); q -= kSolveSlices) {
        const zc l = wrow[r - q];
#pragma unroll
        for (int cc = 0; cc < kSolveCols; ++cc) {
          const zc y = ring[(q & mask) * kSolveCols + cc];
          s[cc].re += l.re * y.re - l.im * y.im;
          s[cc].im += l.re * y.im + l.im * y.re;
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < kSolveCols; ++cc) part[h][rr][cc] = s[cc];
    __syncthreads();
    if (lead && lr < nr && lc < ncol) {
      zc t = xat(r0 + lr, lc);
      for (int q = 0; q < kSolveSlices; ++q) t = csub(t, part[q][lr][lc]);
      yb[lr][lc] = t;
    }
    __syncthreads();
    for (int kk = 0; kk < nr - 1; ++kk) {
      // rows below kk within the block take its contribution
      if (lead && lr > kk && lr < nr && lc < ncol)
        yb[lr][lc] = csub(yb[lr][lc], cmul(tri[lr][kk], yb[kk][lc]));
      __syncthreads();
    }
    if (lead && lr < nr) {
      const zc v = lc < ncol ? yb[lr][lc] : zc{0.0, 0.0};
      ring[((r0 + lr) & mask) * kSolveCols + lc] = v;
      if (lc < ncol) xat(r0 + lr, lc) = v;
    }
    __syncthreads();
  }
  // backward: L^T x = D^{-1} y, blocks from the last; the ring now takes the
  // solved x of the rows after the block
  for (int r1 = n; r1 > 0; r1 -= kSolveRows) {
    const int r0 = max(0, r1 - kSolveRows), nr = r1 - r0;
    stage(r0, nr);
    zc s[kSolveCols];
#pragma unroll
    for (int cc = 0; cc < kSolveCols; ++cc) s[cc] = zc{0.0, 0.0};
    if (rr < nr) {
      const int r = r0 + rr;
      const int hi = min(n - 1, r + b);
#pragma unroll 4
      for (int i = r1 + h; i <= hi; i += kSolveSlices) {
        const zc l = W[(size_t)i * ldw + (i - r)];
#pragma unroll
        for (int cc = 0; cc < kSolveCols; ++cc) {
          const zc x = ring[(i & mask) * kSolveCols + cc];
          s[cc].re += l.re * x.re - l.im * x.im;
          s[cc].im += l.re * x.im + l.im * x.re;
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < kSolveCols; ++cc) part[h][rr][cc] = s[cc];
    __syncthreads();
    if (lead && lr < nr && lc < ncol) {
      zc t = cmul(xat(r0 + lr, lc), cinv(piv[lr]));
      for (int q = 0; q < kSolveSlices; ++q) t = csub(t, part[q][lr][lc]);
      yb[lr][lc] = t;
    }
    __syncthreads();
    for (int kk = nr - 1; kk > 0; --kk) {
      if (lead && lr < kk && lc < ncol)
        yb[lr][lc] = csub(yb[lr][lc], cmul(tri[kk][lr], yb[kk][lc]));
      __syncthreads();
    }
    if (lead && lr < nr) {
      const zc v = lc < ncol ? yb[lr][lc] : zc{0.0, 0.0};
      ring[((r0 + lr) & mask) * kSolveCols + lc] = v;
      if (lc < ncol) xat(r0 + lr, lc) = v;
    }
    __syncthreads();
  }
}

// resid[j k + c] = ||B_c - (z_j I - A) X_{j,c}|| / ||B_c|| (0 for B_c = 0),
// in FP64 with A in caller order; one workgroup per system.
__global__ __launch_bounds__(256) void k_band_resid(int n, const int* __restrict__ rowptr,
                                                    const int* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ z,
                                                    const double* __restrict__ B, int ldb, int k,
                                                    const zc* __restrict__ X, int64_t ldx,
                                                    double* __restrict__ resid) {
  const int sys = blockIdx.x, j = sys / k, c = sys % k;
  const double zr = z[2 * j], zi = z[2 * j + 1];
  double rr = 0.0, bb = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    double ar = 0.0, ai = 0.0;
    for (int t = rowptr[i]; t < rowptr[i + 1]; ++t) {
      const zc x = X[(size_t)col[t] * ldx + sys];
      ar += val[t] * x.re;
      ai += val[t] * x.im;
    }
    const zc x = X[(size_t)i * ldx + sys];
    const double bi = B[(size_t)i * ldb + c];
    const double sr = bi - (zr * x.re - zi * x.im - ar);
    const double si = -(zr * x.im + zi * x.re - ai);
    rr += sr * sr + si * si;
    bb += bi * bi;
  }
  __shared__ double red[2][4];
  rr = wave_sum_f64(rr);
  bb = wave_sum_f64(bb);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = rr;
    red[1][wv] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double r2 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double b2 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    resid[sys] = b2 > 0.0 ? sqrt(r2 / b2) : 0.0;
  }
}

}  // namespace

int band_panel_width(int b) {
  (void)b;
  return kBandMaxPanel;
}

size_t band_lds_bytes(int b) {
  (void)b;
  // the panel kernel's dynamic LDS: a chunk of rows below the block
  return (size_t)kPanelRows * (kBandMaxPanel + 1) * sizeof(zc);
}

int band_solve_ring_rows(int b) {
  int rows = kSolveRows;
  while (rows < b + kSolveRows) rows *= 2;
  return rows;
}

bool band_supported(int b) {
  return band_lds_bytes(b) <= 160 * 1024 &&
         (size_t)band_solve_ring_rows(b) * kSolveCols * sizeof(zc) <= kBandSolveRingBytes;
}

hipError_t band_assemble(hipStream_t st, int n, int b, const int* rowptr, const int* col,
                         const double* val, int nz, const double* z, cpx<double>* W) {
  if (n <= 0 || nz <= 0) return hipSuccess;
  dim3 grid((n + 255) / 256, nz);
  hipLaunchKernelGGL(k_band_assemble, grid, dim3(256), 0, st, n, b, rowptr, col, val, z, W,
                     (size_t)n * (b + 1));
  return hipGetLastError();
}

hipError_t band_factor(hipStream_t st, int n, int b, int nz, cpx<double>* W, int* info) {
  if (n <= 0 || nz <= 0) return hipSuccess;
  const int nb = band_panel_width(b);
  const size_t lds = band_lds_bytes(b);
  hipError_t e = hipFuncSetAttribute((const void*)k_band_panel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(info, 0, nz * sizeof(int), st);
  if (e != hipSuccess) return e;
  const size_t stride = (size_t)n * (b + 1);
  // panel by panel, all shifts together: the panel (one workgroup per
  // shift), then its window's Schur complement over many workgroups
  for (int c = 0; c < n; c += nb) {
    hipLaunchKernelGGL(k_band_panel, dim3(nz), dim3(kPanelThreads), lds, st, n, b, nb, c, W,
                       stride, info);
    const int end = std::min(c + nb, n), m = std::min(n, end + b) - end;
    if (m > 0) {
      const int mb = (m + kSchurBlock - 1) / kSchurBlock;
      hipLaunchKernelGGL(k_band_schur, dim3(mb * (mb + 1) / 2, nz), dim3(256), 0, st, n, b, nb,
                         c, W, stride, info);
    }
  }
  return hipGetLastError();
}

hipError_t band_solve(hipStream_t st, int n, int b, int nz, const cpx<double>* W, const int* perm,
                      const double* B, int ldb, int k, cpx<double>* X, int64_t ldx) {
  if (n <= 0 || nz <= 0 || k <= 0) return hipSuccess;
  const int ring = band_solve_ring_rows(b);
  const size_t lds = (size_t)ring * kSolveCols * sizeof(zc);
  if (lds > kBandSolveRingBytes) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_band_solve,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  dim3 grid((k + kSolveCols - 1) / kSolveCols, nz);
  hipLaunchKernelGGL(k_band_solve, grid, dim3(kSolveThreads), lds, st, n, b, W,
                     (size_t)n * (b + 1), perm, B, ldb, k, X, ldx, ring);
  return hipGetLastError();
}

hipError_t band_resid(hipStream_t st, int n, const int* rowptr, const int* col, const double* val,
                      int nz, const double* z, const double* B, int ldb, int k,
                      const cpx<double>* X, int64_t ldx, double* resid) {
  if (n <= 0 || nz <= 0 || k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_resid, dim3(nz * k), dim3(256), 0, st, n, rowptr, col, val, z, B,
                     ldb, k, X, ldx, resid);
  return hipGetLastError();
}

}  // namespace rafeast
