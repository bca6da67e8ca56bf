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
// Factorization: one workgroup per shift, panels of nb columns.  The panel's
// rows (its nb rows and the b rows below that the band reaches) are staged in
// LDS, factorized there column by column (the multipliers l = m / d and their
// rank-one updates within the panel), written back, and the Schur complement
// of the b x b window below the panel is updated in 4 x 4 register tiles:
// W(i, j) -= sum_k l_ik d_k l_jk.  Solves: one workgroup per (shift, group of
// right-hand sides); blocks of 32 rows, each first reduced by the solved rows
// within the band, then solved within the block in LDS; forward with L, then
// D, then backward with L^T.
#include "device.h"
#include "kernels.h"

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

constexpr int kFactorThreads = 512;
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

// In-place band LDL^T of W_j (workgroup j).  info[j] = 0 on success, else
// 1 + the row whose pivot was zero or not finite (the factorization stops
// there).  LDS: the panel, (b + nb) rows of nb + 1 entries, then nb pivots.
__global__ __launch_bounds__(kFactorThreads) void k_band_factor(int n, int b, int nb,
                                                                zc* __restrict__ Wall,
                                                                size_t stride,
                                                                int* __restrict__ info) {
  extern __shared__ zc P[];
  const int j = blockIdx.x;
  zc* __restrict__ W = Wall + (size_t)j * stride;
  const int ldw = b + 1, ldp = nb + 1;
  zc* __restrict__ Dp = P + (size_t)(b + nb) * ldp;
  __shared__ int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) bad = 0;
  for (int c = 0; c < n; c += nb) {
    const int e = min(c + nb, n), w = e - c, rend = min(n, e + b), rows = rend - c;
    // stage the panel's rows, panel columns: P[i - c][k - c] = M(i, k)
    for (int idx = tid; idx < rows * nb; idx += nt) {
      const int i = c + idx / nb, kk = idx % nb, k = c + kk;
      zc v{0.0, 0.0};
      if (kk < w && k <= i && i - k <= b) v = W[(size_t)i * ldw + (i - k)];
      P[(idx / nb) * ldp + kk] = v;
    }
    __syncthreads();
    for (int kk = 0; kk < w; ++kk) {
      const zc d = P[kk * ldp + kk];
      const bool ok = cfinite(d) && (d.re != 0.0 || d.im != 0.0);
      if (!ok) {
        if (tid == 0) {
          bad = 1;
          info[j] = c + kk + 1;
        }
      }
      __syncthreads();
      if (bad) return;  // uniform: every thread read the flag after the barrier
      const zc inv = cinv(d);
      // multipliers of column k for the rows below it
      for (int ii = kk + 1 + tid; ii < rows; ii += nt) P[ii * ldp + kk] = cmul(P[ii * ldp + kk], inv);
      if (tid == 0) Dp[kk] = d;
      __syncthreads();
      // rank-one update of the panel's remaining columns
      const int rem = w - kk - 1;
      if (rem > 0) {
        const int cnt = (rows - kk - 1) * rem;
        for (int idx = tid; idx < cnt; idx += nt) {
          const int ii = kk + 1 + idx / rem, jj = kk + 1 + idx % rem;
          if (jj > ii) continue;
          const zc t = cmul(cmul(P[ii * ldp + kk], d), P[jj * ldp + kk]);
          P[ii * ldp + jj] = csub(P[ii * ldp + jj], t);
        }
      }
      __syncthreads();
    }
    // write the panel back: multipliers below the diagonal, pivots on it
    for (int idx = tid; idx < rows * w; idx += nt) {
      const int ii = idx / w, kk = idx % w, i = c + ii, k = c + kk;
      if (k <= i && i - k <= b) W[(size_t)i * ldw + (i - k)] = P[ii * ldp + kk];
    }
    // Schur complement of the window below the panel, lower triangle, in
    // 4 x 4 tiles: W(i, jc) -= sum_k l_ik d_k l_jc,k for e <= jc <= i < rend
    const int m = rend - e;
    if (m > 0) {
      const int ntile = (m + 3) / 4;
      const int count = ntile * (ntile + 1) / 2;
      const int o = e - c;  // first window row within the panel
      for (int t = tid; t < count; t += nt) {
        int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        const int tj = t - ti * (ti + 1) / 2;
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
            const int ri = min(o + 4 * ti + u, rows - 1);
            const int rj = min(o + 4 * tj + u, rows - 1);
            a[u] = cmul(P[ri * ldp + kk], dk);
            bv[u] = P[rj * ldp + kk];
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
            const int i = e + 4 * ti + u, jc = e + 4 * tj + v;
            if (i < rend && jc <= i) {
              zc* p = W + (size_t)i * ldw + (i - jc);
              *p = csub(*p, acc[u][v]);
            }
          }
      }
    }
    __syncthreads();
  }
  if (tid == 0) info[j] = 0;
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
  // the largest power of two up to 32 whose panel fits 144 KiB of LDS
  int nb = 32;
  while (nb > 1 && (size_t)(b + nb) * (nb + 1) * sizeof(zc) + nb * sizeof(zc) > 147456) nb /= 2;
  return nb;
}

size_t band_lds_bytes(int b) {
  const int nb = band_panel_width(b);
  return (size_t)(b + nb) * (nb + 1) * sizeof(zc) + nb * sizeof(zc);
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
  hipError_t e = hipFuncSetAttribute((const void*)k_band_factor,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_factor, dim3(nz), dim3(kFactorThreads), lds, st, n, b, nb, W,
                     (size_t)n * (b + 1), info);
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
