// Small dense kernels of the RA-FEAST path, one workgroup each (k <= 192):
//  - CholQR factor: column scaling, Cholesky G = R^T R (shifted when it
//    fails), R^{-1};  Y <- Y diag(1/sqrt(g_ii)) R^{-1} orthonormalises Y
//    (the QR step of Algorithms 1 and 2);
//  - parallel cyclic Jacobi for the reduced eigenproblem of Rayleigh-Ritz;
//  - Phase-1 truncation: keep the m0 Ritz vectors with largest |op| value.
#include "device.h"
#include "kernels.h"

namespace rafeast {

constexpr int kSmallThreads = 1024;
constexpr int kSmallMaxK = 192;

__device__ __forceinline__ int packed_index(int k, int i, int j) {  // i <= j
  return i * k - (i * (i - 1)) / 2 + (j - i);
}

// Sum over an aligned group of 2^lg lanes (lg = 2, 3 or 4, inside a 16-lane
// row), in every lane of the group: the butterfly over lanes l ^ 1, l ^ 2,
// l ^ 4, l ^ 8 as DPP steps.  After the first two steps all lanes of a quad
// hold the same value, so the half-row and row mirrors fetch the values the
// l ^ 4 and l ^ 8 partners hold, and each sum is formed as in the butterfly.
__device__ __forceinline__ double group_sum_f64(double v, int lg) {
  v += dpp_f64(v, 0);
  v += dpp_f64(v, 1);
  if (lg >= 3) v += dpp_f64(v, 2);
  if (lg >= 4) v += dpp_f64(v, 3);
  return v;
}

// ============================================================================
// CholQR factor.  LDS: dsc[k] (column scales) | U (packed upper, k(k+1)/2)
// [| X = U^{-1} (packed upper) when kXInLds].  Right-looking Cholesky with
// one barrier per column: step j reads the unscaled pivot d_j = U[j][j]
// (every thread, so the failure test is uniform), updates the trailing block
// by U[i][l] -= U[j][i] U[j][l] / d_j from the unscaled row j, and scales
// row j-1 (which no thread of step j reads) by 1/sqrt(d_{j-1}).  The inverse
// is built column by column, X[j][j] = 1/U[j][j] and
// X[i][j] = -(sum_{t=i}^{j-1} X[i][t] U[t][j]) / U[j][j], in LDS when it fits
// (else directly in M, global), then its rows are scaled by dsc.
// ============================================================================
template <bool kXInLds>
__global__ __launch_bounds__(kSmallThreads) void k_chol_inv(int k, double shift_unit,
                                                            const double* __restrict__ G,
                                                            int ldg, double* __restrict__ M,
                                                            int ldm, int* __restrict__ flag) {
  extern __shared__ double sm[];
  double* dsc = sm;
  double* U = sm + k;
  double* X = U + (size_t)k * (k + 1) / 2;  // used when kXInLds
  __shared__ int s_fail;
  const int tid = threadIdx.x;
  if (tid == 0) s_fail = 0;
  __syncthreads();
  for (int i = tid; i < k; i += kSmallThreads) {
    const double d = G[(size_t)i * ldg + i];
    if (d > 0.0 && isfinite(d)) {
      dsc[i] = 1.0 / sqrt(d);
    } else {
      dsc[i] = 0.0;
      s_fail = 1;
    }
  }
  __syncthreads();
  int status = 0;
  if (s_fail) {
    status = 2;
  } else {
    for (int attempt = 0; attempt < 2; ++attempt) {
      const double shift = attempt == 0 ? 0.0 : shift_unit;
      for (int e = tid; e < k * k; e += kSmallThreads) {
        const int i = e / k, j = e % k;
        if (j < i) continue;
        double g = 0.5 * (G[(size_t)i * ldg + j] + G[(size_t)j * ldg + i]) * dsc[i] * dsc[j];
        if (i == j) g = 1.0 + shift;  // unit diagonal after scaling
        U[packed_index(k, i, j)] = g;
      }
      __syncthreads();
      bool ok = true;
      for (int j = 0; j < k; ++j) {
        const double d = U[packed_index(k, j, j)];
        if (!(d > 0.0) || !isfinite(d)) {
          ok = false;
          break;
        }
        if (j > 0) {  // finish row j - 1
          const int r = j - 1;
          const double piv = sqrt(U[packed_index(k, r, r)]);
          for (int l = r + 1 + tid; l < k; l += kSmallThreads) U[packed_index(k, r, l)] /= piv;
        }
        const double inv_d = 1.0 / d;
        // trailing block rows ii, columns ll >= ii, on a 32 x 32 thread grid
        const int rj = packed_index(k, j, j);  // U[j][c] = U[rj + c - j]
        for (int ii = j + 1 + (tid >> 5); ii < k; ii += kSmallThreads / 32) {
          const double a = U[rj + ii - j] * inv_d;
          const int ri = packed_index(k, ii, ii);  // U[ii][c] = U[ri + c - ii]
          for (int ll = ii + (tid & 31); ll < k; ll += 32) U[ri + ll - ii] -= a * U[rj + ll - j];
        }
        __syncthreads();
        if (j > 0 && tid == 0) {
          const int r = j - 1;
          U[packed_index(k, r, r)] = sqrt(U[packed_index(k, r, r)]);
        }
      }
      if (ok) {
        // last row: only its diagonal; the previous diagonal write is
        // ordered by this barrier
        if (tid == 0) U[packed_index(k, k - 1, k - 1)] = sqrt(U[packed_index(k, k - 1, k - 1)]);
        __syncthreads();
        status = attempt;
        break;
      }
      status = 2;
      __syncthreads();
    }
  }
  if (status == 2) {
    for (int e = tid; e < k * k; e += kSmallThreads) {
      const int i = e / k, j = e % k;
      M[(size_t)i * ldm + j] = (i == j) ? dsc[i] : 0.0;
    }
    if (tid == 0) *flag = 2;
    return;
  }
  // L lanes of one wave share row i and split the sum (L = 16 for k <= 64,
  // 8 for k <= 128, else 4: L k <= 1024 threads).
  const int lg = k <= 64 ? 4 : (k <= 128 ? 3 : 2);
  const int L = 1 << lg;
  const int i = tid >> lg, qd = tid & (L - 1);
  if constexpr (kXInLds) {
    for (int j = 0; j < k; ++j) {
      const double ujj = U[packed_index(k, j, j)];
      double part = 0.0;
      if (i < j) {
        for (int t = i + qd; t < j; t += L)
          part += X[packed_index(k, i, t)] * U[packed_index(k, t, j)];
      }
      part = group_sum_f64(part, lg);
      if (i < j && qd == 0) X[packed_index(k, i, j)] = -part / ujj;
      if (tid == kSmallThreads - 1) X[packed_index(k, j, j)] = 1.0 / ujj;
      __syncthreads();
    }
    for (int e = tid; e < k * k; e += kSmallThreads) {
      const int r = e / k, c = e % k;
      M[(size_t)r * ldm + c] = c >= r ? X[packed_index(k, r, c)] * dsc[r] : 0.0;
    }
  } else {
    for (int e = tid; e < k * k; e += kSmallThreads) {
      const int r = e / k, c = e % k;
      if (c < r) M[(size_t)r * ldm + c] = 0.0;
    }
    for (int j = 0; j < k; ++j) {
      const double ujj = U[packed_index(k, j, j)];
      double part = 0.0;
      if (i < j) {
        for (int t = i + qd; t < j; t += L)
          part += M[(size_t)i * ldm + t] * U[packed_index(k, t, j)];
      }
      part = group_sum_f64(part, lg);
      if (i < j && qd == 0) M[(size_t)i * ldm + j] = -part / ujj;
      if (tid == kSmallThreads - 1) M[(size_t)j * ldm + j] = 1.0 / ujj;
      __syncthreads();
    }
    for (int e = tid; e < k * k; e += kSmallThreads) {
      const int r = e / k, c = e % k;
      if (c >= r) M[(size_t)r * ldm + c] *= dsc[r];
    }
  }
  if (tid == 0) *flag = status;
}

// Dynamic LDS budget of the one-workgroup kernels (the static arrays of
// k_jacobi take under 8 KB of the 160 KB).
constexpr size_t kSmallLdsMax = 160 * 1024 - 8192;

hipError_t launch_chol_inv(hipStream_t st, int k, int64_t nrows, const double* G, int ldg,
                           double* M, int ldm, int* flag) {
  if (k < 1 || k > kSmallMaxK) return hipErrorInvalidValue;
  // Shifted CholQR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020):
  // s = 11 (m n + n (n+1)) u ||X||_2^2 with ||X||_2^2 <= trace(G) = k after scaling.
  const double u = 0x1.0p-53;
  const double shift = 11.0 * ((double)nrows * k + (double)k * (k + 1)) * u * (double)k;
  const size_t base = sizeof(double) * ((size_t)k + (size_t)k * (k + 1) / 2);
  const size_t with_x = base + sizeof(double) * (size_t)k * (k + 1) / 2;
  const bool x_lds = with_x <= kSmallLdsMax;
  const size_t lds = x_lds ? with_x : base;
  const void* fn = x_lds ? (const void*)k_chol_inv<true> : (const void*)k_chol_inv<false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (x_lds)
    hipLaunchKernelGGL(k_chol_inv<true>, dim3(1), dim3(kSmallThreads), lds, st, k, shift, G, ldg,
                       M, ldm, flag);
  else
    hipLaunchKernelGGL(k_chol_inv<false>, dim3(1), dim3(kSmallThreads), lds, st, k, shift, G, ldg,
                       M, ldm, flag);
  return hipGetLastError();
}

// ============================================================================
// Parallel cyclic Jacobi (round-robin pairing).  Each round rotates k/2
// disjoint pairs (p, q) at once: the rotation J (J_pp = J_qq = c, J_pq = s,
// J_qp = -s) zeroing H_pq follows Golub & Van Loan, Alg. 8.5.1.  H <- J^T H J
// is applied per (row pair, column pair) 2x2 block, each block by one thread,
// and V <- V J per (row, pair).  H lives in LDS for k <= 128, else in global
// workspace; V lives in LDS too when both fit, else in global workspace.
// ============================================================================
template <bool kHInLds, bool kVInLds>
__global__ __launch_bounds__(kSmallThreads) void k_jacobi(int k, const double* __restrict__ Hin,
                                                          int ldh, double* __restrict__ theta,
                                                          double* __restrict__ S, int lds,
                                                          double* __restrict__ work) {
  extern __shared__ double sh_h[];
  __shared__ int rp[kSmallMaxK / 2 + 1], rq[kSmallMaxK / 2 + 1], perm[kSmallMaxK];
  __shared__ double rc[kSmallMaxK / 2 + 1], rs[kSmallMaxK / 2 + 1], dg[kSmallMaxK];
  __shared__ double red[2][kSmallThreads / 64];
  // In LDS, H and V rows are k | 1 doubles apart (an odd stride): the rows a
  // wave touches in one access then start in different banks.
  const int hs = kHInLds ? (k | 1) : k, vs = kVInLds ? (k | 1) : k;
  double* H = kHInLds ? sh_h : work;
  double* V = kVInLds ? sh_h + (size_t)k * hs : work + (size_t)k * k;
  const int tid = threadIdx.x;
  for (int e = tid; e < k * k; e += kSmallThreads) {
    const int i = e / k, j = e % k;
    H[i * hs + j] = 0.5 * (Hin[(size_t)i * ldh + j] + Hin[(size_t)j * ldh + i]);
    V[i * vs + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kk = k + (k & 1);
  const int np = kk / 2;
  const int players = kk - 1;  // the last player stays fixed
  const float inv_np = 1.0f / (float)np;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test on the off-diagonal mass
    double off = 0.0, tot = 0.0;
    for (int i = tid >> 5; i < k; i += kSmallThreads / 32)
      for (int j = tid & 31; j < k; j += 32) {
        const double h = H[i * hs + j];
        tot += h * h;
        if (i != j) off += h * h;
      }
    off = wave_sum(off);
    tot = wave_sum(tot);
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = off;
      red[1][tid >> 6] = tot;
    }
    __syncthreads();
    off = 0.0;
    tot = 0.0;
    for (int w = 0; w < kSmallThreads / 64; ++w) {
      off += red[0][w];
      tot += red[1][w];
    }
    __syncthreads();
    // converged once the off-diagonal mass is at the rounding floor: each
    // of the k (k - 1) off-diagonal entries is then a few units of roundoff
    // of the diagonal, so off / tot ~ k u^2; 64 k u^2 leaves a margin of 8 u
    // per entry (u = 2^-53)
    if (k == 1 || off <= 64.0 * k * 0x1.0p-106 * tot) break;
    for (int r = 0; r < players; ++r) {
      for (int t = tid; t < np; t += kSmallThreads) {
        int p, q;
        if (t == 0) {
          p = r;
          q = kk - 1;
        } else {
          p = (r + t) % players;
          q = (r - t + players) % players;
        }
        double c = 1.0, s = 0.0;
        if (p < k && q < k) {
          const double apq = H[p * hs + q];
          if (fabs(apq) >= 0x1.0p-1000) {
            // this phase is one wave's latency per round: reciprocals and
            // square roots from Newton-refined hardware estimates (a few ulp;
            // the rotation stays orthogonal to working precision)
            const double tau = (H[q * hs + q] - H[p * hs + p]) * rcp_nr(2.0 * apq);
            double tt;
            if (fabs(tau) > 1e150) {
              tt = 0.5 / tau;
            } else {
              const double w = fma(tau, tau, 1.0);
              tt = (tau >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(tau) + w * rsq_nr(w));
            }
            c = rsq_nr(fma(tt, tt, 1.0));
            s = tt * c;
          } else if (apq != 0.0) {
            const double tau = (H[q * hs + q] - H[p * hs + p]) / (2.0 * apq);
            const double tt = fabs(tau) > 1e150 ? 0.5 / tau
                              : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        rp[t] = p;
        rq[t] = q;
        rc[t] = c;
        rs[t] = s;
      }
      __syncthreads();
      for (int b = tid; b < np * np; b += kSmallThreads) {
        // b / np in float: exact for b, e < 2^15 and np <= 96
        const int t1 = (int)(((float)b + 0.5f) * inv_np), t2 = b - t1 * np;
        const int p1 = rp[t1], q1 = rq[t1], p2 = rp[t2], q2 = rq[t2];
        const double c1 = rc[t1], s1 = rs[t1], c2 = rc[t2], s2 = rs[t2];
        const bool v_p1 = p1 < k, v_q1 = q1 < k, v_p2 = p2 < k, v_q2 = q2 < k;
        const double h00 = (v_p1 && v_p2) ? H[p1 * hs + p2] : 0.0;
        const double h01 = (v_p1 && v_q2) ? H[p1 * hs + q2] : 0.0;
        const double h10 = (v_q1 && v_p2) ? H[q1 * hs + p2] : 0.0;
        const double h11 = (v_q1 && v_q2) ? H[q1 * hs + q2] : 0.0;
        // rows: J^T
        const double g00 = c1 * h00 - s1 * h10, g01 = c1 * h01 - s1 * h11;
        const double g10 = s1 * h00 + c1 * h10, g11 = s1 * h01 + c1 * h11;
        // columns: J
        const double f00 = c2 * g00 - s2 * g01, f01 = s2 * g00 + c2 * g01;
        const double f10 = c2 * g10 - s2 * g11, f11 = s2 * g10 + c2 * g11;
        if (v_p1 && v_p2) H[p1 * hs + p2] = f00;
        if (v_p1 && v_q2) H[p1 * hs + q2] = f01;
        if (v_q1 && v_p2) H[q1 * hs + p2] = f10;
        if (v_q1 && v_q2) H[q1 * hs + q2] = f11;
      }
      for (int e = tid; e < k * np; e += kSmallThreads) {
        const int row = (int)(((float)e + 0.5f) * inv_np), t = e - row * np;
        const int p = rp[t], q = rq[t];
        if (p < k && q < k) {
          const double c = rc[t], s = rs[t];
          const double vp = V[row * vs + p], vq = V[row * vs + q];
          V[row * vs + p] = c * vp - s * vq;
          V[row * vs + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < k; i += kSmallThreads) dg[i] = H[i * hs + i];
  __syncthreads();
  for (int i = tid; i < k; i += kSmallThreads) {
    const double d = dg[i];
    int rank = 0;
    for (int j = 0; j < k; ++j) rank += (dg[j] < d) || (dg[j] == d && j < i);
    theta[rank] = d;
    perm[rank] = i;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += kSmallThreads) {
    const int row = e / k, c = e % k;
    S[(size_t)row * lds + c] = V[row * vs + perm[c]];
  }
}

hipError_t launch_jacobi(hipStream_t st, int k, const double* H, int ldh, double* theta,
                         double* S, int lds, double* work) {
  if (k < 1 || k > kSmallMaxK) return hipErrorInvalidValue;
  // H (and V) in LDS with rows k | 1 doubles apart
  const size_t hb = sizeof(double) * (size_t)k * (size_t)(k | 1);
  if (2 * hb <= kSmallLdsMax) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jacobi<true, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * hb));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_jacobi<true, true>), dim3(1), dim3(kSmallThreads), 2 * hb, st, k, H,
                       ldh, theta, S, lds, work);
  } else if (k <= 128) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jacobi<true, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)hb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_jacobi<true, false>), dim3(1), dim3(kSmallThreads), hb, st, k, H, ldh,
                       theta, S, lds, work);
  } else {
    hipLaunchKernelGGL((k_jacobi<false, false>), dim3(1), dim3(kSmallThreads), 0, st, k, H, ldh,
                       theta, S, lds, work);
  }
  return hipGetLastError();
}

// ============================================================================
// Phase-1 truncation: f_i = |a + b theta_i + c theta_i^2| is the op-value of
// Ritz value theta_i; keep the m0 largest (ties to the lower index), in
// ascending-theta order.
// ============================================================================
__global__ __launch_bounds__(256) void k_select(int k, int m0, const double* __restrict__ theta,
                                                const double* __restrict__ S, int lds, double a,
                                                double b, double c, double* __restrict__ Ssel,
                                                double* __restrict__ info) {
  __shared__ double f[kSmallMaxK];
  __shared__ int rank[kSmallMaxK], pos[kSmallMaxK];
  const int tid = threadIdx.x;
  for (int i = tid; i < k; i += 256) {
    const double t = theta[i];
    f[i] = fabs(a + b * t + c * t * t);
  }
  __syncthreads();
  for (int i = tid; i < k; i += 256) {
    int r = 0;
    for (int j = 0; j < k; ++j) r += (f[j] > f[i]) || (f[j] == f[i] && j < i);
    rank[i] = r;
  }
  __syncthreads();
  for (int i = tid; i < k; i += 256) {
    int ps = 0;
    for (int j = 0; j < i; ++j) ps += rank[j] < m0;
    pos[i] = rank[i] < m0 ? ps : -1;
    if (rank[i] == m0 - 1) info[0] = f[i];
    if (rank[i] == m0) info[1] = f[i];
  }
  if (tid == 0 && k <= m0) info[1] = __builtin_nan("");
  __syncthreads();
  for (int e = tid; e < k * k; e += 256) {
    const int row = e / k, i = e % k;
    if (pos[i] >= 0) Ssel[(size_t)row * m0 + pos[i]] = S[(size_t)row * lds + i];
  }
}

hipError_t launch_select(hipStream_t st, int k, int m0, const double* theta, const double* S,
                         int lds, double a, double b, double c, double* Ssel, double* info) {
  if (k < 1 || k > kSmallMaxK || m0 > k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_select, dim3(1), dim3(256), 0, st, k, m0, theta, S, lds, a, b, c, Ssel,
                     info);
  return hipGetLastError();
}

}  // namespace rafeast
