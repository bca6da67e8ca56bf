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

// ============================================================================
// CholQR factor.  LDS: dsc[k] (column scales) | U (packed upper, k(k+1)/2).
// The inverse X = U^{-1} is built column by column directly in M (global,
// visible across the workgroup after each barrier), then rows scaled by dsc.
// ============================================================================
__global__ __launch_bounds__(kSmallThreads) void k_chol_inv(int k, double shift_unit,
                                                            const double* __restrict__ G,
                                                            int ldg, double* __restrict__ M,
                                                            int ldm, int* __restrict__ flag) {
  extern __shared__ double sm[];
  double* dsc = sm;
  double* U = sm + k;
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
      for (int j = 0; j < k; ++j) {
        if (tid == 0) {
          const double d = U[packed_index(k, j, j)];
          if (!(d > 0.0) || !isfinite(d))
            s_fail = 1;
          else
            U[packed_index(k, j, j)] = sqrt(d);
        }
        __syncthreads();
        if (s_fail) break;
        const double piv = U[packed_index(k, j, j)];
        for (int l = j + 1 + tid; l < k; l += kSmallThreads) U[packed_index(k, j, l)] /= piv;
        __syncthreads();
        const int m = k - 1 - j;
        for (int e = tid; e < m * m; e += kSmallThreads) {
          const int ii = j + 1 + e / m, ll = j + 1 + e % m;
          if (ll < ii) continue;
          U[packed_index(k, ii, ll)] -= U[packed_index(k, j, ii)] * U[packed_index(k, j, ll)];
        }
        __syncthreads();
      }
      if (!s_fail) {
        status = attempt;
        break;
      }
      status = 2;
      __syncthreads();
      if (tid == 0) s_fail = 0;
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
  // X = U^{-1}, column j: X[j][j] = 1/U[j][j];
  // X[i][j] = -(sum_{t=i}^{j-1} X[i][t] U[t][j]) / U[j][j] for i < j.
  // Four lanes of one wave share row i and split the sum.
  for (int e = tid; e < k * k; e += kSmallThreads) {
    const int i = e / k, j = e % k;
    if (j < i) M[(size_t)i * ldm + j] = 0.0;
  }
  for (int j = 0; j < k; ++j) {
    const double ujj = U[packed_index(k, j, j)];
    const int i = tid >> 2, qd = tid & 3;
    double part = 0.0;
    if (i < j) {
      for (int t = i + qd; t < j; t += 4)
        part += M[(size_t)i * ldm + t] * U[packed_index(k, t, j)];
    }
    part += __shfl_xor(part, 1, 64);
    part += __shfl_xor(part, 2, 64);
    if (i < j && qd == 0) M[(size_t)i * ldm + j] = -part / ujj;
    if (tid == kSmallThreads - 1) M[(size_t)j * ldm + j] = 1.0 / ujj;
    __syncthreads();
  }
  for (int e = tid; e < k * k; e += kSmallThreads) {
    const int i = e / k, j = e % k;
    if (j >= i) M[(size_t)i * ldm + j] *= dsc[i];
  }
  if (tid == 0) *flag = status;
}

hipError_t launch_chol_inv(hipStream_t st, int k, int64_t nrows, const double* G, int ldg,
                           double* M, int ldm, int* flag) {
  if (k < 1 || k > kSmallMaxK) return hipErrorInvalidValue;
  // Shifted CholQR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020):
  // s = 11 (m n + n (n+1)) u ||X||_2^2 with ||X||_2^2 <= trace(G) = k after scaling.
  const double u = 0x1.0p-53;
  const double shift = 11.0 * ((double)nrows * k + (double)k * (k + 1)) * u * (double)k;
  const size_t lds = sizeof(double) * ((size_t)k + (size_t)k * (k + 1) / 2);
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_inv,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kSmallThreads), lds, st, k, shift, G, ldg, M, ldm,
                     flag);
  return hipGetLastError();
}

// ============================================================================
// Parallel cyclic Jacobi (round-robin pairing).  Each round rotates k/2
// disjoint pairs (p, q) at once: the rotation J (J_pp = J_qq = c, J_pq = s,
// J_qp = -s) zeroing H_pq follows Golub & Van Loan, Alg. 8.5.1.  H <- J^T H J
// is applied per (row pair, column pair) 2x2 block, each block by one thread,
// and V <- V J per (row, pair).  H lives in LDS for k <= 128, else in global
// workspace; V is in global workspace.
// ============================================================================
template <bool kHInLds>
__global__ __launch_bounds__(kSmallThreads) void k_jacobi(int k, const double* __restrict__ Hin,
                                                          int ldh, double* __restrict__ theta,
                                                          double* __restrict__ S, int lds,
                                                          double* __restrict__ work) {
  extern __shared__ double sh_h[];
  __shared__ int rp[kSmallMaxK / 2 + 1], rq[kSmallMaxK / 2 + 1], perm[kSmallMaxK];
  __shared__ double rc[kSmallMaxK / 2 + 1], rs[kSmallMaxK / 2 + 1], dg[kSmallMaxK];
  __shared__ double red[2][kSmallThreads / 64];
  double* H = kHInLds ? sh_h : work;
  double* V = work + (size_t)k * k;
  const int tid = threadIdx.x;
  for (int e = tid; e < k * k; e += kSmallThreads) {
    const int i = e / k, j = e % k;
    H[e] = 0.5 * (Hin[(size_t)i * ldh + j] + Hin[(size_t)j * ldh + i]);
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kk = k + (k & 1);
  const int np = kk / 2;
  const int players = kk - 1;  // the last player stays fixed
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test on the off-diagonal mass
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < k * k; e += kSmallThreads) {
      const double h = H[e];
      tot += h * h;
      if (e / k != e % k) off += h * h;
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
    if (k == 1 || off <= 1e-30 * tot) break;
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
          const double apq = H[p * k + q];
          if (apq != 0.0) {
            const double tau = (H[q * k + q] - H[p * k + p]) / (2.0 * apq);
            double tt;
            if (fabs(tau) > 1e150)
              tt = 0.5 / tau;
            else
              tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
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
        const int t1 = b / np, t2 = b % np;
        const int p1 = rp[t1], q1 = rq[t1], p2 = rp[t2], q2 = rq[t2];
        const double c1 = rc[t1], s1 = rs[t1], c2 = rc[t2], s2 = rs[t2];
        const bool v_p1 = p1 < k, v_q1 = q1 < k, v_p2 = p2 < k, v_q2 = q2 < k;
        const double h00 = (v_p1 && v_p2) ? H[p1 * k + p2] : 0.0;
        const double h01 = (v_p1 && v_q2) ? H[p1 * k + q2] : 0.0;
        const double h10 = (v_q1 && v_p2) ? H[q1 * k + p2] : 0.0;
        const double h11 = (v_q1 && v_q2) ? H[q1 * k + q2] : 0.0;
        // rows: J^T
        const double g00 = c1 * h00 - s1 * h10, g01 = c1 * h01 - s1 * h11;
        const double g10 = s1 * h00 + c1 * h10, g11 = s1 * h01 + c1 * h11;
        // columns: J
        const double f00 = c2 * g00 - s2 * g01, f01 = s2 * g00 + c2 * g01;
        const double f10 = c2 * g10 - s2 * g11, f11 = s2 * g10 + c2 * g11;
        if (v_p1 && v_p2) H[p1 * k + p2] = f00;
        if (v_p1 && v_q2) H[p1 * k + q2] = f01;
        if (v_q1 && v_p2) H[q1 * k + p2] = f10;
        if (v_q1 && v_q2) H[q1 * k + q2] = f11;
      }
      for (int e = tid; e < k * np; e += kSmallThreads) {
        const int row = e / np, t = e % np;
        const int p = rp[t], q = rq[t];
        if (p < k && q < k) {
          const double c = rc[t], s = rs[t];
          const double vp = V[row * k + p], vq = V[row * k + q];
          V[row * k + p] = c * vp - s * vq;
          V[row * k + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < k; i += kSmallThreads) dg[i] = H[i * k + i];
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
    S[(size_t)row * lds + c] = V[row * k + perm[c]];
  }
}

hipError_t launch_jacobi(hipStream_t st, int k, const double* H, int ldh, double* theta,
                         double* S, int lds, double* work) {
  if (k < 1 || k > kSmallMaxK) return hipErrorInvalidValue;
  if (k <= 128) {
    const size_t bytes = sizeof(double) * (size_t)k * k;
    hipError_t e = hipFuncSetAttribute((const void*)k_jacobi<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_jacobi<true>, dim3(1), dim3(kSmallThreads), bytes, st, k, H, ldh, theta,
                       S, lds, work);
  } else {
    hipLaunchKernelGGL(k_jacobi<false>, dim3(1), dim3(kSmallThreads), 0, st, k, H, ldh, theta, S,
                       lds, work);
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
