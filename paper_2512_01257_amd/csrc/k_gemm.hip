// Products with the dense operators of the statistical workloads (Section 4):
// kernel PCA, A = K (symmetric n x n); sample covariance, A = scale Xd^T Xd
// with the centred data Xd (rows x n).  Every product is one GEMM form,
//   C (M x N, row-major) = alpha op(A) B + beta C,
// run on the matrix cores: v_mfma_f64_16x16x4f64 in FP64 and
// v_mfma_f32_16x16x4f32 in FP32.
//
// Tiling: a 256-thread workgroup owns a 128 x 32 TN tile of C; its four
// waves own 64 x 16 TN quarters, 4 x TN MFMA tiles of 16 x 16 each, so every
// operand fragment read from LDS feeds several MFMAs (TN = 4 in FP32, 2 in
// FP64).  The inner dimension advances in
// steps of 16: the step's A (128 x 16) and B (16 x 128) panels are staged in
// LDS (two buffers; the next step's global loads are issued before the
// current step's MFMAs and stored after them, one barrier per step).  A may
// be stored by rows or by columns (op(A)(i, k) at A[i lda + k] or
// A[k lda + i]); B and C by rows.  Products with a long inner dimension and
// few output tiles are split into chunks of the inner dimension (grid.z), each
// chunk's product written to a slab of a workspace, and the slabs summed in
// chunk order by a second kernel: no atomics, the same sums every run.
#include "device.h"
#include "kernels.h"

namespace rafeast {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kBM = 128, kGT = 256;
#ifndef RAFEAST_GEMM_BK32
#define RAFEAST_GEMM_BK32 32
#endif
#ifndef RAFEAST_GEMM_BK64
#define RAFEAST_GEMM_BK64 16
#endif
#ifndef RAFEAST_GEMM_TN64
#define RAFEAST_GEMM_TN64 2
#endif
#ifndef RAFEAST_GEMM_TN32
#define RAFEAST_GEMM_TN32 4
#endif
#ifndef RAFEAST_GEMM_XCD
#define RAFEAST_GEMM_XCD 1
#endif
#ifndef RAFEAST_GEMM_VEC_BYTES
#define RAFEAST_GEMM_VEC_BYTES 16
#endif
constexpr int kGemmVecBytes = RAFEAST_GEMM_VEC_BYTES;  // bytes per vector load

// MFMA operand layout (lane l of the wave):
//   A (16 x 4): A[l % 16][l / 16]     B (4 x 16): B[l / 16][l % 16]
//   D (16 x 16): register v of lane l holds D[row(l, v)][l % 16]
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef v4d Acc;
  static __device__ __forceinline__ Acc step(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef v4f Acc;
  static __device__ __forceinline__ Acc step(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// ACOL: op(A)(i, k) = A[k lda + i] (else A[i lda + k]).  BK: inner indices
// per LDS step.  VEC: elements per global load along each operand's
// contiguous dimension (the host takes VEC > 1 only when the operands'
// addresses and leading dimensions are multiples of VEC elements).  part != nullptr:
// chunk z covers inner indices [z kc, min(K, (z + 1) kc)) and its
// raw product goes to part + z M N (row-major, ld N); otherwise C is written.
template <typename T, bool ACOL, int BK, int VEC, int TN>
__global__ __launch_bounds__(kGT) void k_gemm(int M, int N, int K, int kc,
                                              const T* __restrict__ A, int64_t lda,
                                              const T* __restrict__ B, int64_t ldb,
                                              T* __restrict__ C, int64_t ldc, T alpha, T beta,
                                              T* __restrict__ part) {
  // rows padded by one element: the transposing stores of a row-major A
  // spread over the banks
  constexpr int BN = 32 * TN;                   // block tile width
  __shared__ T As[2][BK][kBM + 1];
  __shared__ T Bs[2][BK][BN + 1];
  typedef typename Mfma<T>::Acc Acc;
  constexpr int NVA = kBM * BK / (kGT * VEC);  // vectors per thread: A panel
  constexpr int NVB = BN * BK / (kGT * VEC);   // and B panel
  constexpr int CA = ACOL ? kBM : BK;          // A panel: contiguous length
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // Workgroups go to the eight XCDs in turn (linear id b to XCD b mod 8).
  // With a grid of a multiple of eight workgroups, XCD x takes the x-th
  // contiguous eighth of the tiles in (chunk, row tile, column tile) order,
  // so the workgroups that share an A row panel or a chunk share one L2.
  const int gx = gridDim.x, gy = gridDim.y;
  const int G = gx * gy * (int)gridDim.z;
  const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int l = (RAFEAST_GEMM_XCD && G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int tn = l % gx, tm = (l / gx) % gy, tz = l / (gx * gy);
  const int i0 = tm * kBM, j0 = tn * BN;
  const int kbeg = tz * kc;
  const int kend = min(K, kbeg + kc);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

  T ra[NVA][VEC], rb[NVB][VEC];
  Acc acc[4][TN];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < TN; ++nt) acc[mt][nt] = Acc{T(0), T(0), T(0), T(0)};

  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NVA; ++q) {
      const int e = (tid + q * kGT) * VEC;
      const int ca = e % CA, oa = e / CA;
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        if (ACOL)
          As[buf][oa][ca + u] = ra[q][u];
        else
          As[buf][ca + u][oa] = ra[q][u];
      }
    }
#pragma unroll
    for (int q = 0; q < NVB; ++q) {
      const int e = (tid + q * kGT) * VEC;
#pragma unroll
      for (int u = 0; u < VEC; ++u) Bs[buf][e / BN][e % BN + u] = rb[q][u];
    }
  };
  const int fr = lane >> 4, fc = lane & 15;
  // The fragments of sub-step ks + 4 are read from LDS while the MFMAs of
  // sub-step ks issue (two register sets), so LDS latency overlaps the
  // matrix work.
  auto mfma_step = [&](int cur) {
    T a[2][4], b[2][TN];
    auto frag = [&](int set, int ks) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) a[set][mt] = As[cur][ks + fr][wm * 64 + mt * 16 + fc];
#pragma unroll
      for (int nt = 0; nt < TN; ++nt) b[set][nt] = Bs[cur][ks + fr][wn * 16 * TN + nt * 16 + fc];
    };
    frag(0, 0);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int set = (ks / 4) & 1;
      if (ks + 4 < BK) frag(set ^ 1, ks + 4);
      // keep the look-ahead reads ahead of this sub-step's MFMAs
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < TN; ++nt)
          acc[mt][nt] = Mfma<T>::step(a[set][mt], b[set][nt], acc[mt][nt]);
    }
  };

  // The fast path needs whole steps of the inner dimension.  Rows of op(A)
  // past M and columns of B past N feed only outputs that are never stored,
  // so a vector that starts past the edge is simply read from the tile's
  // first row or column instead; a vector may not straddle the edge (M, N a
  // multiple of VEC when the tile is cut there).
  const bool a_fast = !ACOL || i0 + kBM <= M || M % VEC == 0;
  const bool b_fast = j0 + BN <= N || N % VEC == 0;
  if (a_fast && b_fast && (kend - kbeg) % BK == 0) {
    // Per-thread operand pointers advanced by one step each time,
    // whole-vector loads, no bounds tests in the loop.
    typedef T VT __attribute__((ext_vector_type(VEC)));
    const T* pa[NVA];
    const T* pb[NVB];
#pragma unroll
    for (int q = 0; q < NVA; ++q) {
      const int e = (tid + q * kGT) * VEC;
      const int ca = e % CA, oa = e / CA;
      int gi = i0 + (ACOL ? ca : oa);
      if (gi >= M) gi = i0;
      pa[q] = ACOL ? A + (int64_t)(kbeg + oa) * lda + gi : A + (int64_t)gi * lda + (kbeg + ca);
    }
#pragma unroll
    for (int q = 0; q < NVB; ++q) {
      const int e = (tid + q * kGT) * VEC;
      int gj = j0 + e % BN;
      if (gj >= N) gj = j0;
      pb[q] = B + (int64_t)(kbeg + e / BN) * ldb + gj;
    }
    const int64_t da = ACOL ? (int64_t)BK * lda : BK, db = (int64_t)BK * ldb;
    auto load = [&]() {
#pragma unroll
      for (int q = 0; q < NVA; ++q) {
        const VT va = *reinterpret_cast<const VT*>(pa[q]);
#pragma unroll
        for (int u = 0; u < VEC; ++u) ra[q][u] = va[u];
        pa[q] += da;
      }
#pragma unroll
      for (int q = 0; q < NVB; ++q) {
        const VT vb = *reinterpret_cast<const VT*>(pb[q]);
#pragma unroll
        for (int u = 0; u < VEC; ++u) rb[q][u] = vb[u];
        pb[q] += db;
      }
    };
    if (nk > 0) {
      load();
      store(0);
    }
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
      const int cur = t & 1;
      if (t + 1 < nk) load();
      mfma_step(cur);
      if (t + 1 < nk) store(cur ^ 1);
      __syncthreads();
    }
  } else {
    // Other edge tiles: element loads from addresses clamped into the
    // matrix, the elements outside it zeroed.
    auto load = [&](int k0) {
#pragma unroll
      for (int q = 0; q < NVA; ++q) {
        const int e = (tid + q * kGT) * VEC;
        const int ca = e % CA, oa = e / CA;
#pragma unroll
        for (int u = 0; u < VEC; ++u) {
          const int gi = i0 + (ACOL ? ca + u : oa), gk = k0 + (ACOL ? oa : ca + u);
          const int ci = min(gi, M - 1), ck = min(gk, kend - 1);
          const T va = A[ACOL ? (int64_t)ck * lda + ci : (int64_t)ci * lda + ck];
          ra[q][u] = (gi < M && gk < kend) ? va : T(0);
        }
      }
#pragma unroll
      for (int q = 0; q < NVB; ++q) {
        const int e = (tid + q * kGT) * VEC;
#pragma unroll
        for (int u = 0; u < VEC; ++u) {
          const int gj = j0 + e % BN + u, gb = k0 + e / BN;
          const int cj = min(gj, N - 1), cb = min(gb, kend - 1);
          const T vb = B[(int64_t)cb * ldb + cj];
          rb[q][u] = (gj < N && gb < kend) ? vb : T(0);
        }
      }
    };
    if (nk > 0) {
      load(kbeg);
      store(0);
    }
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
      const int cur = t & 1;
      if (t + 1 < nk) load(kbeg + (t + 1) * BK);
      mfma_step(cur);
      if (t + 1 < nk) store(cur ^ 1);
      __syncthreads();
    }
  }

  T* __restrict__ slab = part ? part + (size_t)tz * (size_t)M * N : nullptr;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < TN; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wm * 64 + mt * 16 + Mfma<T>::row(lane, v);
        const int gj = j0 + wn * 16 * TN + nt * 16 + fc;
        if (gi >= M || gj >= N) continue;
        if (slab) {
          slab[(size_t)gi * N + gj] = acc[mt][nt][v];
        } else {
          T c = alpha * acc[mt][nt][v];
          if (beta != T(0)) c += beta * C[(int64_t)gi * ldc + gj];
          C[(int64_t)gi * ldc + gj] = c;
        }
      }
}

// C = alpha sum_z slab_z + beta C, slabs in chunk order.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_reduce(int M, int N, int S,
                                                     const T* __restrict__ part,
                                                     T* __restrict__ C, int64_t ldc, T alpha,
                                                     T beta) {
  const int64_t MN = (int64_t)M * N;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= MN) return;
  T s = T(0);
  for (int z = 0; z < S; ++z) s += part[(size_t)z * MN + e];
  const int64_t i = e / N, j = e % N;
  T c = alpha * s;
  if (beta != T(0)) c += beta * C[i * ldc + j];
  C[i * ldc + j] = c;
}

__global__ __launch_bounds__(256) void k_axpy(int64_t count, double a, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) y[e] += a * x[e];
}

template <typename T, int BK, int TN>
hipError_t launch_tiles(hipStream_t st, bool acol, bool vec, dim3 grid, int M, int N, int K,
                        int kc, const T* A, int64_t lda, const T* B, int64_t ldb, T* C,
                        int64_t ldc, T alpha, T beta, T* part) {
  constexpr int V = kGemmVecBytes / (int)sizeof(T) > 0 ? kGemmVecBytes / (int)sizeof(T) : 1;
  if (acol && vec)
    hipLaunchKernelGGL((k_gemm<T, true, BK, V, TN>), grid, dim3(kGT), 0, st, M, N, K, kc, A, lda,
                       B, ldb, C, ldc, alpha, beta, part);
  else if (acol)
    hipLaunchKernelGGL((k_gemm<T, true, BK, 1, TN>), grid, dim3(kGT), 0, st, M, N, K, kc, A, lda,
                       B, ldb, C, ldc, alpha, beta, part);
  else if (vec)
    hipLaunchKernelGGL((k_gemm<T, false, BK, V, TN>), grid, dim3(kGT), 0, st, M, N, K, kc, A,
                       lda, B, ldb, C, ldc, alpha, beta, part);
  else
    hipLaunchKernelGGL((k_gemm<T, false, BK, 1, TN>), grid, dim3(kGT), 0, st, M, N, K, kc, A,
                       lda, B, ldb, C, ldc, alpha, beta, part);
  return hipGetLastError();
}

// C = alpha op(A) B + beta C.  work (nullable, work_elems elements) holds the
// chunk slabs: the inner dimension is split when the output has fewer tiles
// than two per CU and the chunks stay at least 512 long.
template <typename T>
hipError_t gemm(hipStream_t st, bool acol, int M, int N, int K, const T* A, int64_t lda,
                const T* B, int64_t ldb, T* C, int64_t ldc, T alpha, T beta, T* work,
                size_t work_elems) {
  if (M <= 0 || N <= 0) return hipSuccess;
  // MFMA column tiles per wave: up to four in FP32 (128-wide blocks), up to
  // two in FP64 (64-wide blocks: half the accumulators, so two waves fit a
  // SIMD); narrow products (the few live columns at the end of a solve) take
  // one or two, so a block does not compute many columns it throws away
  constexpr int TNmax = sizeof(T) == 8 ? RAFEAST_GEMM_TN64 : RAFEAST_GEMM_TN32;
  const int TN = N <= 32 ? 1 : (N <= 64 || TNmax == 2) ? 2 : 4;
  const int BN = 32 * TN;
  // inner indices per LDS step (FP64: 16, so that the staging buffers leave
  // room for two workgroups per CU)
  constexpr int BK = sizeof(T) == 8 ? RAFEAST_GEMM_BK64 : RAFEAST_GEMM_BK32;
  const int tiles = ((M + kBM - 1) / kBM) * ((N + BN - 1) / BN);
  int S = 1;
  if (work && K >= 1024) {
    const int want = (512 + tiles - 1) / tiles;
    const int by_len = K / 512;
    const int by_room = (int)std::min<size_t>(work_elems / ((size_t)M * N), 64);
    S = std::max(1, std::min(want, std::min(by_len, by_room)));
  }
  int kc = (K + S - 1) / S;
  kc = (kc + BK - 1) / BK * BK;
  if (K <= 0) kc = BK;
  S = K > 0 ? (K + kc - 1) / kc : 1;
  T* part = S > 1 ? work : nullptr;
  dim3 grid((N + BN - 1) / BN, (M + kBM - 1) / kBM, S);
  // vector loads when every operand row starts on a vector boundary
  constexpr int V = kGemmVecBytes / (int)sizeof(T) > 0 ? kGemmVecBytes / (int)sizeof(T) : 1;
  const bool vec = V > 1 && lda % V == 0 && ldb % V == 0 &&
                   reinterpret_cast<uintptr_t>(A) % (V * sizeof(T)) == 0 &&
                   reinterpret_cast<uintptr_t>(B) % (V * sizeof(T)) == 0;
  hipError_t e;
  if (TN == 1)
    e = launch_tiles<T, BK, 1>(st, acol, vec, grid, M, N, K, kc, A, lda, B, ldb, C, ldc, alpha,
                               beta, part);
  else if (TN == 2)
    e = launch_tiles<T, BK, 2>(st, acol, vec, grid, M, N, K, kc, A, lda, B, ldb, C, ldc, alpha,
                               beta, part);
  else
    e = launch_tiles<T, BK, TNmax>(st, acol, vec, grid, M, N, K, kc, A, lda, B, ldb, C, ldc,
                                   alpha, beta, part);
  if (e != hipSuccess || S == 1) return e;
  const int64_t MN = (int64_t)M * N;
  hipLaunchKernelGGL(k_gemm_reduce<T>, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, M,
                     N, S, part, C, ldc, alpha, beta);
  return hipGetLastError();
}

bool fits_int(int64_t v) { return v >= 0 && v < ((int64_t)1 << 31); }

// Y = alpha A X + beta Y for one dense operator, in T.
template <typename T>
hipError_t dense_apply(const DenseOp& A, hipStream_t st, int k, const T* X, int ldx, T* Y,
                       int ldy, T alpha, T beta, const T* a, T* t) {
  if (k == 0) return hipSuccess;
  if (k < 0 || !a || !fits_int(A.n) || !fits_int(A.rows) || ldx < k || ldy < k)
    return hipErrorInvalidValue;
  const int n = (int)A.n, rows = (int)A.rows;
  if (A.kind == 1) {
    // K is symmetric: K(i, kk) = K[kk n + i], the column-major reading; the
    // workspace serves products up to tcols wide
    const size_t room = t && k <= A.tcols ? (size_t)A.wslabs * n * A.tcols : 0;
    return gemm<T>(st, true, n, k, n, a, n, X, ldx, Y, ldy, alpha, beta, t, room);
  }
  if (A.kind != 2 || !t || k > A.tcols) return hipErrorInvalidValue;
  // T (rows x k, ld kt) = Xd X: Xd(r, j) = a[j rows + r]; the chunk slabs
  // follow T in the workspace.  kt rounds k up to a multiple of 4, so that
  // the second product reads T in whole vectors.
  const int kt = (k + 3) / 4 * 4 <= A.tcols ? (k + 3) / 4 * 4 : k;
  const size_t room = (size_t)(A.wslabs - 1) * rows * A.tcols;
  hipError_t e = gemm<T>(st, true, rows, k, n, a, rows, X, ldx, t, kt, T(1), T(0),
                         t + (size_t)rows * A.tcols, room);
  if (e != hipSuccess) return e;
  // Y = alpha scale Xd^T T + beta Y: Xd^T(i, r) = a[i rows + r]
  return gemm<T>(st, false, n, k, rows, a, rows, t, kt, Y, ldy, alpha * T(A.scale), beta,
                 nullptr, 0);
}

}  // namespace

hipError_t dense_apply_f64(const DenseOp& A, hipStream_t st, int k, const double* X, int ldx,
                           double* Y, int ldy, double alpha, double beta) {
  return dense_apply<double>(A, st, k, X, ldx, Y, ldy, alpha, beta, A.a64, A.t64);
}

hipError_t dense_apply_f32(const DenseOp& A, hipStream_t st, int k, const float* X, int ldx,
                           float* Y, int ldy) {
  return dense_apply<float>(A, st, k, X, ldx, Y, ldy, 1.0f, 0.0f, A.a32, A.t32);
}

hipError_t dense_axpy(hipStream_t st, int64_t count, double a, const double* x, double* y) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, a,
                     x, y);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(hipStream_t st, bool acol, int M, int N, int K, const double* A,
                           int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                           double alpha, double beta, double* work, size_t work_elems) {
  return gemm<double>(st, acol, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, work, work_elems);
}

hipError_t launch_gemm_f32(hipStream_t st, bool acol, int M, int N, int K, const float* A,
                           int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                           float alpha, float beta, float* work, size_t work_elems) {
  return gemm<float>(st, acol, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, work, work_elems);
}

}  // namespace rafeast
