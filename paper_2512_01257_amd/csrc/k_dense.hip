// Dense and sparse x dense kernels of the RA-FEAST path on gfx950:
//  - CSR SpMM with FP64 real blocks (Rayleigh-Ritz W = A Q, Phase-1 operator
//    applications, eq. rand-range and eq. B-def),
//  - tall-skinny Gram X^T Y and X S products on FP64 MFMA (Rayleigh-Ritz
//    projection Q^T A Q and CholQR),
//  - Ritz residuals, filter combination (eq. projector-quad), the Philox
//    Gaussian sketch (Algorithm 2, Phase 1) and layout helpers.
#include "device.h"
#include "kernels.h"

namespace rafeast {

// ============================================================================
// SpMM, FP64 real: Y = alpha*A*X + beta*X + gamma*X2.  One wave per row; the
// row's nonzeros are wave-uniform (scalar loads), lanes run over the columns
// of the block, so every gathered row X[j, :] is one coalesced read.
// ============================================================================
__global__ __launch_bounds__(256) void k_spmm_f64(int n, int k, const int* __restrict__ rowptr,
                                                  const int* __restrict__ col,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ X, int ldx,
                                                  double* __restrict__ Y, int ldy, double alpha,
                                                  double beta, const double* __restrict__ X2,
                                                  int ldx2, double gamma) {
  const int row = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (row >= n) return;
  const int lane = threadIdx.x & 63;
  const int s = rowptr[row], e = rowptr[row + 1];
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int c = c0 + lane;
    const bool ok = c < k;
    // four gathered rows in flight per wave; even and odd nonzeros go to two
    // partial sums in row order
    double acc0 = 0.0, acc1 = 0.0;
    int t = s;
    for (; t + 3 < e; t += 4) {
      const int j0 = col[t], j1 = col[t + 1], j2 = col[t + 2], j3 = col[t + 3];
      const double a0 = val[t], a1 = val[t + 1], a2 = val[t + 2], a3 = val[t + 3];
      if (ok) {
        const double x0 = X[(size_t)j0 * ldx + c], x1 = X[(size_t)j1 * ldx + c];
        const double x2 = X[(size_t)j2 * ldx + c], x3 = X[(size_t)j3 * ldx + c];
        acc0 += a0 * x0;
        acc1 += a1 * x1;
        acc0 += a2 * x2;
        acc1 += a3 * x3;
      }
    }
    for (; t + 1 < e; t += 2) {
      const int j0 = col[t], j1 = col[t + 1];
      const double a0 = val[t], a1 = val[t + 1];
      if (ok) {
        acc0 += a0 * X[(size_t)j0 * ldx + c];
        acc1 += a1 * X[(size_t)j1 * ldx + c];
      }
    }
    if (t < e && ok) acc0 += val[t] * X[(size_t)col[t] * ldx + c];
    if (ok) {
      double y = alpha * (acc0 + acc1);
      if (beta != 0.0) y += beta * X[(size_t)row * ldx + c];
      if (X2 != nullptr) y += gamma * X2[(size_t)row * ldx2 + c];
      Y[(size_t)row * ldy + c] = y;
    }
  }
}

// Entry U of a round, loaded by lane U of each group of L lanes, handed to
// every lane of its group (a row's lanes): a lane swizzle within 32 lanes,
// or a read of lane U when the row has the whole wave.
template <int L, int U>
__device__ __forceinline__ int group_bcast(int v) {
  if constexpr (L == 64)
    return __builtin_amdgcn_readlane(v, U);
  else
    return __builtin_amdgcn_ds_swizzle(v, (0x1f & ~(L - 1)) | (U << 5));
}

template <int L, int U, int C>
struct RoundBcast {
  __device__ __forceinline__ static void run(int jv, double av, int* j, double* a) {
    j[U] = group_bcast<L, U>(jv);
    const long long ab = __double_as_longlong(av);
    const int lo = group_bcast<L, U>((int)(ab & 0xffffffffLL));
    const int hi = group_bcast<L, U>((int)(ab >> 32));
    a[U] = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    RoundBcast<L, U + 1, C>::run(jv, av, j, a);
  }
};
template <int L, int C>
struct RoundBcast<L, C, C> {
  __device__ __forceinline__ static void run(int, double, int*, double*) {}
};

// A row's extent and the first round of its entries (lane u < C of the
// row's lanes holds entry u), loaded ahead of the row's gathers.
struct RowHead {
  int s, e, jv;
  double av;
};

// Every load of the SpMM below runs on every lane, at an index that is in
// range whether or not its value is used (an unused row reads row 0, an
// unused entry reads entry 0, an unused gather reads row j of entry 0 or
// column grp * kg), and unused values are dropped where they are consumed:
// with no lane-masked branch around the loads and no select right after
// them, the compiler counts the loads in flight and waits only for the ones
// a step needs.  The matrix has at least one nonzero (checked at launch).
__device__ __forceinline__ void head_bounds(RowHead& h, int row, bool live,
                                            const int* __restrict__ rowptr) {
  const int r = live ? row : 0;
  h.s = __builtin_nontemporal_load(rowptr + r);
  h.e = __builtin_nontemporal_load(rowptr + r + 1);
}

template <int C>
__device__ __forceinline__ void head_entries(RowHead& h, int sub, int t0,
                                             const int* __restrict__ col,
                                             const double* __restrict__ val) {
  // the matrix streams past L2 (it is read once per column group), which
  // keeps L2 for the gathered rows of X
  const int t = sub < C && t0 + sub < h.e ? t0 + sub : 0;
  h.jv = __builtin_nontemporal_load(col + t);
  h.av = __builtin_nontemporal_load(val + t);
}

// One row of Y (the columns of group grp) for the lanes of sub-index sub.
// h holds the row's extent and its first round of entries; later rounds and
// later column passes load their own.
template <int L>
__device__ __forceinline__ void spmm_x2_row(int row, int sub, int grp, int k, int kg,
                                            const RowHead& h, const int* __restrict__ col,
                                            const double* __restrict__ val,
                                            const double* __restrict__ X, int ldx,
                                            double* __restrict__ Y, int ldy, double alpha,
                                            double beta, const double* __restrict__ X2, int ldx2,
                                            double gamma) {
  constexpr int C = L < 8 ? L : 8;  // nonzeros per round
  const int s = h.s, e = h.e;
  const int cend = min(k, (grp + 1) * kg);
  // round 0 (positions s .. s + C - 1): lane u < C of the row's lanes holds
  // entry u; handed round the row's lanes once, kept for every column pass
  int j0[C];
  double a0[C];
  RoundBcast<L, 0, C>::run(h.jv, h.av, j0, a0);
  for (int c0 = grp * kg; c0 < cend; c0 += 2 * L) {
    const int c = c0 + 2 * sub;
    const bool ok = c < cend;
    const int cs = ok ? c : grp * kg;  // an in-range column for the idle lanes
    double2 acc0 = make_double2(0.0, 0.0), acc1 = acc0;
    // the gathered rows of a round are loaded together; even and odd
    // positions of the row go to two partial sums, in order (a round of one
    // entry alternates between them)
    {
      double2 x[C];
#pragma unroll
      for (int u = 0; u < C; ++u)
        x[u] = *reinterpret_cast<const double2*>(X + (size_t)j0[u] * ldx + cs);
#pragma unroll
      for (int u = 0; u < C; ++u) {
        if (s + u < e) {
          if (u & 1) {
            acc1.x += a0[u] * x[u].x;
            acc1.y += a0[u] * x[u].y;
          } else {
            acc0.x += a0[u] * x[u].x;
            acc0.y += a0[u] * x[u].y;
          }
        }
      }
    }
    // later rounds (rows longer than C): their entries are loaded here
    for (int t0 = s + C; t0 < e; t0 += C) {
      RowHead r = h;
      head_entries<C>(r, sub, t0, col, val);
      int j[C];
      double a[C];
      RoundBcast<L, 0, C>::run(r.jv, r.av, j, a);
      double2 x[C];
#pragma unroll
      for (int u = 0; u < C; ++u)
        x[u] = *reinterpret_cast<const double2*>(X + (size_t)j[u] * ldx + cs);
#pragma unroll
      for (int u = 0; u < C; ++u) {
        if (t0 + u < e) {
          const bool odd = C == 1 ? ((t0 - s) & 1) != 0 : (u & 1) != 0;
          if (odd) {
            acc1.x += a[u] * x[u].x;
            acc1.y += a[u] * x[u].y;
          } else {
            acc0.x += a[u] * x[u].x;
            acc0.y += a[u] * x[u].y;
          }
        }
      }
    }
    if (ok) {
      double2 y = make_double2(alpha * (acc0.x + acc1.x), alpha * (acc0.y + acc1.y));
      if (beta != 0.0) {
        const double2 xr = *reinterpret_cast<const double2*>(X + (size_t)row * ldx + c);
        y.x += beta * xr.x;
        y.y += beta * xr.y;
      }
      if (X2 != nullptr) {
        const double2 x2r = *reinterpret_cast<const double2*>(X2 + (size_t)row * ldx2 + c);
        y.x += gamma * x2r.x;
        y.y += gamma * x2r.y;
      }
      // Y is not read again here: streamed past L2, which keeps the gathered rows
      typedef double d2v __attribute__((ext_vector_type(2)));
      d2v yv;
      yv.x = y.x;
      yv.y = y.y;
      __builtin_nontemporal_store(yv, reinterpret_cast<d2v*>(Y + (size_t)row * ldy + c));
    }
  }
}

// Two columns per lane (16-byte loads) and 64 / L rows per wave, L the
// power of two of lanes that covers kg / 2 column pairs (k even, ld even and
// 16-byte aligned blocks): each load instruction moves twice the bytes of the
// one-column form, and a wave serves several short rows at once.  Nonzeros
// go to two partial sums (even and odd positions) in row order.
//
// Placement: workgroup b runs on XCD b mod 8 (dispatch deals workgroup ids
// to the eight XCDs in turn).  XCD x owns the x-th contiguous eighth of the
// row blocks (rbx of them) and sweeps it once per group of kg columns, in
// row order, so a gathered row X[j, group] is fetched into that XCD's L2
// once and reused by the rows around j that need it, as long as the rows
// within the matrix's span of j fit in L2 for one group (the host picks kg
// for that).  A workgroup takes rpb consecutive row blocks of 4 * 64 / L
// rows, one after the other, as a pipeline: while a block's gathers are in
// flight, the next block's first entries and the extents of the block after
// it are loaded.
template <int L>
__global__ __launch_bounds__(256) void k_spmm_f64_x2(int n, int k, int kg, int rbx, int rpb,
                                                     const int* __restrict__ rowptr,
                                                     const int* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ X, int ldx,
                                                     double* __restrict__ Y, int ldy, double alpha,
                                                     double beta, const double* __restrict__ X2,
                                                     int ldx2, double gamma) {
  constexpr int RW = 64 / L;  // rows per wave
  constexpr int C = L < 8 ? L : 8;
  const int b = (int)blockIdx.x;
  const int i = b >> 3;
  const int nbx = (rbx + rpb - 1) / rpb;  // workgroups per XCD and group
  const int grp = i / nbx;
  const int rb0 = (i - grp * nbx) * rpb;
  const int rb1 = min(rbx, rb0 + rpb);
  const int lane = threadIdx.x & 63;
  const int sub = lane % L;
  auto row_of = [&](int rbl) {
    return (((b & 7) * rbx + rbl) * 4 + (int)(threadIdx.x >> 6)) * RW + lane / L;
  };
  auto live = [&](int rbl, int r) { return rbl < rb1 && r < n; };
  int row = row_of(rb0), nrow = row_of(rb0 + 1);
  RowHead h, nh;
  head_bounds(h, row, live(rb0, row), rowptr);
  head_bounds(nh, nrow, live(rb0 + 1, nrow), rowptr);
  head_entries<C>(h, sub, h.s, col, val);
  for (int rbl = rb0; rbl < rb1; ++rbl) {
    if (row >= n) break;
    const int nnrow = row_of(rbl + 2);
    RowHead nnh;
    head_bounds(nnh, nnrow, live(rbl + 2, nnrow), rowptr);
    head_entries<C>(nh, sub, nh.s, col, val);
    spmm_x2_row<L>(row, sub, grp, k, kg, h, col, val, X, ldx, Y, ldy, alpha, beta, X2, ldx2,
                   gamma);
    h = nh;
    nh = nnh;
    row = nrow;
    nrow = nnrow;
  }
}

// Row blocks a workgroup of the two-column SpMM sweeps.
#ifndef RAFEAST_SPMM_RPB
#define RAFEAST_SPMM_RPB 4
#endif

// Bytes of an XCD's L2 (4 MiB) given to the gathered rows of one column group.
#ifndef RAFEAST_SPMM_L2_BYTES
#define RAFEAST_SPMM_L2_BYTES (3 << 20)
#endif

int spmm_group_cols(int k, int64_t span) {
  // the rows a gather can reach around row j span 2 * span + 1 rows of a
  // group's kg FP64 columns: the fewest equal groups (kg even, at least 8)
  // whose rows fit the budget
  for (int ng = 1;; ++ng) {
    int kg = (k + ng - 1) / ng;
    kg += kg & 1;
    if (kg <= 8 || (2 * span + 1) * (int64_t)kg * 8 <= (int64_t)RAFEAST_SPMM_L2_BYTES)
      return kg < k ? kg : k;
  }
}

hipError_t launch_spmm_f64(hipStream_t st, int n, int k, const int* rowptr, const int* col,
                           const double* val, int64_t nnz, const double* X, int ldx, double* Y,
                           int ldy, double alpha, double beta, const double* X2, int ldx2,
                           double gamma, int64_t span) {
  if (n <= 0 || k <= 0) return hipSuccess;
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const bool x2_ok = X2 == nullptr || (ldx2 % 2 == 0 && al16(X2));
  if (nnz > 0 && k % 2 == 0 && ldx % 2 == 0 && ldy % 2 == 0 && al16(X) && al16(Y) && x2_ok) {
    const int kg = span > 0 ? spmm_group_cols(k, span) : k;
    const int ng = (k + kg - 1) / kg;
    // lanes per row: the power of two covering kg / 2 column pairs (<= 64)
    int L = 1;
    while (L < 64 && 2 * L < kg) L *= 2;
    const int rw = 64 / L;
    const int rblocks = (n + 4 * rw - 1) / (4 * rw);
    const int rbx = (rblocks + 7) / 8;
    const int rpb = RAFEAST_SPMM_RPB;
    const dim3 grid((unsigned)(8 * ng * ((rbx + rpb - 1) / rpb)));
#define RAFEAST_SPMM_X2(LL)                                                                     \
  hipLaunchKernelGGL(k_spmm_f64_x2<LL>, grid, dim3(256), 0, st, n, k, kg, rbx, rpb, rowptr, col, \
                     val, X, ldx, Y, ldy, alpha, beta, X2, ldx2, gamma)
    switch (L) {
      case 1: RAFEAST_SPMM_X2(1); break;
      case 2: RAFEAST_SPMM_X2(2); break;
      case 4: RAFEAST_SPMM_X2(4); break;
      case 8: RAFEAST_SPMM_X2(8); break;
      case 16: RAFEAST_SPMM_X2(16); break;
      case 32: RAFEAST_SPMM_X2(32); break;
      default: RAFEAST_SPMM_X2(64); break;
    }
#undef RAFEAST_SPMM_X2
    return hipGetLastError();
  }
  dim3 grid((n + 3) / 4);
  hipLaunchKernelGGL(k_spmm_f64, grid, dim3(256), 0, st, n, k, rowptr, col, val, X, ldx, Y, ldy,
                     alpha, beta, X2, ldx2, gamma);
  return hipGetLastError();
}

// ============================================================================
// Gram G = X^T Y on v_mfma_f64_16x16x4f64.
// Operand layout of the 16x16x4 FP64 MFMA (per lane l of the wave):
//   A (16 x 4):  A[l % 16][l / 16]        B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): D[l / 16 + 4 v][l % 16], v = 0..3
// For G = X^T Y the A operand is a 4-row slab of X transposed and B the same
// rows of Y, so lane l reads X[r + l/16][a0 + l%16] and Y[r + l/16][b0 + l%16]:
// 16 consecutive doubles of a row per quarter-wave.
// Rows are split into chunks (grid.x); each wave owns one 16-row tile strip of
// G and four 16-column tiles; partial Grams are summed in chunk order.
// ============================================================================
// Word 3 of a raw buffer descriptor on gfx9-family GPUs (no format, no
// swizzle, stride 0): reads past num_records bytes return zero.
constexpr int kBufferWord3 = 0x00020000;

int gram_chunks(int64_t n) {
  int64_t c = (n + 127) / 128;
  if (c > 256) c = 256;
  if (c < 1) c = 1;
  return (int)c;
}

size_t gram_partial_doubles(int64_t n, int k1, int k2) {
  return (size_t)gram_chunks(n) * (size_t)k1 * (size_t)k2;
}

// A workgroup owns a TA x TB block of 16 x 16 output tiles of one row chunk;
// its 4 waves split the chunk's rows (wave w takes batches w, w + 4, ...)
// and add their partial blocks through LDS in a fixed order.  Per 4-row step a
// wave loads TA + TB operand fragments and issues TA * TB MFMAs on them.
// Rows go in batches of U steps (4 U rows) whose loads are issued together,
// unconditionally (a column past k reads column k - 1, which only feeds rows
// or columns of G that are not stored; a row past the chunk reads zero), and
// every tile's MFMA is issued, so no branch separates the loads from the
// MFMAs.
template <int TA, int TB, int U>
__global__ __launch_bounds__(256) void k_gram_partial(int64_t n, int k1, int k2,
                                                      const double* __restrict__ X, int ldx,
                                                      const double* __restrict__ Y, int ldy,
                                                      double* __restrict__ part,
                                                      int64_t rows_per_chunk) {
  constexpr int kBlockVals = TA * TB * 256;  // one wave's partial block
  __shared__ double sh[2 * kBlockVals];
  const int chunk = blockIdx.x;
  const int64_t r_begin = (int64_t)chunk * rows_per_chunk;
  int64_t r_end = r_begin + rows_per_chunk;
  if (r_end > n) r_end = n;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int tb_n = (k2 + 15) >> 4;
  const int bb_n = (tb_n + TB - 1) / TB;  // tile blocks per block row
  const int blk = blockIdx.y;
  const int ta0 = (blk / bb_n) * TA, tb0 = (blk % bb_n) * TB;
  const int li = lane & 15, lk = lane >> 4;
  int a_col[TA], b_col[TB];
#pragma unroll
  for (int i = 0; i < TA; ++i) a_col[i] = (ta0 + i) * 16 + li;
#pragma unroll
  for (int j = 0; j < TB; ++j) b_col[j] = (tb0 + j) * 16 + li;
  v4d acc[TA][TB];
#pragma unroll
  for (int i = 0; i < TA; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  // Loads go through buffer descriptors covering exactly the chunk's rows of
  // X and Y: an address is a per-lane 32-bit byte offset (lane row lk, tile
  // column) plus a wave-uniform row offset, and a read past the chunk's last
  // row returns zero, so the last partial batch needs no guard.
  constexpr int BR = 4 * U;  // rows per batch
  const int64_t nrows = r_end > r_begin ? r_end - r_begin : 0;
  const int64_t nbatch = (nrows + BR - 1) / BR;
  const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(X + r_begin * ldx), (short)0, (int)(nrows * ldx * 8), kBufferWord3);
  const __amdgpu_buffer_rsrc_t ys = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(Y + r_begin * ldy), (short)0, (int)(nrows * ldy * 8), kBufferWord3);
  int xo[TA], yo[TB];
#pragma unroll
  for (int i = 0; i < TA; ++i) xo[i] = (lk * ldx + min(a_col[i], k1 - 1)) * 8;
#pragma unroll
  for (int j = 0; j < TB; ++j) yo[j] = (lk * ldy + min(b_col[j], k2 - 1)) * 8;
  for (int64_t bt = wave; bt < nbatch; bt += 4) {
    const int r = (int)(bt * BR);  // row within the chunk
    double a[U][TA], b[U][TB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int xrow = (r + 4 * u) * ldx * 8, yrow = (r + 4 * u) * ldy * 8;
#pragma unroll
      for (int i = 0; i < TA; ++i)
        a[u][i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(xs, xo[i], xrow, 0));
#pragma unroll
      for (int j = 0; j < TB; ++j)
        b[u][j] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(ys, yo[j], yrow, 0));
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < TA; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][i], b[u][j], acc[i][j], 0, 0, 0);
  }
  // the 4 waves' blocks summed in a fixed order, (w0 + w2) + (w1 + w3), in
  // two rounds through half the LDS; element (i, j, v, l) of a block is
  // D[l / 16 + 4 v][l % 16] of tile (i, j)
  auto idx = [&](int i, int j, int v) { return ((i * TB + j) * 4 + v) * 64 + lane; };
  if (wave >= 2) {
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) sh[(wave - 2) * kBlockVals + idx(i, j, v)] = acc[i][j][v];
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][j][v] += sh[wave * kBlockVals + idx(i, j, v)];
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) sh[idx(i, j, v)] = acc[i][j][v];
  }
  __syncthreads();
  if (wave == 0) {
    double* P = part + (size_t)chunk * k1 * k2;
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = (ta0 + i) * 16 + lk + 4 * v;
          const int gj = (tb0 + j) * 16 + li;
          if (gi < k1 && gj < k2) P[(size_t)gi * k2 + gj] = acc[i][j][v] + sh[idx(i, j, v)];
        }
  }
}

__global__ __launch_bounds__(256) void k_gram_reduce(int chunks, int k1, int k2,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ G, int ldg) {
  __shared__ double sh[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e = blockIdx.x * 64 + lane;
  const int total = k1 * k2;
  const size_t stride = (size_t)total;
  const int q = (chunks + 3) / 4;
  const int c0 = wave * q, c1 = min(chunks, c0 + q);
  double s = 0.0;
  if (e < total)
    for (int c = c0; c < c1; ++c) s += part[(size_t)c * stride + e];
  sh[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && e < total)
    G[(size_t)(e / k2) * ldg + (e % k2)] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

hipError_t launch_gram(hipStream_t st, int64_t n, int k1, int k2, const double* X, int ldx,
                       const double* Y, int ldy, double* G, int ldg, double* part) {
  return launch_gram_chunks(st, n, k1, k2, X, ldx, Y, ldy, G, ldg, part, gram_chunks(n));
}

hipError_t launch_gram_chunks(hipStream_t st, int64_t n, int k1, int k2, const double* X,
                              int ldx, const double* Y, int ldy, double* G, int ldg, double* part,
                              int chunks) {
  if (k1 <= 0 || k2 <= 0) return hipSuccess;
  if (chunks < 1) chunks = 1;
  if (chunks > gram_chunks(n)) chunks = gram_chunks(n);
  int64_t rpc = (n + chunks - 1) / chunks;
  rpc = (rpc + 3) & ~int64_t(3);
  // a chunk's rows are addressed through 32-bit buffer offsets
  if (rpc * (int64_t)(ldx > ldy ? ldx : ldy) * 8 > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  const int ta_n = (k1 + 15) / 16, tb_n = (k2 + 15) / 16;
  // one workgroup per tile block and chunk: 3 x 3 blocks when that still
  // gives twelve or more per chunk, else 2 x 2
  auto nblk = [&](int ta, int tb) { return ((ta_n + ta - 1) / ta) * ((tb_n + tb - 1) / tb); };
  const bool big = nblk(3, 3) >= 12;
  const int blocks = big ? nblk(3, 3) : nblk(2, 2);
  dim3 grid(chunks, blocks);
  if (big)
    hipLaunchKernelGGL((k_gram_partial<3, 3, 2>), grid, dim3(256), 0, st, n, k1, k2, X, ldx, Y,
                       ldy, part, rpc);
  else
    hipLaunchKernelGGL((k_gram_partial<2, 2, 4>), grid, dim3(256), 0, st, n, k1, k2, X, ldx, Y,
                       ldy, part, rpc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3((k1 * k2 + 63) / 64), dim3(256), 0, st, chunks, k1,
                     k2, part, G, ldg);
  return hipGetLastError();
}

// ============================================================================
// TSMM Y = X S on v_mfma_f64_16x16x4f64: each wave computes a 16-row strip of
// Y for TB 16-column tiles; A operand lane l reads X[r0 + l%16][a0 + l/16],
// B operand reads S[a0 + l/16][b0 + l%16].
// ============================================================================
template <int TB>
__global__ __launch_bounds__(256) void k_tsmm(int64_t n, int k, int k2,
                                              const double* __restrict__ X, int ldx,
                                              const double* __restrict__ S, int lds,
                                              double* __restrict__ Y, int ldy) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (r0 >= n) return;
  const int tb_n = (k2 + 15) >> 4;
  const int tb0 = blockIdx.y * TB;
  const int nb = min(TB, tb_n - tb0);  // wave-uniform
  const int li = lane & 15, lk = lane >> 4;
  v4d acc[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t arow = r0 + li;
  const bool r_ok = arow < n;
  int bcol[TB];
  bool bok[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    bcol[t] = (tb0 + t) * 16 + li;
    bok[t] = t < nb && bcol[t] < k2;
  }
  for (int a0 = 0; a0 < k; a0 += 4) {
    const int acol = a0 + lk;
    const bool aok = acol < k;
    const double a = (aok && r_ok) ? X[arow * ldx + acol] : 0.0;
#pragma unroll
    for (int t = 0; t < TB; ++t) {
      if (t >= nb) continue;
      const double bv = (aok && bok[t]) ? S[(size_t)acol * lds + bcol[t]] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    if (!bok[t]) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = r0 + lk + 4 * v;
      if (r < n) Y[r * ldy + bcol[t]] = acc[t][v];
    }
  }
}

// The same product with the workgroup's TB * 16 columns of S staged in LDS
// (zero past k and k2) and read from there by every wave, where k_tsmm
// re-reads them from L2 for each 16-row strip.  A workgroup of 8 waves
// takes RW blocks of 128 rows (16 per wave) in turn; a wave loads its A
// fragments 8 k-steps at a time, all issued together through a buffer
// descriptor over its 16 rows (a row past n reads zero; a column past k
// reads column k - 1, which meets a zero row of S), then issues the MFMAs.
constexpr int kTsmmThreads = 512;
constexpr int kTsmmRW = 4;
constexpr int kTsmmMaxLds = 128 * 1024;

template <int TB>
__global__ __launch_bounds__(kTsmmThreads) void k_tsmm_lds(int64_t n, int k, int k2,
                                                           const double* __restrict__ X, int ldx,
                                                           const double* __restrict__ S, int lds,
                                                           double* __restrict__ Y, int ldy) {
  extern __shared__ double sl[];  // kp x (16 TB), row-major
  constexpr int SC = 16 * TB;
  const int kp = (k + 3) & ~3;
  const int tb0 = blockIdx.y * TB;
  for (int e = threadIdx.x; e < kp * SC; e += kTsmmThreads) {
    const int a = e / SC, gc = tb0 * 16 + e % SC;
    sl[e] = (a < k && gc < k2) ? S[(size_t)a * lds + gc] : 0.0;
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int nsteps = kp >> 2;
  constexpr int KB = 8;  // k-steps per batch of A loads
  for (int rb = 0; rb < kTsmmRW; ++rb) {
    const int64_t r0 = (((int64_t)blockIdx.x * kTsmmRW + rb) * (kTsmmThreads / 64) + wave) * 16;
    if (r0 >= n) break;  // wave-uniform
    const int rows = (int)min<int64_t>(16, n - r0);
    const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(X + r0 * ldx), (short)0, rows * ldx * 8, kBufferWord3);
    v4d acc[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int s0 = 0; s0 < nsteps; s0 += KB) {
      double a[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int col = min(4 * (s0 + u) + lk, k - 1);
        a[u] = __builtin_bit_cast(double,
                                  __builtin_amdgcn_raw_buffer_load_b64(xs, (li * ldx + col) * 8, 0, 0));
      }
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        // steps past kp meet rows of sl that do not exist: skip them (uniform)
        if (s0 + u >= nsteps) break;
        const double* srow = sl + (4 * (s0 + u) + lk) * SC + li;
#pragma unroll
        for (int t = 0; t < TB; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], srow[16 * t], acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < TB; ++t) {
      const int c = (tb0 + t) * 16 + li;
      if (c >= k2) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + lk + 4 * v;
        if (r < n) Y[r * ldy + c] = acc[t][v];
      }
    }
  }
}

hipError_t launch_tsmm(hipStream_t st, int64_t n, int k, int k2, const double* X, int ldx,
                       const double* S, int lds, double* Y, int ldy) {
  if (n <= 0 || k2 <= 0) return hipSuccess;
  const int tb_n = (k2 + 15) / 16;
  // one wave covers up to six column tiles, so X is read once for k2 <= 96
  constexpr int TB = 6;
  const size_t lds_bytes = (size_t)((k + 3) & ~3) * 16 * TB * sizeof(double);
  // staging S pays once there are enough rows to give every CU a workgroup
  // of 512 rows; below that the per-strip kernel spreads wider
  if (k >= 1 && lds_bytes <= (size_t)kTsmmMaxLds && n >= (int64_t)1 << 17) {
    hipError_t e = hipFuncSetAttribute((const void*)k_tsmm_lds<TB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    const int64_t rows_per_wg = (int64_t)kTsmmRW * (kTsmmThreads / 64) * 16;
    dim3 grid((unsigned)((n + rows_per_wg - 1) / rows_per_wg), (tb_n + TB - 1) / TB);
    hipLaunchKernelGGL(k_tsmm_lds<TB>, grid, dim3(kTsmmThreads), lds_bytes, st, n, k, k2, X, ldx,
                       S, lds, Y, ldy);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((n + 63) / 64), (tb_n + TB - 1) / TB);
  hipLaunchKernelGGL(k_tsmm<TB>, grid, dim3(256), 0, st, n, k, k2, X, ldx, S, lds, Y, ldy);
  return hipGetLastError();
}

// ============================================================================
// Ritz residuals R = W - Q diag(theta) and column norms.  Threads are laid out
// 4 rows x 64 columns; per-thread sums are combined in a fixed order.
// ============================================================================
__global__ __launch_bounds__(256) void k_resid_partial(int64_t n, int k,
                                                       const double* __restrict__ W,
                                                       const double* __restrict__ Q, int ld,
                                                       const double* __restrict__ theta,
                                                       double* __restrict__ R,
                                                       double* __restrict__ part,
                                                       int64_t rows_per_chunk) {
  __shared__ double sh[2][4][64];
  const int chunk = blockIdx.x;
  const int64_t rb = (int64_t)chunk * rows_per_chunk;
  int64_t re = rb + rows_per_chunk;
  if (re > n) re = n;
  const int ty = threadIdx.x >> 6, tx = threadIdx.x & 63;
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int c = c0 + tx;
    double s1 = 0.0, s2 = 0.0;
    if (c < k) {
      const double th = theta[c];
      for (int64_t r = rb + ty; r < re; r += 4) {
        const double q = Q[r * ld + c];
        const double v = W[r * ld + c] - th * q;
        R[r * ld + c] = v;
        s1 += v * v;
        s2 += q * q;
      }
    }
    sh[0][ty][tx] = s1;
    sh[1][ty][tx] = s2;
    __syncthreads();
    if (ty == 0 && c < k) {
      const double a = ((sh[0][0][tx] + sh[0][1][tx]) + sh[0][2][tx]) + sh[0][3][tx];
      const double b = ((sh[1][0][tx] + sh[1][1][tx]) + sh[1][2][tx]) + sh[1][3][tx];
      part[(size_t)chunk * 2 * k + c] = a;
      part[(size_t)chunk * 2 * k + k + c] = b;
    }
    __syncthreads();
  }
}

__global__ void k_resid_final(int chunks, int k, const double* __restrict__ part, double s_win,
                              double* __restrict__ res, double* __restrict__ qn) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double a = 0.0, b = 0.0;
  for (int ch = 0; ch < chunks; ++ch) {
    a += part[(size_t)ch * 2 * k + c];
    b += part[(size_t)ch * 2 * k + k + c];
  }
  const double q = sqrt(b);
  res[c] = sqrt(a) / (s_win * q);
  qn[c] = q;
}

hipError_t launch_residual(hipStream_t st, int64_t n, int k, const double* W, const double* Q,
                           int ld, const double* theta, double s_win, double* R, double* res,
                           double* qn, double* part) {
  const int chunks = gram_chunks(n);
  const int64_t rpc = (n + chunks - 1) / chunks;
  hipLaunchKernelGGL(k_resid_partial, dim3(chunks), dim3(256), 0, st, n, k, W, Q, ld, theta, R,
                     part, rpc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_resid_final, dim3((k + 63) / 64), dim3(64), 0, st, chunks, k, part, s_win,
                     res, qn);
  return hipGetLastError();
}

// ============================================================================
// Filter combination (eq. projector-quad, upper-half nodes, real part).
// ============================================================================
__global__ void k_gamma(int nc, int k, const double* __restrict__ zw,
                        const double* __restrict__ theta, double* __restrict__ gamma) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc * k) return;
  const int j = e / k, i = e % k;
  const zd z{zw[2 * j], zw[2 * j + 1]};
  const zd w{zw[2 * nc + 2 * j], zw[2 * nc + 2 * j + 1]};
  const zd g = zdiv(w, zd{z.re - theta[i], z.im});
  gamma[2 * e] = g.re;
  gamma[2 * e + 1] = g.im;
}

hipError_t launch_gamma(hipStream_t st, int nc, int k, const double* zw, const double* theta,
                        double* gamma) {
  const int tot = nc * k;
  hipLaunchKernelGGL(k_gamma, dim3((tot + 255) / 256), dim3(256), 0, st, nc, k, zw, theta, gamma);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_combine(int64_t n, int nc, int k,
                                                 const double* __restrict__ gamma,
                                                 const double* __restrict__ zw, int residual,
                                                 const double* __restrict__ Q, int ldq,
                                                 const cpx<T>* __restrict__ D, int ldd,
                                                 double* __restrict__ Qt, int ldt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * k) return;
  const int64_t r = e / k;
  const int i = (int)(e % k);
  double acc = 0.0;
  if (residual) {
    const double q = Q[r * ldq + i];
    for (int j = 0; j < nc; ++j) {
      const cpx<T> d = D[r * ldd + (size_t)j * k + i];
      const double gr = gamma[2 * (j * k + i)], gi = gamma[2 * (j * k + i) + 1];
      acc += gr * (q + (double)d.re) - gi * (double)d.im;
    }
  } else {
    for (int j = 0; j < nc; ++j) {
      const cpx<T> d = D[r * ldd + (size_t)j * k + i];
      const double wr = zw[2 * nc + 2 * j], wi = zw[2 * nc + 2 * j + 1];
      acc += wr * (double)d.re - wi * (double)d.im;
    }
  }
  Qt[r * ldt + i] = acc;
}

hipError_t launch_combine(hipStream_t st, int64_t n, int nc, int k, const double* gamma,
                          const double* zw, bool residual_form, const double* Q, int ldq,
                          const void* D, int ldd, bool d32, double* Qt, int ldt) {
  const int64_t tot = n * k;
  dim3 grid((unsigned)((tot + 255) / 256));
  if (d32)
    hipLaunchKernelGGL(k_combine<float>, grid, dim3(256), 0, st, n, nc, k, gamma, zw,
                       residual_form ? 1 : 0, Q, ldq, (const cpx<float>*)D, ldd, Qt, ldt);
  else
    hipLaunchKernelGGL(k_combine<double>, grid, dim3(256), 0, st, n, nc, k, gamma, zw,
                       residual_form ? 1 : 0, Q, ldq, (const cpx<double>*)D, ldd, Qt, ldt);
  return hipGetLastError();
}

// ============================================================================
// Gaussian sketch: Philox4x32-10 (Salmon et al., SC'11) + Box-Muller.
// ============================================================================
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    const uint32_t lo0 = M0 * c[0], hi0 = __umulhi(M0, c[0]);
    const uint32_t lo1 = M1 * c[2], hi1 = __umulhi(M1, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ void k_gaussian(int64_t n, int w, uint32_t s0, uint32_t s1, double* __restrict__ O,
                           int ld) {
  const int pairs = (w + 1) >> 1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * pairs) return;
  const int64_t i = e / pairs;
  const int kp = (int)(e % pairs);
  uint32_t c[4] = {(uint32_t)(i & 0xFFFFFFFF), (uint32_t)((uint64_t)i >> 32), (uint32_t)kp, 0u};
  philox10(c, s0, s1);
  const uint64_t x1 = ((uint64_t)c[0] << 32) | c[1];
  const uint64_t x2 = ((uint64_t)c[2] << 32) | c[3];
  const double u1 = (double)(x1 >> 11) * 0x1.0p-53 + 0x1.0p-54;
  const double u2 = (double)(x2 >> 11) * 0x1.0p-53 + 0x1.0p-54;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586476925287 * u2;
  O[i * ld + 2 * kp] = rad * cos(ang);
  if (2 * kp + 1 < w) O[i * ld + 2 * kp + 1] = rad * sin(ang);
}

hipError_t launch_gaussian(hipStream_t st, int64_t n, int w, uint64_t seed, double* O, int ld) {
  const int64_t tot = n * ((w + 1) / 2);
  hipLaunchKernelGGL(k_gaussian, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, w,
                     (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), O, ld);
  return hipGetLastError();
}

// ============================================================================
// Layout helpers.
// ============================================================================
__global__ void k_col2row(int64_t n, int k, const double* __restrict__ src,
                          double* __restrict__ dst, int ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t r = e / k;
  const int c = (int)(e % k);
  dst[r * ldd + c] = src[(int64_t)c * n + r];
}

hipError_t launch_colmajor_to_rowmajor(hipStream_t st, int64_t n, int k, const double* src,
                                       double* dst, int ldd) {
  const int64_t tot = n * k;
  hipLaunchKernelGGL(k_col2row, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, k, src,
                     dst, ldd);
  return hipGetLastError();
}

__global__ void k_copy_cols(int64_t n, int k, const double* __restrict__ src, int lds,
                            double* __restrict__ dst, int ldd, const int* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  if (status && *status == 2) return;  // a failed factorization: dst keeps its values
  const int64_t r = e / k;
  const int c = (int)(e % k);
  dst[r * ldd + c] = src[r * lds + c];
}

hipError_t launch_copy_cols(hipStream_t st, int64_t n, int k, const double* src, int lds,
                            double* dst, int ldd, const int* status) {
  const int64_t tot = n * k;
  hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, k,
                     src, lds, dst, ldd, status);
  return hipGetLastError();
}

// p[0..n) = v.  A kernel, not a memset node, so it can sit in a captured graph.
__global__ void k_fill_int(int* __restrict__ p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_int(hipStream_t st, int* p, int v, int n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

__global__ void k_row2col(int64_t n, int k, const double* __restrict__ src, int lds,
                          double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int c = (int)(e / n);
  const int64_t r = e % n;
  dst[e] = src[r * lds + c];
}

hipError_t launch_rowmajor_to_colmajor(hipStream_t st, int64_t n, int k, const double* src,
                                       int lds, double* dst) {
  const int64_t tot = n * k;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row2col, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, k, src,
                     lds, dst);
  return hipGetLastError();
}

// One block per exported column: norm, first index of the largest |entry|,
// then the scaled column into column-major dst.
__global__ __launch_bounds__(256) void k_export(int64_t n, const int* __restrict__ sel,
                                                const double* __restrict__ src, int lds,
                                                double* __restrict__ dst) {
  __shared__ double s_sq[4], s_mx[4];
  __shared__ int64_t s_ix[4];
  const int c = blockIdx.x;
  const int col = sel[c];
  double sq = 0.0, mx = -1.0;
  int64_t ix = n;
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    const double v = src[r * lds + col];
    sq += v * v;
    const double a = fabs(v);
    if (a > mx) {  // rows visited in increasing order: keeps the first maximum
      mx = a;
      ix = r;
    }
  }
  // wave reduction: (max, lowest index) and sum
  for (int off = 32; off > 0; off >>= 1) {
    const double omx = __shfl_xor(mx, off, 64);
    const int64_t oix = __shfl_xor(ix, off, 64);
    if (omx > mx || (omx == mx && oix < ix)) {
      mx = omx;
      ix = oix;
    }
    sq += __shfl_xor(sq, off, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_sq[wv] = sq;
    s_mx[wv] = mx;
    s_ix[wv] = ix;
  }
  __syncthreads();
  double tsq = 0.0, tmx = -1.0;
  int64_t tix = n;
  for (int w = 0; w < 4; ++w) {
    tsq += s_sq[w];
    if (s_mx[w] > tmx || (s_mx[w] == tmx && s_ix[w] < tix)) {
      tmx = s_mx[w];
      tix = s_ix[w];
    }
  }
  const double sgn = (tix < n && src[tix * lds + col] < 0.0) ? -1.0 : 1.0;
  const double sc = sgn / sqrt(tsq);
  for (int64_t r = threadIdx.x; r < n; r += 256) dst[(int64_t)c * n + r] = src[r * lds + col] * sc;
}

hipError_t launch_export_vectors(hipStream_t st, int64_t n, int cnt, const int* sel,
                                 const double* src, int lds, double* dst, double* part) {
  (void)part;
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export, dim3(cnt), dim3(256), 0, st, n, sel, src, lds, dst);
  return hipGetLastError();
}

}  // namespace rafeast
