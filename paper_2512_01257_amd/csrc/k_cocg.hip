// COCG for the shifted systems (z_j I - A) d = b of the FEAST filter
// (Section 2.1: the dominant cost, one solve per quadrature node and subspace
// column).  COCG (van der Vorst & Melissen, 1990) is CG with the unconjugated
// bilinear form x^T y, valid for the complex-symmetric z I - A.
//
// Resident engine: one 1024-thread workgroup owns one system for its whole
// solve.  The search direction p (gathered by the SpMM) and the residual r
// live in LDS; w = (zI - A) p and the iterate x live in registers (RPT slots
// per thread).  A is streamed from L2 in the row-sorted SELL-64 layout of
// kernels.h, coalesced across the wave, with the column already an LDS byte
// offset: in FP32 a float value and a 16-bit offset per nonzero, eight per
// lane in three 16-byte loads (the pace of this SpMV is set by the number of
// load instructions, not by the bytes); in FP64 16 bytes per nonzero.  Both COCG
// reductions per iteration are workgroup reductions: no grid-wide
// synchronisation, and systems with different iteration counts retire
// independently.  Workgroups take systems from an atomic work counter in the
// order given (longest first).  A work item names a graph, a shift and a
// right-hand-side column, so one launch can serve the systems of several
// matrices (the batching form); a workgroup reloads the graph's descriptor
// only when its next item belongs to another graph.
//
// Per system: b is scaled to unit norm.  COCG runs in T (float or double;
// per-thread sums in T, cross-thread sums in FP64) with reliable updates in
// FP64: whenever the recursive residual has dropped by the factor delta
// (0.1 in FP32, 1e-4 in FP64) since the last check, or below tol, the
// correction accumulated in T is added to the FP64 solution x_hi (a
// per-workgroup global buffer, indexed by slot) and the true residual
// s = b - (zI - A) x_hi is formed in FP64 with FP64 values of A.  If
// ||s|| > tol the recurrence continues from r = s with the same search
// direction (beta = s^T s / rho_prev), which removes the drift between the
// recursive and the true residual that FP32 storage causes without throwing
// the Krylov recurrence away.  It restarts from p = s only after a breakdown
// (p^T w = 0 or a non-finite step), when ||s|| has not at least halved since
// the previous check, or after a stall: no drop by delta within twice the
// previous check interval (and twice the first interval after the last
// start, at least 256 iterations) sends the system to an early check, which
// bounds the iterations an FP32 recurrence can spend drifting away from the
// true residual on an ill-conditioned system.  At most
// max_refine checks per system.
#include "device.h"
#include "kernels.h"

#include <algorithm>
#include <vector>

namespace rafeast {

constexpr int kResThreads = 1024;
constexpr int kResWaves = kResThreads / 64;

// Sums of values over the 16 lanes of row 0, read from lane 0: the DPP
// steps of wave_sum_f64 stay inside a row of 16 lanes, so rows 1 to 3 (which
// the callers fill with copies) take no part.
template <int NV>
__device__ __forceinline__ void row0_sums_f64(double (&v)[NV]) {
  // step by step over all values, so that the NV chains interleave
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += dpp_f64(v[q], c);
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = readlane_f64(v[q], 0);
}
static_assert(kResWaves == 16, "wave 0 sums the per-wave partials over one 16-lane row");

// wave_sum_f32 / wave_sum_f64 of NV values at once, step by step over all
// values so that the chains interleave (each value's arithmetic unchanged)
template <int NV, typename A>
__device__ __forceinline__ void wave_sums(const A (&part)[NV], double (&ws)[NV]) {
  A v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = part[q];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if constexpr (sizeof(A) == 4)
        v[q] += dpp_f32(v[q], c);
      else
        v[q] += dpp_f64(v[q], c);
    }
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if constexpr (sizeof(A) == 4) {
      const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[q]), 0));
      const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[q]), 16));
      const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[q]), 32));
      const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[q]), 48));
      ws[q] = (double)((r0 + r1) + (r2 + r3));
    } else {
      ws[q] = (readlane_f64(v[q], 0) + readlane_f64(v[q], 16)) +
              (readlane_f64(v[q], 32) + readlane_f64(v[q], 48));
    }
  }
}

// Workgroup sum of NV values given per-thread partials of type A (float or
// double): DPP wave sums (no LDS), one LDS slot per wave, a barrier, then
// wave 0 adds the kResWaves wave sums in FP64 (fixed order) and publishes the
// totals in LDS for a second barrier.  One wave finishing the sum, instead of
// every wave repeating it, frees the SIMDs for the other waves' work.  Wave
// 0 reads all NV slots unconditionally (lane l reads wave l mod 16's), so
// the reads are in flight together.
template <int NV, typename A>
__device__ __forceinline__ void block_sum(const A (&part)[NV], double (&v)[NV],
                                          double (*red)[kResWaves][4], int set) {
  const int wv = threadIdx.x >> 6;
  double ws[NV];
  wave_sums(part, ws);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[set][wv][q] = ws[q];
  }
  __syncthreads();
  // wave 0: lane w < kResWaves reads wave w's sum, a DPP sum over the wave;
  // the totals overwrite wave 0's slots (read before they are written).
  // Every caller passes another barrier after reading the totals and before
  // the next call on the same set writes its partials.
  const int ln = threadIdx.x & 63;
  if (wv == 0) {
    double x[NV], t[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) x[q] = red[set][ln & (kResWaves - 1)][q];
    row0_sums_f64(x);
#pragma unroll
    for (int q = 0; q < NV; ++q) t[q] = x[q];
    if (ln == 0) {
#pragma unroll
      for (int q = 0; q < NV; ++q) red[set][0][q] = t[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = red[set][0][q];
}

// As block_sum, but wave 0 also maps the NV totals to NO published values
// (the COCG step lengths), so no other wave repeats that arithmetic.
template <int NV, int NO, typename A, typename F>
__device__ __forceinline__ void block_sum_fin(const A (&part)[NV], double (&o)[NO],
                                              double (*red)[kResWaves][4], int set, F fin) {
  const int wv = threadIdx.x >> 6;
  double ws[NV];
  wave_sums(part, ws);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[set][wv][q] = ws[q];
  }
  __syncthreads();
  const int ln = threadIdx.x & 63;
  double* flat = &red[set][0][0];
  if (wv == 0) {
    double x[NV], t[NV], r[NO];
#pragma unroll
    for (int q = 0; q < NV; ++q) x[q] = red[set][ln & (kResWaves - 1)][q];
    row0_sums_f64(x);
#pragma unroll
    for (int q = 0; q < NV; ++q) t[q] = x[q];
    fin(t, r);
    if (ln == 0) {
#pragma unroll
      for (int q = 0; q < NO; ++q) flat[q] = r[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NO; ++q) o[q] = flat[q];
}


template <typename T>
__device__ __forceinline__ cpx<T> gather(const char* __restrict__ base, int byte_off) {
  return *reinterpret_cast<const cpx<T>*>(base + byte_off);
}

// Gather from an absolute LDS byte address: p is the first object of the
// kernel's LDS (no static LDS; checked at launch), so the stored offset is
// the address and the load needs no address arithmetic.
template <typename T>
__device__ __forceinline__ cpx<T> lds_gather(int byte_addr) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const __attribute__((address_space(3))) cpx<T> lds_t;
  return *reinterpret_cast<lds_t*>((size_t)(unsigned)byte_addr);
#else
  (void)byte_addr;  // device-only function; the host pass never calls it
  return cpx<T>{T(0), T(0)};
#endif
}

// sum_k a_k v[c_k] over one slot's entries (width a multiple of 4), in
// batches of four entry loads issued before their gathers.
template <typename T, typename AccT, typename E>
__device__ __forceinline__ void sell_dot(const E* __restrict__ ep, int wdt,
                                         const char* __restrict__ vbase, AccT& ar, AccT& ai) {
  for (int kk = 0; kk < wdt; kk += 4) {
    E e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) e[u] = ep[(kk + u) * 64];
    cpx<T> g[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) g[u] = gather<T>(vbase, e[u].c);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ar += (AccT)e[u].v * (AccT)g[u].re;
      ai += (AccT)e[u].v * (AccT)g[u].im;
    }
  }
}

template <typename E>
__device__ __forceinline__ E load_entry(const E* __restrict__ base, unsigned idx) {
  // 32-bit byte offset from a uniform base: one VGPR of address per load
  return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) +
                                     idx * (unsigned)sizeof(E));
}

#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) ResGraph ConstGraph;
__device__ __forceinline__ ConstGraph* const_graph(const ResGraph* graphs, int g) {
  return reinterpret_cast<ConstGraph*>((size_t)graphs) + g;
}
#else
__device__ __forceinline__ const ResGraph* const_graph(const ResGraph* graphs, int g) {
  return graphs + g;  // device-only function; the host pass never calls it
}
#endif

// MULTI false: every item belongs to the graph whose fields are the scalar
// kernel arguments (scalar loads from the argument segment).  MULTI true:
// item (g, j, i) reads graphs[g] at its start; the scalar graph arguments
// are unused.
template <typename T, int RPT, bool MULTI>
__global__ __launch_bounds__(kResThreads) void k_cocg_resident(
    int a_nslices, const int* __restrict__ a_sbase, const int* __restrict__ a_perm,
    const void* __restrict__ a_ent, const SellEntry64* __restrict__ a_ent64, int a_n32, int nitems,
    const int* __restrict__ items, const double* __restrict__ a_zs,
    const double* __restrict__ a_B, int a_ldb, int a_kcols, void* __restrict__ a_D, int a_ldd,
    double tol, int maxit, int max_refine, int* __restrict__ counter, int* __restrict__ a_iters,
    int* __restrict__ a_stats, double* __restrict__ a_resid, cpx<double>* __restrict__ xhi_all,
    int a_zero_base, const int* __restrict__ a_wave_slices, const ResGraph* __restrict__ graphs,
    int max_npad) {
  // Dynamic LDS only (so p starts at address 0 and a gather address is the
  // entry's stored byte offset): p | r (sized for the graph of the current
  // item) ... | zero row | trash row | reduction slots | work item (after
  // room for the largest graph).  The vector loops read every slot
  // unconditionally, so that a wave issues all its LDS loads before the
  // first wait: a slot past the wave's last slice reads the zero row (its
  // terms are exact zeros) and writes the trash row, which nothing reads.
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* P = reinterpret_cast<cpx<T>*>(smem_raw);
  const int zoff = 2 * max_npad, toff = zoff + 64;
  double(*red)[kResWaves][4] = reinterpret_cast<double(*)[kResWaves][4]>(
      smem_raw + ((size_t)max_npad * 2 + 128) * sizeof(cpx<T>));
  int& s_item = *reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(red) +
                                        2 * kResWaves * 4 * sizeof(double));
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  double tol2 = tol * tol;  // of the current graph
  cpx<double>* __restrict__ XH = xhi_all + (size_t)blockIdx.x * max_npad;

  // The graph of the current item.  A descriptor from the array is read
  // through the constant address space: scalar, invariant loads the compiler
  // may repeat instead of keeping every field live in registers.  With a
  // single graph, everything is read once, before the work loop.
  int nslices = 0, zero_base = 0, ldb = 0, kcols = 0, ldd = 0, n32 = 0;
  const int* __restrict__ sbase = nullptr;
  const int* __restrict__ perm = nullptr;
  const void* __restrict__ ent = nullptr;
  const SellEntry64* __restrict__ ent64 = nullptr;
  const double* __restrict__ Bm = nullptr;
  cpx<T>* __restrict__ D = nullptr;
  const double* __restrict__ zs = nullptr;
  int* __restrict__ iters = nullptr;
  double* __restrict__ resid_out = nullptr;
  int* __restrict__ stats = nullptr;
  cpx<T>* R = P;
  int slc[RPT];  // this wave's slices (-1: none), widest first
  auto load_graph = [&](const auto& G) {
    nslices = G.nslices;
    zero_base = G.zero_base;
    ldb = G.ldb;
    kcols = G.kcols;
    ldd = G.ldd;
    sbase = G.sbase;
    perm = G.perm;
    ent = G.ent;
    n32 = G.n32;
    ent64 = G.ent64;
    Bm = G.B;
    D = reinterpret_cast<cpx<T>*>(G.D);
    zs = G.zs;
    iters = G.iters;
    resid_out = G.resid;
    stats = G.stats;
    tol2 = G.tol * G.tol;
    R = P + nslices * 64;
#pragma unroll
    for (int t = 0; t < RPT; ++t) slc[t] = G.wave_slices[wv * RPT + t];
  };
  if constexpr (!MULTI) {
    ResGraph g0;
    g0.nslices = a_nslices;
    g0.zero_base = a_zero_base;
    g0.ldb = a_ldb;
    g0.kcols = a_kcols;
    g0.ldd = a_ldd;
    g0.sbase = a_sbase;
    g0.perm = a_perm;
    g0.ent = a_ent;
    g0.ent64 = a_ent64;
    g0.n32 = a_n32;
    g0.wave_slices = a_wave_slices;
    g0.B = a_B;
    g0.D = a_D;
    g0.zs = a_zs;
    g0.iters = a_iters;
    g0.resid = a_resid;
    g0.stats = a_stats;
    g0.tol = tol;
    load_graph(g0);
  }

  cpx<T> w[RPT], xr[RPT];
  if (tid < 64) P[zoff + tid] = cpx<T>{T(0), T(0)};  // ordered by the loop's first barrier

  for (;;) {
    if (tid == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= nitems) break;
    const int g = __builtin_amdgcn_readfirstlane(items[3 * item]);
    const int j = __builtin_amdgcn_readfirstlane(items[3 * item + 1]);
    const int ci = __builtin_amdgcn_readfirstlane(items[3 * item + 2]);
    if constexpr (MULTI) load_graph(*const_graph(graphs, g));
    const double zr = zs[2 * j], zi = zs[2 * j + 1];
    const int ocol = j * kcols + ci;

    // ---- right-hand side, scaled to unit norm ----
    double acc1[1] = {0.0};
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int slice = slc[t];
      if (slice >= 0) {
        const int row = perm[slice * 64 + lane];
        const double b = row >= 0 ? Bm[(unsigned)row * (unsigned)ldb + ci] : 0.0;
        acc1[0] += b * b;
      }
    }
    double bsum[1];
    block_sum<1>(acc1, bsum, red, 0);
    const double bn2 = bsum[0];
    if (!(bn2 > 0.0) || !isfinite(bn2)) {
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int slice = slc[t];
        if (slice >= 0) {
          const int row = perm[slice * 64 + lane];
          if (row >= 0) D[(unsigned)row * (unsigned)ldd + ocol] = cpx<T>{T(0), T(0)};
        }
      }
      if (tid == 0) {
        iters[ocol] = 0;
        if (resid_out) resid_out[ocol] = 0.0;
      }
      // see the barrier that ends an item
      __syncthreads();
      continue;
    }
    const double scale = 1.0 / sqrt(bn2);
#pragma unroll
    for (int t = 0; t < RPT; ++t) xr[t] = cpx<T>{T(0), T(0)};
    double rho3[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int slice = slc[t];
      if (slice >= 0) {
        const int s = slice * 64 + lane;
        const int row = perm[s];
        const double b = row >= 0 ? Bm[(unsigned)row * (unsigned)ldb + ci] * scale : 0.0;
        const cpx<T> rv{T(b), T(0)};
        P[s] = rv;
        R[s] = rv;
        const double rr = (double)rv.re;
        rho3[0] += rr * rr;
      }
    }
    double rho_s[3];
    block_sum<3>(rho3, rho_s, red, 1);
    double rho_re = rho_s[0], rho_im = 0.0;
    int it = 0, nref = 0, nbd = 0;
    double last_res = 1.0;
    // x_hi is first written at the first check (kept out of L2 before)
    bool first_cycle = true;
    // next check when the recursive residual is below
    // max(tol, delta * ||s at the last check||)
    const double delta = sizeof(T) == 4 ? 0.1 : 1e-4;
    double cyc_tol2 = fmax(tol2, delta * delta * rho_s[0]);
    // check bookkeeping: iteration of the last check and of the last start,
    // length of the previous interval and of the longest first interval
    // after a start, ||s||^2 at the last check
    int lastit = 0, rstart = 0, span = 0, span0 = 0;
    double sprev = rho_s[0];

    for (;;) {
      bool verify = false, restart = false;
      // Slot addresses are cheap to recompute; hiding the lane index from
      // loop-invariant code motion keeps them out of the register budget.
      int ln = lane;
      asm volatile("" : "+v"(ln));
      // ---- w = (zI - A) p,  mu = p^T w ----
      T acc_re[RPT], acc_im[RPT];
      int bse[RPT], wde[RPT];
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        acc_re[t] = T(0);
        acc_im[t] = T(0);
        const int slice = slc[t];
        bse[t] = slice >= 0 ? sbase[slice] : zero_base;
        wde[t] = slice >= 0 ? (sbase[slice + 1] - bse[t]) >> 6 : 0;
      }
      if constexpr (sizeof(T) == 4) {
        // FP32: the SpMV issues few wide loads (the load instruction count,
        // not the bytes, sets its pace): per lane and slot, eight entries
        // take three 16-byte loads (eight values, eight 16-bit LDS offsets)
        // and a trailing four take two; slots go in pairs so that the loads
        // of two slots are in flight together; slots past their width load
        // nothing (wave-uniform bounds).
        const float* __restrict__ vals = reinterpret_cast<const float*>(ent);
        const unsigned short* __restrict__ offs =
            reinterpret_cast<const unsigned short*>(vals + n32);
#pragma unroll
        for (int t = 0; t < RPT; t += 2) {
          const int ta = t, tb = t + 1 < RPT ? t + 1 : t;
          const int na = wde[ta] >> 3, nb = tb != ta ? wde[tb] >> 3 : 0;
          for (int o = 0; o < na; ++o) {
            const int ba = bse[ta] + o * 512;
            const float4 va0 = load_entry(reinterpret_cast<const float4*>(vals + ba), (unsigned)ln);
            const float4 va1 =
                load_entry(reinterpret_cast<const float4*>(vals + ba + 256), (unsigned)ln);
            const uint4 oa = load_entry(reinterpret_cast<const uint4*>(offs + ba), (unsigned)ln);
            float4 vb0 = make_float4(0.f, 0.f, 0.f, 0.f), vb1 = vb0;
            uint4 ob = make_uint4(0u, 0u, 0u, 0u);
            const bool hb = o < nb;
            if (hb) {
              const int bb = bse[tb] + o * 512;
              vb0 = load_entry(reinterpret_cast<const float4*>(vals + bb), (unsigned)ln);
              vb1 = load_entry(reinterpret_cast<const float4*>(vals + bb + 256), (unsigned)ln);
              ob = load_entry(reinterpret_cast<const uint4*>(offs + bb), (unsigned)ln);
            }
            const float va[8] = {va0.x, va0.y, va0.z, va0.w, va1.x, va1.y, va1.z, va1.w};
            const unsigned oaw[4] = {oa.x, oa.y, oa.z, oa.w};
            cpx<T> ga[8];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              ga[2 * u] = lds_gather<T>((int)(oaw[u] & 0xffffu));
              ga[2 * u + 1] = lds_gather<T>((int)(oaw[u] >> 16));
            }
            if (hb) {
              const float vbv[8] = {vb0.x, vb0.y, vb0.z, vb0.w, vb1.x, vb1.y, vb1.z, vb1.w};
              const unsigned obw[4] = {ob.x, ob.y, ob.z, ob.w};
              cpx<T> gb[8];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                gb[2 * u] = lds_gather<T>((int)(obw[u] & 0xffffu));
                gb[2 * u + 1] = lds_gather<T>((int)(obw[u] >> 16));
              }
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                acc_re[tb] += vbv[u] * gb[u].re;
                acc_im[tb] += vbv[u] * gb[u].im;
              }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              acc_re[ta] += va[u] * ga[u].re;
              acc_im[ta] += va[u] * ga[u].im;
            }
          }
          // remaining octs of slot tb cannot exist (widths are non-increasing
          // within a wave); trailing quads of both slots
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int tq = q == 0 ? ta : tb;
            if ((q == 0 || tb != ta) && (wde[tq] & 4)) {
              const int bq = bse[tq] + (wde[tq] >> 3) * 512;
              const float4 v = load_entry(reinterpret_cast<const float4*>(vals + bq), (unsigned)ln);
              const uint2 oq = load_entry(reinterpret_cast<const uint2*>(offs + bq), (unsigned)ln);
              const cpx<T> g0 = lds_gather<T>((int)(oq.x & 0xffffu));
              const cpx<T> g1 = lds_gather<T>((int)(oq.x >> 16));
              const cpx<T> g2 = lds_gather<T>((int)(oq.y & 0xffffu));
              const cpx<T> g3 = lds_gather<T>((int)(oq.y >> 16));
              acc_re[tq] += v.x * g0.re + v.y * g1.re + v.z * g2.re + v.w * g3.re;
              acc_im[tq] += v.x * g0.im + v.y * g1.im + v.z * g2.im + v.w * g3.im;
            }
          }
        }
      } else {
        // FP64: 16-byte entries, two per lane and slot per batch, the loads
        // of all slots issued before any gather
        constexpr int KB = 2;
        const SellEntry64* __restrict__ e64 = reinterpret_cast<const SellEntry64*>(ent);
        for (int kk = 0; kk < wde[0]; kk += KB) {
          SellEntry64 e[RPT][KB];
#pragma unroll
          for (int t = 0; t < RPT; ++t) {
            const SellEntry64* __restrict__ ep =
                kk < wde[t] ? e64 + bse[t] + kk * 64 : e64 + zero_base;
#pragma unroll
            for (int u = 0; u < KB; ++u) e[t][u] = ep[u * 64 + ln];
          }
          cpx<T> g[RPT][KB];
#pragma unroll
          for (int t = 0; t < RPT; ++t) {
#pragma unroll
            for (int u = 0; u < KB; ++u) g[t][u] = lds_gather<T>(e[t][u].c);
          }
#pragma unroll
          for (int t = 0; t < RPT; ++t) {
#pragma unroll
            for (int u = 0; u < KB; ++u) {
              acc_re[t] += e[t][u].v * g[t][u].re;
              acc_im[t] += e[t][u].v * g[t][u].im;
            }
          }
        }
      }
      T mu_t[2] = {T(0), T(0)};
      const T zrt = T(zr), zit = T(zi);
      // this thread's p and r stay in registers until the p update (p is
      // not written before it, r only by this thread's own update)
      cpx<T> pv[RPT], rv[RPT];
#pragma unroll
      for (int t = 0; t < RPT; ++t) pv[t] = P[(slc[t] >= 0 ? slc[t] * 64 : zoff) + ln];
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        // an empty slot has p = 0 and no entries: w = 0, no term
        w[t].re = zrt * pv[t].re - zit * pv[t].im - acc_re[t];
        w[t].im = zrt * pv[t].im + zit * pv[t].re - acc_im[t];
        mu_t[0] += pv[t].re * w[t].re - pv[t].im * w[t].im;
        mu_t[1] += pv[t].re * w[t].im + pv[t].im * w[t].re;
      }
      double mo[4];
      block_sum_fin<2, 4>(mu_t, mo, red, 0, [&](const double* t, double* r) {
        const zd a = zdiv_fast(zd{rho_re, rho_im}, zd{t[0], t[1]});
        r[0] = t[0];
        r[1] = t[1];
        r[2] = a.re;
        r[3] = a.im;
      });
      const double mu[2] = {mo[0], mo[1]};
      const zd alpha{mo[2], mo[3]};
      if (!(isfinite(alpha.re) && isfinite(alpha.im)) || (mu[0] == 0.0 && mu[1] == 0.0)) {
        ++nbd;
        verify = true;
        restart = true;
      } else {
        // ---- x += alpha p, r -= alpha w, rho' = r^T r, ||r||^2 ----
        T s3_t[3] = {T(0), T(0), T(0)};
        const T alr = T(alpha.re), ali = T(alpha.im);
        const int roff = (int)(R - P);
#pragma unroll
        for (int t = 0; t < RPT; ++t) rv[t] = P[(slc[t] >= 0 ? roff + slc[t] * 64 : zoff) + ln];
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          // empty slots: p = w = r = 0, so x stays 0 and no term is added
          xr[t].re += alr * pv[t].re - ali * pv[t].im;
          xr[t].im += alr * pv[t].im + ali * pv[t].re;
          rv[t].re -= alr * w[t].re - ali * w[t].im;
          rv[t].im -= alr * w[t].im + ali * w[t].re;
          P[(slc[t] >= 0 ? roff + slc[t] * 64 : toff) + ln] = rv[t];
          s3_t[0] += rv[t].re * rv[t].re - rv[t].im * rv[t].im;
          s3_t[1] += T(2) * rv[t].re * rv[t].im;
          s3_t[2] += rv[t].re * rv[t].re + rv[t].im * rv[t].im;
        }
        double so[5];
        block_sum_fin<3, 5>(s3_t, so, red, 1, [&](const double* t, double* r) {
          const zd b = zdiv_fast(zd{t[0], t[1]}, zd{rho_re, rho_im});
          r[0] = t[0];
          r[1] = t[1];
          r[2] = t[2];
          r[3] = b.re;
          r[4] = b.im;
        });
        const double s3[3] = {so[0], so[1], so[2]};
        ++it;
        const bool stall =
            span > 0 && it - lastit > max(2 * max(span, span0), 256);
        if (s3[2] <= cyc_tol2 || it >= maxit || stall) {
          verify = true;
        } else {
          const zd beta{so[3], so[4]};
          rho_re = s3[0];
          rho_im = s3[1];
          const T br = T(beta.re), bi = T(beta.im);
#pragma unroll
          for (int t = 0; t < RPT; ++t)
            P[(slc[t] >= 0 ? slc[t] * 64 : toff) + ln] =
                cpx<T>{rv[t].re + br * pv[t].re - bi * pv[t].im,
                       rv[t].im + br * pv[t].im + bi * pv[t].re};
          __syncthreads();
        }
      }
      if (!verify) continue;

      // ---- x_hi += x; true residual s = b - (zI - A) x_hi in FP64 ----
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int slice = slc[t];
        if (slice >= 0) {
          const int s = slice * 64 + ln;
          const cpx<T> xl = xr[t];
          xr[t] = cpx<T>{T(0), T(0)};
          cpx<double> xh{0.0, 0.0};
          if (!first_cycle) xh = XH[s];
          xh.re += (double)xl.re;
          xh.im += (double)xl.im;
          XH[s] = xh;
        }
      }
      first_cycle = false;
      __syncthreads();
      double s3p[3] = {0.0, 0.0, 0.0}, s3[3];
      const char* XHb = reinterpret_cast<const char*>(XH);
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int slice = slc[t];
        if (slice >= 0) {
          const int s = slice * 64 + ln;
          const int base = sbase[slice];
          const int wdt = (sbase[slice + 1] - base) >> 6;
          double ar = 0.0, ai = 0.0;
          sell_dot<double, double>(ent64 + base + ln, wdt, XHb, ar, ai);
          const cpx<double> xr = XH[s];
          const int row = perm[s];
          const double b = row >= 0 ? Bm[(unsigned)row * (unsigned)ldb + ci] * scale : 0.0;
          const double sr = b - (zr * xr.re - zi * xr.im - ar);
          const double si = -(zr * xr.im + zi * xr.re - ai);
          w[t] = cpx<T>{T(sr), T(si)};  // the next cycle's residual
          s3p[0] += sr * sr - si * si;
          s3p[1] += 2.0 * sr * si;
          s3p[2] += sr * sr + si * si;
        }
      }
      block_sum<3>(s3p, s3, red, 0);
      last_res = sqrt(s3[2]);
      if (s3[2] <= tol2 || nref >= max_refine || it >= maxit || nbd > 3) break;
      ++nref;
      // reliable update (keep p, beta = s^T s / rho_prev) or restart (p = s)
      zd beta{0.0, 0.0};
      if (!restart && s3[2] <= 0.25 * sprev) {
        beta = zdiv_fast(zd{s3[0], s3[1]}, zd{rho_re, rho_im});
        if (!(isfinite(beta.re) && isfinite(beta.im))) beta = zd{0.0, 0.0};
      }
      const bool keep = beta.re != 0.0 || beta.im != 0.0;
      span = it - lastit;
      if (lastit == rstart) span0 = max(span0, span);
      lastit = it;
      if (!keep) rstart = it;
      sprev = s3[2];
      rho_re = s3[0];
      rho_im = s3[1];
      cyc_tol2 = fmax(tol2, delta * delta * s3[2]);
      const T br = T(beta.re), bi = T(beta.im);
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int slice = slc[t];
        if (slice >= 0) {
          const int s = slice * 64 + ln;
          const cpx<T> rv = w[t];
          cpx<T> pv = rv;
          if (keep) {
            const cpx<T> pr = P[s];
            pv = cpx<T>{rv.re + br * pr.re - bi * pr.im, rv.im + br * pr.im + bi * pr.re};
          }
          P[s] = pv;
          R[s] = rv;
        }
      }
      __syncthreads();
    }

    const double bn = sqrt(bn2);
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int slice = slc[t];
      if (slice >= 0) {
        const int row = perm[slice * 64 + lane];
        const cpx<double> xh = XH[slice * 64 + lane];
        if (row >= 0)
          D[(unsigned)row * (unsigned)ldd + ocol] = cpx<T>{T(xh.re * bn), T(xh.im * bn)};
      }
    }
    if (tid == 0) {
      iters[ocol] = it;
      if (resid_out) resid_out[ocol] = last_res;
      if (nref) atomicAdd(&stats[0], nref);
      if (nbd > 3) atomicAdd(&stats[1], 1);
    }
    // A barrier between this thread-0 block and the thread-0 fetch of the
    // next item: without it the compiler may merge the two blocks and send
    // the other threads straight to the fetch's barrier, where they would
    // read the old item again while thread 0 still waits to run.
    __syncthreads();
  }
}

size_t cocg_resident_xhi_slots(int n, int blocks) {
  return (size_t)blocks * (size_t)((n + 63) / 64) * 64;
}

// p and r in LDS: 16 B per slot in FP32, 32 B in FP64.
int cocg_resident_max_n(bool fp32) { return (fp32 ? 8 : 4) * kResWaves * 64; }

int cocg_resident_waves() { return kResWaves; }

// Slice-to-wave table: contiguous runs of the width-sorted slices, as many
// per wave as keep (slots x widest width) under a common bound C, with C the
// smallest bound for which kResWaves waves of at most rpt slots suffice.  A
// wave's batch loop runs to its widest slot and loads every slot at each
// step, so its cost is its slot count times its widest width.
std::vector<int> cocg_resident_wave_table(const std::vector<int>& widths, int rpt) {
  const int nsl = (int)widths.size();
  auto place = [&](long long C, std::vector<int>* out) {
    int s = 0;
    for (int wv = 0; wv < kResWaves; ++wv) {
      int k = 0;
      if (s < nsl) {
        const long long w0 = widths[s] > 0 ? widths[s] : 1;
        k = (int)std::min<long long>(rpt, C / w0);
        if (k < 1) return false;
        k = std::min(k, nsl - s);
      }
      if (out)
        for (int t = 0; t < rpt; ++t) (*out)[wv * rpt + t] = t < k ? s + t : -1;
      s += k;
    }
    return s >= nsl;
  };
  long long lo = 1, hi = 1;
  for (int w : widths) hi = std::max<long long>(hi, (long long)w * rpt);
  if (!place(hi, nullptr)) return {};
  while (lo < hi) {
    const long long mid = (lo + hi) / 2;
    if (place(mid, nullptr))
      hi = mid;
    else
      lo = mid + 1;
  }
  std::vector<int> tab((size_t)kResWaves * rpt, -1);
  place(hi, &tab);
  return tab;
}

size_t cocg_resident_lds(int n, bool fp32) {
  const size_t nsl = (size_t)(n + 63) / 64;
  // p and r, the zero and trash rows, the reduction slots, the work item
  return (nsl * 64 * 2 + 128) * (fp32 ? sizeof(cpx<float>) : sizeof(cpx<double>)) +
         2 * kResWaves * 4 * sizeof(double) + 16;
}

template <typename T, int RPT, bool MULTI>
static hipError_t launch_res(hipStream_t st, const ResGraph& g0, const ResGraph* graphs, int max_n,
                             const CocgLaunch& L, int blocks) {
  auto kern = k_cocg_resident<T, RPT, MULTI>;
  // the gathers address LDS absolutely: the kernel must own no static LDS
  hipFuncAttributes fa;
  hipError_t fe = hipFuncGetAttributes(&fa, (const void*)kern);
  if (fe != hipSuccess) return fe;
  if (fa.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
  const size_t lds = cocg_resident_lds(max_n, sizeof(T) == 4);
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int max_npad = (max_n + 63) / 64 * 64;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kResThreads), lds, st, g0.nslices, g0.sbase,
                     g0.perm, g0.ent, g0.ent64, g0.n32, L.nitems, L.items, g0.zs, g0.B, g0.ldb,
                     g0.kcols, g0.D, g0.ldd, L.tol, L.maxit, L.max_refine, L.counter, g0.iters,
                     g0.stats,
                     g0.resid, (cpx<double>*)L.xhi, g0.zero_base, g0.wave_slices, graphs,
                     max_npad);
  return hipGetLastError();
}

template <typename T, int RPT, bool MULTI>
static hipError_t prepare_res(int max_n) {
  const size_t lds = cocg_resident_lds(max_n, sizeof(T) == 4);
  return hipFuncSetAttribute((const void*)k_cocg_resident<T, RPT, MULTI>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t prepare_cocg_resident(int max_n, int rpt, bool fp32) {
  if (max_n < 1 || max_n > cocg_resident_max_n(fp32)) return hipErrorInvalidValue;
  if (fp32) {
    if (rpt == 1) return prepare_res<float, 1, true>(max_n);
    if (rpt == 2) return prepare_res<float, 2, true>(max_n);
    if (rpt == 4) return prepare_res<float, 4, true>(max_n);
    if (rpt == 8) return prepare_res<float, 8, true>(max_n);
    return hipErrorInvalidValue;
  }
  if (rpt == 1) return prepare_res<double, 1, true>(max_n);
  if (rpt == 2) return prepare_res<double, 2, true>(max_n);
  if (rpt == 4) return prepare_res<double, 4, true>(max_n);
  return hipErrorInvalidValue;
}

template <typename T, int RPT>
static hipError_t launch_res2(hipStream_t st, const ResGraph* g0, const ResGraph* graphs,
                              int max_n, const CocgLaunch& L, int blocks) {
  if (g0) return launch_res<T, RPT, false>(st, *g0, nullptr, max_n, L, blocks);
  return launch_res<T, RPT, true>(st, ResGraph{}, graphs, max_n, L, blocks);
}

hipError_t launch_cocg_resident(hipStream_t st, const ResGraph* g0, const ResGraph* graphs,
                                int max_n, int rpt, const CocgLaunch& L, bool fp32,
                                int num_blocks) {
  if (max_n < 1 || max_n > cocg_resident_max_n(fp32)) return hipErrorInvalidValue;
  if (L.nitems <= 0) return hipSuccess;
  if ((g0 == nullptr) == (graphs == nullptr)) return hipErrorInvalidValue;
  if (!(rpt == 1 || rpt == 2 || rpt == 4 || rpt == 8)) return hipErrorInvalidValue;
  int blocks = num_blocks < L.nitems ? num_blocks : L.nitems;
  if (blocks < 1) blocks = 1;
  const size_t max_npad = (size_t)(max_n + 63) / 64 * 64;
  if (L.xhi == nullptr || (size_t)blocks * max_npad > L.xhi_slots) return hipErrorInvalidValue;
  if (fp32) {
    if (rpt == 1) return launch_res2<float, 1>(st, g0, graphs, max_n, L, blocks);
    if (rpt == 2) return launch_res2<float, 2>(st, g0, graphs, max_n, L, blocks);
    if (rpt == 4) return launch_res2<float, 4>(st, g0, graphs, max_n, L, blocks);
    return launch_res2<float, 8>(st, g0, graphs, max_n, L, blocks);
  }
  if (rpt == 1) return launch_res2<double, 1>(st, g0, graphs, max_n, L, blocks);
  if (rpt == 2) return launch_res2<double, 2>(st, g0, graphs, max_n, L, blocks);
  if (rpt == 4) return launch_res2<double, 4>(st, g0, graphs, max_n, L, blocks);
  return hipErrorInvalidValue;
}

}  // namespace rafeast
