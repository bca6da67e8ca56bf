// Learned polynomial preconditioner for the shifted solves: training-data
// generation, the coefficient network (forward, backward, Adam), and COCG
// preconditioned by p(A) = sum_{k<8} c_k T_k(A^).
//
// Spectral map A^ = a A + b I (a = 2/(hi - lo), b = -(hi + lo)/(hi - lo)) for
// the Gershgorin interval [lo, hi]; T_k the Chebyshev polynomials.
//
// Training data for a real residual r at shift z: with T_k = T_k(A^) r and
// S_k = A^ T_k = (T_{k+1} + T_{k-1}) / 2 (S_0 = T_1), the vectors
// v_k = (zI - A) T_k = zeta T_k - S_k / a with zeta = z + b/a, so
// G_kl = v_k^H v_l and h_k = v_k^H r follow, for every shift, from the real
// Gram matrix of the 16 vectors {T_k, S_k} of r.
//
// Network: features (Re z^, Im z^, theta^_lo, theta^_hi) -> 64 -> 64 -> 64
// (exact GELU) -> 16 = (Re c_0, Im c_0, ..., Re c_7, Im c_7).  Weights are
// kept in FP32 (Adam's master copy) and used in BF16 (round to nearest even);
// layer inputs are rounded to BF16, sums accumulate in FP32.  One wave per
// sample, one lane per neuron.  Loss per sample:
// (c^H G c - 2 Re(c^H h) + rr) / rr, averaged over the minibatch.
#include <cstdio>
#include <utility>

#include "device.h"
#include "kernels.h"

namespace rafeast {

namespace {

constexpr int kPairs = 136;  // pairs p <= q of 16 vectors
constexpr int kMlpIn = 4, kMlpH = 64, kMlpOut = 16;
// flat parameter offsets (W row-major out x in, then b, per layer)
constexpr int kW1 = 0, kB1 = kW1 + kMlpH * kMlpIn;
constexpr int kW2 = kB1 + kMlpH, kB2 = kW2 + kMlpH * kMlpH;
constexpr int kW3 = kB2 + kMlpH, kB3 = kW3 + kMlpH * kMlpH;
constexpr int kW4 = kB3 + kMlpH, kB4 = kW4 + kMlpOut * kMlpH;
constexpr int kNPar = kB4 + kMlpOut;
static_assert(kNPar == 9680, "parameter count");
// After the trained weights: the input standardization x' = (x - mu) / sd
// (mu[4], sd[4]), fixed from the training features, never rounded to BF16
// and never changed by training.
constexpr int kMu = kNPar, kSd = kNPar + kMlpIn;
constexpr int kNTot = kNPar + 2 * kMlpIn;

__device__ __forceinline__ float bf16_round(float x) {
  // round to nearest even on the upper 16 bits (finite inputs)
  unsigned u = __float_as_uint(x);
  const unsigned lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ float gelu_f(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
         x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

// Orders this wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void pair_index(int t, int& p, int& q) {
  // t enumerates p <= q row by row: (0,0), (0,1), ..., (0,15), (1,1), ...
  p = 0;
  int rem = t;
  while (rem >= 16 - p) {
    rem -= 16 - p;
    ++p;
  }
  q = p + rem;
}

}  // namespace

// ---------------------------------------------------------------------------
// training data
// T: 9 blocks T_0..T_8 (n x kc row-major each, block stride n * kc).
// Partial Gram sums of column i over a row chunk: part[(chunk * kc + i) * 136 + t].
__global__ __launch_bounds__(256) void k_cheb_gram(int64_t n, int kc, const double* __restrict__ T,
                                                   int64_t rows_per_chunk,
                                                   double* __restrict__ part) {
  const int i = blockIdx.x, chunk = blockIdx.y;
  const int t = threadIdx.x;
  if (t >= kPairs) return;
  int p, q;
  pair_index(t, p, q);
  const int64_t r0 = (int64_t)chunk * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  const size_t bs = (size_t)n * kc;
  // vector v of the 16 at row r: T_v for v < 8, S_{v-8} otherwise
  auto val = [&](int v, int64_t r) -> double {
    const size_t o = (size_t)r * kc + i;
    if (v < 8) return T[(size_t)v * bs + o];
    const int k = v - 8;
    if (k == 0) return T[bs + o];
    return 0.5 * (T[(size_t)(k + 1) * bs + o] + T[(size_t)(k - 1) * bs + o]);
  };
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += val(p, r) * val(q, r);
  part[((size_t)chunk * kc + i) * kPairs + t] = s;
}

// Per sample s = j * kc + i: features, G (8 x 8 complex), h (8 complex), rr.
__global__ void k_pc_assemble(int nz, int kc, int nchunks, const double* __restrict__ part,
                              const double* __restrict__ zs, double a, double b, double th_lo,
                              double th_hi, double* __restrict__ X, double* __restrict__ G,
                              double* __restrict__ h, double* __restrict__ rr) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nz * kc) return;
  const int j = s / kc, i = s % kc;
  double Q[16][16];
  for (int t = 0; t < kPairs; ++t) {
    double acc = 0.0;
    for (int c = 0; c < nchunks; ++c) acc += part[((size_t)c * kc + i) * kPairs + t];
    int p, q;
    pair_index(t, p, q);
    Q[p][q] = acc;
    Q[q][p] = acc;
  }
  const double zr = zs[2 * j], zi = zs[2 * j + 1];
  const double er = zr + b / a, ei = zi;  // zeta
  const double al = 1.0 / a, z2 = er * er + ei * ei;
  for (int k = 0; k < 8; ++k) {
    for (int l = 0; l < 8; ++l) {
      // |zeta|^2 T.T - conj(zeta) al T_k.S_l - zeta al S_k.T_l + al^2 S.S
      const double tt = Q[k][l], ts = Q[k][8 + l], st = Q[8 + k][l], ss = Q[8 + k][8 + l];
      const double gr = z2 * tt - al * er * (ts + st) + al * al * ss;
      const double gi = al * ei * (ts - st);
      G[((size_t)s * 64 + k * 8 + l) * 2] = gr;
      G[((size_t)s * 64 + k * 8 + l) * 2 + 1] = gi;
    }
    // h_k = conj(zeta) T_k.r - al S_k.r, r = T_0
    h[((size_t)s * 8 + k) * 2] = er * Q[k][0] - al * Q[8 + k][0];
    h[((size_t)s * 8 + k) * 2 + 1] = -ei * Q[k][0];
  }
  rr[s] = Q[0][0];
  X[(size_t)s * 4] = a * zr + b;
  X[(size_t)s * 4 + 1] = a * zi;
  X[(size_t)s * 4 + 2] = a * th_lo + b;
  X[(size_t)s * 4 + 3] = a * th_hi + b;
}

hipError_t launch_pc_gram_assemble(hipStream_t st, int64_t n, int kc, const double* T, int nz,
                                   const double* zs, double a, double b, double th_lo,
                                   double th_hi, double* part, int nchunks, double* X, double* G,
                                   double* h, double* rr) {
  const int64_t per = (n + nchunks - 1) / nchunks;
  hipLaunchKernelGGL(k_cheb_gram, dim3(kc, nchunks), dim3(256), 0, st, n, kc, T, per, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ns = nz * kc;
  hipLaunchKernelGGL(k_pc_assemble, dim3((ns + 63) / 64), dim3(64), 0, st, nz, kc, nchunks, part,
                     zs, a, b, th_lo, th_hi, X, G, h, rr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// network
__global__ void k_to_bf16(int n, const float* __restrict__ w, float* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = i < kNPar ? bf16_round(w[i]) : w[i];  // the standardization stays FP32
}

// Forward pass of one sample in one wave; weights wb (BF16 values held in
// FP32) in LDS.  On return act[l][*] hold the BF16-rounded inputs of layer
// l (l = 0..3), pre[l] the lane's pre-activation of hidden layer l (lane =
// neuron) and y (lanes < 16) the output.
struct Fwd {
  float pre[3];
  float y;
};

__device__ __forceinline__ Fwd mlp_fwd_wave(const float* __restrict__ wb, const double* x,
                                            float (*act)[kMlpH]) {
  const int lane = threadIdx.x & 63;
  Fwd f;
  if (lane < kMlpIn)
    act[0][lane] = bf16_round((float)((x[lane] - (double)wb[kMu + lane]) / (double)wb[kSd + lane]));
  wave_sync();
  float s = wb[kB1 + lane];
  for (int i = 0; i < kMlpIn; ++i) s += wb[kW1 + lane * kMlpIn + i] * act[0][i];
  f.pre[0] = s;
  act[1][lane] = bf16_round(gelu_f(s));
  wave_sync();
  s = wb[kB2 + lane];
  for (int i = 0; i < kMlpH; ++i) s += wb[kW2 + lane * kMlpH + i] * act[1][i];
  f.pre[1] = s;
  act[2][lane] = bf16_round(gelu_f(s));
  wave_sync();
  s = wb[kB3 + lane];
  for (int i = 0; i < kMlpH; ++i) s += wb[kW3 + lane * kMlpH + i] * act[2][i];
  f.pre[2] = s;
  act[3][lane] = bf16_round(gelu_f(s));
  wave_sync();
  f.y = 0.0f;
  if (lane < kMlpOut) {
    s = wb[kB4 + lane];
    for (int i = 0; i < kMlpH; ++i) s += wb[kW4 + lane * kMlpH + i] * act[3][i];
    f.y = s;
  }
  return f;
}

constexpr int kMlpWaves = 4;

// Y[s][0..16) for s < ns (FP32 outputs).
__global__ __launch_bounds__(256) void k_mlp_forward(int ns, const double* __restrict__ X,
                                                     const float* __restrict__ wb_g,
                                                     float* __restrict__ Y) {
  __shared__ float wb[kNTot];
  __shared__ float act[kMlpWaves][4][kMlpH];
  for (int i = threadIdx.x; i < kNTot; i += blockDim.x) wb[i] = wb_g[i];
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int s = blockIdx.x * kMlpWaves + wv; s < ns; s += gridDim.x * kMlpWaves) {
    const Fwd f = mlp_fwd_wave(wb, X + (size_t)s * 4, act[wv]);
    if (lane < kMlpOut) Y[(size_t)s * kMlpOut + lane] = f.y;
    wave_sync();
  }
}

// Forward and backward over the samples idx[0..nb) of a minibatch: each
// wave accumulates the gradient of its samples' mean loss (1/nb weight) in
// registers (lane = neuron: its rows of W2, W3, W4, W1 and biases) and
// writes it to part[wave][0..9680); loss partials to lpart[wave].
__global__ __launch_bounds__(256) void k_mlp_backward(
    int nb, const int* __restrict__ idx, const double* __restrict__ X,
    const double* __restrict__ G, const double* __restrict__ h, const double* __restrict__ rr,
    const float* __restrict__ wb_g, float* __restrict__ part, double* __restrict__ lpart) {
  __shared__ float wb[kNTot];
  __shared__ float act[kMlpWaves][4][kMlpH];
  __shared__ float dlt[kMlpWaves][kMlpH];
  for (int i = threadIdx.x; i < kNTot; i += blockDim.x) wb[i] = wb_g[i];
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gw = blockIdx.x * kMlpWaves + wv, nw = gridDim.x * kMlpWaves;
  float g1[kMlpIn], g2[kMlpH], g3[kMlpH], g4[kMlpH];
  float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, gb4 = 0.f;
  for (int i = 0; i < kMlpIn; ++i) g1[i] = 0.f;
  for (int i = 0; i < kMlpH; ++i) g2[i] = g3[i] = g4[i] = 0.f;
  double lsum = 0.0;
  const float inv = 1.0f / (float)nb;
  for (int t = gw; t < nb; t += nw) {
    const int s = idx[t];
    const Fwd f = mlp_fwd_wave(wb, X + (size_t)s * 4, act[wv]);
    // coefficients c = y / Im z^ (the network predicts c scaled by the
    // shift's distance from the real axis, an O(1) quantity)
    const double cs = 1.0 / X[(size_t)s * 4 + 1];
    // loss and dL/dy: lanes k < 8 form (G c - h)_k
    dlt[wv][lane] = lane < kMlpOut ? (float)(f.y * cs) : 0.0f;
    wave_sync();
    const double* Gs = G + (size_t)s * 128;
    const double* hs = h + (size_t)s * 16;
    const double rrs = rr[s];
    double gre = 0.0, gim = 0.0, cre = 0.0, cim = 0.0;
    if (lane < 8) {
      for (int l = 0; l < 8; ++l) {
        const double ar = Gs[(lane * 8 + l) * 2], ai = Gs[(lane * 8 + l) * 2 + 1];
        const double br = dlt[wv][2 * l], bi = dlt[wv][2 * l + 1];
        gre += ar * br - ai * bi;
        gim += ar * bi + ai * br;
      }
      cre = dlt[wv][2 * lane];
      cim = dlt[wv][2 * lane + 1];
    }
    // per-lane part of c^H G c - 2 Re(c^H h): Re(conj(c_k) (Gc)_k) - 2 Re(conj(c_k) h_k)
    double lp = 0.0;
    if (lane < 8) {
      lp = cre * gre + cim * gim - 2.0 * (cre * hs[2 * lane] + cim * hs[2 * lane + 1]);
    }
    const double lw = wave_sum(lp);
    lsum += (lw + rrs) / rrs;
    wave_sync();
    // dL/dy (mean over the minibatch)
    float d4 = 0.0f;
    if (lane < 8) {
      const double sc = 2.0 / rrs * cs;  // dL/dy = dL/dc / Im z^
      dlt[wv][2 * lane] = (float)((gre - hs[2 * lane]) * sc) * inv;
      dlt[wv][2 * lane + 1] = (float)((gim - hs[2 * lane + 1]) * sc) * inv;
    }
    wave_sync();
    if (lane < kMlpOut) d4 = dlt[wv][lane];
    // layer 4: dW4[j][i] += d4_j a3_i (lanes j < 16)
    if (lane < kMlpOut) {
      for (int i = 0; i < kMlpH; ++i) g4[i] += d4 * act[wv][3][i];
      gb4 += d4;
    }
    // delta3_i = gelu'(pre3_i) sum_j W4[j][i] d4_j
    wave_sync();
    float s3 = 0.0f;
    for (int j = 0; j < kMlpOut; ++j) s3 += wb[kW4 + j * kMlpH + lane] * dlt[wv][j];
    const float d3 = s3 * gelu_grad_f(f.pre[2]);
    wave_sync();
    dlt[wv][lane] = d3;
    wave_sync();
    for (int i = 0; i < kMlpH; ++i) g3[i] += d3 * act[wv][2][i];
    gb3 += d3;
    float s2 = 0.0f;
    for (int j = 0; j < kMlpH; ++j) s2 += wb[kW3 + j * kMlpH + lane] * dlt[wv][j];
    const float d2 = s2 * gelu_grad_f(f.pre[1]);
    wave_sync();
    dlt[wv][lane] = d2;
    wave_sync();
    for (int i = 0; i < kMlpH; ++i) g2[i] += d2 * act[wv][1][i];
    gb2 += d2;
    float s1 = 0.0f;
    for (int j = 0; j < kMlpH; ++j) s1 += wb[kW2 + j * kMlpH + lane] * dlt[wv][j];
    const float d1 = s1 * gelu_grad_f(f.pre[0]);
    for (int i = 0; i < kMlpIn; ++i) g1[i] += d1 * act[wv][0][i];
    gb1 += d1;
    wave_sync();
  }
  float* o = part + (size_t)gw * kNPar;
  for (int i = 0; i < kMlpIn; ++i) o[kW1 + lane * kMlpIn + i] = g1[i];
  o[kB1 + lane] = gb1;
  for (int i = 0; i < kMlpH; ++i) o[kW2 + lane * kMlpH + i] = g2[i];
  o[kB2 + lane] = gb2;
  for (int i = 0; i < kMlpH; ++i) o[kW3 + lane * kMlpH + i] = g3[i];
  o[kB3 + lane] = gb3;
  if (lane < kMlpOut) {
    for (int i = 0; i < kMlpH; ++i) o[kW4 + lane * kMlpH + i] = g4[i];
    o[kB4 + lane] = gb4;
  }
  if (lane == 0) lpart[gw] = lsum;
}

// grad[i] = sum over waves (fixed order) of part[w][i]; loss = sum lpart / nb.
__global__ void k_mlp_reduce(int nwaves, const float* __restrict__ part, float* __restrict__ grad,
                             const double* __restrict__ lpart, int nb, double* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kNPar) {
    float s = 0.0f;
    for (int w = 0; w < nwaves; ++w) s += part[(size_t)w * kNPar + i];
    grad[i] = s;
  } else if (i < kNTot) {
    grad[i] = 0.0f;  // the standardization is not trained
  }
  if (i == 0 && loss) {
    double l = 0.0;
    for (int w = 0; w < nwaves; ++w) l += lpart[w];
    *loss = l / nb;
  }
}

// Adam step t (1-based) on the FP32 master weights; refreshes the BF16 copy.
__global__ void k_adam(int n, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps,
                       float c1, float c2, float* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = bf16_round(wi);
}

// dst (n x 2k real, row-major) <- the real parts of columns c0..c0+k of the
// complex block src (n x ld), then their imaginary parts.
__global__ void k_split_complex(int64_t n, int ld, int c0, int k,
                                const cpx<double>* __restrict__ src, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t r = e / k;
  const int i = (int)(e % k);
  const cpx<double> v = src[r * ld + c0 + i];
  dst[r * 2 * k + i] = v.re;
  dst[r * 2 * k + k + i] = v.im;
}

hipError_t launch_split_complex(hipStream_t st, int64_t n, int ld, int c0, int k,
                                const cpx<double>* src, double* dst) {
  const int64_t total = n * k;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_complex, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n,
                     ld, c0, k, src, dst);
  return hipGetLastError();
}

int mlp_param_count() { return kNTot; }
int mlp_backward_waves(int nb) {
  int w = (nb + 3) / 4;  // about four samples per wave
  if (w > 1024) w = 1024;
  if (w < kMlpWaves) w = kMlpWaves;
  return (w + kMlpWaves - 1) / kMlpWaves * kMlpWaves;
}

hipError_t launch_mlp_bf16(hipStream_t st, const float* w, float* wb) {
  hipLaunchKernelGGL(k_to_bf16, dim3((kNTot + 255) / 256), dim3(256), 0, st, kNTot, w, wb);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(hipStream_t st, int ns, const double* X, const float* wb, float* Y) {
  int blocks = (ns + kMlpWaves - 1) / kMlpWaves;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(64 * kMlpWaves), 0, st, ns, X, wb, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(hipStream_t st, int nb, const int* idx, const double* X,
                           const double* G, const double* h, const double* rr, const float* wb,
                           float* part, double* lpart, float* grad, double* loss) {
  const int waves = mlp_backward_waves(nb);
  hipLaunchKernelGGL(k_mlp_backward, dim3(waves / kMlpWaves), dim3(64 * kMlpWaves), 0, st, nb,
                     idx, X, G, h, rr, wb, part, lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNTot + 255) / 256), dim3(256), 0, st, waves, part, grad,
                     lpart, nb, loss);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t st, float* w, float* m, float* v, const float* g, float lr,
                       int step, float* wb) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((kNPar + 255) / 256), dim3(256), 0, st, kNPar, w, m, v, g, lr,
                     b1, b2, eps, c1, c2, wb);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Preconditioned COCG (FP64, all columns in lock step).  Vectors are
// n x Bc complex FP64 blocks, row-major; a workgroup owns a contiguous row
// range and 256 columns (thread = column); per-column partial sums go to
// part[(block * Bc + c) * NQ + q] and are summed in a fixed order.
namespace {
constexpr int kPcT = 256;

struct PcRows {
  int64_t r0, r1;
};
__device__ __forceinline__ PcRows pc_rows(int64_t n) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  return {r0 < n ? r0 : n, r0 + per < n ? r0 + per : n};
}
__device__ __forceinline__ cpx<double> cm(cpx<double> a, cpx<double> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
}  // namespace

// out = coef_c r + s * (a A bk1 + b bk1) - bk2 (bk1, bk2 nullable = 0);
// with part, partials of r^T out.
__global__ __launch_bounds__(kPcT) void k_pc_cheb(
    int64_t n, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ val, double a, double b, int Bc,
    const double* __restrict__ coef /*[Bc] complex*/, double sA, const cpx<double>* __restrict__ r,
    const cpx<double>* __restrict__ bk1, const cpx<double>* __restrict__ bk2,
    cpx<double>* __restrict__ out, double* __restrict__ part) {
  const int c = blockIdx.y * kPcT + threadIdx.x;
  if (c >= Bc) return;
  const cpx<double> cf{coef[2 * c], coef[2 * c + 1]};
  double pr = 0.0, pi = 0.0;
  const PcRows rg = pc_rows(n);
  for (int64_t row = rg.r0; row < rg.r1; ++row) {
    const size_t o = (size_t)row * Bc + c;
    const cpx<double> rv = r[o];
    cpx<double> y = cm(cf, rv);
    if (bk1) {
      double ar = 0.0, ai = 0.0;
      for (int t = rowptr[row]; t < rowptr[row + 1]; ++t) {
        const cpx<double> v = bk1[(size_t)col[t] * Bc + c];
        ar += val[t] * v.re;
        ai += val[t] * v.im;
      }
      const cpx<double> own = bk1[o];
      y.re += sA * (a * ar + b * own.re);
      y.im += sA * (a * ai + b * own.im);
    }
    if (bk2) {
      const cpx<double> v = bk2[o];
      y.re -= v.re;
      y.im -= v.im;
    }
    out[o] = y;
    pr += rv.re * y.re - rv.im * y.im;
    pi += rv.re * y.im + rv.im * y.re;
  }
  if (part) {
    part[((size_t)blockIdx.x * Bc + c) * 2] = pr;
    part[((size_t)blockIdx.x * Bc + c) * 2 + 1] = pi;
  }
}

// p = u + beta p (own and gathered rows; pnew written), w = z p - A p,
// partials of p^T w.
__global__ __launch_bounds__(kPcT) void k_pc_spmm(
    int64_t n, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ val, int Bc, const double* __restrict__ zc,
    const double* __restrict__ beta, const cpx<double>* __restrict__ u,
    const cpx<double>* __restrict__ pold, cpx<double>* __restrict__ pnew,
    cpx<double>* __restrict__ w, double* __restrict__ part) {
  const int c = blockIdx.y * kPcT + threadIdx.x;
  if (c >= Bc) return;
  const cpx<double> bt{beta[2 * c], beta[2 * c + 1]};
  const cpx<double> z{zc[2 * c], zc[2 * c + 1]};
  double mr = 0.0, mi = 0.0;
  const PcRows rg = pc_rows(n);
  for (int64_t row = rg.r0; row < rg.r1; ++row) {
    const size_t o = (size_t)row * Bc + c;
    const cpx<double> pb = cm(bt, pold[o]);
    const cpx<double> pv{u[o].re + pb.re, u[o].im + pb.im};
    double ar = 0.0, ai = 0.0;
    for (int t = rowptr[row]; t < rowptr[row + 1]; ++t) {
      const size_t q = (size_t)col[t] * Bc + c;
      const cpx<double> pq = cm(bt, pold[q]);
      ar += val[t] * (u[q].re + pq.re);
      ai += val[t] * (u[q].im + pq.im);
    }
    const cpx<double> zp = cm(z, pv);
    const cpx<double> wv{zp.re - ar, zp.im - ai};
    pnew[o] = pv;
    w[o] = wv;
    mr += pv.re * wv.re - pv.im * wv.im;
    mi += pv.re * wv.im + pv.im * wv.re;
  }
  part[((size_t)blockIdx.x * Bc + c) * 2] = mr;
  part[((size_t)blockIdx.x * Bc + c) * 2 + 1] = mi;
}

// x += alpha p, r -= alpha w; partials of ||r||^2 and r^T r.
__global__ __launch_bounds__(kPcT) void k_pc_update(int64_t n, int Bc,
                                                   const double* __restrict__ alpha,
                                                   cpx<double>* __restrict__ x,
                                                   cpx<double>* __restrict__ r,
                                                   const cpx<double>* __restrict__ p,
                                                   const cpx<double>* __restrict__ w,
                                                   double* __restrict__ part) {
  const int c = blockIdx.y * kPcT + threadIdx.x;
  if (c >= Bc) return;
  const cpx<double> al{alpha[2 * c], alpha[2 * c + 1]};
  double s2 = 0.0, sr = 0.0, si = 0.0;
  const PcRows rg = pc_rows(n);
  for (int64_t row = rg.r0; row < rg.r1; ++row) {
    const size_t o = (size_t)row * Bc + c;
    const cpx<double> ap = cm(al, p[o]), aw = cm(al, w[o]);
    x[o].re += ap.re;
    x[o].im += ap.im;
    cpx<double> rv = r[o];
    rv.re -= aw.re;
    rv.im -= aw.im;
    r[o] = rv;
    s2 += rv.re * rv.re + rv.im * rv.im;
    sr += rv.re * rv.re - rv.im * rv.im;
    si += 2.0 * rv.re * rv.im;
  }
  part[((size_t)blockIdx.x * Bc + c) * 3] = s2;
  part[((size_t)blockIdx.x * Bc + c) * 3 + 1] = sr;
  part[((size_t)blockIdx.x * Bc + c) * 3 + 2] = si;
}

// Start (init) or true-residual check: for columns with flag set,
// s = b - (zI - A) x (x = 0 at the start), r = s; partials of ||s||^2 and
// s^T s.  Column c takes B[:, c % kb].
__global__ __launch_bounds__(kPcT) void k_pc_resid(
    int64_t n, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ val, int Bc, const double* __restrict__ zc,
    const double* __restrict__ B, int ldb, int kb, const int* __restrict__ flag, int init,
    cpx<double>* __restrict__ x, cpx<double>* __restrict__ r, double* __restrict__ part) {
  const int c = blockIdx.y * kPcT + threadIdx.x;
  if (c >= Bc) return;
  const bool on = init || flag[c] != 0;
  const cpx<double> z{zc[2 * c], zc[2 * c + 1]};
  double s2 = 0.0, sr = 0.0, si = 0.0;
  const PcRows rg = pc_rows(n);
  for (int64_t row = rg.r0; row < rg.r1; ++row) {
    if (!on) break;
    const size_t o = (size_t)row * Bc + c;
    const double bv = B[(size_t)row * ldb + c % kb];
    cpx<double> s{bv, 0.0};
    if (init) {
      x[o] = cpx<double>{0.0, 0.0};
    } else {
      double ar = 0.0, ai = 0.0;
      for (int t = rowptr[row]; t < rowptr[row + 1]; ++t) {
        const cpx<double> xv = x[(size_t)col[t] * Bc + c];
        ar += val[t] * xv.re;
        ai += val[t] * xv.im;
      }
      const cpx<double> zx = cm(z, x[o]);
      s.re -= zx.re - ar;
      s.im -= zx.im - ai;
    }
    r[o] = s;
    s2 += s.re * s.re + s.im * s.im;
    sr += s.re * s.re - s.im * s.im;
    si += 2.0 * s.re * s.im;
  }
  part[((size_t)blockIdx.x * Bc + c) * 3] = s2;
  part[((size_t)blockIdx.x * Bc + c) * 3 + 1] = sr;
  part[((size_t)blockIdx.x * Bc + c) * 3 + 2] = si;
}

// Per-column scalars (one thread per column, fixed-order sums over blocks).
//  mode 0 (start):  bn2 = ||b||^2; active = bn2 > 0; done columns get x = 0
//  mode 1 (mu):     alpha = rho / mu for active columns, else 0
//  mode 2 (resid):  it += 1 for active; pending = ||r||^2 <= tol^2 bn2 or
//                   it >= maxit; without a preconditioner also rho_new = r^T r
//  mode 3 (check):  for pending: res = ||s||/||b||; done if <= tol or it >= maxit
//  mode 4 (rho):    beta = rho_new / rho, rho = rho_new for active columns
__global__ void k_pc_fin(int mode, int Bc, int nb, const double* __restrict__ part, int nq,
                         PcCols cols, double tol, int maxit, int precond,
                         int* __restrict__ counts) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Bc) return;
  double s[3] = {0.0, 0.0, 0.0};
  for (int bb = 0; bb < nb; ++bb)
    for (int q = 0; q < nq; ++q) s[q] += part[((size_t)bb * Bc + c) * nq + q];
  const bool act = cols.active[c] != 0;
  switch (mode) {
    case 0:
      cols.bn2[c] = s[0];
      cols.active[c] = s[0] > 0.0 ? 1 : 0;
      if (s[0] > 0.0) atomicAdd(&counts[1], 1);
      cols.it[c] = 0;
      cols.pending[c] = 0;
      cols.res[c] = 0.0;
      cols.beta[2 * c] = cols.beta[2 * c + 1] = 0.0;
      if (!precond) {
        cols.rho[2 * c] = s[1];
        cols.rho[2 * c + 1] = s[2];
      }
      break;
    case 1: {
      double ar = 0.0, ai = 0.0;
      if (act) {
        const zd al = zdiv(zd{cols.rho[2 * c], cols.rho[2 * c + 1]}, zd{s[0], s[1]});
        if (isfinite(al.re) && isfinite(al.im)) {
          ar = al.re;
          ai = al.im;
        } else {
          cols.active[c] = 0;  // breakdown: stop the column, report its residual
          cols.pending[c] = 1;
          atomicAdd(&counts[0], 1);
        }
      }
      cols.alpha[2 * c] = ar;
      cols.alpha[2 * c + 1] = ai;
      break;
    }
    case 2:
      if (act) {
        cols.it[c] += 1;
        if (s[0] <= tol * tol * cols.bn2[c] || cols.it[c] >= maxit) {
          cols.pending[c] = 1;
          atomicAdd(&counts[0], 1);
        }
        if (!precond) {
          cols.rhon[2 * c] = s[1];
          cols.rhon[2 * c + 1] = s[2];
        }
      }
      break;
    case 3:
      if (cols.pending[c]) {
        cols.pending[c] = 0;
        cols.res[c] = sqrt(s[0] / cols.bn2[c]);
        if (s[0] <= tol * tol * cols.bn2[c] || cols.it[c] >= maxit) cols.active[c] = 0;
        if (!precond) {  // the replaced residual's r^T r
          cols.rhon[2 * c] = s[1];
          cols.rhon[2 * c + 1] = s[2];
        }
      }
      if (cols.active[c]) atomicAdd(&counts[1], 1);
      break;
    case 4:
      if (precond) {
        cols.rhon[2 * c] = s[0];
        cols.rhon[2 * c + 1] = s[1];
      }
      if (act) {
        const zd bt = zdiv(zd{cols.rhon[2 * c], cols.rhon[2 * c + 1]},
                           zd{cols.rho[2 * c], cols.rho[2 * c + 1]});
        const bool ok = isfinite(bt.re) && isfinite(bt.im);
        cols.beta[2 * c] = ok ? bt.re : 0.0;
        cols.beta[2 * c + 1] = ok ? bt.im : 0.0;
        cols.rho[2 * c] = cols.rhon[2 * c];
        cols.rho[2 * c + 1] = cols.rhon[2 * c + 1];
      } else {
        cols.beta[2 * c] = cols.beta[2 * c + 1] = 0.0;  // p = u stays bounded
      }
      break;
  }
}

int pc_blocks(int64_t n, int num_cu) {
  int64_t nb = (int64_t)num_cu * 4;
  if (nb > n) nb = n;
  return nb < 1 ? 1 : (int)nb;
}

hipError_t run_pc_cocg(hipStream_t st, const PcSolve& S) {
  const int Bc = S.Bc;
  const int nb = pc_blocks(S.n, S.num_cu);
  const dim3 grid(nb, (Bc + kPcT - 1) / kPcT), blk(kPcT), fg((Bc + 255) / 256), fb(256);
  const bool pre = S.coef != nullptr;
  auto fin = [&](int mode, int nq) {
    hipLaunchKernelGGL(k_pc_fin, fg, fb, 0, st, mode, Bc, nb, S.part, nq, S.cols, S.tol, S.maxit,
                       pre ? 1 : 0, S.counts);
    return hipGetLastError();
  };
#define PCL(...)                     \
  do {                               \
    hipLaunchKernelGGL(__VA_ARGS__); \
    hipError_t _e = hipGetLastError(); \
    if (_e != hipSuccess) return _e; \
  } while (0)
#define PCE(expr)                    \
  do {                               \
    hipError_t _e = (expr);          \
    if (_e != hipSuccess) return _e; \
  } while (0)
  cpx<double>* X = S.x;
  cpx<double>* R = S.r;
  cpx<double>* U = pre ? S.u : S.r;  // no preconditioner: u is r itself
  cpx<double>* Pa = S.p0;
  cpx<double>* Pb = S.p1;
  cpx<double>* W = S.w;
  // M r by Clenshaw: b_7 = c_7 r; b_k = c_k r + 2 A^ b_{k+1} - b_{k+2}
  // (k = 6..1); u = c_0 r + A^ b_1 - b_2; partials of r^T u
  auto apply_m = [&]() -> hipError_t {
    cpx<double>* bb[3] = {S.t0, S.t1, S.t2};  // b_{k+2}, b_{k+1}, b_k (rotating)
    const size_t cs = (size_t)Bc * 2;
    PCL(k_pc_cheb, grid, blk, 0, st, S.n, S.rowptr, S.col, S.val, S.a, S.b, Bc, S.coef + 7 * cs,
        0.0, R, (const cpx<double>*)nullptr, (const cpx<double>*)nullptr, bb[1], (double*)nullptr);
    for (int k = 6; k >= 1; --k) {
      PCL(k_pc_cheb, grid, blk, 0, st, S.n, S.rowptr, S.col, S.val, S.a, S.b, Bc,
          S.coef + k * cs, 2.0, R, bb[1], k == 6 ? (const cpx<double>*)nullptr : bb[0], bb[2],
          (double*)nullptr);
      cpx<double>* t = bb[0];
      bb[0] = bb[1];
      bb[1] = bb[2];
      bb[2] = t;
    }
    PCL(k_pc_cheb, grid, blk, 0, st, S.n, S.rowptr, S.col, S.val, S.a, S.b, Bc, S.coef, 1.0, R,
        bb[1], bb[0], U, S.part);
    return hipSuccess;
  };
  // start: x = 0, r = b, u = M r, rho = r^T u
  PCE(hipMemsetAsync(S.counts, 0, 2 * sizeof(int), st));
  PCL(k_pc_resid, grid, blk, 0, st, S.n, S.rowptr, S.col, S.val, Bc, S.zc, S.B, S.ldb, S.kb,
      (const int*)nullptr, 1, X, R, S.part);
  PCE(fin(0, 3));
  if (pre) {
    PCE(apply_m());
    PCE(fin(4, 2));  // rho = r^T u (beta from a zero rho_old is discarded: p_old = 0)
    PCE(hipMemsetAsync(Pa, 0, (size_t)S.n * Bc * sizeof(cpx<double>), st));
  } else {
    PCE(hipMemsetAsync(Pa, 0, (size_t)S.n * Bc * sizeof(cpx<double>), st));
  }
  int host_counts[2] = {0, 0};
  PCE(hipMemcpyAsync(host_counts, S.counts, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  PCE(hipStreamSynchronize(st));
  int live = host_counts[1];
  for (int it = 0; it < S.maxit && live > 0; ++it) {
    PCE(hipMemsetAsync(S.counts, 0, 2 * sizeof(int), st));
    PCL(k_pc_spmm, grid, blk, 0, st, S.n, S.rowptr, S.col, S.val, Bc, S.zc, S.cols.beta, U, Pa,
        Pb, W, S.part);
    std::swap(Pa, Pb);
    PCE(fin(1, 2));
    PCL(k_pc_update, grid, blk, 0, st, S.n, Bc, S.cols.alpha, X, R, Pa, W, S.part);
    PCE(fin(2, 3));
    PCE(hipMemcpyAsync(host_counts, S.counts, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    PCE(hipStreamSynchronize(st));
    if (host_counts[0] > 0) {
      PCL(k_pc_resid, grid, blk, 0, st, S.n, S.rowptr, S.col, S.val, Bc, S.zc, S.B, S.ldb, S.kb,
          S.cols.pending, 0, X, R, S.part);
      PCE(fin(3, 3));
      PCE(hipMemcpyAsync(host_counts, S.counts, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      PCE(hipStreamSynchronize(st));
      live = host_counts[1];
      if (live == 0) break;
    }
    if (S.progress && (it + 1) % 500 == 0)
      std::fprintf(stderr, "rafeast: preconditioned COCG iteration %d, %d systems left\n", it + 1,
                   live);
    if (pre) {
      PCE(apply_m());
      PCE(fin(4, 2));
    } else {
      PCE(fin(4, 3));
    }
  }
#undef PCL
#undef PCE
  return hipSuccess;
}

}  // namespace rafeast
