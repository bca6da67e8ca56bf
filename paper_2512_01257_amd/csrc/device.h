// Device-side helpers shared by the RA-FEAST kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rafeast {

constexpr int kWave = 64;

template <typename T>
struct __align__(2 * sizeof(T)) cpx {
  T re, im;
};

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Wave-wide sum without LDS traffic: DPP butterflies within each 16-lane row
// (xor 1, xor 2 by quad permutes, then the half-row and row mirrors, which
// act as xor 4 and xor 8 once the smaller groups are uniform), then the four
// row sums combined through lane reads.  The result is wave-uniform.
__device__ __forceinline__ float dpp_f32(float v, int ctrl_sel) {
  int x = __float_as_int(v);
  switch (ctrl_sel) {
    case 0: x = __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); break;   // quad [1,0,3,2]
    case 1: x = __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false); break;   // quad [2,3,0,1]
    case 2: x = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false); break;  // row half mirror
    default: x = __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false); break; // row mirror
  }
  return __int_as_float(x);
}

__device__ __forceinline__ float wave_sum_f32(float v) {
  v += dpp_f32(v, 0);
  v += dpp_f32(v, 1);
  v += dpp_f32(v, 2);
  v += dpp_f32(v, 3);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ double dpp_f64(double v, int ctrl_sel) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
  lo = __float_as_int(dpp_f32(__int_as_float(lo), ctrl_sel));
  hi = __float_as_int(dpp_f32(__int_as_float(hi), ctrl_sel));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64(v, 0);
  v += dpp_f64(v, 1);
  v += dpp_f64(v, 2);
  v += dpp_f64(v, 3);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Complex helpers in double.
struct zd {
  double re, im;
};
__device__ __forceinline__ zd zmul(zd a, zd b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ zd zdiv(zd a, zd b) {
  // Smith's algorithm for complex division
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  double r = b.re / b.im, d = b.im + b.re * r;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

// 1/d from the hardware reciprocal estimate refined by two Newton steps
// (each squares the relative error), and Smith's complex division on top of
// it: the COCG step lengths need a few ulp, not a correctly rounded quotient,
// and this costs far fewer FP64 instructions than three IEEE divisions.
__device__ __forceinline__ double rcp_nr(double d) {
  double x = __builtin_amdgcn_rcp(d);
  x = fma(x, fma(-d, x, 1.0), x);
  x = fma(x, fma(-d, x, 1.0), x);
  return x;
}
// 1/sqrt(x) for positive normal x from the hardware estimate refined by two
// Newton steps y <- y (3 - x y^2) / 2 (each squares the relative error).
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
__device__ __forceinline__ zd zdiv_fast(zd a, zd b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im * rcp_nr(b.re), inv = rcp_nr(b.re + b.im * r);
    return {(a.re + a.im * r) * inv, (a.im - a.re * r) * inv};
  }
  const double r = b.re * rcp_nr(b.im), inv = rcp_nr(b.im + b.re * r);
  return {(a.re * r + a.im) * inv, (a.im * r - a.re) * inv};
}

}  // namespace rafeast
