// Device helpers shared by the HIP kernels: stored-type loads of X, fixed-tree
// reductions, affine-map scans (the linear recurrences of the tridiagonal
// LDL^T sweeps) and 2x2 projective products (its continued fraction).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "flr_internal.h"

namespace flr {

// ---------------------------------------------------------------------------
// stored-type loads: 16 bytes per lane, widened to double
// ---------------------------------------------------------------------------
template <typename XT> struct XV;
template <> struct XV<double> {
  static constexpr int V = 2;
  using raw = double2;
  __device__ static inline void cvt(const raw& v, double* o) { o[0] = v.x; o[1] = v.y; }
  __device__ static inline void cvt(const raw& v, float* o) { o[0] = (float)v.x; o[1] = (float)v.y; }
};
template <> struct XV<float> {
  static constexpr int V = 4;
  using raw = float4;
  __device__ static inline void cvt(const raw& v, double* o) {
    o[0] = (double)v.x; o[1] = (double)v.y; o[2] = (double)v.z; o[3] = (double)v.w;
  }
  __device__ static inline void cvt(const raw& v, float* o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
};
template <> struct XV<uint16_t> {  // bfloat16 bit patterns
  static constexpr int V = 8;
  using raw = uint4;
  __device__ static inline double lo(uint32_t w) { return (double)__uint_as_float(w << 16); }
  __device__ static inline double hi(uint32_t w) { return (double)__uint_as_float(w & 0xffff0000u); }
  __device__ static inline void cvt(const raw& v, double* o) {
    o[0] = lo(v.x); o[1] = hi(v.x); o[2] = lo(v.y); o[3] = hi(v.y);
    o[4] = lo(v.z); o[5] = hi(v.z); o[6] = lo(v.w); o[7] = hi(v.w);
  }
  __device__ static inline float lof(uint32_t w) { return __uint_as_float(w << 16); }
  __device__ static inline float hif(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
  __device__ static inline void cvt(const raw& v, float* o) {
    o[0] = lof(v.x); o[1] = hif(v.x); o[2] = lof(v.y); o[3] = hif(v.y);
    o[4] = lof(v.z); o[5] = hif(v.z); o[6] = lof(v.w); o[7] = hif(v.w);
  }
};

template <typename XT>
__device__ inline typename XV<XT>::raw load16(const XT* p) {
  return *reinterpret_cast<const typename XV<XT>::raw*>(p);
}

// ---------------------------------------------------------------------------
// reductions and scans over one 256-thread workgroup (fixed trees)
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup; every thread receives the result.  lds: 4 doubles.
__device__ inline double wg_sum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) lds[w] = v;
  __syncthreads();
  return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// Four sums over the workgroup at once (one pair of barriers).  lds: 16 doubles.
__device__ inline void wg_sum4(double* v, double* lds) {
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) lds[4 * w + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (lds[k] + lds[4 + k]) + (lds[8 + k] + lds[12 + k]);
}

// Affine map t -> a t + b.  compose(E, L) applies E first, then L.
struct Aff {
  double a, b;
};
__device__ inline Aff compose(Aff E, Aff Lm) { return {Lm.a * E.a, Lm.a * E.b + Lm.b}; }

// Inclusive scan in thread order 0..255 (recurrence t_j = a_j t_{j-1} + b_j).
// lds: 8 doubles.
__device__ inline Aff wg_scan_fwd(Aff m, double* lds) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double pa = __shfl_up(m.a, d, 64), pb = __shfl_up(m.b, d, 64);
    if (l >= d) m = compose({pa, pb}, m);
  }
  __syncthreads();
  if (l == 63) { lds[2 * w] = m.a; lds[2 * w + 1] = m.b; }
  __syncthreads();
  Aff pre = {1.0, 0.0};
  for (int v = 0; v < w; ++v) pre = compose(pre, {lds[2 * v], lds[2 * v + 1]});
  return compose(pre, m);
}

// Inclusive scan in thread order 255..0 (recurrence t_j = a_j t_{j+1} + b_j).
__device__ inline Aff wg_scan_rev(Aff m, double* lds) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double pa = __shfl_down(m.a, d, 64), pb = __shfl_down(m.b, d, 64);
    if (l + d < 64) m = compose({pa, pb}, m);
  }
  __syncthreads();
  if (l == 0) { lds[2 * w] = m.a; lds[2 * w + 1] = m.b; }
  __syncthreads();
  Aff pre = {1.0, 0.0};
  for (int v = 3; v > w; --v) pre = compose(pre, {lds[2 * v], lds[2 * v + 1]});
  return compose(pre, m);
}

// Inclusive scans over the 64 lanes of one wave (no barriers).
__device__ inline Aff wave_scan_fwd(Aff m) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double pa = __shfl_up(m.a, d, 64), pb = __shfl_up(m.b, d, 64);
    if (l >= d) m = compose({pa, pb}, m);
  }
  return m;
}
__device__ inline Aff wave_scan_rev(Aff m) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double pa = __shfl_down(m.a, d, 64), pb = __shfl_down(m.b, d, 64);
    if (l + d < 64) m = compose({pa, pb}, m);
  }
  return m;
}

// 2x2 projective (Moebius) product used for the continued fraction
// D_j = d_j - e_j^2 / D_{j-1} of the tridiagonal LDL^T factorization.
struct Mob {
  double m00, m01, m10, m11;
};
__device__ inline Mob mob_norm(Mob o) {
  double mx = fmax(fmax(fabs(o.m00), fabs(o.m01)), fmax(fabs(o.m10), fabs(o.m11)));
  if (mx > 0.0 && isfinite(mx)) {
    int ex = ilogb(mx);
    o.m00 = ldexp(o.m00, -ex); o.m01 = ldexp(o.m01, -ex);
    o.m10 = ldexp(o.m10, -ex); o.m11 = ldexp(o.m11, -ex);
  }
  return o;
}
// L * R (R acts first)
__device__ inline Mob mob_mul(Mob Lm, Mob R) {
  return mob_norm({Lm.m00 * R.m00 + Lm.m01 * R.m10, Lm.m00 * R.m01 + Lm.m01 * R.m11,
                   Lm.m10 * R.m00 + Lm.m11 * R.m10, Lm.m10 * R.m01 + Lm.m11 * R.m11});
}

__device__ inline void copy_state(const State* sin, State* sout, const State& s) {
  (void)sin;
  if (blockIdx.x == 0 && threadIdx.x == 0) *sout = s;
}

}  // namespace flr
