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

// Workgroup barrier that orders LDS only: each wave waits for its own LDS
// operations (lgkmcnt 0) but not for its outstanding global loads, which may
// stay in flight across the barrier (a plain __syncthreads waits for them,
// which defeats loads issued ahead).  The wavefront-scope fences generate no
// code; they keep the compiler from moving memory operations across.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // gfx9 encoding: lgkmcnt(0), vmcnt and expcnt left at their maximum
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
// LDL^T of a symmetric tridiagonal matrix (diagonal d, sub-diagonal
// e_j = M_{j,j-1}, e_0 = 0): L_j = e_j / D_{j-1}, D_j = d_j - e_j L_j.  The
// pivots form one dependent chain, so a single wave runs it: the lanes stage
// 64 (d, e) pairs at a time through this wave's LDS and prefetch the next 64
// from memory while the chain runs on broadcast reads; lane t keeps element t
// of the chunk for one coalesced store.  1/D_j is the hardware reciprocal
// refined by two Newton steps (within an ulp or two of the quotient), so the
// chain carries one multiply, one fma, the reciprocal and four fmas per
// element.  Called by all 64 lanes of one wave; stage: 128 doubles of LDS
// that no other wave touches meanwhile.
__device__ inline void tri_factor_wave(const double* d, const double* e, double* L, double* invD, int64_t p,
                                       double* stage) {
  const int lane = threadIdx.x & 63;
  double rprev = 0.0;  // 1/D_{-1}: e_0 = 0 makes L_0 = 0, D_0 = d_0
  double dn = lane < p ? d[lane] : 1.0;
  double en = lane < p ? e[lane] : 0.0;
  for (int64_t c0 = 0; c0 < p; c0 += 64) {
    stage[2 * lane] = dn;
    stage[2 * lane + 1] = en;
    const int64_t jn = c0 + 64 + lane;
    dn = jn < p ? d[jn] : 1.0;
    en = jn < p ? e[jn] : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double Lout = 0.0, Iout = 0.0;
#pragma unroll 16
    for (int t = 0; t < 64; ++t) {
      const double dt = stage[2 * t], et = stage[2 * t + 1];
      const double Lt = et * rprev;
      const double Dt = fma(-et, Lt, dt);
      double r = __builtin_amdgcn_rcp(Dt);
      r = fma(r, fma(-Dt, r, 1.0), r);
      r = fma(r, fma(-Dt, r, 1.0), r);
      rprev = r;
      Lout = lane == t ? Lt : Lout;
      Iout = lane == t ? r : Iout;
    }
    const int64_t j = c0 + lane;
    if (j < p) {
      L[j] = Lout;
      invD[j] = Iout;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__device__ inline void copy_state(const State* sin, State* sout, const State& s) {
  (void)sin;
  if (blockIdx.x == 0 && threadIdx.x == 0) *sout = s;
}

}  // namespace flr
