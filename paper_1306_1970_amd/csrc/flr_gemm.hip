// FP64 matrix-core products of the lambda-grid solver (see flr_gemm.h).
//
// Tiling: a workgroup (4 wave64) owns a 64 x 64 output tile, each wave a
// 32 x 32 quarter computed as 2 x 2 blocks of v_mfma_f64_16x16x4f64.  The
// reduction runs over K in tiles of 32 staged through LDS (double-buffered:
// the next tile's global loads are in flight while the matrix cores work on
// the current one; one barrier per tile).  Inside an MFMA the four reduction
// slots are fed by the four 16-lane groups of the wave; group g takes the
// reduction indices 4g .. 4g + 3 of a 16-wide slice over four consecutive
// instructions, so every lane reads its four operands as one contiguous
// 32-byte LDS load (A and B use the same assignment, so the sum is the same).
// X is widened to FP64 as it is staged, in its stored type.
//
// Workgroup ids are mapped to tiles so that the tiles of one row band of X
// (all column tiles of one split-K slice) land on the same XCD (dispatch is
// round-robin over the 8 XCDs by workgroup id), where they share X in L2.
// Each output element is a fixed-order sum that depends only on X and its own
// operand column, never on the batch size or on the column's slot.
#include <hip/hip_runtime.h>

#include "flr_device.h"
#include "flr_gemm.h"

namespace flr {

typedef double dx4 __attribute__((ext_vector_type(4)));

// Eight consecutive stored elements widened to FP64 (16-byte loads).
template <typename XT>
__device__ inline void load8x(const XT* p, double (&v)[8]) {
  constexpr int V = XV<XT>::V;
#pragma unroll
  for (int q = 0; q < 8 / V; ++q) XV<XT>::cvt(load16(p + q * V), v + q * V);
}

__device__ inline void load8d(const double* p, double (&v)[8]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double2 t = *reinterpret_cast<const double2*>(p + 2 * q);
    v[2 * q] = t.x;
    v[2 * q + 1] = t.y;
  }
}

// TR = false: C (M = n) = X O, reduction over the columns of X, split over K
//             into nslice partial outputs.
// TR = true:  C (M = p_pad) = X^T U, reduction over the n rows of X.
// BX (with TR): the right operand is X as well, C = X^T X (the Gram matrix).
template <typename XT, bool TR, bool BX = false>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g) {
  constexpr int MT = kGemmMT, NT = kGemmNT, KT = kGemmKT, LDK = KT + 2;
  __shared__ __align__(16) double As[2][MT * LDK];  // [m][k]
  __shared__ __align__(16) double Bs[2][NT * LDK];  // [n][k]
  const int T = g.tiles_m * g.tiles_n * g.nslice;
  const int per = (T + 7) / 8;
  const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (t >= T) return;
  const int tn = t % g.tiles_n;
  const int rest = t / g.tiles_n;
  const int tm = rest % g.tiles_m;
  const int ts = rest / g.tiles_m;
  const int m0 = tm * MT, n0 = tn * NT;
  const int64_t kbase = (int64_t)ts * g.K;
  const XT* X = reinterpret_cast<const XT*>(g.X);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  double ra[8], rb[8];
  // staging: every thread loads 8 consecutive elements of A and of B per tile
  auto load_tile = [&](int kt) {
    const int64_t k0 = kbase + (int64_t)kt * KT;
    if (!TR) {
      const int r = tid >> 2, c = (tid & 3) * 8;  // row m0 + r of X, columns k0 + c ..
      if (m0 + r < g.M) {
        load8x(X + (int64_t)(m0 + r) * g.ldx + k0 + c, ra);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[e] = 0.0;
      }
    } else {
      const int kr = tid >> 3, c = (tid & 7) * 8;  // row k0 + kr of X, columns m0 + c ..
      if (k0 + kr < g.K) {
        load8x(X + (k0 + kr) * g.ldx + m0 + c, ra);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[e] = 0.0;
      }
    }
    if (BX) {  // B(n, k) = X[k][n]: row k0 + kr of X, columns n0 + c ..
      const int kr = tid >> 3, c = (tid & 7) * 8;
      if (k0 + kr < g.K) {
        load8x(X + (k0 + kr) * g.ldx + n0 + c, rb);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) rb[e] = 0.0;
      }
      return;
    }
    const int cn = tid >> 2, cc = (tid & 3) * 8;  // operand column n0 + cn, entries k0 + cc ..
    if (n0 + cn < g.N) {
      load8d(g.Bm + (int64_t)(n0 + cn) * g.ldb + k0 + cc, rb);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = 0.0;
    }
  };
  auto store_tile = [&](int buf) {
    if (!TR) {
      const int r = tid >> 2, c = (tid & 3) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][r * LDK + c + e] = ra[e];
    } else {
      const int kr = tid >> 3, c = (tid & 7) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][(c + e) * LDK + kr] = ra[e];
    }
    if (BX) {
      const int kr = tid >> 3, c = (tid & 7) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][(c + e) * LDK + kr] = rb[e];
      return;
    }
    const int cn = tid >> 2, cc = (tid & 3) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) Bs[buf][cn * LDK + cc + e] = rb[e];
  };

  const int wm = wave & 1, wn = wave >> 1;
  const int g4 = (lane >> 4) * 4, i16 = lane & 15;
  // The FP64 MFMA returns row i of its 16 x 16 block in lane group i % 4,
  // register i / 4.  Feeding A row sig(i) = 4 (i % 4) + i / 4 into MFMA row i
  // makes lane l hold the output rows 4 (l / 16) + r, r = 0..3: four
  // consecutive rows of one column, stored as one 32-byte write.
  const int sig = 4 * (i16 & 3) + (i16 >> 2);
  dx4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dx4{0.0, 0.0, 0.0, 0.0};

  const int nk = (g.K + KT - 1) / KT;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_tile(kt + 1);
#pragma unroll
    for (int h = 0; h < KT / 16; ++h) {
      dx4 av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[q] = *reinterpret_cast<const dx4*>(&As[buf][(wm * 32 + q * 16 + sig) * LDK + h * 16 + g4]);
        bv[q] = *reinterpret_cast<const dx4*>(&Bs[buf][(wn * 32 + q * 16 + i16) * LDK + h * 16 + g4]);
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][kk], bv[b][kk], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }
  // lane holds C[m = 4 (lane / 16) + r][n = lane % 16] of each 16 x 16 block (rows permuted above)
  double* Cs = g.C + (int64_t)ts * g.cslice;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int n = n0 + wn * 32 + b * 16 + i16;
      const int m = m0 + wm * 32 + a * 16 + g4;
      if (n < g.N) *reinterpret_cast<dx4*>(Cs + (int64_t)n * g.ldc + m) = acc[a][b];
    }
}

template <typename XT, bool TR, bool BX = false>
static hipError_t launch_t(const GemmArgs& g, hipStream_t st) {
  const int T = g.tiles_m * g.tiles_n * g.nslice;
  const int grid = 8 * ((T + 7) / 8);
  hipLaunchKernelGGL((k_gemm_f64<XT, TR, BX>), dim3(grid), dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_gram(int dtype, const GemmArgs& g, hipStream_t st) {
  switch (dtype) {
    case 0: return launch_t<double, true, true>(g, st);
    case 1: return launch_t<float, true, true>(g, st);
    default: return launch_t<uint16_t, true, true>(g, st);
  }
}

hipError_t launch_gemm_xo(int dtype, const GemmArgs& g, hipStream_t st) {
  switch (dtype) {
    case 0: return launch_t<double, false>(g, st);
    case 1: return launch_t<float, false>(g, st);
    default: return launch_t<uint16_t, false>(g, st);
  }
}

hipError_t launch_gemm_xtu(int dtype, const GemmArgs& g, hipStream_t st) {
  switch (dtype) {
    case 0: return launch_t<double, true>(g, st);
    case 1: return launch_t<float, true>(g, st);
    default: return launch_t<uint16_t, true>(g, st);
  }
}

}  // namespace flr
