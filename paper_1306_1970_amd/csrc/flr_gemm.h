// Batched products of the lambda-grid solver on the gfx950 matrix cores.
//
// Every PCG step of Algorithm 2 needs X^T X p for each column p of the grid;
// over B columns these are two dense products that share X:
//   U = X O      (n x B, reduction over the p columns of X)
//   V = X^T U    (p x B, reduction over the n rows of X)
// Both run as FP64 MFMA (v_mfma_f64_16x16x4f64) with X read in its stored
// type (f64 / f32 / bf16) and widened exactly to FP64 while a tile is staged
// into LDS, so X is never copied and the products equal FP64 GEMMs on the
// stored instance.  The reduced-precision variant (bf16 MFMA with split
// operands, FP32 accumulation) shares the tiling.
//
// Operand layouts (all column-major in the sense "column s contiguous"):
//   X  row-major n x p_pad, row stride ldx
//   O  column s at O + s * ldo, K = p_pad contiguous
//   U  column s at U + s * ldu, ldu >= n rounded up to the tile (64)
//   V  column s at V + s * ldv, ldv = p_pad
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace flr {

struct GemmArgs {
  const void* X;     // stored X
  int64_t ldx;       // row stride of X (elements)
  const double* Bm;  // right operand, column s at Bm + s * ldb (K contiguous)
  int64_t ldb;
  double* C;         // output, column s at C + s * ldc (+ slice * cslice)
  int64_t ldc;
  int64_t cslice;    // stride between split-K partial outputs
  int32_t M, N, K;   // output M x N; K = reduction length of one slice
  int32_t tiles_m, tiles_n, nslice;
};

constexpr int kGemmMT = 64;  // output rows per workgroup tile
constexpr int kGemmNT = 64;  // output columns per workgroup tile
constexpr int kGemmKT = 32;  // reduction depth staged per LDS tile

hipError_t launch_gemm_xo(int dtype, const GemmArgs& g, hipStream_t st);   // U = X O (split over K)
hipError_t launch_gemm_xtu(int dtype, const GemmArgs& g, hipStream_t st);  // V = X^T U
hipError_t launch_gram(int dtype, const GemmArgs& g, hipStream_t st);      // C = X^T X (M = N = columns)

}  // namespace flr
