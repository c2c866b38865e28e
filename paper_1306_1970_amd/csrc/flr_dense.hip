// Algorithm 1 (section 3.1) on the GPU: each MM iteration forms the whole
// system Q = X^T X + lambda1 A + lambda2 B and solves Q b = X^T y through its
// Cholesky factor - the route the paper recommends when M is not banded (a
// general edge set, e.g. all pairs).  X^T X is formed once per problem on the
// FP64 matrix cores (flr_gemm.hip); per MM iteration:
//   reweight  a_j = 1/(|b_j| + eps), w_e = 1/(|b_j - b_k| + eps)
//   assemble  Q (column-major, order nd = p rounded up to 64; the padding is
//             the identity, so the factor of the leading p x p block is that
//             of Q itself)
//   factor    blocked right-looking Cholesky, blocks of 64: a panel launch
//             (every workgroup factors the diagonal block in LDS and solves
//             its own 64 rows of the panel against it) and an MFMA update of
//             the trailing lower triangle, tile by tile
//   solve     L z = c, then L^T b = z, blocked by 64 in one workgroup
//   objective f(b) in FP64: 1/2 ||y - X b||^2 (one pass over X) + penalties
// The host drives the MM loop: one MM step's launches are captured once per
// solve as a HIP graph and replayed every iteration, with one
// synchronization per iteration for f and the pivot flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "flr_device.h"
#include "flr_gemm.h"
#include "flr_problem.h"

namespace flr {

constexpr int kNB = 64;                 // Cholesky block
constexpr int64_t kDenseMaxP = 8192;    // Algorithm 1 keeps two nd x nd FP64 matrices

typedef double dx4v __attribute__((ext_vector_type(4)));

// a_j and the per-CSR-entry weights of the current iterate (majorizer at b).
__global__ __launch_bounds__(kWG) void k_dense_reweight(int64_t p, const double* __restrict__ x,
                                                        const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, double eps,
                                                        double* __restrict__ a, double* __restrict__ w) {
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (j >= p) return;
  const double xj = x[j];
  a[j] = 1.0 / (fabs(xj) + eps);
  for (int q = rowptr[j]; q < rowptr[j + 1]; ++q) w[q] = 1.0 / (fabs(xj - x[col[q]]) + eps);
}

// Column j of Q = G + lambda1 diag(a) + lambda2 L_w (one workgroup per column).
__global__ __launch_bounds__(kWG) void k_dense_assemble(int64_t p, int64_t nd, const double* __restrict__ G,
                                                        double* __restrict__ Q, const double* __restrict__ a,
                                                        const double* __restrict__ w,
                                                        const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col, double l1, double l2) {
  const int64_t j = blockIdx.x;
  double* qc = Q + j * nd;
  const double* gc = G + j * nd;
  for (int64_t i = threadIdx.x; i < nd; i += kWG) qc[i] = j < p ? gc[i] : (i == j ? 1.0 : 0.0);
  __syncthreads();
  if (j >= p) return;
  // edges of row j: distinct rows of column j, so no two threads touch one entry
  for (int q = rowptr[j] + threadIdx.x; q < rowptr[j + 1]; q += kWG) qc[col[q]] -= l2 * w[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    double ws = 0.0;
    for (int q = rowptr[j]; q < rowptr[j + 1]; ++q) ws += w[q];
    qc[j] += l1 * a[j] + l2 * ws;
  }
}

// Panel kb of the blocked factor: the unblocked right-looking Cholesky of
// the tall panel (the diagonal block and the row blocks below it, columns kb
// .. kb + 63).  Workgroup g holds the diagonal block (every workgroup needs
// its pivots and columns) and row blocks 1 + kPR g .. kPR (g + 1) of the
// panel: lane l of wave s keeps row l of each of those blocks, columns
// 16 s .. 16 s + 15, in registers.  At column c the owning wave publishes the
// column of every block it holds in LDS (double-buffered by step parity: one
// barrier per column) and every wave applies the rank-1 update to its own
// columns.  Workgroup 0 writes the factored diagonal block to `diag` (others
// may still be reading it from Q; the update launch moves it into Q); every
// workgroup writes its own row blocks of L back into Q.  Q column-major, ld
// nd; nrb = row blocks in the panel, the diagonal one included; *bad set on a
// pivot that is not positive and finite.
// Panel row blocks per workgroup besides the diagonal block.  One is the
// fastest measured (order 512: factorization 275 us against 310 us with two
// and 345 us with three): fewer registers per lane, more workgroups per panel.
constexpr int kPR = 1;

__global__ __launch_bounds__(kWG) void k_chol_panel(double* __restrict__ Q, int64_t nd, int64_t kb, int nrb,
                                                    int* bad, double* __restrict__ diag) {
  __shared__ __align__(16) double cbuf[2][(1 + kPR) * kNB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int first = 1 + kPR * (int)blockIdx.x;          // first row block beyond the diagonal one
  const int nset = 1 + min(kPR, max(0, nrb - first));   // row sets held, the diagonal block included
  double v[1 + kPR][16];
#pragma unroll
  for (int m = 0; m <= kPR; ++m) {
    const int64_t row = kb + (m == 0 ? 0 : (int64_t)(first + m - 1) * kNB) + lane;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) v[m][kk] = m < nset ? Q[(kb + 16 * wave + kk) * nd + row] : 0.0;
  }
  bool ok = true;
#pragma unroll
  for (int cs = 0; cs < 4; ++cs) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int c = 16 * cs + k;
      double* col = cbuf[c & 1];
      if (wave == cs) {
#pragma unroll
        for (int m = 0; m <= kPR; ++m) col[m * kNB + lane] = v[m][k];
      }
      __syncthreads();
      const double piv = col[c];
      ok = ok && piv > 0.0 && isfinite(piv);
      const double rp = 1.0 / piv;
      double q[1 + kPR];  // a_rc / a_cc for each held row: L_rc L_jc = a_rc a_jc / a_cc
#pragma unroll
      for (int m = 0; m <= kPR; ++m) q[m] = col[m * kNB + lane] * rp;
      if (wave > cs) {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const double lc = col[16 * wave + kk];
#pragma unroll
          for (int m = 0; m <= kPR; ++m) v[m][kk] = fma(-q[m], lc, v[m][kk]);
        }
      } else if (wave == cs) {
#pragma unroll
        for (int kk = k + 1; kk < 16; ++kk) {
          const double lc = col[16 * cs + kk];
#pragma unroll
          for (int m = 0; m <= kPR; ++m) v[m][kk] = fma(-q[m], lc, v[m][kk]);
        }
        const double d = sqrt(piv), rd = 1.0 / d;
        v[0][k] = lane == c ? d : lane > c ? col[lane] * rd : 0.0;
#pragma unroll
        for (int m = 1; m <= kPR; ++m) v[m][k] = col[m * kNB + lane] * rd;
      }
    }
  }
  if (!ok) {  // the same decision in every thread
    if (tid == 0 && blockIdx.x == 0) *bad = 1;
    return;
  }
  if (blockIdx.x == 0) {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) diag[(16 * wave + kk) * kNB + lane] = v[0][kk];
  }
#pragma unroll
  for (int m = 1; m <= kPR; ++m) {
    if (m < nset) {
      const int64_t row = kb + (int64_t)(first + m - 1) * kNB + lane;
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) Q[(kb + 16 * wave + kk) * nd + row] = v[m][kk];
    }
  }
}

// The factored diagonal block of panel kb from `diag` into Q (lower triangle).
__device__ inline void put_diag(double* __restrict__ Q, int64_t nd, int64_t kb, const double* __restrict__ diag) {
  for (int e = threadIdx.x; e < kNB * kNB; e += kWG) {
    const int r = e % kNB, c = e / kNB;
    if (r >= c) Q[(kb + c) * nd + kb + r] = diag[c * kNB + r];
  }
}

__global__ __launch_bounds__(kWG) void k_chol_put_diag(double* __restrict__ Q, int64_t nd, int64_t kb,
                                                       const double* __restrict__ diag) {
  put_diag(Q, nd, kb, diag);
}

// Trailing update after panel kb (workgroup 0 also moves the factored
// diagonal block into Q): tile (bi, bj), bi >= bj, of the lower triangle
// below and right of the panel: C -= L_i L_j^T with K = 64 (the panel
// columns), on v_mfma_f64_16x16x4f64 (same lane assignment as the grid
// products: A rows fed in the order 4 (i % 4) + i / 4, so each lane holds four
// consecutive rows of one output column).
__global__ __launch_bounds__(kWG) void k_chol_update(double* __restrict__ Q, int64_t nd, int64_t kb, int nt,
                                                     const double* __restrict__ diag) {
  constexpr int LDK = kNB + 4;
  if (blockIdx.x == 0) put_diag(Q, nd, kb, diag);  // disjoint from every tile read or written below
  __shared__ __align__(16) double As[kNB * LDK];
  __shared__ __align__(16) double Bs[kNB * LDK];
  // tile index -> (bi, bj) with bi >= bj over nt blocks
  int t = blockIdx.x, bj = 0;
  while (t >= nt - bj) {
    t -= nt - bj;
    ++bj;
  }
  const int bi = bj + t;
  const int64_t base = kb + kNB;
  const int64_t i0 = base + (int64_t)bi * kNB, j0 = base + (int64_t)bj * kNB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kNB * kNB; e += kWG) {
    const int m = e % kNB, k = e / kNB;  // coalesced along m
    As[m * LDK + k] = Q[(kb + k) * nd + i0 + m];
    Bs[m * LDK + k] = Q[(kb + k) * nd + j0 + m];
  }
  __syncthreads();
  const int wm = wave & 1, wn = wave >> 1;
  const int g4 = (lane >> 4) * 4, i16 = lane & 15;
  const int sig = 4 * (i16 & 3) + (i16 >> 2);
  dx4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dx4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int h = 0; h < kNB / 16; ++h) {
    dx4v av[2], bv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      av[q] = *reinterpret_cast<const dx4v*>(&As[(wm * 32 + q * 16 + sig) * LDK + h * 16 + g4]);
      bv[q] = *reinterpret_cast<const dx4v*>(&Bs[(wn * 32 + q * 16 + i16) * LDK + h * 16 + g4]);
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][kk], bv[b][kk], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t n = j0 + wn * 32 + b * 16 + i16;
      const int64_t m = i0 + wm * 32 + a * 16 + g4;
      dx4v* dst = reinterpret_cast<dx4v*>(Q + n * nd + m);
      *dst = *dst - acc[a][b];
    }
}

// Lane l's value of v, in every lane (v_readlane; l uniform).
__device__ inline double lane_value(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Triangular solves with the factor (one workgroup): forward L z = rhs, then
// backward L^T out = z, both blocked by 64 and right-looking.  Per block one
// wave substitutes through the diagonal block (staged in LDS with the
// reciprocals of its diagonal; the solved value passed between lanes by
// readlane) while the other three waves stage the next diagonal block into
// the second LDS buffer; then all 256 threads subtract the solved block from
// every row still to come - forward, row i reads L[i][block] (64 coalesced
// loads); backward, row j reads L[block][j], 64 consecutive entries of column
// j - so each block costs one round of loads instead of one per earlier block.
__global__ __launch_bounds__(kWG) void k_chol_solve(const double* __restrict__ Q, int64_t nd, int64_t p,
                                                    const double* __restrict__ rhs, double* __restrict__ z,
                                                    double* __restrict__ out) {
  constexpr int LD = kNB + 1;
  __shared__ double Lb[2][kNB * LD];  // Lb[.][c * LD + r] = L[b*64 + r][b*64 + c]
  __shared__ double rdg[2][kNB];      // 1 / L[b*64 + r][b*64 + r]
  __shared__ double zb[kNB];          // the block just solved
  const int tid = threadIdx.x, r = tid & 63, wave = tid >> 6;
  const int nb = (int)(nd / kNB);
  // diagonal block b into buffer u by the threads first .. kWG - 1
  auto stage = [&](int b, int u, int first) {
    const int64_t o = (int64_t)b * kNB;
    for (int e = tid - first; e < kNB * kNB; e += kWG - first) {
      const int c = e >> 6, rr = e & 63;
      Lb[u][c * LD + rr] = Q[(o + c) * nd + o + rr];
    }
    if (tid - first < kNB && tid >= first) rdg[u][tid - first] = 1.0 / Q[(o + tid - first) * nd + o + tid - first];
  };
  for (int64_t i = tid; i < nd; i += kWG) z[i] = i < p ? rhs[i] : 0.0;
  stage(0, 0, 0);
  __syncthreads();
  // forward: z holds the running right-hand side; block b is final once blocks < b are applied
  for (int b = 0; b < nb; ++b) {
    const int u = b & 1;
    if (wave == 0) {
      const int64_t i = (int64_t)b * kNB + r;
      double t = z[i];
      for (int c = 0; c < kNB; ++c) {
        const double zc = lane_value(t, c) * rdg[u][c];
        if (r == c) t = zc;
        else if (r > c) t = fma(-Lb[u][c * LD + r], zc, t);
      }
      z[i] = t;
      zb[r] = t;
    } else if (b + 1 < nb) {
      stage(b + 1, u ^ 1, 64);
    }
    __syncthreads();
    const double* Lc = Q + (int64_t)b * kNB * nd;  // column b*64 of L
    for (int64_t i = (int64_t)(b + 1) * kNB + tid; i < nd; i += kWG) {
      double s = 0.0;
#pragma unroll 16
      for (int c = 0; c < kNB; ++c) s = fma(Lc[(int64_t)c * nd + i], zb[c], s);
      z[i] -= s;
    }
    __syncthreads();
  }
  // backward: z now holds the running right-hand side of L^T out = z
  stage(nb - 1, (nb - 1) & 1, 0);
  __syncthreads();
  for (int b = nb - 1; b >= 0; --b) {
    const int u = b & 1;
    if (wave == 0) {
      const int64_t i = (int64_t)b * kNB + r;  // column of L
      double t = z[i];
      for (int c = kNB - 1; c >= 0; --c) {
        const double xc = lane_value(t, c) * rdg[u][c];
        if (r == c) t = xc;
        else if (r < c) t = fma(-Lb[u][r * LD + c], xc, t);
      }
      out[i] = t;
      zb[r] = t;
    } else if (b > 0) {
      stage(b - 1, u ^ 1, 64);
    }
    __syncthreads();
    for (int64_t j = tid; j < (int64_t)b * kNB; j += kWG) {
      const double* qc = Q + j * nd + (int64_t)b * kNB;  // L[b*64 .. b*64+63][j]
      double s = 0.0;
#pragma unroll 16
      for (int c = 0; c < kNB; ++c) s = fma(qc[c], zb[c], s);
      z[j] -= s;
    }
    __syncthreads();
  }
}

// Per-row squared residual (y_i - X_i b)^2, one wave per row.
template <typename XT>
__global__ __launch_bounds__(kWG) void k_dense_rowres(const XT* __restrict__ X, int64_t ldx, int64_t n, int64_t p_pad,
                                                      const double* __restrict__ y, const double* __restrict__ b,
                                                      double* __restrict__ rr) {
  constexpr int V = XV<XT>::V;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j0 = (int64_t)lane * V; j0 < p_pad; j0 += 64 * V) {
    double xv[V];
    XV<XT>::cvt(load16(X + i * ldx + j0), xv);
#pragma unroll
    for (int v = 0; v < V; ++v) s = fma(xv[v], b[j0 + v], s);
  }
  s = wave_sum(s);
  if (lane == 0) {
    const double d = y[i] - s;
    rr[i] = d * d;
  }
}

// The pivot flag cleared by a kernel (graphs here record no memset nodes).
__global__ __launch_bounds__(kWG) void k_clear_flag(int* __restrict__ flag) {
  if (threadIdx.x == 0) *flag = 0;
}

// G[j][j] = 1 for j < p (the Gram matrix of X = I; the rest stays zero).
__global__ __launch_bounds__(kWG) void k_unit_diagonal(double* __restrict__ G, int64_t nd, int64_t p) {
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (j < p) G[j * nd + j] = 1.0;
}

// X = I: the row residuals are (y_j - b_j)^2.
__global__ __launch_bounds__(kWG) void k_dense_rowres_id(int64_t p, const double* __restrict__ y,
                                                         const double* __restrict__ b, double* __restrict__ rr) {
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (j < p) {
    const double d = y[j] - b[j];
    rr[j] = d * d;
  }
}

// f(b) = 1/2 sum of the row residuals + lambda1 ||b||_1 + lambda2 sum_E |b_j - b_k|
// (one workgroup, fixed order); out[0] = f.
__global__ __launch_bounds__(kWG) void k_dense_objective(int64_t n, int64_t p, const double* __restrict__ rr,
                                                         const double* __restrict__ b,
                                                         const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col, double l1, double l2,
                                                         double* __restrict__ out) {
  __shared__ double red[8];
  double loss = 0.0, pen = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kWG) loss += rr[i];
  for (int64_t j = threadIdx.x; j < p; j += kWG) {
    double e = 0.0;
    for (int q = rowptr[j]; q < rowptr[j + 1]; ++q)
      if (col[q] > j) e += fabs(b[j] - b[col[q]]);
    pen += l1 * fabs(b[j]) + l2 * e;
  }
  const double L = wg_sum(loss, red);
  const double P = wg_sum(pen, red + 4);
  if (threadIdx.x == 0) out[0] = 0.5 * L + P;
}

}  // namespace flr

using namespace flr;

namespace flr {
void set_last_error(const std::string& s);
hipError_t launch_init(const Dims& D, const Bufs& B, const double* warm, int use_warm, hipStream_t st);
bool is_device_pointer(const void* p);

struct DenseOut {
  double f;
  int bad;
  int pad;
};

struct DenseWork {
  int64_t nd = 0;
  double* G = nullptr;    // X^T X, nd x nd column-major (padding zero)
  double* Q = nullptr;    // the system, then its Cholesky factor
  double* a = nullptr;
  double* w = nullptr;
  double* z = nullptr;
  double* xn = nullptr;   // solution of the current MM step
  double* rr = nullptr;   // n row residuals
  double* scal = nullptr; // f
  double* diag = nullptr; // factored diagonal block in flight (64 x 64)
  int* bad = nullptr;
  DenseOut* h_out = nullptr;  // pinned: f of the candidate and the pivot flag of the last step
  size_t bytes = 0;
};

void dense_free(flr_problem h) {
  DenseWork* dw = h->dense;
  if (!dw) return;
  for (void* p : {(void*)dw->G, (void*)dw->Q, (void*)dw->a, (void*)dw->w, (void*)dw->z, (void*)dw->xn, (void*)dw->rr,
                  (void*)dw->scal, (void*)dw->diag, (void*)dw->bad})
    if (p) (void)hipFree(p);
  if (dw->h_out) (void)hipHostFree(dw->h_out);
  h->footprint -= dw->bytes;
  delete dw;
  h->dense = nullptr;
}

static flr_status dfail(flr_status st, const std::string& m) {
  set_last_error(m);
  return st;
}

#define DCK(expr)                                                                                           \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) {                                                                                 \
      (void)hipGetLastError(); /* a failed call also leaves its error for the next check */                 \
      return dfail(e_ == hipErrorOutOfMemory ? FLR_ERR_OUT_OF_MEMORY : FLR_ERR_DEVICE,                      \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                                      \
    }                                                                                                       \
  } while (0)

// Workspace and X^T X, on the first Algorithm 1 solve of a handle; on any
// failure the partial workspace is released, so a later call starts over.
static flr_status dense_prepare_once(flr_problem h);

static flr_status dense_prepare(flr_problem h) {
  if (h->dense) return FLR_OK;
  const flr_status st = dense_prepare_once(h);
  if (st != FLR_OK) {
    (void)hipStreamSynchronize(h->stream);
    dense_free(h);
  }
  return st;
}

static flr_status dense_prepare_once(flr_problem h) {
  const Dims& D = h->D;
  DenseWork* dw = new DenseWork;
  h->dense = dw;
  dw->nd = (D.p + kNB - 1) / kNB * kNB;
  const size_t nd2 = (size_t)dw->nd * (size_t)dw->nd;
  auto al = [&](auto** ptr, size_t count, size_t elem) -> hipError_t {
    const size_t b = std::max<size_t>(count, 1) * elem;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(ptr), b);
    if (e == hipSuccess) {
      dw->bytes += b;
      h->footprint += b;
      e = hipMemsetAsync(*ptr, 0, b, h->stream);
    }
    return e;
  };
  DCK(al(&dw->G, nd2, sizeof(double)));
  DCK(al(&dw->Q, nd2, sizeof(double)));
  DCK(al(&dw->a, (size_t)D.p, sizeof(double)));
  DCK(al(&dw->w, (size_t)std::max<int64_t>(h->nnz, 1), sizeof(double)));
  DCK(al(&dw->z, (size_t)dw->nd, sizeof(double)));
  DCK(al(&dw->xn, (size_t)std::max<int64_t>(dw->nd, D.p_pad), sizeof(double)));  // the solve writes nd entries
  DCK(al(&dw->rr, (size_t)D.n, sizeof(double)));
  DCK(al(&dw->scal, 4, sizeof(double)));
  DCK(al(&dw->diag, (size_t)kNB * kNB, sizeof(double)));
  DCK(al(&dw->bad, 1, sizeof(int)));
  DCK(hipHostMalloc(reinterpret_cast<void**>(&dw->h_out), sizeof(DenseOut), hipHostMallocDefault));
  if (D.flsa) {  // X = I: X^T X = I on the leading p x p block (G was zeroed on this stream)
    hipLaunchKernelGGL(k_unit_diagonal, dim3((unsigned)((D.p + kWG - 1) / kWG)), dim3(kWG), 0, h->stream, dw->G,
                       dw->nd, D.p);
    DCK(hipGetLastError());
  } else {
    GemmArgs g{};
    g.X = h->B.X;
    g.ldx = D.ldx;
    g.C = dw->G;
    g.ldc = dw->nd;
    g.M = (int32_t)dw->nd;
    g.N = (int32_t)dw->nd;
    g.K = (int32_t)D.n;
    g.tiles_m = g.tiles_n = (int32_t)(dw->nd / kGemmMT);
    g.nslice = 1;
    DCK(launch_gram(D.dtype, g, h->stream));
  }
  DCK(hipStreamSynchronize(h->stream));
  return FLR_OK;
}

// f(b) for b in device memory (FP64; one pass over X).
static hipError_t dense_objective(flr_problem h, const double* b, double l1, double l2) {
  DenseWork* dw = h->dense;
  const Dims& D = h->D;
  const unsigned rows = (unsigned)((D.n + 3) / 4);
  if (D.flsa) {
    hipLaunchKernelGGL(k_dense_rowres_id, dim3((unsigned)((D.p + kWG - 1) / kWG)), dim3(kWG), 0, h->stream, D.p,
                       h->B.y, b, dw->rr);
  } else {
    switch (D.dtype) {
      case 0:
        hipLaunchKernelGGL(k_dense_rowres<double>, dim3(rows), dim3(kWG), 0, h->stream,
                           reinterpret_cast<const double*>(h->B.X), D.ldx, D.n, D.p_pad, h->B.y, b, dw->rr);
        break;
      case 1:
        hipLaunchKernelGGL(k_dense_rowres<float>, dim3(rows), dim3(kWG), 0, h->stream,
                           reinterpret_cast<const float*>(h->B.X), D.ldx, D.n, D.p_pad, h->B.y, b, dw->rr);
        break;
      default:
        hipLaunchKernelGGL(k_dense_rowres<uint16_t>, dim3(rows), dim3(kWG), 0, h->stream,
                           reinterpret_cast<const uint16_t*>(h->B.X), D.ldx, D.n, D.p_pad, h->B.y, b, dw->rr);
        break;
    }
  }
  hipLaunchKernelGGL(k_dense_objective, dim3(1), dim3(kWG), 0, h->stream, D.n, D.p, dw->rr, b, h->B.rowptr,
                     h->B.col, l1, l2, dw->scal);
  return hipGetLastError();
}

// Q = L L^T in place (lower triangle); *bad set on a failed pivot.
static hipError_t dense_factor(flr_problem h) {
  DenseWork* dw = h->dense;
  const int64_t nd = dw->nd;
  for (int64_t kb = 0; kb < nd; kb += kNB) {
    const int nrb = (int)((nd - kb) / kNB);
    const unsigned groups = (unsigned)std::max(1, (nrb - 1 + kPR - 1) / kPR);
    hipLaunchKernelGGL(k_chol_panel, dim3(groups), dim3(kWG), 0, h->stream, dw->Q, nd, kb, nrb, dw->bad, dw->diag);
    const int nt = nrb - 1;
    if (nt > 0)
      hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(kWG), 0, h->stream, dw->Q, nd, kb,
                         nt, dw->diag);
    else
      hipLaunchKernelGGL(k_chol_put_diag, dim3(1), dim3(kWG), 0, h->stream, dw->Q, nd, kb, dw->diag);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One MM step of Algorithm 1 enqueued on the problem's stream: reweighting
// at the iterate, assembly of Q, its factorization and the two triangular
// solves into the candidate xn, the candidate's objective, and copies of that
// objective and of the pivot flag into pinned host memory.
static hipError_t dense_step(flr_problem h, double l1, double l2, double eps) {
  const Dims& D = h->D;
  DenseWork* dw = h->dense;
  const unsigned pb = (unsigned)((D.p + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_dense_reweight, dim3(pb), dim3(kWG), 0, h->stream, D.p, h->B.x, h->B.rowptr, h->B.col, eps,
                     dw->a, dw->w);
  hipLaunchKernelGGL(k_dense_assemble, dim3((unsigned)dw->nd), dim3(kWG), 0, h->stream, D.p, dw->nd, dw->G, dw->Q,
                     dw->a, dw->w, h->B.rowptr, h->B.col, l1, l2);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(kWG), 0, h->stream, dw->bad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = dense_factor(h)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(kWG), 0, h->stream, dw->Q, dw->nd, D.p, h->B.c, dw->z, dw->xn);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = dense_objective(h, dw->xn, l1, l2)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(&dw->h_out->f, dw->scal, sizeof(double), hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
    return e;
  return hipMemcpyAsync(&dw->h_out->bad, dw->bad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
}

// One solve by Algorithm 1: the MM loop with an exact (Cholesky) solve per
// iteration.  Same outer test, initialization, warm starts and outputs as the
// PCG path (cg_iters = 0, rel_residual = 0).
flr_status dense_run(flr_problem h, double l1, double l2, double tol, const flr_solve_opts* o, double* beta_out,
                     flr_result* res) {
  auto t0 = std::chrono::steady_clock::now();
  const Dims& D = h->D;
  if (D.p > kDenseMaxP)
    return dfail(FLR_ERR_INVALID_ARG, "Algorithm 1 keeps two dense p x p matrices: p must be <= " +
                                          std::to_string(kDenseMaxP) + " (use Algorithm 2)");
  flr_status ps = dense_prepare(h);
  if (ps != FLR_OK) return ps;
  DenseWork* dw = h->dense;
  const double eps = o->eps > 0.0 ? o->eps : 1e-8;
  const int32_t max_iter = o->max_iter > 0 ? o->max_iter : 10000;
  // initialization / warm start into the handle's iterate (shared with the PCG path)
  const double* warm = nullptr;
  int use_warm = 0;
  if (o->warm_start) {
    if (is_device_pointer(o->warm_start)) {
      warm = o->warm_start;
    } else {
      DCK(hipMemcpyAsync(h->B.r, o->warm_start, D.p * sizeof(double), hipMemcpyHostToDevice, h->stream));
      warm = h->B.r;
    }
    use_warm = 1;
  } else if (o->use_last && h->has_solution) {
    warm = h->B.x;
    use_warm = 1;
  }
  DCK(launch_init(D, h->B, warm, use_warm, h->stream));
  double* x = h->B.x;
  DCK(dense_objective(h, x, l1, l2));
  double f_old = 0.0;
  DCK(hipMemcpyAsync(&f_old, dw->scal, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  DCK(hipStreamSynchronize(h->stream));
  int status = FLR_ERR_MAX_ITER;
  double re = 0.0, f_new = f_old;
  int32_t it = 0;
  // One MM step's device work is captured once per solve as a HIP graph and
  // replayed every iteration (FLR_DENSE_GRAPH=0: launched eagerly instead);
  // the candidate is accepted into the iterate outside the graph, since a
  // failed pivot must leave the iterate as it was.
  const char* gv = std::getenv("FLR_DENSE_GRAPH");
  const bool use_graph = !(gv && gv[0] == '0');
  struct GraphGuard {  // on every return: a replay still in flight finishes before its graph goes
    hipStream_t st;
    hipGraphExec_t exec = nullptr;
    ~GraphGuard() {
      if (!exec) return;
      (void)hipStreamSynchronize(st);
      (void)hipGraphExecDestroy(exec);
    }
  } gg{h->stream};
  if (use_graph) {
    DCK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t body = dense_step(h, l1, l2, eps);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->stream, &graph);
    if (body != hipSuccess && graph) (void)hipGraphDestroy(graph);
    DCK(body);
    DCK(ec);
    const hipError_t ei = hipGraphInstantiate(&gg.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    DCK(ei);
  }
  while (it < max_iter) {
    if (gg.exec)
      DCK(hipGraphLaunch(gg.exec, h->stream));
    else
      DCK(dense_step(h, l1, l2, eps));
    DCK(hipStreamSynchronize(h->stream));
    if (dw->h_out->bad) {
      status = FLR_ERR_NUMERICAL;
      break;
    }
    DCK(hipMemcpyAsync(x, dw->xn, (size_t)D.p * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    f_new = dw->h_out->f;
    ++it;
    re = f_old != 0.0 ? std::fabs(f_new - f_old) / std::fabs(f_old) : std::fabs(f_new - f_old);
    f_old = f_new;
    if (!std::isfinite(f_new)) {
      status = FLR_ERR_NUMERICAL;
      break;
    }
    if (re <= tol) {
      status = FLR_OK;
      break;
    }
  }
  DCK(hipStreamSynchronize(h->stream));
  if (beta_out) DCK(hipMemcpy(beta_out, x, D.p * sizeof(double), hipMemcpyDefault));
  h->has_solution = true;
  if (res) {
    res->objective = f_new;
    res->rel_change = re;
    res->rel_residual = 0.0;
    res->cg_iters = 0;
    res->mm_iters = it;
    res->status = status;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status == FLR_ERR_NUMERICAL) set_last_error("Cholesky pivot not positive or non-finite objective (Algorithm 1)");
  if (status == FLR_ERR_MAX_ITER) set_last_error("MM iteration cap reached");
  return (flr_status)status;
}

// Average durations (us, HIP events on the problem's stream) of the three
// stages of one Algorithm 1 step at the current iterate: reweighting plus
// assembly of Q, the blocked Cholesky factor, and the two triangular solves.
// Writes only Q, a, w, z and xn; the iterate and the last result stay intact.
flr_status dense_profile(flr_problem h, double l1, double l2, int32_t reps, double* avg_us) {
  const Dims& D = h->D;
  DenseWork* dw = h->dense;
  if (!dw) return dfail(FLR_ERR_INVALID_ARG, "profiling Algorithm 1 needs a completed Algorithm 1 solve");
  const unsigned pb = (unsigned)((D.p + kWG - 1) / kWG);
  hipEvent_t ev[4];
  for (auto& e : ev) DCK(hipEventCreate(&e));
  float ms[3] = {0.f, 0.f, 0.f};
  for (int stage = 0; stage < 3; ++stage) {
    DCK(hipEventRecord(ev[0], h->stream));
    for (int i = 0; i < reps; ++i) {
      // the factor needs a fresh Q each time: its assembly runs outside the timed span
      if (stage == 0 || stage == 1) {
        hipLaunchKernelGGL(k_dense_reweight, dim3(pb), dim3(kWG), 0, h->stream, D.p, h->B.x, h->B.rowptr, h->B.col,
                           1e-8, dw->a, dw->w);  // the weights' values do not change the work
        hipLaunchKernelGGL(k_dense_assemble, dim3((unsigned)dw->nd), dim3(kWG), 0, h->stream, D.p, dw->nd, dw->G,
                           dw->Q, dw->a, dw->w, h->B.rowptr, h->B.col, l1, l2);
        DCK(hipGetLastError());
      }
      if (stage == 1) {
        DCK(hipEventRecord(ev[2], h->stream));
        DCK(dense_factor(h));
        DCK(hipEventRecord(ev[3], h->stream));
        DCK(hipStreamSynchronize(h->stream));
        float t = 0.f;
        DCK(hipEventElapsedTime(&t, ev[2], ev[3]));
        ms[1] += t;
      }
      if (stage == 2) {
        hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(kWG), 0, h->stream, dw->Q, dw->nd, D.p, h->B.c, dw->z, dw->xn);
        DCK(hipGetLastError());
      }
    }
    DCK(hipEventRecord(ev[1], h->stream));
    DCK(hipStreamSynchronize(h->stream));
    if (stage != 1) DCK(hipEventElapsedTime(&ms[stage], ev[0], ev[1]));
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  for (int k = 0; k < 3; ++k) avg_us[k] = 1000.0 * ms[k] / reps;
  return FLR_OK;
}

}  // namespace flr
