// Batched solver for a grid of (lambda1, lambda2) settings on one resident
// problem (flr_solve_grid).  Every column is an independent MM solve
// (section 3.1, Algorithm 2); what they share is X, so the two products of
// each PCG step become dense GEMMs over all columns:
//   U = X O^T   (n x B)      O[b] = p_b in a PCG step, x_b at an MM boundary
//   V = X^T U   (p x B)
// run as FP64 matrix-core products that read X in its stored type
// (flr_gemm.hip).
// Everything else of a step is one fused kernel per column (k_col, one
// workgroup owns one column): the Laplacian product, p^T Q p, the CG updates,
// the whole tridiagonal preconditioner solve as a chunked two-level scan, the
// stopping tests, and at an MM boundary the objective, relative-change test,
// reweighting, LDL^T factorization and the new residual.  Columns advance at
// their own pace: each keeps its own phase; finished columns contribute zero
// operands.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "flr_band.h"
#include "flr_device.h"
#include "flr_gemm.h"
#include "flr_problem.h"

namespace flr {

struct ColState {
  int32_t phase, status, first, mm_iter, cg_iter, jacobi;
  int64_t cg_total;
  double rz, f_old, f_new, rel_change, rel_res, pad;
};

struct GridParams {
  double eps, tol, inner_tol, cnorm;
  int32_t max_iter, max_cg;
  int32_t band;  // W = bandwidth + 1 when columns with lambda1 > 0 use M's banded Cholesky factor, else 0
  int32_t pad;
};

struct GridDev {
  int64_t n, p, p_pad, nnz;
  int64_t ldu;   // leading dimension of U (n rounded up to the product tile)
  int32_t B, pad;
  const double* y;
  const double* c;
  const double* s;
  const int32_t* rowptr;
  const int32_t* col;
  const int32_t* prevpos;
  double* x;     // B x p_pad
  double* r;
  double* pv;
  double* g;
  double* z;
  double* O;     // GEMM operand, B x p_pad (column-major p_pad x B)
  double* U;     // n x B (column-major, ld ldu)
  double* V;     // p_pad x B (column-major, ld p_pad)
  double* a;
  double* d;
  double* e;
  double* L;
  double* invD;
  double* w;     // B x nnz
  const double* lam1;
  const double* lam2;
  ColState* st;
  const GridParams* prm;
  const int32_t* map;  // GEMM slot -> column (active columns only, in slot order)
  double* Lb;          // banded factor by columns, B x p x W (banded mode)
  double* LbT;         // the same by rows
};

constexpr int kE = 8;              // consecutive elements per thread in a chunk
constexpr int kCH = kWG * kE;      // chunk of the two-level scans

// Exclusive value for this thread from the inclusive maps of all threads:
// the composition of threads 0..t-1 (forward) or t+1..255 (reverse) applied to t_in.
__device__ inline double exclusive_apply(Aff inc, double t_in, bool reverse, double* sh2) {
  const int tid = threadIdx.x;
  __syncthreads();
  sh2[2 * tid] = inc.a;
  sh2[2 * tid + 1] = inc.b;
  __syncthreads();
  const int src = reverse ? tid + 1 : tid - 1;
  if (src < 0 || src >= kWG) return t_in;
  return fma(sh2[2 * src], t_in, sh2[2 * src + 1]);
}

// z = M^-1 r for one column with the LDL^T factors (L, invD) of the
// tridiagonal preconditioner: forward g_j = r_j - L_j g_{j-1}, backward
// z_j = g_j / D_j - L_{j+1} z_{j+1}.  Chunks of 256 x 8 elements; inside a
// chunk each thread sweeps 8 consecutive elements, the workgroup scans the
// threads' affine maps, and the chunk's end value carries to the next chunk.
__device__ void col_tri_solve(const double* __restrict__ r, const double* __restrict__ L,
                              const double* __restrict__ invD, double* __restrict__ g, double* __restrict__ z,
                              int64_t p, double* lds, double* sh2) {
  const int tid = threadIdx.x;
  const int nch = (int)((p + kCH - 1) / kCH);
  double carry = 0.0;
  for (int ch = 0; ch < nch; ++ch) {
    const int64_t j0 = (int64_t)ch * kCH + (int64_t)tid * kE;
    double rv[kE], lv[kE];
#pragma unroll
    for (int i = 0; i < kE; ++i) {
      const int64_t j = j0 + i;
      rv[i] = j < p ? r[j] : 0.0;
      lv[i] = j < p ? L[j] : 0.0;
    }
    double loc = 0.0, A = 1.0;
#pragma unroll
    for (int i = 0; i < kE; ++i) {
      loc = fma(-lv[i], loc, rv[i]);
      A = -lv[i] * A;
    }
    const Aff inc = wg_scan_fwd({A, loc}, lds);
    double gv = exclusive_apply(inc, carry, false, sh2);
#pragma unroll
    for (int i = 0; i < kE; ++i) {
      gv = fma(-lv[i], gv, rv[i]);
      const int64_t j = j0 + i;
      if (j < p) g[j] = gv;
    }
    // chunk end value: the last thread's end equals its inclusive map applied to the chunk inflow
    carry = fma(sh2[2 * (kWG - 1)], carry, sh2[2 * (kWG - 1) + 1]);
  }
  __syncthreads();
  carry = 0.0;
  for (int ch = nch - 1; ch >= 0; --ch) {
    const int64_t j0 = (int64_t)ch * kCH + (int64_t)tid * kE;
    double gv[kE], dv[kE], ln[kE];
#pragma unroll
    for (int i = 0; i < kE; ++i) {
      const int64_t j = j0 + i;
      gv[i] = j < p ? g[j] : 0.0;
      dv[i] = j < p ? invD[j] : 0.0;
      ln[i] = j + 1 < p ? L[j + 1] : 0.0;
    }
    double loc = 0.0, A = 1.0;
#pragma unroll
    for (int i = kE - 1; i >= 0; --i) {
      loc = fma(-ln[i], loc, gv[i] * dv[i]);
      A = -ln[i] * A;
    }
    const Aff inc = wg_scan_rev({A, loc}, lds);
    double zv = exclusive_apply(inc, carry, true, sh2);
#pragma unroll
    for (int i = kE - 1; i >= 0; --i) {
      zv = fma(-ln[i], zv, gv[i] * dv[i]);
      const int64_t j = j0 + i;
      if (j < p) z[j] = zv;
    }
    carry = fma(sh2[0], carry, sh2[1]);  // thread 0's inclusive map covers the whole chunk
  }
  __syncthreads();
}

// LDL^T factorization of one column's tridiagonal M: the continued fraction
// D_j = d_j - e_j L_j with L_j = e_j / D_{j-1}, walked in order by the first
// wave (a projective-product scan loses accuracy when fused edges make the
// weights span many decades).  Writes L_j and 1 / D_j.
__device__ void col_factor(const double* __restrict__ d, const double* __restrict__ e, double* __restrict__ L,
                           double* __restrict__ invD, int64_t p, double* sh4) {
  if (threadIdx.x < 64) tri_factor_wave(d, e, L, invD, p, sh4);
  __syncthreads();
}

// (M v)_j for column b: lambda1 a_j v_j + lambda2 sum_k w_jk (v_j - v_k)
__device__ inline double col_apply_m(const GridDev& G, int b, int64_t j, const double* v, double l1, double l2) {
  const double* a = G.a + (int64_t)b * G.p_pad;
  const double* w = G.w + (int64_t)b * G.nnz;
  const double vj = v[j];
  double lap = 0.0;
  for (int q = G.rowptr[j]; q < G.rowptr[j + 1]; ++q) lap = fma(w[q], vj - v[G.col[q]], lap);
  return l1 * a[j] * vj + l2 * lap;
}

// One workgroup per active column.  The GEMM operand and products (O, U, V)
// are indexed by the column's slot in the active list; everything else by the
// column itself.  BAND: columns with lambda1 > 0 apply M^-1 through its banded
// Cholesky factor (graphs of bandwidth >= 2), the others the tridiagonal part.
// hold: a column that has reached its MM boundary (PH_END) waits in this
// launch; its operand O = x is unchanged, so the boundary it runs later sees
// the same products U = X x, V = X^T X x.
template <bool BAND>
__global__ __launch_bounds__(kWG) void k_col(GridDev G, int hold) {
  const int slot = blockIdx.x, tid = threadIdx.x;
  const int b = G.map[slot];
  __shared__ double lds[24];
  __shared__ double sh2[2 * kWG];
  __shared__ double sh4[4 * kWG];
  __shared__ double bl[BAND ? kBandLds : 1];
  ColState s = G.st[b];
  if (s.phase == PH_DONE || (hold && s.phase == PH_END)) return;
  const GridParams prm = *G.prm;
  const bool use_band = BAND && !s.jacobi;
  const int W = prm.band;
  double* Lbb = BAND ? G.Lb + (int64_t)b * G.p * W : nullptr;
  double* LbTb = BAND ? G.LbT + (int64_t)b * G.p * W : nullptr;
  const double l1 = G.lam1[b], l2 = G.lam2[b];
  const int64_t p = G.p, P = G.p_pad, off = (int64_t)b * P;
  double* x = G.x + off;
  double* r = G.r + off;
  double* pv = G.pv + off;
  double* z = G.z + off;
  double* O = G.O + (int64_t)slot * P;
  const double* V = G.V + (int64_t)slot * P;
  const double* U = G.U + (int64_t)slot * G.ldu;

  const bool cg = s.phase == PH_CG;
  if (cg) {
    // q = X^T X p + M p (kept in z), p^T q
    double part = 0.0;
    for (int64_t j = tid; j < p; j += kWG) {
      const double q = V[j] + col_apply_m(G, b, j, pv, l1, l2);
      z[j] = q;
      part = fma(pv[j], q, part);
    }
    const double pq = wg_sum(part, lds);
    const double nu = s.rz / pq;
    if (!(pq > 0.0) || !isfinite(nu)) {
      if (tid == 0) {
        s.phase = PH_DONE;
        s.status = ST_NUMERICAL;
        G.st[b] = s;
      }
      for (int64_t j = tid; j < P; j += kWG) O[j] = 0.0;
      return;
    }
    for (int64_t j = tid; j < p; j += kWG) {
      x[j] = fma(nu, pv[j], x[j]);
      r[j] = fma(-nu, z[j], r[j]);
    }
    __syncthreads();
  } else {
    // ---- MM boundary: U = X x, V = X^T X x for this column ----
    double lp = 0.0;
    for (int64_t i = tid; i < G.n; i += kWG) {
      const double dlt = G.y[i] - U[i];
      lp = fma(dlt, dlt, lp);
    }
    double pp = 0.0;
    for (int64_t j = tid; j < p; j += kWG) {
      const double xj = x[j];
      double pen2 = 0.0;
      for (int q = G.rowptr[j]; q < G.rowptr[j + 1]; ++q) {
        const int k = G.col[q];
        if (k > j) pen2 += fabs(xj - x[k]);
      }
      pp += l1 * fabs(xj) + l2 * pen2;
    }
    const double loss = wg_sum(lp, lds);
    const double pen = wg_sum(pp, lds);
    const double f_new = 0.5 * loss + pen;
    s.f_new = f_new;
    bool finish = false;
    if (!isfinite(f_new)) {
      s.status = ST_NUMERICAL;
      finish = true;
    } else if (s.first) {
      s.first = 0;
    } else {
      s.mm_iter += 1;
      const double re = s.f_old != 0.0 ? fabs(f_new - s.f_old) / fabs(s.f_old) : fabs(f_new - s.f_old);
      s.rel_change = re;
      if (re <= prm.tol) {
        s.status = ST_OK;
        finish = true;
      } else if (s.mm_iter >= prm.max_iter) {
        s.status = ST_MAX_ITER;
        finish = true;
      }
    }
    if (finish) {
      s.phase = PH_DONE;
      for (int64_t j = tid; j < P; j += kWG) O[j] = 0.0;
      if (tid == 0) G.st[b] = s;
      return;
    }
    s.f_old = f_new;
    s.cg_iter = 0;
    // reweighting (majorizer at the current iterate) and the tridiagonal part of M
    double* a = G.a + off;
    double* w = G.w + (int64_t)b * G.nnz;
    double* d = G.d + off;
    double* e = G.e + off;
    for (int64_t j = tid; j < p; j += kWG) {
      const double xj = x[j];
      const double aj = 1.0 / (fabs(xj) + prm.eps);
      a[j] = aj;
      double wsum = 0.0, ej = 0.0;
      for (int q = G.rowptr[j]; q < G.rowptr[j + 1]; ++q) {
        const int k = G.col[q];
        const double wq = 1.0 / (fabs(xj - x[k]) + prm.eps);
        w[q] = wq;
        wsum += wq;
        if (k == j - 1 && !s.jacobi) ej = -l2 * wq;
      }
      double dj = l1 * aj + l2 * wsum;
      if (s.jacobi) dj += G.s[j];
      d[j] = dj;
      e[j] = ej;
    }
    __syncthreads();
    if (use_band) {
      band_assemble(d, G.rowptr, G.col, w, l2, p, W, Lbb);
      if (!band_factor(Lbb, LbTb, G.invD + off, p, W, bl)) {
        s.status = ST_NUMERICAL;
        s.phase = PH_DONE;
        for (int64_t j = tid; j < P; j += kWG) O[j] = 0.0;
        if (tid == 0) G.st[b] = s;
        return;
      }
    } else {
      col_factor(d, e, G.L + off, G.invD + off, p, sh4);
    }
    // r0 = c - (X^T X + M) x
    for (int64_t j = tid; j < p; j += kWG) r[j] = G.c[j] - (V[j] + col_apply_m(G, b, j, x, l1, l2));
    __syncthreads();
  }
  // z = M^-1 r (one call site for both branches)
  if (use_band)
    band_solve(r, G.g + off, z, Lbb, LbTb, G.invD + off, p, W, bl);
  else
    col_tri_solve(r, G.L + off, G.invD + off, G.g + off, z, p, lds, sh2);
  double rzp = 0.0, rrp = 0.0;
  for (int64_t j = tid; j < p; j += kWG) {
    rzp = fma(r[j], z[j], rzp);
    rrp = fma(r[j], r[j], rrp);
  }
  const double rz = wg_sum(rzp, lds);
  const double rr = wg_sum(rrp, lds);
  const double rn = sqrt(rr) / prm.cnorm;
  s.rel_res = rn;
  if (cg) {
    s.cg_iter += 1;
    s.cg_total += 1;
    const bool done = !(rn > prm.inner_tol) || s.cg_iter >= prm.max_cg;
    if (done) {
      s.phase = PH_END;
      for (int64_t j = tid; j < P; j += kWG) O[j] = j < p ? x[j] : 0.0;
    } else {
      const double gamma = rz / s.rz;
      for (int64_t j = tid; j < p; j += kWG) {
        const double v = fma(gamma, pv[j], z[j]);
        pv[j] = v;
        O[j] = v;
      }
      s.rz = rz;
    }
  } else {
    s.rz = rz;
    // Algorithm 2's inner loop is repeat-until: at least one PCG step after
    // r0, unless r0 is exactly zero (nu would be 0/0)
    const bool done = !(rr > 0.0);
    if (done) {
      s.phase = PH_END;
      for (int64_t j = tid; j < P; j += kWG) O[j] = j < p ? x[j] : 0.0;
    } else {
      s.phase = PH_CG;
      for (int64_t j = tid; j < P; j += kWG) {
        const double v = j < p ? z[j] : 0.0;
        pv[j] = v;
        O[j] = v;
      }
    }
  }
  if (tid == 0) G.st[b] = s;
}

// Start of a grid solve: x_b = warm start or X_j^T y / X_j^T X_j, operand O_b = x_b,
// state at the MM boundary (first evaluation of f).
__global__ __launch_bounds__(kWG) void k_col_init(GridDev G, const double* __restrict__ warm, int use_warm,
                                                  const int32_t* __restrict__ jacobi) {
  const int b = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  const int64_t off = (int64_t)b * G.p_pad;
  if (j < G.p_pad) {
    double v = 0.0;
    if (j < G.p) v = use_warm ? warm[off + j] : (G.s[j] > 0.0 ? G.c[j] / G.s[j] : 0.0);
    G.x[off + j] = v;
    G.O[off + j] = v;
    G.pv[off + j] = 0.0;
    G.r[off + j] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ColState s{};
    s.phase = PH_END;
    s.status = ST_OK;
    s.first = 1;
    s.jacobi = jacobi[b];
    G.st[b] = s;
  }
}

// Compaction of the GEMM operand: new slot t takes the column that sat in old
// slot from[t].
__global__ __launch_bounds__(kWG) void k_gather_cols(const double* __restrict__ Oold, double* __restrict__ Onew,
                                                     const int32_t* __restrict__ from, int64_t P) {
  const int t = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (j < P) Onew[(int64_t)t * P + j] = Oold[(int64_t)from[t] * P + j];
}

// U = sum of the split-K partial products, in slice order (fixed, so the
// result does not depend on timing).
__global__ __launch_bounds__(kWG) void k_sum_parts(const double* __restrict__ parts, double* __restrict__ out,
                                                   int64_t cnt, int nparts) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= cnt) return;
  double acc = parts[i];
  for (int q = 1; q < nparts; ++q) acc += parts[(int64_t)q * cnt + i];
  out[i] = acc;
}

}  // namespace flr

using namespace flr;

// The whole device workspace of a grid solve is one block: the allocating
// entry point takes it from hipMalloc (kept on the handle and charged to its
// footprint), the no-allocation entry point from a static device array.
// GridCarve places every buffer in it (256-byte aligned); run with a null
// base it only measures.
struct GridCarve {
  char* base = nullptr;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t b = (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += b;
    return p;
  }
};

struct GridWork {
  int cap = 0;                // columns the workspace holds
  bool band = false;          // holds a banded factor per column
  GridDev G{};
  char* block = nullptr;      // device workspace
  size_t bytes = 0;
  bool owned = false;         // block from hipMalloc (freed with the handle)
  GridParams* d_prm = nullptr;
  double* d_lam = nullptr;    // 2 x cap
  int32_t* d_jac = nullptr;   // cap
  int32_t* d_map = nullptr;   // cap
  int32_t* d_from = nullptr;  // cap
  double* O2 = nullptr;       // second operand buffer for compaction
  int splitk = 1;             // K slices of U = X O
  double* Upart = nullptr;    // splitk x ldu x cap partial products
  ColState* h_st = nullptr;   // host copy of the column states (pinned on the allocating path)
  hipEvent_t ev = nullptr;    // polling event (allocating path; the no-allocation path synchronizes)
};

namespace flr {

// K slices of U = X O: a product over all p columns has only ceil(n/64)
// row tiles per 64 columns, so it is split over K until about 256 row-band
// tiles exist (slices of at least 512, a multiple of the K tile).  Fixed per
// problem shape, so a column's products never depend on the batch.
static int grid_splitk(const Dims& D) {
  const int64_t tm = (D.n + kGemmMT - 1) / kGemmMT;
  int sk = 1;
  while (sk < 8 && tm * sk * 2 <= 256 && D.p_pad % ((int64_t)sk * 2 * kGemmKT) == 0 && D.p_pad / (sk * 2) >= 512)
    sk *= 2;
  return sk;
}

static void grid_carve(GridCarve& c, GridWork& gw, const Dims& D, int cap, int64_t nnz, int band_w, bool band) {
  GridDev& G = gw.G;
  const size_t PB = (size_t)D.p_pad * (size_t)cap;
  const int64_t ldu = (D.n + kGemmMT - 1) / kGemmMT * kGemmMT;
  G.ldu = ldu;
  G.x = c.take<double>(PB);
  G.r = c.take<double>(PB);
  G.pv = c.take<double>(PB);
  G.g = c.take<double>(PB);
  G.z = c.take<double>(PB);
  G.O = c.take<double>(PB);
  gw.O2 = c.take<double>(PB);
  G.V = c.take<double>(PB);
  G.a = c.take<double>(PB);
  G.d = c.take<double>(PB);
  G.e = c.take<double>(PB);
  G.L = c.take<double>(PB);
  G.invD = c.take<double>(PB);
  G.U = c.take<double>((size_t)ldu * (size_t)cap);
  G.w = c.take<double>((size_t)std::max<int64_t>(nnz, 1) * (size_t)cap);
  gw.splitk = grid_splitk(D);
  gw.Upart = gw.splitk > 1 ? c.take<double>((size_t)gw.splitk * (size_t)ldu * (size_t)cap) : nullptr;
  if (band) {
    G.Lb = c.take<double>((size_t)cap * (size_t)D.p * (size_t)band_w);
    G.LbT = c.take<double>((size_t)cap * (size_t)D.p * (size_t)band_w);
  } else {
    G.Lb = G.LbT = nullptr;
  }
  gw.d_lam = c.take<double>(2 * (size_t)cap);
  G.st = c.take<ColState>((size_t)cap);
  gw.d_prm = c.take<GridParams>(1);
  gw.d_jac = c.take<int32_t>((size_t)cap);
  gw.d_map = c.take<int32_t>((size_t)cap);
  gw.d_from = c.take<int32_t>((size_t)cap);
}

// Static fields of the column view for a problem.
static void grid_bind(GridWork& gw, flr_problem h) {
  GridDev& G = gw.G;
  const Dims& D = h->D;
  G.n = D.n;
  G.p = D.p;
  G.p_pad = D.p_pad;
  G.nnz = std::max<int64_t>(h->nnz, 1);
  G.y = h->B.y;
  G.c = h->B.c;
  G.s = h->B.s;
  G.rowptr = h->B.rowptr;
  G.col = h->B.col;
  G.prevpos = h->B.prevpos;
  G.prm = gw.d_prm;
  G.map = gw.d_map;
}

// Workspace bytes of a grid solve with `cap` columns on this problem.
size_t grid_workspace_bytes(flr_problem h, int cap, bool band) {
  GridCarve c;
  GridWork gw;
  grid_carve(c, gw, h->D, cap, h->nnz, h->band_w, band);
  return c.used;
}

void grid_free(flr_problem h) {
  GridWork* gw = h->grid;
  if (!gw) return;
  if (gw->owned && gw->block) {
    (void)hipFree(gw->block);
    h->footprint -= gw->bytes;
  }
  if (gw->h_st) (void)hipHostFree(gw->h_st);
  if (gw->ev) (void)hipEventDestroy(gw->ev);
  delete gw;
  h->grid = nullptr;
}
bool is_device_pointer(const void* p);

__global__ __launch_bounds__(kWG) void k_fill_zero(double* __restrict__ p, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * kWG;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < count; i += stride) p[i] = 0.0;
}

// U = X O, then V = X^T U, for the first nact operand columns.
static hipError_t grid_products(flr_problem h, const GridWork& gw, const GridDev& G, const double* O, int nact) {
  const Dims& D = h->D;
  if (D.flsa) {  // X = I: U = O (its p rows) and V = X^T U = O
    hipError_t e = hipMemcpy2DAsync(G.U, (size_t)G.ldu * sizeof(double), O, (size_t)D.p_pad * sizeof(double),
                                    (size_t)D.p * sizeof(double), (size_t)nact, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(G.V, O, (size_t)nact * (size_t)D.p_pad * sizeof(double), hipMemcpyDeviceToDevice,
                          h->stream);
  }
  GemmArgs a{};
  a.X = h->B.X;
  a.ldx = D.ldx;
  a.Bm = O;
  a.ldb = D.p_pad;
  a.C = gw.splitk > 1 ? gw.Upart : G.U;
  a.ldc = G.ldu;
  a.cslice = G.ldu * (int64_t)nact;
  a.M = (int32_t)D.n;
  a.N = nact;
  a.K = (int32_t)(D.p_pad / gw.splitk);
  a.tiles_m = (int32_t)((D.n + kGemmMT - 1) / kGemmMT);
  a.tiles_n = (nact + kGemmNT - 1) / kGemmNT;
  a.nslice = gw.splitk;
  hipError_t e = launch_gemm_xo(D.dtype, a, h->stream);
  if (e != hipSuccess) return e;
  if (gw.splitk > 1) {
    const int64_t cnt = G.ldu * (int64_t)nact;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((cnt + kWG - 1) / kWG)), dim3(kWG), 0, h->stream, gw.Upart, G.U,
                       cnt, gw.splitk);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  GemmArgs b{};
  b.X = h->B.X;
  b.ldx = D.ldx;
  b.Bm = G.U;
  b.ldb = G.ldu;
  b.C = G.V;
  b.ldc = D.p_pad;
  b.cslice = 0;
  b.M = (int32_t)D.p_pad;
  b.N = nact;
  b.K = (int32_t)D.n;
  b.tiles_m = (int32_t)(D.p_pad / kGemmMT);
  b.tiles_n = (nact + kGemmNT - 1) / kGemmNT;
  b.nslice = 1;
  return launch_gemm_xtu(D.dtype, b, h->stream);
}

}  // namespace flr

static flr_status gfail(flr_status st, const std::string& m) {
  set_last_error(m);
  return st;
}

#define GCK(expr)                                                                                           \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) {                                                                                 \
      (void)hipGetLastError(); /* a failed call also leaves its error for the next check */                 \
      return gfail(e_ == hipErrorOutOfMemory ? FLR_ERR_OUT_OF_MEMORY : FLR_ERR_DEVICE,                      \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                                      \
    }                                                                                                       \
  } while (0)

// Workspace of the allocating entry point: kept on the handle while it holds
// at least B columns (and a banded factor when one is needed), else replaced.
// On any failure the partial workspace is released, so that a later call
// does not take it for a usable one.
static flr_status grid_prepare_once(flr_problem h, int B, bool band);

static flr_status grid_prepare(flr_problem h, int B, bool band) {
  if (h->grid && h->grid->cap >= B && (h->grid->band || !band)) return FLR_OK;
  grid_free(h);
  const flr_status st = grid_prepare_once(h, B, band);
  if (st != FLR_OK) {
    (void)hipStreamSynchronize(h->stream);
    grid_free(h);
  }
  return st;
}

static flr_status grid_prepare_once(flr_problem h, int B, bool band) {
  GridWork* gw = new GridWork;
  h->grid = gw;
  gw->cap = B;
  gw->band = band;
  GridCarve c;
  grid_carve(c, *gw, h->D, B, h->nnz, h->band_w, band);
  gw->bytes = c.used;
  GCK(hipMalloc(reinterpret_cast<void**>(&gw->block), gw->bytes));
  gw->owned = true;
  h->footprint += gw->bytes;
  c.base = gw->block;
  c.used = 0;
  grid_carve(c, *gw, h->D, B, h->nnz, h->band_w, band);
  grid_bind(*gw, h);
  hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(kWG), 0, h->stream, reinterpret_cast<double*>(gw->block),
                     (int64_t)(gw->bytes / sizeof(double)));
  GCK(hipGetLastError());
  GCK(hipHostMalloc(reinterpret_cast<void**>(&gw->h_st), sizeof(ColState) * (size_t)B, hipHostMallocDefault));
  GCK(hipEventCreateWithFlags(&gw->ev, hipEventDisableTiming));
  return FLR_OK;
}

// Host-side arrays of a grid solve (B entries each).
struct GridHost {
  double* lam;   // 2B
  int32_t* jac;
  int32_t* act;
  int32_t* nxt;
  int32_t* from;
};

static flr_status grid_run(flr_problem h, GridWork* gw, GridHost hb, const double* l1, const double* l2, int32_t B,
                           double tol, const flr_solve_opts* o, double* beta_out, flr_result* res) {
  auto t0 = std::chrono::steady_clock::now();
  GridDev G = gw->G;
  G.B = B;
  const Dims& D = h->D;
  GridParams P{};
  P.eps = o->eps > 0.0 ? o->eps : 1e-8;
  P.tol = tol;
  P.inner_tol = o->inner_tol > 0.0 ? o->inner_tol : tol;
  P.cnorm = h->cnorm > 0.0 ? h->cnorm : 1.0;
  P.max_iter = o->max_iter > 0 ? o->max_iter : 10000;
  P.max_cg = o->max_cg > 0 ? o->max_cg : (int32_t)std::min<int64_t>(D.p, INT32_MAX);
  const int pre0 = o->preconditioner;
  const bool band = gw->band;
  for (int i = 0; i < B; ++i) {
    hb.lam[i] = l1[i];
    hb.lam[B + i] = l2[i];
    int pre = pre0;
    if (pre == FLR_PRECOND_AUTO) pre = l1[i] > 0.0 ? FLR_PRECOND_TRIDIAG : FLR_PRECOND_JACOBI;
    if ((pre == FLR_PRECOND_TRIDIAG || pre == FLR_PRECOND_BAND) && !(l1[i] > 0.0))
      return gfail(FLR_ERR_INVALID_ARG, "the tridiagonal and banded preconditioners need lambda1 > 0");
    hb.jac[i] = pre == FLR_PRECOND_JACOBI ? 1 : 0;
  }
  P.band = band ? h->band_w : 0;
  G.lam1 = gw->d_lam;
  G.lam2 = gw->d_lam + B;
  GCK(hipMemcpyAsync(gw->d_lam, hb.lam, 2 * (size_t)B * sizeof(double), hipMemcpyHostToDevice, h->stream));
  GCK(hipMemcpyAsync(gw->d_jac, hb.jac, (size_t)B * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  GCK(hipMemcpyAsync(gw->d_prm, &P, sizeof(P), hipMemcpyHostToDevice, h->stream));
  const double* warm = nullptr;
  if (o->warm_start) {
    // B rows of p values into the padded rows of a work buffer (k_col_init reads only j < p)
    GCK(hipMemcpy2DAsync(G.g, (size_t)D.p_pad * sizeof(double), o->warm_start, (size_t)D.p * sizeof(double),
                         (size_t)D.p * sizeof(double), (size_t)B, hipMemcpyDefault, h->stream));
    warm = G.g;
  }
  hipLaunchKernelGGL(k_col_init, dim3((unsigned)((D.p_pad + kWG - 1) / kWG), (unsigned)B), dim3(kWG), 0, h->stream,
                     G, warm, warm ? 1 : 0, gw->d_jac);
  GCK(hipGetLastError());
  const int check_every = 8;
  // Banded columns gather their MM boundaries into every hold_period-th
  // launch while at least kHoldMinCols columns run: a boundary factors the
  // band in one workgroup (tens of ms at bandwidth 100), and columns reach
  // their boundaries at different steps, so without this almost every launch
  // would wait for some column's factorization.  A held column only idles;
  // its arithmetic is unchanged.  FLR_GRID_HOLD overrides the period (0 or 1:
  // no holding).
  constexpr int kHoldMinCols = 8;
  int hold_period = band ? 16 : 1;
  if (const char* hv = std::getenv("FLR_GRID_HOLD")) hold_period = std::max(1, std::atoi(hv));
  // every column needs at most max_iter * (max_cg + 2 + hold_period) + 1
  // steps; the host sees a finished batch up to two polling periods later
  const int64_t max_steps =
      (int64_t)P.max_iter * ((int64_t)P.max_cg + 2 + hold_period) + 4 + 3 * check_every;
  // active columns in slot order; compacted when enough of them have finished
  int nact = B;
  for (int i = 0; i < B; ++i) hb.act[i] = i;
  GCK(hipMemcpyAsync(gw->d_map, hb.act, (size_t)B * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  GCK(hipStreamSynchronize(h->stream));
  double* Ospare = gw->O2;
  bool done = false;
  int64_t step = 0;
  bool pending = false;
  // FLR_PROGRESS=1: a line on stderr every few seconds from the polling loop
  const char* prog_env = std::getenv("FLR_PROGRESS");
  const bool progress = prog_env && prog_env[0] && prog_env[0] != '0';
  auto t_prog = std::chrono::steady_clock::now();
  auto poll = [&]() -> hipError_t {  // column states to the host: async + event, or synchronously
    hipError_t e = hipMemcpyAsync(gw->h_st, G.st, sizeof(ColState) * (size_t)B, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return e;
    return gw->ev ? hipEventRecord(gw->ev, h->stream) : hipStreamSynchronize(h->stream);
  };
  // One batched step: the two products (and the split-K sum) for the active
  // columns, then the fused per-column kernel.
  auto one_step = [&](int64_t st) -> hipError_t {
    hipError_t e = grid_products(h, *gw, G, G.O, nact);
    if (e != hipSuccess) return e;
    const int hold = hold_period > 1 && nact >= kHoldMinCols && st % hold_period != 0 ? 1 : 0;
    if (P.band)
      hipLaunchKernelGGL(k_col<true>, dim3((unsigned)nact), dim3(kWG), 0, h->stream, G, hold);
    else
      hipLaunchKernelGGL(k_col<false>, dim3((unsigned)nact), dim3(kWG), 0, h->stream, G, hold);
    return hipGetLastError();
  };
  // The allocating entry point replays whole polling periods (check_every
  // steps) as HIP graphs, one per hold pattern of the period, captured for the
  // current set of active columns and operand buffer and captured again after
  // a compaction.  The no-allocation entry point (no event) launches eagerly,
  // since instantiating a graph may allocate; FLR_GRID_GRAPH=0 does the same.
  const char* gv = std::getenv("FLR_GRID_GRAPH");
  const bool use_graphs = gw->ev && !(gv && gv[0] == '0');
  struct Period {
    unsigned mask;
    hipGraphExec_t exec;
  };
  std::vector<Period> graphs;
  auto drop_graphs = [&]() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  };
  struct GraphGuard {  // on every return: replays still in flight finish before their graphs go
    hipStream_t st;
    std::function<void()> f;
    ~GraphGuard() {
      (void)hipStreamSynchronize(st);
      f();
    }
  } guard{h->stream, drop_graphs};
  auto run_period = [&](int64_t st) -> hipError_t {
    unsigned mask = 0;
    for (int k = 0; k < check_every; ++k)
      if (hold_period > 1 && nact >= kHoldMinCols && (st + k) % hold_period != 0) mask |= 1u << k;
    for (auto& g : graphs)
      if (g.mask == mask) return hipGraphLaunch(g.exec, h->stream);
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t body = hipSuccess;
    for (int k = 0; k < check_every && body == hipSuccess; ++k) body = one_step(st + k);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(h->stream, &graph);
    if (body != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return body;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    graphs.push_back({mask, exec});
    return hipGraphLaunch(exec, h->stream);
  };
  while (!done) {
    if (step >= max_steps) return gfail(FLR_ERR_DEVICE, "grid solve did not terminate within its step bound");
    if (progress && std::chrono::steady_clock::now() - t_prog > std::chrono::seconds(5)) {
      t_prog = std::chrono::steady_clock::now();
      std::fprintf(stderr, "flr grid: %lld batched steps, %d of %d columns active\n", (long long)step, nact, B);
    }
    if (use_graphs && step % check_every == 0) {
      GCK(run_period(step));
      step += check_every;
    } else {
      GCK(one_step(step));
      ++step;
    }
    if (step % check_every == 0) {
      if (pending) {
        if (gw->ev) GCK(hipEventSynchronize(gw->ev));
        int still = 0;
        for (int i = 0; i < nact; ++i) still += gw->h_st[hb.act[i]].phase != PH_DONE;
        if (still == 0) {
          done = true;
        } else if (nact - still >= std::max(8, nact / 8)) {
          // drain, then keep only the columns still running; their operand
          // columns move to the front of the spare buffer
          GCK(hipMemcpyAsync(gw->h_st, G.st, sizeof(ColState) * (size_t)B, hipMemcpyDeviceToHost, h->stream));
          GCK(hipStreamSynchronize(h->stream));
          int cnt = 0;
          for (int i = 0; i < nact; ++i) {
            if (gw->h_st[hb.act[i]].phase != PH_DONE) {
              hb.nxt[cnt] = hb.act[i];
              hb.from[cnt] = i;
              ++cnt;
            }
          }
          if (cnt == 0) {
            done = true;
          } else {
            GCK(hipMemcpyAsync(gw->d_from, hb.from, (size_t)cnt * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
            GCK(hipMemcpyAsync(gw->d_map, hb.nxt, (size_t)cnt * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
            hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((D.p_pad + kWG - 1) / kWG), (unsigned)cnt), dim3(kWG),
                               0, h->stream, G.O, Ospare, gw->d_from, D.p_pad);
            GCK(hipGetLastError());
            // the host arrays are read by the copies above before they change again
            GCK(hipStreamSynchronize(h->stream));
            std::swap(G.O, Ospare);
            std::swap(hb.act, hb.nxt);
            nact = cnt;
            drop_graphs();  // captured for the old columns and operand buffer
          }
          pending = false;
          continue;
        }
      }
      GCK(poll());
      pending = true;
    }
  }
  GCK(hipMemcpyAsync(gw->h_st, G.st, sizeof(ColState) * (size_t)B, hipMemcpyDeviceToHost, h->stream));
  if (beta_out)
    GCK(hipMemcpy2DAsync(beta_out, (size_t)D.p * sizeof(double), G.x, (size_t)D.p_pad * sizeof(double),
                         (size_t)D.p * sizeof(double), (size_t)B, hipMemcpyDefault, h->stream));
  GCK(hipStreamSynchronize(h->stream));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  flr_status first = FLR_OK;
  for (int b = 0; b < B; ++b) {
    const ColState& s = gw->h_st[b];
    const flr_status st = s.status == ST_OK ? FLR_OK : s.status == ST_MAX_ITER ? FLR_ERR_MAX_ITER : FLR_ERR_NUMERICAL;
    if (st != FLR_OK && first == FLR_OK) first = st;
    if (res) {
      res[b].objective = s.f_new;
      res[b].rel_change = s.rel_change;
      res[b].rel_residual = s.rel_res;
      res[b].cg_iters = s.cg_total;
      res[b].mm_iters = s.mm_iter;
      res[b].status = st;
      res[b].seconds = secs;
    }
  }
  return first;
}

// Argument checks shared by the grid entry points; *band: the columns with
// lambda1 > 0 apply M^-1 through its banded factor.
static flr_status grid_check(flr_problem h, const double* l1, const double* l2, int32_t B, double tol,
                             const flr_solve_opts* o, bool* band) {
  if (!h || !l1 || !l2 || B < 1) return gfail(FLR_ERR_INVALID_ARG, "bad grid arguments");
  for (int32_t i = 0; i < B; ++i) {
    if (!(std::isfinite(l1[i]) && l1[i] >= 0.0) || !(std::isfinite(l2[i]) && l2[i] >= 0.0))
      return gfail(FLR_ERR_INVALID_ARG, "lambda1 and lambda2 must be finite and >= 0");
  }
  if (!(std::isfinite(tol) && tol > 0.0)) return gfail(FLR_ERR_INVALID_ARG, "tol must be finite and > 0");
  if (o->precision != FLR_PREC_FP64) return gfail(FLR_ERR_INVALID_ARG, "grid solves run in FP64 (no mixed-precision grid path)");
  if (o->method != FLR_METHOD_PCG) return gfail(FLR_ERR_INVALID_ARG, "the grid runs Algorithm 2 (PCG) only");
  if (!(o->eps >= 0.0) || !(o->inner_tol >= 0.0) || o->max_iter < 0 || o->max_cg < 0)
    return gfail(FLR_ERR_INVALID_ARG, "options out of range");
  const int pre0 = o->preconditioner;
  if (pre0 < FLR_PRECOND_AUTO || pre0 > FLR_PRECOND_BAND) return gfail(FLR_ERR_INVALID_ARG, "unknown preconditioner");
  if (pre0 == FLR_PRECOND_BAND && !h->band_w)
    return gfail(FLR_ERR_INVALID_ARG, "banded preconditioner: the edge set has bandwidth < 2 or its band is too wide");
  if (o->warm_start && is_device_pointer(o->warm_start))
    return gfail(FLR_ERR_INVALID_ARG, "grid warm starts are host arrays (B x p)");
  *band = h->band_w && (pre0 == FLR_PRECOND_AUTO || pre0 == FLR_PRECOND_BAND);
  return FLR_OK;
}

extern "C" flr_status flr_solve_grid(flr_problem h, const double* l1, const double* l2, int32_t B, double tol,
                                     const flr_solve_opts* opts, double* beta_out, flr_result* res) {
  flr_solve_opts dflt;
  flr_default_opts(&dflt);
  const flr_solve_opts* o = opts ? opts : &dflt;
  bool band = false;
  flr_status cs = grid_check(h, l1, l2, B, tol, o, &band);
  if (cs != FLR_OK) return cs;
  std::unique_lock<std::mutex> lk(h->busy, std::try_to_lock);
  if (!lk.owns_lock()) return gfail(FLR_ERR_BUSY, "problem handle in use by another thread");
  if (hipSetDevice(h->ctx->device) != hipSuccess) return gfail(FLR_ERR_DEVICE, "hipSetDevice failed");
  flr_status ps = grid_prepare(h, B, band);
  if (ps != FLR_OK) return ps;
  std::vector<double> lam(2 * (size_t)B);
  std::vector<int32_t> ints(4 * (size_t)B);
  GridHost hb{lam.data(), ints.data(), ints.data() + B, ints.data() + 2 * (size_t)B, ints.data() + 3 * (size_t)B};
  return grid_run(h, h->grid, hb, l1, l2, B, tol, o, beta_out, res);
}

extern "C" flr_status flr_profile_grid(flr_problem h, int32_t B, int32_t reps, double* avg_us) {
  if (!h || !avg_us || reps < 1 || B < 1) return gfail(FLR_ERR_INVALID_ARG, "flr_profile_grid: bad arguments");
  std::unique_lock<std::mutex> lk(h->busy, std::try_to_lock);
  if (!lk.owns_lock()) return gfail(FLR_ERR_BUSY, "problem handle in use by another thread");
  if (!h->grid || h->grid->cap < B)
    return gfail(FLR_ERR_INVALID_ARG, "flr_profile_grid: needs a completed grid solve with at least B columns");
  if (h->D.flsa) return gfail(FLR_ERR_INVALID_ARG, "flr_profile_grid: an X = I problem has no products to time");
  if (hipSetDevice(h->ctx->device) != hipSuccess) return gfail(FLR_ERR_DEVICE, "hipSetDevice failed");
  GridWork* gw = h->grid;
  const GridDev& G = gw->G;
  const Dims& D = h->D;
  hipEvent_t e[3];
  for (auto& ev : e) GCK(hipEventCreate(&ev));
  // the spare operand buffer, as in a batched PCG step
  auto gemm_u = [&]() {
    GemmArgs a{};
    a.X = h->B.X;
    a.ldx = D.ldx;
    a.Bm = gw->O2;
    a.ldb = D.p_pad;
    a.C = gw->splitk > 1 ? gw->Upart : G.U;
    a.ldc = G.ldu;
    a.cslice = G.ldu * (int64_t)B;
    a.M = (int32_t)D.n;
    a.N = B;
    a.K = (int32_t)(D.p_pad / gw->splitk);
    a.tiles_m = (int32_t)((D.n + kGemmMT - 1) / kGemmMT);
    a.tiles_n = (B + kGemmNT - 1) / kGemmNT;
    a.nslice = gw->splitk;
    hipError_t er = launch_gemm_xo(D.dtype, a, h->stream);
    if (er == hipSuccess && gw->splitk > 1) {
      const int64_t cnt = G.ldu * (int64_t)B;
      hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((cnt + kWG - 1) / kWG)), dim3(kWG), 0, h->stream, gw->Upart,
                         G.U, cnt, gw->splitk);
      er = hipGetLastError();
    }
    return er;
  };
  auto gemm_v = [&]() {
    GemmArgs b{};
    b.X = h->B.X;
    b.ldx = D.ldx;
    b.Bm = G.U;
    b.ldb = G.ldu;
    b.C = G.V;
    b.ldc = D.p_pad;
    b.M = (int32_t)D.p_pad;
    b.N = B;
    b.K = (int32_t)D.n;
    b.tiles_m = (int32_t)(D.p_pad / kGemmMT);
    b.tiles_n = (B + kGemmNT - 1) / kGemmNT;
    b.nslice = 1;
    return launch_gemm_xtu(D.dtype, b, h->stream);
  };
  flr_status st = FLR_OK;
  double tot[2] = {0.0, 0.0};
  for (int pass = 0; pass < 2 && st == FLR_OK; ++pass) {  // pass 0 warms up
    if (hipEventRecord(e[0], h->stream) != hipSuccess) st = FLR_ERR_DEVICE;
    for (int i = 0; i < reps && st == FLR_OK; ++i)
      if (gemm_u() != hipSuccess) st = FLR_ERR_DEVICE;
    if (st == FLR_OK && hipEventRecord(e[1], h->stream) != hipSuccess) st = FLR_ERR_DEVICE;
    for (int i = 0; i < reps && st == FLR_OK; ++i)
      if (gemm_v() != hipSuccess) st = FLR_ERR_DEVICE;
    if (st == FLR_OK && hipEventRecord(e[2], h->stream) != hipSuccess) st = FLR_ERR_DEVICE;
    if (st == FLR_OK && hipEventSynchronize(e[2]) != hipSuccess) st = FLR_ERR_DEVICE;
    float m0 = 0.f, m1 = 0.f;
    if (st == FLR_OK && (hipEventElapsedTime(&m0, e[0], e[1]) != hipSuccess ||
                         hipEventElapsedTime(&m1, e[1], e[2]) != hipSuccess))
      st = FLR_ERR_DEVICE;
    tot[0] = 1e3 * m0 / reps;
    tot[1] = 1e3 * m1 / reps;
  }
  for (auto& ev : e) (void)hipEventDestroy(ev);
  if (st != FLR_OK) return gfail(st, "flr_profile_grid: a launch or event call failed");
  avg_us[0] = tot[0];
  avg_us[1] = tot[1];
  return FLR_OK;
}


// ---------------------------------------------------------------------------
// No-allocation grid solve: the workspace is a fixed static device array
// (scratch) instead of memory the library allocates.  In host code the name
// `scratch` is only a stand-in for the symbol; its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
// ---------------------------------------------------------------------------
static constexpr size_t kGridScratchBytes = (size_t)FLR_GRID_STATIC_BYTES;
static constexpr int kGridStaticMaxCols = FLR_GRID_STATIC_MAX_COLS;
static __device__ __align__(256) char scratch[kGridScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use with
// the device current).
flr_status scratch_address(int device, char** out) {
  if (device < 0 || device >= kMaxDevices) return gfail(FLR_ERR_DEVICE, "device id beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return gfail(FLR_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return FLR_OK;
}
}  // namespace

extern "C" flr_status flr_solve_grid_static(flr_problem h, const double* l1, const double* l2, int32_t B, double tol,
                                            const flr_solve_opts* opts, double* beta_out, flr_result* res) {
  flr_solve_opts dflt;
  flr_default_opts(&dflt);
  const flr_solve_opts* o = opts ? opts : &dflt;
  bool band = false;
  flr_status cs = grid_check(h, l1, l2, B, tol, o, &band);
  if (cs != FLR_OK) return cs;
  if (B > kGridStaticMaxCols)
    return gfail(FLR_ERR_INVALID_ARG, "flr_solve_grid_static: at most " + std::to_string(kGridStaticMaxCols) +
                                          " columns per call");
  std::unique_lock<std::mutex> lk(h->busy, std::try_to_lock);
  if (!lk.owns_lock()) return gfail(FLR_ERR_BUSY, "problem handle in use by another thread");
  if (hipSetDevice(h->ctx->device) != hipSuccess) return gfail(FLR_ERR_DEVICE, "hipSetDevice failed");
  GridWork gw;
  gw.cap = B;
  gw.band = band;
  GridCarve c;
  grid_carve(c, gw, h->D, B, h->nnz, h->band_w, band);
  if (c.used > kGridScratchBytes)
    return gfail(FLR_ERR_INVALID_ARG, "flr_solve_grid_static: the workspace needs " + std::to_string(c.used) +
                                          " bytes, more than the " + std::to_string(kGridScratchBytes) +
                                          "-byte static array (fewer columns, or flr_solve_grid)");
  char* base = nullptr;
  flr_status ss = scratch_address(h->ctx->device, &base);
  if (ss != FLR_OK) return ss;
  c.base = base;
  c.used = 0;
  grid_carve(c, gw, h->D, B, h->nnz, h->band_w, band);
  grid_bind(gw, h);
  gw.block = base;
  gw.bytes = c.used;
  gw.owned = false;
  // host arrays without allocation: per-thread static storage
  static thread_local ColState st_host[kGridStaticMaxCols];
  static thread_local double lam_host[2 * kGridStaticMaxCols];
  static thread_local int32_t int_host[4 * kGridStaticMaxCols];
  gw.h_st = st_host;
  gw.ev = nullptr;
  GridHost hb{lam_host, int_host, int_host + B, int_host + 2 * B, int_host + 3 * B};
  const flr_status st = grid_run(h, &gw, hb, l1, l2, B, tol, o, beta_out, res);
  gw.h_st = nullptr;  // static storage: nothing to free
  return st;
}
