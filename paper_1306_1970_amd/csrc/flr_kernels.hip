// HIP kernels (gfx950) of the device-resident MM / PCG loop for fused lasso
// regression.  Method: section 3.1 (perturbed objective, majorizer, linear
// system with A and B), Algorithm 2 (MM with PCG, preconditioner
// M = lambda1 A + lambda2 B).  See flr_internal.h for the launch rotation.
//
// Numerics: all p-scale arithmetic, dot products, the objective and every
// stopping test are FP64.  X is read in its stored type (f64 / f32 / bf16)
// and widened exactly; products accumulate in FP64.  Every reduction has a
// fixed tree, so a solve is bitwise repeatable and does not depend on what
// else runs on the device.
#include <hip/hip_runtime.h>

#include <cmath>

#include "flr_device.h"
#include "flr_band.h"
#include "flr_internal.h"

namespace flr {

// ---------------------------------------------------------------------------
// Setup: partial column sums of X_ij y_i and X_ij^2 over row panels
// ---------------------------------------------------------------------------
template <typename XT>
__global__ __launch_bounds__(kWG) void k_setup_partial(Dims D, const XT* __restrict__ X, const double* __restrict__ y,
                                                        double* __restrict__ cpart, double* __restrict__ spart) {
  constexpr int V = XV<XT>::V;
  const int wg = blockIdx.x, cb = wg % D.cb2, rb = wg / D.cb2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)rb * D.r2, r1 = min<int64_t>(D.n, r0 + D.r2);
  const int64_t c0 = (int64_t)cb * D.c2 + lane * V;
  double ac[V], as[V];
#pragma unroll
  for (int v = 0; v < V; ++v) { ac[v] = 0.0; as[v] = 0.0; }
  for (int64_t i = r0 + wave; i < r1; i += 4) {
    double xv[V];
    XV<XT>::cvt(load16(X + i * D.ldx + c0), xv);
    const double yi = y[i];
#pragma unroll
    for (int v = 0; v < V; ++v) { ac[v] = fma(xv[v], yi, ac[v]); as[v] = fma(xv[v], xv[v], as[v]); }
  }
  __shared__ double red[2][4][64 * 8];
#pragma unroll
  for (int v = 0; v < V; ++v) { red[0][wave][lane * V + v] = ac[v]; red[1][wave][lane * V + v] = as[v]; }
  __syncthreads();
  for (int t = threadIdx.x; t < 64 * V; t += kWG) {
    const int64_t j = (int64_t)cb * D.c2 + t;
    cpart[(int64_t)rb * D.p_pad + j] = (red[0][0][t] + red[0][1][t]) + (red[0][2][t] + red[0][3][t]);
    spart[(int64_t)rb * D.p_pad + j] = (red[1][0][t] + red[1][1][t]) + (red[1][2][t] + red[1][3][t]);
  }
}

__global__ __launch_bounds__(kWG) void k_setup_final(Dims D, const double* __restrict__ cpart,
                                                      const double* __restrict__ spart, double* __restrict__ c,
                                                      double* __restrict__ s) {
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (j >= D.p_pad) return;
  double sc = 0.0, ss = 0.0;
  for (int rb = 0; rb < D.rb2; ++rb) {
    sc += cpart[(int64_t)rb * D.p_pad + j];
    ss += spart[(int64_t)rb * D.p_pad + j];
  }
  c[j] = j < D.p ? sc : 0.0;
  s[j] = j < D.p ? ss : 0.0;
}

// Initial iterate (initialization of Algorithms 1 and 2: b_j = X_j^T y / X_j^T X_j,
// 0 for a zero column) or a warm start; both state buffers start at the MM
// boundary so the first rotation evaluates f(b0) and sets up the first PCG.
__global__ __launch_bounds__(kWG) void k_init(Dims D, Bufs B, const double* __restrict__ warm, int use_warm) {
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (j < D.p_pad) {
    double v = 0.0;
    if (j < D.p) v = use_warm ? warm[j] : (B.s[j] > 0.0 ? B.c[j] / B.s[j] : 0.0);
    B.x[j] = v;
    B.r[j] = 0.0;
    B.yv[j] = 0.0;
    B.pbuf[j] = 0.0;
    B.pbuf[D.p_pad + j] = 0.0;
    // the banded mode rebuilds z from yv alone (gains and carries stay zero)
    B.sig[j] = 0.0;
    B.psi[j] = 0.0;
  }
  if (j < 2 * (int64_t)D.nblk) B.carry[j] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    State s;
    s.phase = PH_END;
    s.status = ST_OK;
    s.first = 1;
    s.first_cg = 1;
    s.mm_iter = 0;
    s.cg_iter = 0;
    s.cg_total = 0;
    s.rz = 0.0;
    s.f_old = 0.0;
    s.f_new = 0.0;
    s.rel_change = 0.0;
    s.rel_res = 0.0;
    s.nu = 0.0;
    s.gamma = 0.0;
    s.rres = 0.0;
    B.st[0] = s;
    B.st[1] = s;
  }
}

// Rows r0..r1 of one column panel: u_part[cb][i] = sum_j X_ij v_j, with the
// first pair of rows already in registers and the next pair always in flight.
// ACC = double (FP64 path) or float (the inner PCG products of the mixed path).
template <typename XT, typename ACC>
__device__ inline void rows_a(const Dims& D, const Bufs& B, const XT* Xb, int cb, int64_t r0, int64_t r1, int64_t c0,
                              int lane, int wave, const double* sh_v, typename XV<XT>::raw (&cur0)[4],
                              typename XV<XT>::raw (&cur1)[4]) {
  constexpr int V = XV<XT>::V;
  constexpr int NV = 4;
  using RAW = typename XV<XT>::raw;
  ACC pl[NV][V];
#pragma unroll
  for (int t = 0; t < NV; ++t)
#pragma unroll
    for (int v = 0; v < V; ++v) pl[t][v] = (ACC)sh_v[(t * 64 + lane) * V + v];
  for (int64_t i = r0 + wave; i < r1; i += 8) {
    const int64_t i1 = i + 4, in0 = i + 8, in1 = i + 12;
    const bool has1 = i1 < r1;
    RAW nx0[NV], nx1[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int64_t col = c0 + (int64_t)(t * 64 + lane) * V;
      if (in0 < r1) nx0[t] = load16(Xb + in0 * D.ldx + col);
      if (in1 < r1) nx1[t] = load16(Xb + in1 * D.ldx + col);
    }
    ACC acc0 = 0, acc1 = 0;
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      ACC xv[V];
      XV<XT>::cvt(cur0[t], xv);
#pragma unroll
      for (int v = 0; v < V; ++v) acc0 = fma(xv[v], pl[t][v], acc0);
      if (has1) {
        ACC xw[V];
        XV<XT>::cvt(cur1[t], xw);
#pragma unroll
        for (int v = 0; v < V; ++v) acc1 = fma(xw[v], pl[t][v], acc1);
      }
    }
    const double s0 = wave_sum((double)acc0);
    const double s1 = wave_sum((double)acc1);
    if (lane == 0) {
      B.upart[(int64_t)cb * D.n + i] = s0;
      if (has1) B.upart[(int64_t)cb * D.n + i1] = s1;
    }
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      cur0[t] = nx0[t];
      cur1[t] = nx1[t];
    }
  }
}

// ---------------------------------------------------------------------------
// A: row-panel GEMV u_part[cb] = X[rb, cb] v[cb].  In a PCG step v is the new
// direction p = z + gamma p_old, where z = M^-1 r is rebuilt from the local
// block solutions and the carries that the last C workgroup combined
// (z_j = y_j + sigma_j G_k + psi_j Z_k).  Once PCG has converged, or at the
// MM boundary, v is the iterate x.  The state is read through a restrict
// pointer (scalar loads), so it does not wait behind the X loads.
// ---------------------------------------------------------------------------
template <typename XT, bool MX>
__device__ __forceinline__ void gemv_a_body(const Dims& D, const Bufs& B, const State* __restrict__ sin,
                                            State* __restrict__ sout, const int wg) {
  constexpr int V = XV<XT>::V;
  constexpr int NV = 4;  // 16-byte loads per lane per row (the panel is 256 V columns)
  using RAW = typename XV<XT>::raw;
  const State s = *sin;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cb = wg % D.cb1, rb = wg / D.cb1;
  if (wg == 0 && tid == 0) *sout = s;
  if (s.phase == PH_DONE) return;
  const int64_t c0 = (int64_t)cb * D.c1;
  const int64_t r0 = (int64_t)rb * D.r1, r1 = min<int64_t>(D.n, r0 + D.r1);
  const XT* Xb = reinterpret_cast<const XT*>(B.X);

  // operand-slice inputs first (small, needed first), then the wave's first
  // two X rows, so that waiting for the former does not wait for the latter
  __shared__ double sh_v[kMaxC1];
  const bool cg = s.phase == PH_CG;
  const double* pold = B.pbuf + (int64_t)(s.cg_iter & 1) * D.p_pad;
  double* pnew = B.pbuf + (int64_t)((s.cg_iter + 1) & 1) * D.p_pad;
  const int K = D.nblk;
  double fy[V], fs[V], fp[V], fo[V], fg[V], fz[V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int64_t j = c0 + tid + u * kWG;
    const int k = (int)(j / kBlk);
    if (cg) {
      fy[u] = B.yv[j];
      fs[u] = B.sig[j];
      fp[u] = B.psi[j];
      fo[u] = pold[j];
      fg[u] = B.carry[k];
      fz[u] = B.carry[K + k];
    } else {
      fy[u] = B.x[j];
    }
  }
  RAW cur0[NV], cur1[NV];
  if (!D.flsa) {
    const int64_t i0 = r0 + wave, i1 = i0 + 4;
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int64_t col = c0 + (int64_t)(t * 64 + lane) * V;
      if (i0 < r1) cur0[t] = load16(Xb + i0 * D.ldx + col);
      if (i1 < r1) cur1[t] = load16(Xb + i1 * D.ldx + col);
    }
  }
  if (cg) {
    const double gamma = s.gamma;
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int64_t j = c0 + tid + u * kWG;
      const double z = fma(fs[u], fg[u], fma(fp[u], fz[u], fy[u]));
      const double v = fma(gamma, fo[u], z);
      if (rb == 0) pnew[j] = v;
      sh_v[tid + u * kWG] = v;
    }
  } else {
#pragma unroll
    for (int u = 0; u < V; ++u) sh_v[tid + u * kWG] = fy[u];
  }
  __syncthreads();
  if (D.flsa) return;  // X = I: the column-panel kernel uses the operand itself

  if (MX && s.phase == PH_CG)
    rows_a<XT, float>(D, B, Xb, cb, r0, r1, c0, lane, wave, sh_v, cur0, cur1);
  else
    rows_a<XT, double>(D, B, Xb, cb, r0, r1, c0, lane, wave, sh_v, cur0, cur1);
}

template <typename XT, bool MX>
__global__ __launch_bounds__(kWG) void k_gemv_a(Dims D, Bufs B, const State* __restrict__ sin,
                                                State* __restrict__ sout) {
  gemv_a_body<XT, MX>(D, B, sin, sout, blockIdx.x);
}

// (M v)_j = lambda1 a_j v_j + lambda2 sum_k w_jk (v_j - v_k)  (A and B of the linear system)
__device__ inline double apply_m(const Bufs& B, const Params& prm, int64_t j, const double* v) {
  const double vj = v[j];
  double lap = 0.0;
  for (int q = B.rowptr[j]; q < B.rowptr[j + 1]; ++q) lap = fma(B.w[q], vj - v[B.col[q]], lap);
  return prm.lam1 * B.a[j] * vj + prm.lam2 * lap;
}

// Rows r0..r1 of one column panel for this lane's V columns:
// out[v] = sum_i X_{i, c0+v} u_i (rows of this wave, RU rows in flight).
template <typename XT, typename ACC, int RU>
__device__ inline void cols_b(const Dims& D, const XT* Xb, int64_t r0, int64_t r1, int64_t c0, int wave,
                              const double* sh_u, typename XV<XT>::raw (&cur)[RU], double* out) {
  constexpr int V = XV<XT>::V;
  using RAW = typename XV<XT>::raw;
  ACC acc[V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = 0;
  for (int64_t i = r0 + wave; i < r1; i += 4 * RU) {
    RAW nxt[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t ii = i + 4 * RU + 4 * u;
      if (ii < r1) nxt[u] = load16(Xb + ii * D.ldx + c0);
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t ii = i + 4 * u;
      if (ii < r1) {
        ACC xv[V];
        XV<XT>::cvt(cur[u], xv);
        const ACC uu = (ACC)sh_u[ii - r0];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = fma(xv[v], uu, acc[v]);
      }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) cur[u] = nxt[u];
  }
#pragma unroll
  for (int v = 0; v < V; ++v) out[v] = (double)acc[v];
}

// ---------------------------------------------------------------------------
// B: column-panel GEMV q_part[rb] = X[rb, :]^T u[rb] (u summed from the A
// partials).  PCG step: panel row 0 adds M p and each workgroup emits its
// share of p^T Q p.  MM boundary: the same product for the new residual, the
// loss partials 1/2 ||y - X b||^2, and (first nblk workgroups) reweighting
// a_j = 1/(|b_j|+eps), w_jk = 1/(|b_j - b_k|+eps), the tridiagonal part of M,
// the penalty sums of f, and each block's factorization product.
// ---------------------------------------------------------------------------
template <typename XT, bool MX>
__device__ __forceinline__ void gemv_b_body(const Dims& D, const Bufs& B, const State* __restrict__ sin,
                                            State* __restrict__ sout, const Params* __restrict__ prmp,
                                            const int wg) {
  constexpr int V = XV<XT>::V;
  constexpr int RU = 8;  // rows per wave in flight
  using RAW = typename XV<XT>::raw;
  const State s = *sin;
  const int tid = threadIdx.x;
  if (wg == 0 && tid == 0) *sout = s;
  if (s.phase == PH_DONE) return;
  const int lane = tid & 63, wave = tid >> 6;
  const int ngemm = D.cb2 * D.rb2;
  const int cb = wg % D.cb2, rb = wg / D.cb2;
  const int64_t r0 = (int64_t)rb * D.r2, r1 = wg < ngemm ? min<int64_t>(D.n, r0 + D.r2) : r0;
  const int64_t c0 = (int64_t)cb * D.c2 + lane * V;
  const XT* Xb = reinterpret_cast<const XT*>(B.X);
  const Params prm = *prmp;
  const bool cg = s.phase == PH_CG;
  const double* pv = cg ? (B.pbuf + (int64_t)((s.cg_iter + 1) & 1) * D.p_pad) : B.x;

  __shared__ double sh_u[kMaxR2];
  __shared__ double sh_red[4][64 * 8];
  __shared__ double sh_s[16];

  // u for the first 256 panel rows (sum of the A partials), issued before
  // the X rows so that waiting for it does not wait for them
  constexpr int CBMAX = 12;
  const int nr = (int)(r1 - r0);
  double upre[CBMAX];
  RAW cur[RU];
  if (!D.flsa) {
#pragma unroll
    for (int q = 0; q < CBMAX; ++q) upre[q] = (tid < nr && q < D.cb1) ? B.upart[(int64_t)q * D.n + r0 + tid] : 0.0;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t i = r0 + wave + 4 * u;
      if (i < r1) cur[u] = load16(Xb + i * D.ldx + c0);
    }
  }

  if (D.flsa && wg < ngemm) {
    // X = I (one row panel): X^T X v = v; at an MM boundary the loss partial
    // 1/2 ||y - x||^2 runs over this panel's coordinates
    double dotp = 0.0, loss = 0.0;
    for (int t = tid; t < 64 * V; t += kWG) {
      const int64_t j = (int64_t)cb * D.c2 + t;
      double q = 0.0;
      if (j < D.p) {
        q = pv[j];
        if (cg) q += apply_m(B, prm, j, pv);
        if (!cg) {
          const double dlt = B.y[j] - pv[j];
          loss = fma(dlt, dlt, loss);
        }
      }
      B.qpart[j] = q;
      if (cg) dotp = fma(pv[j], q, dotp);
    }
    if (cg) {
      const double tot = wg_sum(dotp, sh_s);
      if (tid == 0) B.pqpart[wg] = tot;
    } else {
      const double tot = wg_sum(loss, sh_s);
      if (tid == 0) B.losspart[cb] = tot;
    }
  } else if (wg < ngemm) {
    double loss = 0.0;
    for (int t = tid; t < nr; t += kWG) {
      double u = 0.0;
      if (t == tid) {
#pragma unroll
        for (int q = 0; q < CBMAX; ++q) u += upre[q];
        for (int q = CBMAX; q < D.cb1; ++q) u += B.upart[(int64_t)q * D.n + r0 + t];
      } else {
        for (int q = 0; q < D.cb1; ++q) u += B.upart[(int64_t)q * D.n + r0 + t];
      }
      sh_u[t] = u;
      if (!cg && cb == 0) {  // loss partials (used at an MM boundary)
        const double dlt = B.y[r0 + t] - u;
        loss = fma(dlt, dlt, loss);
      }
    }
    __syncthreads();
    if (MX && cg)
      cols_b<XT, float, RU>(D, Xb, r0, r1, c0, wave, sh_u, cur, &sh_red[wave][lane * V]);
    else
      cols_b<XT, double, RU>(D, Xb, r0, r1, c0, wave, sh_u, cur, &sh_red[wave][lane * V]);
    __syncthreads();
    double dotp = 0.0;
    for (int t = tid; t < 64 * V; t += kWG) {
      const int64_t j = (int64_t)cb * D.c2 + t;
      double q = (sh_red[0][t] + sh_red[1][t]) + (sh_red[2][t] + sh_red[3][t]);
      if (cg && rb == 0 && j < D.p) q += apply_m(B, prm, j, pv);
      B.qpart[(int64_t)rb * D.p_pad + j] = q;
      if (cg) dotp = fma(pv[j], q, dotp);
    }
    if (cg) {
      const double tot = wg_sum(dotp, sh_s);
      if (tid == 0) B.pqpart[wg] = tot;
    } else if (cb == 0) {
      const double tot = wg_sum(loss, sh_s);
      if (tid == 0) B.losspart[rb] = tot;
    }
  } else if (cg) {
    if (tid == 0) B.pqpart[wg] = 0.0;
  }

  const bool mmb = s.phase == PH_END;  // an MM boundary (not a refinement's residual refresh)
  if (mmb && wg < D.nblk) {
    // reweighting and the tridiagonal part of M, penalties
    const int64_t j = (int64_t)wg * kBlk + tid;
    double pen = 0.0, dj = 1.0, ej = 0.0;
    if (j < D.p) {
      const double xj = B.x[j];
      const double aj = 1.0 / (fabs(xj) + prm.eps);
      B.a[j] = aj;
      double wsum = 0.0;
      double pen2 = 0.0;
      for (int q = B.rowptr[j]; q < B.rowptr[j + 1]; ++q) {
        const int k = B.col[q];
        const double dlt = fabs(xj - B.x[k]);
        const double wq = 1.0 / (dlt + prm.eps);
        B.w[q] = wq;
        wsum += wq;
        if (k > j) pen2 += dlt;
        if (k == j - 1 && !prm.jacobi) ej = -prm.lam2 * wq;
      }
      pen = prm.lam1 * fabs(xj) + prm.lam2 * pen2;
      dj = prm.lam1 * aj + prm.lam2 * wsum;
      if (prm.jacobi) dj += B.s[j];
      B.d[j] = dj;
      B.e[j] = ej;
    } else if (j < D.p_pad) {
      B.d[j] = 1.0;
      B.e[j] = 0.0;
    }
    const double tot = wg_sum(pen, sh_s);
    if (tid == 0) B.penpart[wg] = tot;
  }
  if (mmb) {
    // The last workgroup to finish factors M = L D L^T over all p elements
    // (one wave runs the pivot chain); writes L and 1/D for the C launch.
    __shared__ int sh_flag;
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      const unsigned prev = atomicAdd(B.counter + 16, 1u);
      const bool last = prev == (unsigned)(D.gridB - 1);
      if (last) __threadfence();
      sh_flag = last;
    }
    __syncthreads();
    if (sh_flag) {
      if (wave == 0 && !prm.band) tri_factor_wave(B.d, B.e, B.L, B.invD, D.p, &sh_red[0][0]);
      if (tid == 0) B.counter[16] = 0u;
    }
  }
}

template <typename XT, bool MX>
__global__ __launch_bounds__(kWG) void k_gemv_b(Dims D, Bufs B, const State* __restrict__ sin,
                                                State* __restrict__ sout, const Params* __restrict__ prmp) {
  gemv_b_body<XT, MX>(D, B, sin, sout, prmp, blockIdx.x);
}

// Zero-inflow local solve of the block for the current residual r_j and the
// block scalars that the next A launch combines into the global solution:
//   forward  g_j = r_j - L_j g_{j-1}           (L D L^T, forward sweep)
//   backward y_j = g_j / D_j - L_{j+1} y_{j+1}   (backward sweep)
__device__ inline void block_local_solve(const Dims& D, const Bufs& B, int b, int64_t j, double rj, double Lj,
                                         double Lnext, double invDj, double sigj, double psij, double* lds,
                                         double* lds2) {
  const int tid = threadIdx.x;
  const Aff gf = wg_scan_fwd({-Lj, rj}, lds);
  const double g = gf.b;
  const Aff yb = wg_scan_rev({-Lnext, g * invDj}, lds);
  const double yj = yb.b;
  if (j < D.p_pad) B.yv[j] = yj;
  const int K = D.nblk;
  __syncthreads();
  if (tid == kBlk - 1) lds2[0] = g;
  if (tid == 0) lds2[1] = yj;
  double sums[4] = {rj * yj, rj * sigj, rj * psij, rj * rj};
  wg_sum4(sums, lds);
  if (tid == 0) {
    B.blk[BK_B * K + b] = lds2[0];
    B.blk[BK_YS * K + b] = lds2[1];
    B.blk[BK_RY * K + b] = sums[0];
    B.blk[BK_RS * K + b] = sums[1];
    B.blk[BK_RP * K + b] = sums[2];
    B.blk[BK_RR * K + b] = sums[3];
  }
}

// Reduction of the true residual that one refinement round asks of the
// FP32-product PCG (its products carry errors near 1e-7 relative, so it
// cannot be trusted much further in one round).
constexpr double kRoundReduction = 1e-4;

// Phase after a new residual (its squared norm rr, relative norm rn); also
// records the FP64 residual of a boundary or refresh in o.rres.
// Algorithm 2's inner loop is repeat-until: after the first residual of an
// MM step at least one PCG step runs unless that residual is exactly zero (nu
// would be 0/0).  After a PCG step the inner test decides.  With FP32
// products (mixed precision) a round of PCG stops once its recursive residual
// is kRoundReduction below the round's FP64 starting residual (or meets the
// inner tolerance); then the true residual c - Q x is recomputed in FP64 and
// the MM step ends only if that passes the inner test - else PCG restarts
// from it (iterative refinement).  Refinement also ends when a refresh has
// cut the true residual by less than 10 % (FP32 products can resolve no more
// on this system) or at the PCG step cap.
__device__ inline int32_t next_phase(const Params& prm, State& o, int mode, double rr, double rn) {
  const bool capped = o.cg_iter >= prm.max_cg;
  if (mode == CM_FIRST) {
    o.rres = rn;
    return rr > 0.0 ? PH_CG : PH_END;
  }
  const bool met = !(rn > prm.inner_tol);
  if (mode == CM_REFRESH) {
    const bool stalled = !(rn < 0.9 * o.rres);
    o.rres = rn;
    return (met || capped || stalled) ? PH_END : PH_CG;
  }
  if (capped) return PH_END;
  if (!prm.mixed) return met ? PH_END : PH_CG;
  return (met || !(rn > kRoundReduction * o.rres)) ? PH_RES : PH_CG;
}

// Wave-level variant of combine_blocks for K <= 256 (4 blocks per lane),
// run by wave 0 alone: shuffles only, no barriers.
__device__ void combine_blocks_wave(const Dims& D, const Bufs& B, const Params& prm, State o, double rz_prev,
                                    int mode, State* __restrict__ sout) {
  constexpr int E = 4;
  const int l = threadIdx.x & 63;
  const int K = D.nblk;
  const int e = (K + 63) / 64;
  const double* bk = B.blk;
  const int k0 = l * e;
  double fA[E], fB[E], fRY[E], fRS[E], fRP[E], fRR[E], nPS[E], nYS[E], nSS[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = k0 + i;
    const bool ok = i < e && k < K;
    const bool okn = i < e && k + 1 < K;
    fA[i] = ok ? bk[BK_A * K + k] : 1.0;
    fB[i] = ok ? bk[BK_B * K + k] : 0.0;
    fRY[i] = ok ? bk[BK_RY * K + k] : 0.0;
    fRS[i] = ok ? bk[BK_RS * K + k] : 0.0;
    fRP[i] = ok ? bk[BK_RP * K + k] : 0.0;
    fRR[i] = ok ? bk[BK_RR * K + k] : 0.0;
    nPS[i] = okn ? bk[BK_PSIS * K + k + 1] : 0.0;
    nYS[i] = okn ? bk[BK_YS * K + k + 1] : 0.0;
    nSS[i] = okn ? bk[BK_SIGS * K + k + 1] : 0.0;
  }
  Aff m = {1.0, 0.0};
#pragma unroll
  for (int i = 0; i < E; ++i)
    if (i < e && k0 + i < K) m = compose(m, {fA[i], fB[i]});
  const Aff fin = wave_scan_fwd(m);
  double G = __shfl_up(fin.b, 1, 64);
  if (l == 0) G = 0.0;
  double Gk[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    Gk[i] = G;
    if (i < e && k0 + i < K) G = fma(fA[i], G, fB[i]);
  }
  Aff mb = {1.0, 0.0};
#pragma unroll
  for (int i = E - 1; i >= 0; --i) {
    const int k = k0 + i;
    const double Gn = (i + 1 < e) ? Gk[(i + 1) < E ? i + 1 : 0] : G;
    if (i < e && k < K - 1) {
      mb = compose(mb, {nPS[i], fma(nSS[i], Gn, nYS[i])});
    } else if (i < e && k == K - 1) {
      mb = compose(mb, {0.0, 0.0});
    }
  }
  const Aff finb = wave_scan_rev(mb);
  double Z = __shfl_down(finb.b, 1, 64);
  if (l == 63) Z = 0.0;
  double rzp = 0.0, rrp = 0.0;
#pragma unroll
  for (int i = E - 1; i >= 0; --i) {
    const int k = k0 + i;
    if (i < e && k < K) {
      const double Gn = (i + 1 < e) ? Gk[(i + 1) < E ? i + 1 : 0] : G;
      Z = (k < K - 1) ? fma(nPS[i], Z, fma(nSS[i], Gn, nYS[i])) : 0.0;
      B.carry[k] = Gk[i];
      B.carry[K + k] = Z;
      rzp += fRY[i] + Gk[i] * fRS[i] + Z * fRP[i];
      rrp += fRR[i];
    }
  }
  const double rz = wave_sum(rzp);
  const double rr = wave_sum(rrp);
  if (l == 0) {
    const double rn = sqrt(rr) / prm.cnorm;
    o.phase = next_phase(prm, o, mode, rr, rn);
    o.rel_res = rn;
    o.rz = rz;
    o.gamma = mode != CM_STEP ? 0.0 : rz / rz_prev;
    *sout = o;
    *B.counter = 0u;
  }
}

// Called by every thread of the last C workgroup to finish, once the block
// scalars of all blocks are visible: carries of the partitioned tridiagonal
// solve over the blocks (forward G_k = forward-sweep value entering block k,
// backward Z_k = solution value entering block k from the right), r^T z,
// ||r||, the inner stopping test of Algorithm 2 and gamma = r^T z / r_old^T z_old.
__device__ void combine_blocks(const Dims& D, const Bufs& B, const Params& prm, State o, double rz_prev,
                               int mode, State* __restrict__ sout, double* sh_m, double* sh_G, double* sh_Z) {
  constexpr int EMAX = kMaxBlocks / kWG;
  const int tid = threadIdx.x;
  const int K = D.nblk;
  const int e4 = (K + kWG - 1) / kWG;
  const double* bk = B.blk;
  const int k0 = tid * e4;
  double fA[EMAX], fB[EMAX], fRY[EMAX], fRS[EMAX], fRP[EMAX], fRR[EMAX], nPS[EMAX], nYS[EMAX], nSS[EMAX];
#pragma unroll
  for (int i = 0; i < EMAX; ++i) {
    const int k = k0 + i;
    const bool ok = i < e4 && k < K;
    const bool okn = i < e4 && k + 1 < K;
    fA[i] = ok ? bk[BK_A * K + k] : 1.0;
    fB[i] = ok ? bk[BK_B * K + k] : 0.0;
    fRY[i] = ok ? bk[BK_RY * K + k] : 0.0;
    fRS[i] = ok ? bk[BK_RS * K + k] : 0.0;
    fRP[i] = ok ? bk[BK_RP * K + k] : 0.0;
    fRR[i] = ok ? bk[BK_RR * K + k] : 0.0;
    nPS[i] = okn ? bk[BK_PSIS * K + k + 1] : 0.0;
    nYS[i] = okn ? bk[BK_YS * K + k + 1] : 0.0;
    nSS[i] = okn ? bk[BK_SIGS * K + k + 1] : 0.0;
  }
  Aff m = {1.0, 0.0};
#pragma unroll
  for (int i = 0; i < EMAX; ++i)
    if (i < e4 && k0 + i < K) m = compose(m, {fA[i], fB[i]});
  const Aff fin = wg_scan_fwd(m, sh_m + 8);
  __syncthreads();
  sh_G[kMaxBlocks - 1 - tid] = fin.b;  // scratch: inclusive result per thread
  __syncthreads();
  double G = tid == 0 ? 0.0 : sh_G[kMaxBlocks - tid];
  __syncthreads();
  double Gk[EMAX];
#pragma unroll
  for (int i = 0; i < EMAX; ++i) {
    Gk[i] = G;
    if (i < e4 && k0 + i < K) G = fma(fA[i], G, fB[i]);
  }
  // Z_k = psis_{k+1} Z_{k+1} + ys_{k+1} + sigs_{k+1} G_{k+1},  Z_{K-1} = 0
  Aff mb = {1.0, 0.0};
#pragma unroll
  for (int i = EMAX - 1; i >= 0; --i) {
    const int k = k0 + i;
    const double Gn = (i + 1 < e4) ? Gk[(i + 1) < EMAX ? i + 1 : 0] : G;
    if (i < e4 && k < K - 1) {
      mb = compose(mb, {nPS[i], fma(nSS[i], Gn, nYS[i])});
    } else if (i < e4 && k == K - 1) {
      mb = compose(mb, {0.0, 0.0});
    }
  }
  const Aff finb = wg_scan_rev(mb, sh_m + 8);
  __syncthreads();
  sh_Z[kMaxBlocks - 1 - tid] = finb.b;
  __syncthreads();
  double Z = tid == kWG - 1 ? 0.0 : sh_Z[kMaxBlocks - 2 - tid];
  double rzp = 0.0, rrp = 0.0;
#pragma unroll
  for (int i = EMAX - 1; i >= 0; --i) {
    const int k = k0 + i;
    if (i < e4 && k < K) {
      const double Gn = (i + 1 < e4) ? Gk[(i + 1) < EMAX ? i + 1 : 0] : G;
      Z = (k < K - 1) ? fma(nPS[i], Z, fma(nSS[i], Gn, nYS[i])) : 0.0;
      B.carry[k] = Gk[i];
      B.carry[K + k] = Z;
      rzp += fRY[i] + Gk[i] * fRS[i] + Z * fRP[i];
      rrp += fRR[i];
    }
  }
  const double rz = wg_sum(rzp, sh_m + 8);
  const double rr = wg_sum(rrp, sh_m + 8);
  if (tid == 0) {
    const double rn = sqrt(rr) / prm.cnorm;
    o.phase = next_phase(prm, o, mode, rr, rn);
    o.rel_res = rn;
    o.rz = rz;
    o.gamma = mode != CM_STEP ? 0.0 : rz / rz_prev;
    *sout = o;
    *B.counter = 0u;
  }
}

// True in the one workgroup that finishes last; its loads after this point
// see every other workgroup's block scalars (release by each block before its
// arrival, acquire by the last one).  No workgroup waits for another.
// Only thread 0 wrote the block scalars, so only it needs to publish them;
// the last block's acquire fence by thread 0 precedes the barrier after which
// all of its threads read the other blocks' scalars.
__device__ inline bool arrive_last(const Bufs& B, int nblocks, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(B.counter, 1u);
    const bool last = prev == (unsigned)(nblocks - 1);
    if (last) __threadfence();
    *flag = last;
  }
  __syncthreads();
  return *flag != 0;
}

// ---------------------------------------------------------------------------
// C: per solver block (256 elements).  PCG step: nu = r^T z / p^T Q p,
// x += nu p, r -= nu Q p (the residual update with the minus sign), then the
// local solve of the new residual.  MM boundary: f of the iterate, the
// relative-change test of Algorithm 2, and - if continuing - the LDL^T
// factorization of the tridiagonal M (carry of the block products, then the
// block's own continued fraction), the gain vectors, r0 = c - Q x0 and its
// local solve.  The last workgroup to finish combines the blocks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_body(const Dims& D, const Bufs& B, const State* __restrict__ sin,
                                           State* __restrict__ sout, const Params* __restrict__ prmp,
                                           const int b) {
  constexpr int QMAX = 16;  // row panels whose partial products are prefetched
  const State s = *sin;
  const int tid = threadIdx.x;
  if (s.phase == PH_DONE) {
    if (b == 0 && tid == 0) *sout = s;
    return;
  }
  const int64_t j = (int64_t)b * kBlk + tid;
  const bool real = j < D.p;
  const Params prm = *prmp;
  __shared__ double lds[24];
  __shared__ double lds2[4];
  __shared__ double sh_L[kBlk + 1];
  __shared__ double sh_G[kMaxBlocks], sh_Z[kMaxBlocks];
  __shared__ int sh_flag;

  if (s.phase == PH_CG) {
    // every input of this step in one round of loads
    const double* pv = B.pbuf + (int64_t)((s.cg_iter + 1) & 1) * D.p_pad;
    double part = 0.0;
    for (int q = tid; q < D.gridB; q += kWG) part += B.pqpart[q];
    double qp[QMAX];
#pragma unroll
    for (int rb = 0; rb < QMAX; ++rb) qp[rb] = (real && rb < D.rb2) ? B.qpart[(int64_t)rb * D.p_pad + j] : 0.0;
    double qrest = 0.0;
    for (int rb = QMAX; rb < D.rb2; ++rb) qrest += real ? B.qpart[(int64_t)rb * D.p_pad + j] : 0.0;
    double pj = 0.0, xj = 0.0, rj0 = 0.0, Lj = 0.0, invDj = 0.0, sigj = 0.0, psij = 0.0, Lnb = 0.0;
    if (real) {
      pj = pv[j];
      xj = B.x[j];
      rj0 = B.r[j];
      Lj = B.L[j];
      invDj = B.invD[j];
      sigj = B.sig[j];
      psij = B.psi[j];
    }
    if (tid == 0) Lnb = (j + kBlk < D.p) ? B.L[j + kBlk] : 0.0;
    const double pq = wg_sum(part, lds);
    const double nu = s.rz / pq;
    if (!(pq > 0.0) || !isfinite(nu)) {
      if (b == 0 && tid == 0) {
        State o = s;
        o.phase = PH_DONE;
        o.status = ST_NUMERICAL;
        *sout = o;
      }
      return;
    }
    double rj = 0.0;
    if (real) {
      double q = 0.0;
#pragma unroll
      for (int rb = 0; rb < QMAX; ++rb) q += qp[rb];
      q += qrest;
      B.x[j] = fma(nu, pj, xj);
      rj = fma(-nu, q, rj0);
      B.r[j] = rj;
    }
    if (prm.band) {  // the K launch solves with the new residual
      if (b == 0 && tid == 0) {
        State o = s;
        o.cg_iter = s.cg_iter + 1;
        o.cg_total = s.cg_total + 1;
        o.nu = nu;
        *sout = o;
      }
      return;
    }
    sh_L[tid] = Lj;
    if (tid == 0) sh_L[kBlk] = Lnb;
    __syncthreads();
    block_local_solve(D, B, b, j, rj, Lj, sh_L[tid + 1], invDj, sigj, psij, lds, lds2);
    if (arrive_last(B, D.nblk, &sh_flag)) {
      State o = s;
      o.cg_iter = s.cg_iter + 1;
      o.cg_total = s.cg_total + 1;
      o.nu = nu;
      if (D.nblk <= 4 * 64) {
        if (tid < 64) combine_blocks_wave(D, B, prm, o, s.rz, CM_STEP, sout);
      } else {
        combine_blocks(D, B, prm, o, s.rz, CM_STEP, sout, lds, sh_G, sh_Z);
      }
    }
    return;
  }

  // ---- MM boundary, or an FP64 residual refresh (refinement) ----
  // inputs that do not depend on the decision, loaded up front (L and 1/D come
  // from the sequential factorization at the end of the B launch)
  double cj = 0.0, qsum = 0.0, Lj = 0.0, invDj = 0.0, Lnb = 0.0;
  if (real) {
    cj = B.c[j];
    Lj = B.L[j];
    invDj = B.invD[j];
    for (int rb = 0; rb < D.rb2; ++rb) qsum += B.qpart[(int64_t)rb * D.p_pad + j];
  }
  if (tid == 0) Lnb = (j + kBlk < D.p) ? B.L[j + kBlk] : 0.0;
  if (s.phase == PH_RES) {
    // true residual c - (X^T X + M) x of this MM step's system, in FP64 (the
    // weights and the factorization of M are the ones the PCG used)
    double rj = 0.0;
    if (real) {
      rj = cj - (qsum + apply_m(B, prm, j, B.x));
      B.r[j] = rj;
    }
    if (prm.band) {  // the K launch solves with the existing factor
      if (b == 0 && tid == 0) {
        State o = s;
        o.phase = PH_BANDRES;
        *sout = o;
      }
      return;
    }
    const double sigj = real ? B.sig[j] : 0.0, psij = real ? B.psi[j] : 0.0;
    sh_L[tid] = Lj;
    if (tid == 0) sh_L[kBlk] = Lnb;
    __syncthreads();
    block_local_solve(D, B, b, j, rj, Lj, sh_L[tid + 1], invDj, sigj, psij, lds, lds2);
    if (arrive_last(B, D.nblk, &sh_flag)) {
      if (D.nblk <= 4 * 64) {
        if (tid < 64) combine_blocks_wave(D, B, prm, s, 0.0, CM_REFRESH, sout);
      } else {
        combine_blocks(D, B, prm, s, 0.0, CM_REFRESH, sout, lds, sh_G, sh_Z);
      }
    }
    return;
  }
  // f(b) = loss + penalties (identical arithmetic in every workgroup)
  double fpart = 0.0;
  for (int q = tid; q < D.nloss; q += kWG) fpart += B.losspart[q];
  const double loss = wg_sum(fpart, lds);
  double ppart = 0.0;
  for (int q = tid; q < D.nblk; q += kWG) ppart += B.penpart[q];
  const double pen = wg_sum(ppart, lds);
  const double f_new = 0.5 * loss + pen;
  State o = s;
  o.f_new = f_new;
  bool finish = false;
  if (!isfinite(f_new)) {
    o.status = ST_NUMERICAL;
    finish = true;
  } else if (s.first) {
    o.first = 0;
  } else {
    o.mm_iter = s.mm_iter + 1;
    const double re = s.f_old != 0.0 ? fabs(f_new - s.f_old) / fabs(s.f_old) : fabs(f_new - s.f_old);
    o.rel_change = re;
    if (re <= prm.tol) {
      o.status = ST_OK;
      finish = true;
    } else if (o.mm_iter >= prm.max_iter) {
      o.status = ST_MAX_ITER;
      finish = true;
    }
  }
  if (finish) {
    o.phase = PH_DONE;
    if (b == 0 && tid == 0) *sout = o;
    return;
  }
  o.f_old = f_new;
  o.first_cg = 1;
  o.cg_iter = 0;
  if (prm.band) {  // r0 = c - (X^T X + M) x0; the K launch factors M and solves
    if (real) B.r[j] = cj - (qsum + apply_m(B, prm, j, B.x));
    if (b == 0 && tid == 0) {
      o.phase = PH_BANDMM;
      *sout = o;
    }
    return;
  }
  sh_L[tid] = Lj;
  if (tid == 0) sh_L[kBlk] = Lnb;
  __syncthreads();
  const double Lnext = sh_L[tid + 1];
  // phi_j = prod_{i=start..j} (-L_i); psi_j = prod_{i=j+1..end+1} (-L_i);
  // sigma = zero-inflow backward sweep of phi / D
  const double phi = wg_scan_fwd({-Lj, 0.0}, lds).a;
  const double psi = wg_scan_rev({-Lnext, 0.0}, lds).a;
  const double sig = wg_scan_rev({-Lnext, phi * invDj}, lds).b;
  const double psij = real ? psi : 0.0;
  const double sigj = real ? sig : 0.0;
  if (j < D.p_pad) {
    B.L[j] = Lj;
    B.invD[j] = invDj;
    B.sig[j] = sigj;
    B.psi[j] = psij;
  }
  __syncthreads();
  if (tid == kBlk - 1) lds2[0] = phi;
  if (tid == 0) { lds2[1] = sigj; lds2[3] = psij; }
  __syncthreads();
  if (tid == 0) {
    const int K = D.nblk;
    B.blk[BK_A * K + b] = lds2[0];
    B.blk[BK_SIGS * K + b] = lds2[1];
    B.blk[BK_PSIS * K + b] = lds2[3];
  }
  // r0 = c - (X^T X + M) x0 with x0 the MM iterate (Algorithm 2)
  double rj = 0.0;
  if (real) {
    rj = cj - (qsum + apply_m(B, prm, j, B.x));
    B.r[j] = rj;
  }
  block_local_solve(D, B, b, j, rj, Lj, Lnext, invDj, sigj, psij, lds, lds2);
  if (arrive_last(B, D.nblk, &sh_flag)) {
    if (D.nblk <= 4 * 64) {
      if (tid < 64) combine_blocks_wave(D, B, prm, o, 0.0, CM_FIRST, sout);
    } else {
      combine_blocks(D, B, prm, o, 0.0, CM_FIRST, sout, lds, sh_G, sh_Z);
    }
  }
}

__global__ __launch_bounds__(kWG) void k_block(Dims D, Bufs B, const State* __restrict__ sin,
                                               State* __restrict__ sout, const Params* __restrict__ prmp) {
  block_body(D, B, sin, sout, prmp, blockIdx.x);
}

// ---------------------------------------------------------------------------
// K (banded M, one workgroup): z = M^-1 r through the banded Cholesky factor,
// r^T z, ||r||, the inner stopping test of Algorithm 2 and gamma.  After an
// MM boundary (PH_BANDMM) it first assembles M from the new weights and
// factors it.  A then rebuilds p from z = yv (gains and carries are zero).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void band_body(const Dims& D, const Bufs& B, const State* __restrict__ sin,
                                          State* __restrict__ sout, const Params* __restrict__ prmp) {
  __shared__ double lds[kBandLds];
  __shared__ double red[24];
  const State s = *sin;
  const int tid = threadIdx.x;
  if (s.phase != PH_CG && s.phase != PH_BANDMM && s.phase != PH_BANDRES) {  // nothing to solve
    if (tid == 0) *sout = s;
    return;
  }
  const Params prm = *prmp;
  const int W = prm.band;
  const bool mm = s.phase == PH_BANDMM;
  State o = s;
  if (mm) {
    band_assemble(B.d, B.rowptr, B.col, B.w, prm.lam2, D.p, W, B.Lb);
    if (!band_factor(B.Lb, B.LbT, B.invdb, D.p, W, lds)) {
      if (tid == 0) {
        o.phase = PH_DONE;
        o.status = ST_NUMERICAL;
        *sout = o;
      }
      return;
    }
    __syncthreads();
  }
  band_solve(B.r, B.btmp, B.yv, B.Lb, B.LbT, B.invdb, D.p, W, lds);
  double rzp = 0.0, rrp = 0.0;
  for (int64_t j = tid; j < D.p; j += kWG) {
    const double rj = B.r[j];
    rzp = fma(rj, B.yv[j], rzp);
    rrp = fma(rj, rj, rrp);
  }
  double sums[4] = {rzp, rrp, 0.0, 0.0};
  wg_sum4(sums, red);
  if (tid == 0) {
    const double rz = sums[0], rn = sqrt(sums[1]) / prm.cnorm;
    const int mode = mm ? CM_FIRST : s.phase == PH_BANDRES ? CM_REFRESH : CM_STEP;
    o.phase = next_phase(prm, o, mode, sums[1], rn);
    o.rel_res = rn;
    o.gamma = mode != CM_STEP ? 0.0 : rz / s.rz;
    o.rz = rz;
    *sout = o;
  }
}

__global__ __launch_bounds__(kWG) void k_band(Dims D, Bufs B, const State* __restrict__ sin,
                                              State* __restrict__ sout, const Params* __restrict__ prmp) {
  band_body(D, B, sin, sout, prmp);
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Grouped launches of the ragged batch: one launch of each rotation kernel
// covers every problem of the batch that stores X in the same type; a
// workgroup finds its problem from the offsets of the problems' shares and
// runs that problem's kernel body on its own operands, so each problem's
// arithmetic is that of its solo launch.
// ---------------------------------------------------------------------------
__device__ inline int group_of(const GroupEntry* __restrict__ e, int count, int wg, int which) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int start = which == 0 ? e[mid].wg_a : which == 1 ? e[mid].wg_b : e[mid].wg_c;
    if (start <= wg) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename XT, bool MX>
__global__ __launch_bounds__(kWG) void k_gemv_a_grp(const GroupEntry* __restrict__ e, int count, int par) {
  const GroupEntry& g = e[group_of(e, count, (int)blockIdx.x, 0)];
  gemv_a_body<XT, MX>(g.D, g.B, g.B.st + par, g.B.st + (par ^ 1), (int)blockIdx.x - g.wg_a);
}

template <typename XT, bool MX>
__global__ __launch_bounds__(kWG) void k_gemv_b_grp(const GroupEntry* __restrict__ e, int count, int par) {
  const GroupEntry& g = e[group_of(e, count, (int)blockIdx.x, 1)];
  gemv_b_body<XT, MX>(g.D, g.B, g.B.st + par, g.B.st + (par ^ 1), g.B.prm, (int)blockIdx.x - g.wg_b);
}

__global__ __launch_bounds__(kWG) void k_block_grp(const GroupEntry* __restrict__ e, int count, int par) {
  const GroupEntry& g = e[group_of(e, count, (int)blockIdx.x, 2)];
  block_body(g.D, g.B, g.B.st + par, g.B.st + (par ^ 1), g.B.prm, (int)blockIdx.x - g.wg_c);
}

__global__ __launch_bounds__(kWG) void k_band_grp(const GroupEntry* __restrict__ e, int par) {
  const GroupEntry& g = e[blockIdx.x];
  if (!g.band) {
    if (threadIdx.x == 0) g.B.st[par ^ 1] = g.B.st[par];
    return;
  }
  band_body(g.D, g.B, g.B.st + par, g.B.st + (par ^ 1), g.B.prm);
}

// State of every problem of a batch after a graph launch (slot 0 of each).
__global__ __launch_bounds__(kWG) void k_gather_states(const GroupEntry* __restrict__ e, int count,
                                                       State* __restrict__ out) {
  const int i = (int)blockIdx.x * kWG + threadIdx.x;
  if (i < count) out[i] = e[i].B.st[0];
}

template <typename XT, bool MX>
static hipError_t launch_grouped_t(const GroupEntry* e, int count, int wgs, int par, int which, hipStream_t st) {
  switch (which) {
    case 0: hipLaunchKernelGGL((k_gemv_a_grp<XT, MX>), dim3(wgs), dim3(kWG), 0, st, e, count, par); break;
    case 1: hipLaunchKernelGGL((k_gemv_b_grp<XT, MX>), dim3(wgs), dim3(kWG), 0, st, e, count, par); break;
    case 2: hipLaunchKernelGGL(k_block_grp, dim3(wgs), dim3(kWG), 0, st, e, count, par); break;
    default: hipLaunchKernelGGL(k_band_grp, dim3(count), dim3(kWG), 0, st, e, par); break;
  }
  return hipGetLastError();
}

hipError_t launch_grouped(int dtype, bool mixed, const GroupEntry* e, int count, int wgs, int par, int which,
                          hipStream_t st) {
  switch (dtype) {
    case 0: return mixed ? launch_grouped_t<double, true>(e, count, wgs, par, which, st)
                         : launch_grouped_t<double, false>(e, count, wgs, par, which, st);
    case 1: return mixed ? launch_grouped_t<float, true>(e, count, wgs, par, which, st)
                         : launch_grouped_t<float, false>(e, count, wgs, par, which, st);
    default: return mixed ? launch_grouped_t<uint16_t, true>(e, count, wgs, par, which, st)
                          : launch_grouped_t<uint16_t, false>(e, count, wgs, par, which, st);
  }
}

hipError_t launch_gather_states(const GroupEntry* e, int count, State* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_states, dim3((unsigned)((count + kWG - 1) / kWG)), dim3(kWG), 0, st, e, count, out);
  return hipGetLastError();
}

template <typename XT, bool MX>
static hipError_t launch_rotation_t(const Dims& D, const Bufs& B, int par, int which, hipStream_t st) {
  const State* sin = B.st + par;
  State* sout = B.st + (par ^ 1);
  switch (which) {
    case 0:
      hipLaunchKernelGGL((k_gemv_a<XT, MX>), dim3(D.cb1 * D.rb1), dim3(kWG), 0, st, D, B, sin, sout);
      break;
    case 1:
      hipLaunchKernelGGL((k_gemv_b<XT, MX>), dim3(D.gridB), dim3(kWG), 0, st, D, B, sin, sout, B.prm);
      break;
    case 3:
      hipLaunchKernelGGL(k_band, dim3(1), dim3(kWG), 0, st, D, B, sin, sout, B.prm);
      break;
    default:
      hipLaunchKernelGGL(k_block, dim3(D.nblk), dim3(kWG), 0, st, D, B, sin, sout, B.prm);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_rotation(const Dims& D, const Bufs& B, int par, int which, hipStream_t st, bool mixed) {
  switch (D.dtype) {
    case 0: return mixed ? launch_rotation_t<double, true>(D, B, par, which, st)
                         : launch_rotation_t<double, false>(D, B, par, which, st);
    case 1: return mixed ? launch_rotation_t<float, true>(D, B, par, which, st)
                         : launch_rotation_t<float, false>(D, B, par, which, st);
    default: return mixed ? launch_rotation_t<uint16_t, true>(D, B, par, which, st)
                          : launch_rotation_t<uint16_t, false>(D, B, par, which, st);
  }
}

template <typename XT>
static hipError_t launch_setup_t(const Dims& D, const void* X, const double* y, double* cpart, double* spart,
                                 double* c, double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_setup_partial<XT>, dim3(D.cb2 * D.rb2), dim3(kWG), 0, st, D, reinterpret_cast<const XT*>(X),
                     y, cpart, spart);
  hipLaunchKernelGGL(k_setup_final, dim3((unsigned)((D.p_pad + kWG - 1) / kWG)), dim3(kWG), 0, st, D, cpart, spart,
                     c, s);
  return hipGetLastError();
}

hipError_t launch_setup(const Dims& D, const void* X, const double* y, double* cpart, double* spart, double* c,
                        double* s, hipStream_t st) {
  switch (D.dtype) {
    case 0: return launch_setup_t<double>(D, X, y, cpart, spart, c, s, st);
    case 1: return launch_setup_t<float>(D, X, y, cpart, spart, c, s, st);
    default: return launch_setup_t<uint16_t>(D, X, y, cpart, spart, c, s, st);
  }
}

hipError_t launch_init(const Dims& D, const Bufs& B, const double* warm, int use_warm, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3((unsigned)((D.p_pad + kWG - 1) / kWG)), dim3(kWG), 0, st, D, B, warm, use_warm);
  return hipGetLastError();
}

// Non-finite scan of the stored X (validation at creation).
template <typename XT>
__global__ __launch_bounds__(kWG) void k_check_finite(const XT* __restrict__ X, int64_t count, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * kWG;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < count; i += stride) {
    if constexpr (sizeof(XT) == 2) {
      bad |= (X[i] & 0x7f80u) == 0x7f80u;
    } else {
      bad |= !isfinite((double)X[i]);
    }
  }
  if (bad) *flag = 1;
}

hipError_t launch_check_finite(const void* X, int dtype, int64_t count, int* flag, hipStream_t st) {
  const dim3 g(1024), b(kWG);
  switch (dtype) {
    case 0: hipLaunchKernelGGL(k_check_finite<double>, g, b, 0, st, reinterpret_cast<const double*>(X), count, flag); break;
    case 1: hipLaunchKernelGGL(k_check_finite<float>, g, b, 0, st, reinterpret_cast<const float*>(X), count, flag); break;
    default: hipLaunchKernelGGL(k_check_finite<uint16_t>, g, b, 0, st, reinterpret_cast<const uint16_t*>(X), count, flag); break;
  }
  return hipGetLastError();
}

}  // namespace flr
