// Exact preconditioner solve for graphs whose index bandwidth bw = max |j - k|
// over E is at least 2 (the 2-D lattice, all-pairs fusion): M = lambda1 A +
// lambda2 B is banded with bandwidth bw, and Algorithm 2 applies M^-1 through
// its banded Cholesky factor M = L L^T (Section 3.2; the lattice in the
// paper's 2-D experiments has bw = q).  M changes once per MM iteration, so
// the factor is computed once per MM iteration and every PCG step applies it
// with two triangular sweeps.
//
// Layouts (W = bw + 1 entries per row / column):
//   Lb  column-major band, Lb[j*W + k] = L_{j+k, j}   (column j of L)
//   LbT row-major band,    LbT[i*W + k] = L_{i, i-k}  (row i of L)
//   invd[j] = 1 / L_jj
// Both sweeps walk one dependent chain of length p, so one wave runs each:
// the not-yet-final right-hand sides of the next bw elements sit in a ring of
// 64*NR registers across the wave's lanes (element t in slot t mod 64*NR),
// each step reads the current element from its lane, scales it by 1/L_jj and
// subtracts its multiple from the ring with one fma per register; the other
// three waves of the workgroup stage the multipliers of the coming steps into
// LDS, already permuted to the ring's slot order.
#pragma once
#include "flr_device.h"

namespace flr {

constexpr int kBandLds = 13312;   // doubles of LDS the band routines use (104 KiB)
constexpr int kBandMaxW = 1025;   // widest band the sweeps handle (NR = 17 ring registers)

// Ring registers per lane: 64*NR slots must hold the bw elements ahead of the
// current one plus the 64 of the chunk being consumed.
__host__ __device__ inline int band_nr(int W) {
  const int need = (W + 63 + 63) / 64;
  const int opts[] = {2, 3, 4, 5, 6, 8, 12, 17};
  for (int o : opts)
    if (o >= need) return o;
  return 0;
}

// Band of M below the diagonal, column-major: Lb[k*W] = d_k (the diagonal
// lambda1 a_k + lambda2 sum_q w_q), Lb[k*W + (c - k)] = -lambda2 w_q for every
// edge (k, c) with k < c, zero elsewhere.  Whole workgroup; ends with a barrier.
__device__ inline void band_assemble(const double* __restrict__ d, const int32_t* __restrict__ rowptr,
                                     const int32_t* __restrict__ col, const double* __restrict__ w, double lam2,
                                     int64_t p, int W, double* __restrict__ Lb) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t tot = p * (int64_t)W;
  for (int64_t i = tid; i < tot; i += nt) Lb[i] = 0.0;
  __syncthreads();
  for (int64_t k = tid; k < p; k += nt) {
    Lb[k * W] = d[k];
    for (int q = rowptr[k]; q < rowptr[k + 1]; ++q) {
      const int64_t c = col[q];
      if (c > k && c - k < W) Lb[k * W + (c - k)] = -lam2 * w[q];
    }
  }
  __syncthreads();
}

// Right-looking Cholesky of the assembled band, in place.  Step j takes the
// pivot, writes column j of L (to Lb and, transposed, to LbT) and subtracts
// the outer product of its scaled column from columns j+1 .. j+bw.  Those
// columns live in an LDS ring of W + 1 slots when it fits (column j + W is
// loaded into the slot column j - 1 left), else they are updated in Lb and
// column j is scaled one step later.  256 threads; returns false in every
// thread when a pivot is not positive and finite.
__device__ inline bool band_factor(double* __restrict__ Lb, double* __restrict__ LbT, double* __restrict__ invd,
                                   int64_t p, int W, double* __restrict__ lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int R = W + 1;
  const bool ring = (int64_t)R * W <= kBandLds;
  if (ring) {
    const int64_t ncol = p < W ? p : W;
    for (int64_t i = tid; i < ncol * W; i += nt) lds[i] = Lb[i];
  }
  __syncthreads();
  bool ok = true;
  double inv_prev = 0.0, ljj_prev = 0.0;
  int dmax_prev = -1;
  for (int64_t j = 0; j < p; ++j) {
    const int dmax = (int)((p - 1 - j) < (int64_t)(W - 1) ? (p - 1 - j) : (int64_t)(W - 1));
    if (ring) {
      const double* cj = lds + (j % R) * W;
      const double piv = cj[0];
      if (!(piv > 0.0) || !isfinite(piv)) {
        ok = false;
        break;
      }
      const double ljj = sqrt(piv), inv = 1.0 / ljj;
      for (int d = tid; d <= dmax; d += nt) {
        const double v = d ? cj[d] * inv : ljj;
        Lb[j * W + d] = v;
        LbT[(j + d) * W + d] = v;
      }
      if (tid == 0) invd[j] = inv;
      for (int d1 = 1 + ty; d1 <= dmax; d1 += 16) {
        const double s1 = cj[d1] * inv;
        double* tgt = lds + ((j + d1) % R) * W - d1;
        for (int d2 = d1 + tx; d2 <= dmax; d2 += 16) tgt[d2] = fma(-s1, cj[d2] * inv, tgt[d2]);
      }
      if (j + W < p) {
        double* slot = lds + ((j + W) % R) * W;
        for (int d = tid; d < W; d += nt) slot[d] = Lb[(j + W) * W + d];
      }
      __syncthreads();
    } else {
      double* cj = Lb + j * W;
      const double piv = cj[0];
      if (!(piv > 0.0) || !isfinite(piv)) {
        ok = false;
        break;
      }
      const double ljj = sqrt(piv), inv = 1.0 / ljj;
      double* colj = lds;  // scaled column j
      for (int d = tid; d <= dmax; d += nt) {
        const double v = d ? cj[d] * inv : ljj;
        colj[d] = v;
        LbT[(j + d) * W + d] = v;
      }
      if (tid == 0) invd[j] = inv;
      if (j > 0)  // column j - 1 is final: scale it in place
        for (int d = tid; d <= dmax_prev; d += nt)
          Lb[(j - 1) * W + d] = d ? Lb[(j - 1) * W + d] * inv_prev : ljj_prev;
      __syncthreads();
      for (int d1 = 1 + ty; d1 <= dmax; d1 += 16) {
        const double s1 = colj[d1];
        double* tgt = Lb + (j + d1) * W - d1;
        for (int d2 = d1 + tx; d2 <= dmax; d2 += 16) tgt[d2] = fma(-s1, colj[d2], tgt[d2]);
      }
      inv_prev = inv;
      ljj_prev = ljj;
      dmax_prev = dmax;
      __syncthreads();
    }
  }
  if (ok && !ring && p > 0) {
    for (int d = tid; d <= dmax_prev; d += nt) Lb[(p - 1) * W + d] = d ? Lb[(p - 1) * W + d] * inv_prev : ljj_prev;
    __syncthreads();
  }
  return ok;
}

__device__ inline double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// SC steps of the sweep by wave 0, ring register R0 holding the current chunk.
template <int NR, int SC, int R0>
__device__ __forceinline__ void band_steps(double (&reg)[NR], double& yout, double idv, const double* __restrict__ buf,
                                  int64_t t0, int lc0, int64_t p, int lane) {
#pragma unroll
  for (int l = 0; l < SC; ++l) {
    if (t0 + l >= p) break;
    const int lc = lc0 + l;
    const double yj = readlane_f64(reg[R0], lc) * readlane_f64(idv, lc);
    yout = lane == lc ? yj : yout;
#pragma unroll
    for (int r = 0; r < NR; ++r) reg[r] = fma(-buf[(l * NR + r) * 64 + lane], yj, reg[r]);
  }
}

template <int NR, int SC, int R0>
__device__ __forceinline__ void band_steps_sw(int r0, double (&reg)[NR], double& yout, double idv, const double* buf,
                                     int64_t t0, int lc0, int64_t p, int lane) {
  if constexpr (R0 < NR) {
    if (r0 == R0)
      band_steps<NR, SC, R0>(reg, yout, idv, buf, t0, lc0, p, lane);
    else
      band_steps_sw<NR, SC, R0 + 1>(r0, reg, yout, idv, buf, t0, lc0, p, lane);
  }
}

// One triangular sweep: virtual step t handles element e(t) = t (forward,
// L y = b with the columns of L) or p - 1 - t (backward, L^T z = b with the
// rows of L); the multipliers of step t are Mult[e(t)*W + k] for the element
// k steps further along.  Whole workgroup of 256 threads; stage: kBandLds
// doubles of LDS.  Ends with a barrier.
template <int NR, int SC>
__device__ __forceinline__ void band_sweep_t(const double* __restrict__ b, double* __restrict__ out, const double* __restrict__ Mult,
                             const double* __restrict__ invd, int64_t p, int W, bool fwd, double* __restrict__ stage) {
  constexpr int RS = 64 * NR;
  constexpr int BUF = SC * NR * 64;
  static_assert(2 * BUF <= kBandLds, "stage buffers exceed the LDS budget");
  static_assert(64 % SC == 0, "sub-chunks must tile a chunk");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bw = W - 1;
  const int64_t nsub = (p + SC - 1) / SC;
  auto elem = [&](int64_t t) { return fwd ? t : p - 1 - t; };
  // Waves 1..3 stage sub-chunk s: all PER loads of a thread are issued before
  // any is written to LDS, and they are issued one sub-chunk early (into
  // pend), so their latency hides behind wave 0's steps.
  constexpr int NL = kWG - 64;
  constexpr int PER = (BUF + NL - 1) / NL;
  double pend[PER];
  auto stage_load = [&](int64_t s) {
    const int64_t t0 = s * SC;
    const int r0 = (int)((t0 / 64) % NR);
    const int lc0 = (int)(t0 % 64);
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int i = tid - 64 + NL * m;
      const int l = i / (NR * 64), rem = i - l * (NR * 64), r = rem >> 6, ln = rem & 63;
      const int64_t t = t0 + l;
      int k = ((r - r0 + NR) % NR) * 64 + ln - (lc0 + l);
      if (k < 0) k += RS;
      pend[m] = (i < BUF && t < p && k >= 1 && k <= bw) ? Mult[elem(t) * W + k] : 0.0;
    }
  };
  auto stage_store = [&](double* buf) {
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int i = tid - 64 + NL * m;
      if (i < BUF) buf[i] = pend[m];
    }
  };
  double reg[NR];
  double yout = 0.0, idv = 0.0, nb = 0.0, idv_nx = 0.0, nb_nx = 0.0;
  // 1/L_jj of a chunk's 64 steps and the 64 elements that enter the ring at
  // its end, loaded one chunk ahead
  auto load_chunk = [&](int64_t tc0, double& iv, double& nv) {
    const int64_t tc = tc0 + lane, tn = tc0 + RS + lane;
    iv = tc < p ? invd[elem(tc)] : 0.0;
    nv = tn < p ? b[elem(tn)] : 0.0;
  };
  if (wave == 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int64_t t = r * 64 + lane;
      reg[r] = t < p ? b[elem(t)] : 0.0;
    }
    load_chunk(0, idv_nx, nb_nx);
  } else {
    stage_load(0);
    stage_store(stage);
    if (nsub > 1) stage_load(1);
  }
  __syncthreads();
  for (int64_t s = 0; s < nsub; ++s) {
    double* cur = stage + (s & 1) * BUF;
    if (wave != 0) {
      if (s + 1 < nsub) stage_store(stage + ((s + 1) & 1) * BUF);
      if (s + 2 < nsub) stage_load(s + 2);
    } else {
      const int64_t t0 = s * SC;
      const int r0 = (int)((t0 / 64) % NR);
      const int lc0 = (int)(t0 % 64);
      const int64_t tc0 = t0 - lc0;
      if (lc0 == 0) {
        idv = idv_nx;
        nb = nb_nx;
        load_chunk(tc0 + 64, idv_nx, nb_nx);
      }
      band_steps_sw<NR, SC, 0>(r0, reg, yout, idv, cur, t0, lc0, p, lane);
      if (lc0 + SC == 64 || t0 + SC >= p) {
        const int64_t tc = tc0 + lane;
        if (tc < p) out[elem(tc)] = yout;
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r == r0) reg[r] = nb;
      }
    }
    __syncthreads();
  }
}

template <int NR>
__device__ __forceinline__ void band_solve_nr(const double* r, double* tmp, double* z, const double* Lb, const double* LbT,
                                     const double* invd, int64_t p, int W, double* lds) {
  constexpr int SC = (2 * 32 * NR * 64 <= kBandLds) ? 32 : (2 * 16 * NR * 64 <= kBandLds) ? 16
                     : (2 * 8 * NR * 64 <= kBandLds) ? 8 : 4;
  band_sweep_t<NR, SC>(r, tmp, Lb, invd, p, W, true, lds);
  band_sweep_t<NR, SC>(tmp, z, LbT, invd, p, W, false, lds);
}

// z = M^-1 r = L^-T L^-1 r through tmp (p doubles).  Whole workgroup of 256
// threads; W <= kBandMaxW (checked on the host).  Ends with a barrier.
__device__ __forceinline__ void band_solve(const double* r, double* tmp, double* z, const double* Lb, const double* LbT,
                                  const double* invd, int64_t p, int W, double* lds) {
  switch (band_nr(W)) {
    case 2: band_solve_nr<2>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 3: band_solve_nr<3>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 4: band_solve_nr<4>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 5: band_solve_nr<5>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 6: band_solve_nr<6>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 8: band_solve_nr<8>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 12: band_solve_nr<12>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    default: band_solve_nr<17>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
  }
}

}  // namespace flr
