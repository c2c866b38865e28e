// Exact preconditioner solve for graphs whose index bandwidth bw = max |j - k|
// over E is at least 2 (the 2-D lattice, all-pairs fusion): M = lambda1 A +
// lambda2 B is banded with bandwidth bw, and Algorithm 2 applies M^-1 through
// its banded Cholesky factor M = L L^T (section 3.1, where the PCG
// preconditioner is solved with a banded Cholesky factorization; the lattice
// of the paper's 2-D experiments has bw = q).  M changes once per MM iteration, so
// the factor is computed once per MM iteration and every PCG step applies it
// with two triangular sweeps.
//
// Layouts (W = bw + 1 entries per row / column), stored as the sweeps use
// them, i.e. divided by the diagonal of the step that applies them:
//   Lb  column-major band, Lb[j*W + k]  = L_{j+k, j} / L_jj  (column j; k >= 1)
//   LbT row-major band,    LbT[i*W + k] = L_{i, i-k} / L_ii  (row i; k >= 1)
//   Lb[j*W] = LbT[j*W] = L_jj, invd[j] = 1 / L_jj
// Both sweeps walk one dependent chain of length p, so one wave runs each:
// the not-yet-final right-hand sides of the next bw elements sit in a ring of
// 64*NR registers across the wave's lanes (element t in slot t mod 64*NR),
// each step reads the current element's right-hand side b_j from its lane and
// subtracts b_j times (multiplier / L_jj) from the ring with one fma per
// register; the solution b_j / L_jj of a chunk of 64 elements is formed once
// the chunk is done.  The other three waves of the workgroup stage the
// coming steps' multipliers into LDS in the ring's slot order, straight from
// Lb / LbT: each staging thread owns fixed ring distances k and walks the
// steps of a sub-chunk (one row of W multipliers per step, read coalesced
// across threads), with its loads issued a sub-chunk ahead.
#pragma once
#include <type_traits>

#include "flr_device.h"

namespace flr {

constexpr int kBandLds = 13312;   // doubles of LDS the band routines use (104 KiB)
constexpr int kBandMaxW = 1025;   // widest band the sweeps handle (NR = 17 ring registers)
constexpr int kPanelMaxW = 107;   // widest band the register-panel factorization takes (its LDS window)

// Ring registers per lane: 64*NR slots must hold the bw elements ahead of the
// current one plus the 64 of the chunk being consumed.
__host__ __device__ inline int band_nr(int W) {
  const int need = (W + 63 + 63) / 64;
  const int opts[] = {2, 3, 5, 8, 17};  // a few ring sizes keep the code (and compile time) small
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

__device__ inline double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Blocked right-looking Cholesky of the assembled band for bands too wide for
// the register-panel factorization's LDS window (below).  Panels of nb columns (nb = 16, fewer for very wide
// bands so that a panel fits the band LDS) are loaded into LDS and factored
// there, one pivot per step; the panel's columns of L are written out (Lb
// scaled by 1/L_jj, LbT unscaled, rescaled by the caller), and the triangle
// of the band that the panel reaches - columns j0 + nb .. j0 + nb + W - 2 -
// is updated with one rank-nb pass in global memory (wave w takes every
// fourth column, lanes its rows, coalesced), instead of one pass per pivot.
// 256 threads; returns false in every thread on a pivot that is not
// positive and finite.
__device__ inline bool band_factor_blocked(double* __restrict__ Lb, double* __restrict__ LbT,
                                           double* __restrict__ invd, int64_t p, int W, double* __restrict__ P) {
  __shared__ double sh_inv[16];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int nb = kBandLds / W < 16 ? kBandLds / W : 16;
  for (int64_t j0 = 0; j0 < p; j0 += nb) {
    const int w = (int)((p - j0) < (int64_t)nb ? (p - j0) : (int64_t)nb);
    const double* src = Lb + j0 * W;  // the panel's columns are contiguous
    for (int e = tid; e < w * W; e += nt) P[e] = src[e];
    __syncthreads();
    for (int jj = 0; jj < w; ++jj) {
      const double piv = P[jj * W];
      if (!(piv > 0.0) || !isfinite(piv)) return false;  // the same value in every thread
      const double ljj = sqrt(piv), inv = 1.0 / ljj;
      __syncthreads();  // every thread has the pivot before it is overwritten
      for (int k = tid; k < W; k += nt) P[jj * W + k] = k ? P[jj * W + k] * inv : ljj;
      if (tid == 0) sh_inv[jj] = inv;
      __syncthreads();
      // later panel columns: M(j' + k, j') -= L(j' + k, j) L(j', j), j' = j + d
      const int rem = w - 1 - jj;
      for (int e = tid; e < rem * W; e += nt) {
        const int d = 1 + e / W, k = e - (d - 1) * W;
        if (k < W - d) P[(jj + d) * W + k] = fma(-P[jj * W + k + d], P[jj * W + d], P[(jj + d) * W + k]);
      }
      __syncthreads();
    }
    for (int e = tid; e < w * W; e += nt) {
      const int jj = e / W, k = e - jj * W;
      const int64_t j = j0 + jj;
      const double v = P[e];
      if (k == 0) {
        Lb[j * W] = v;
        LbT[j * W] = v;
        invd[j] = sh_inv[jj];
      } else if (j + k < p) {
        Lb[j * W + k] = v * sh_inv[jj];
        LbT[(j + k) * W + k] = v;
      }
    }
    // trailing triangle: column c = j0 + dcol, row c + di gets the sum over
    // the panel columns whose band reaches both c and c + di
    const int64_t cend = (j0 + w + W - 2) < p - 1 ? (j0 + w + W - 2) : p - 1;
    for (int64_t c = j0 + w + wave; c <= cend; c += 4) {
      const int dcol = (int)(c - j0);
      int dimax = W - 1 < w + W - 2 - dcol ? W - 1 : w + W - 2 - dcol;
      if ((int64_t)dimax > p - 1 - c) dimax = (int)(p - 1 - c);
      for (int di = lane; di <= dimax; di += 64) {
        const int jlo = dcol + di - (W - 1) > 0 ? dcol + di - (W - 1) : 0;
        double sum = 0.0;
        for (int jj = jlo; jj < w; ++jj) sum = fma(P[jj * W + dcol + di - jj], P[jj * W + dcol - jj], sum);
        Lb[c * W + di] -= sum;
      }
    }
    __syncthreads();
  }
  return true;
}

// Right-looking Cholesky of the assembled band in panels of NB columns, for
// bands narrow enough that the active window fits in LDS.  The window -
// columns j0 .. j0 + NB + W - 2 while the panel that starts at column j0 is
// factored - is a ring of R = NB + W - 1 columns of W entries (column c in
// slot c mod R).  Per panel:
//  * wave 0 takes the panel's columns into registers (lane l holds rows
//    j0 + l and j0 + 64 + l) and factors them there: each pivot and the
//    multipliers of the later panel columns come from the lanes that hold
//    them (readlane), so the panel needs no barrier.  It leaves the panel's
//    rows of L in LDS (Lp) and nothing else, to keep this serial part short;
//  * after one barrier waves 1-3 write the panel's columns of L to Lb, LbT
//    and invd while wave 0 moves the next NB columns of the assembled band,
//    loaded one panel earlier, into the panel's freed slots and issues the
//    loads for the panel after (its memory counter then holds only those
//    loads, so waiting for them never waits for the scattered stores); then
//    the workgroup subtracts L21 L21^T (L21: the rows of Lp below the panel)
//    from the trailing triangle (columns j0 + NB .. j0 + NB + W - 2):
//    thread (tx, ty) keeps its entries (row offset tx + 16 c, column offset
//    ty + 16 a) in registers over the panel's NB pivots.
// Every entry receives the same fused multiply-adds in the same pivot order as
// in a one-pivot-per-step right-looking factorization (an update from a pivot
// whose band does not reach the entry multiplies by an exact zero), so the
// factor is the same bit for bit; the trailing triangle makes one LDS round
// trip per NB pivots instead of one per pivot, with two barriers per panel.
// 256 threads; false in every thread on a pivot that is not positive and
// finite.
template <int NB>
__device__ inline bool band_factor_panels(double* __restrict__ Lb, double* __restrict__ LbT,
                                          double* __restrict__ invd, int64_t p, int W, double* __restrict__ lds) {
  constexpr int LP = NB + 1;                   // Lp row stride, odd: 16 consecutive rows in distinct banks
  constexpr int NXT = (NB * kPanelMaxW + 63) / 64;  // entering band entries per lane of wave 0
  constexpr int kTB = 7;                       // 16-wide blocks of the trailing triangle (W - 1 <= 112)
  __shared__ int sh_bad;
  __shared__ double sh_inv[NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx = tid & 15, ty = tid >> 4;
  const int R = NB + W - 1;
  double* Lp = lds + R * W;  // rows j0 .. j0 + R - 1 of the panel's columns of L, LP apart
  const int64_t pw = p * (int64_t)W;
  {
    const int64_t n0 = (p < R ? p : (int64_t)R) * W;
    for (int64_t i = tid; i < n0; i += 256) lds[i] = Lb[i];
  }
  double nxt[NXT];
#pragma unroll
  for (int q = 0; q < NXT; ++q) {
    const int e = lane + 64 * q;
    const int64_t g = (int64_t)R * W + e;
    nxt[q] = (wave == 0 && e < NB * W && g < pw) ? Lb[g] : 0.0;
  }
  if (tid == 0) sh_bad = 0;
  int s0 = 0;  // ring slot of column j0
  for (int64_t j0 = 0; j0 < p; j0 += NB) {
    const int w = (p - j0) < (int64_t)NB ? (int)(p - j0) : NB;
    lds_barrier();
    if (wave == 0) {
      // the panel in registers.  Full panels (all but possibly the last) are
      // compiled without the per-column bounds; LDS reads are unconditional
      // at indices clamped into the column and selected afterwards (a
      // guarded read compiles to a branch), and ring positions wrap once at
      // R W: the slot of column j0 + jj starts at (s0 + jj) W mod R W.
      auto factor_panel = [&](auto full) {
        constexpr bool F = decltype(full)::value;
        const int ww = F ? NB : w;
        const int RW = R * W, base = s0 * W;
        double x0[NB], x1[NB];
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
          const int k0 = lane - jj, k1 = lane + 64 - jj;  // entries of column j0 + jj in the lane's rows
          int a0 = base + jj * W + (k0 < 0 ? 0 : (k0 < W ? k0 : W - 1));
          int a1 = base + jj * W + (k1 < W ? k1 : W - 1);
          a0 = a0 >= RW ? a0 - RW : a0;
          a1 = a1 >= RW ? a1 - RW : a1;
          const double v0 = lds[a0], v1 = lds[a1];
          x0[jj] = ((F || jj < ww) && k0 >= 0 && k0 < W) ? v0 : 0.0;
          x1[jj] = ((F || jj < ww) && k1 < W) ? v1 : 0.0;
        }
        bool bad = false;
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
          if (!F && jj >= ww) break;
          const double piv = readlane_f64(x0[jj], jj);
          if (!(piv > 0.0) || !isfinite(piv)) {
            bad = true;
            break;
          }
          const double ljj = sqrt(piv), rj = 1.0 / ljj;
          if (lane == 0) sh_inv[jj] = rj;
          const double l0 = lane > jj ? x0[jj] * rj : (lane == jj ? ljj : 0.0);
          const double l1 = x1[jj] * rj;
          x0[jj] = l0;
          x1[jj] = l1;
#pragma unroll
          for (int c = jj + 1; c < NB; ++c) {
            if (F || c < ww) {
              const double lc = readlane_f64(l0, c);
              x0[c] = fma(-l0, lc, x0[c]);
              x1[c] = fma(-l1, lc, x1[c]);
            }
          }
        }
        if (bad) {
          if (lane == 0) sh_bad = 1;
        } else {
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) {
            if (lane < R) Lp[lane * LP + jj] = x0[jj];
            if (lane + 64 < R) Lp[(lane + 64) * LP + jj] = x1[jj];
          }
        }
      };
      if (w == NB)
        factor_panel(std::integral_constant<bool, true>());
      else
        factor_panel(std::integral_constant<bool, false>());
    }
    lds_barrier();
    if (sh_bad) return false;
    if (wave == 0) {
      // the panel's slots take the columns entering the window (entry e of
      // them at (s0 W + e) mod R W), then the loads for the next panel go out
      const int RW = R * W;
      const int64_t left = pw - (j0 + R) * W, left2 = left - (int64_t)NB * W;
      const int lim = left < (int64_t)NB * W ? (int)(left > 0 ? left : 0) : NB * W;
      const int lim2 = left2 < (int64_t)NB * W ? (int)(left2 > 0 ? left2 : 0) : NB * W;
#pragma unroll
      for (int q = 0; q < NXT; ++q) {
        const int e = lane + 64 * q, a = s0 * W + e;
        if (e < lim) lds[a >= RW ? a - RW : a] = nxt[q];
      }
      const double* src = Lb + (j0 + NB + R) * W;
#pragma unroll
      for (int q = 0; q < NXT; ++q) {
        const int e = lane + 64 * q;
        nxt[q] = e < lim2 ? src[e] : 0.0;
      }
    } else {
      // the panel's columns of L: Lb scaled by 1/L_jj below the diagonal,
      // LbT unscaled (the caller scales its rows), invd
      const int k = tid - 64;
      for (int jj = 0; jj < w; ++jj) {
        const int64_t j = j0 + jj;
        if (k < W && j + k < p) {
          const double v = Lp[(jj + k) * LP + jj];
          Lb[j * W + k] = k ? v * sh_inv[jj] : v;
          LbT[(j + k) * W + k] = v;
        }
      }
      if (k < w) invd[j0 + k] = sh_inv[k];
    }
    if (j0 + NB < p) {
      const int64_t rest = p - 1 - (j0 + NB);
      const int cmax = rest < (int64_t)(W - 2) ? (int)rest : W - 2;
      double t[kTB][kTB];
#pragma unroll
      for (int a = 0; a < kTB; ++a) {
        const int u = ty + 16 * a, uc = u < W - 2 ? u : W - 2;
        const int slot = s0 + NB + uc < R ? s0 + NB + uc : s0 + NB + uc - R;
#pragma unroll
        for (int c = a; c < kTB; ++c) {
          const int v = tx + 16 * c;
          t[a][c] = (u <= v && v <= cmax) ? lds[slot * W + (v - u)] : 0.0;
        }
      }
#pragma unroll 2
      for (int jj = 0; jj < NB; ++jj) {
        double lu[kTB], lv[kTB];
#pragma unroll
        for (int a = 0; a < kTB; ++a) {
          const int u = ty + 16 * a, v = tx + 16 * a;
          lu[a] = Lp[(NB + (u < W - 2 ? u : W - 2)) * LP + jj];
          lv[a] = Lp[(NB + (v < W - 2 ? v : W - 2)) * LP + jj];
        }
        // every tile entry is updated (entries outside the triangle hold
        // values that are never stored), so no per-entry selects
#pragma unroll
        for (int a = 0; a < kTB; ++a)
#pragma unroll
          for (int c = a; c < kTB; ++c) t[a][c] = fma(-lu[a], lv[c], t[a][c]);
      }
#pragma unroll
      for (int a = 0; a < kTB; ++a) {
        const int u = ty + 16 * a, uc = u < W - 2 ? u : W - 2;
        const int slot = s0 + NB + uc < R ? s0 + NB + uc : s0 + NB + uc - R;
#pragma unroll
        for (int c = a; c < kTB; ++c) {
          const int v = tx + 16 * c;
          if (u <= v && v <= cmax) lds[slot * W + (v - u)] = t[a][c];
        }
      }
    }
    s0 = s0 + NB < R ? s0 + NB : s0 + NB - R;
  }
  return true;
}

// Cholesky factor of the assembled band, in place: the register-panel
// factorization above when its window fits the band LDS (W <= 107), the
// blocked one with the trailing update in global memory otherwise.  256
// threads; returns false in every thread when a pivot is not positive and
// finite.
__device__ inline bool band_factor(double* __restrict__ Lb, double* __restrict__ LbT, double* __restrict__ invd,
                                   int64_t p, int W, double* __restrict__ lds) {
  constexpr int NB = 8;
  const int tid = threadIdx.x, nt = blockDim.x;
  const bool panels = W >= 2 && W <= kPanelMaxW && (int64_t)(NB + W - 1) * (W + NB + 1) <= kBandLds;
  const bool ok = panels ? band_factor_panels<NB>(Lb, LbT, invd, p, W, lds)
                         : band_factor_blocked(Lb, LbT, invd, p, W, lds);
  // the rescale below reads invd (stored by lane 0) and LbT entries stored
  // by other threads: a full barrier orders those global stores (the panel
  // loop's barriers order LDS only)
  __syncthreads();
  if (ok) {  // rows of L scaled by their own 1/L_ii (the backward sweep's multipliers): a wave per row
    for (int64_t i = tid >> 6; i < p; i += nt >> 6) {
      const double s = invd[i];
      for (int k = 1 + (tid & 63); k < W; k += 64) LbT[i * W + k] *= s;
    }
    __syncthreads();
  }
  return ok;
}

// SC steps of the sweep by wave 0: elements t0 .. t0 + SC - 1, held in
// lanes lc0 .. lc0 + SC - 1 of ring register R0.  The staged multipliers
// already include 1/L_jj.  The dependent chain is one fma per step, on values
// every lane holds: bu = b_j (final), and the next element's final value
// b_{j+1} = pre - m b_j, where pre is b_{j+1} after the steps before j (read
// from its lane one step early) and m its multiplier at step j, which the
// lane of element j+1 already holds among the step's ring multipliers (a
// readlane, no LDS read on the chain).  The ring update - one fma per
// register - and those reads stay off that chain; the ring multipliers of a
// step are loaded DP steps ahead.  Elements j + 1, j + 2 live in register R0
// or, in the last two steps of a chunk, in the next ring register R1.
template <int NR, int SC, int R0>
__device__ __forceinline__ void band_steps(double (&reg)[NR], double& bu, double& pre, const double* __restrict__ buf,
                                           int lc0, int lane) {
  constexpr int R1 = (R0 + 1) % NR;
  constexpr int DP = SC < (NR <= 5 ? 4 : 2) ? SC : (NR <= 5 ? 4 : 2);  // steps of multipliers in flight
  double mq[DP][NR];
#pragma unroll
  for (int d = 0; d < DP; ++d)
#pragma unroll
    for (int r = 0; r < NR; ++r) mq[d][r] = buf[(d * NR + r) * 64 + lane];
#pragma unroll
  for (int l = 0; l < SC; ++l) {
    const int lc = lc0 + l;
    const int ln1 = (lc + 1) & 63, ln2 = (lc + 2) & 63;
    double(&mc)[NR] = mq[l % DP];
    const double m1 = readlane_f64(lc + 1 < 64 ? mc[R0] : mc[R1], ln1);
#pragma unroll
    for (int r = 0; r < NR; ++r) reg[r] = fma(-mc[r], bu, reg[r]);
    const double pre2 = readlane_f64(lc + 2 < 64 ? reg[R0] : reg[R1], ln2);
    bu = fma(-m1, bu, pre);
    pre = pre2;
    if (l + DP < SC) {
#pragma unroll
      for (int r = 0; r < NR; ++r) mc[r] = buf[((l + DP) * NR + r) * 64 + lane];
    }
  }
}

template <int NR, int SC, int R0>
__device__ __forceinline__ void band_steps_sw(int r0, double (&reg)[NR], double& bu, double& pre, const double* buf,
                                              int lc0, int lane) {
  if constexpr (R0 < NR) {
    if (r0 == R0)
      band_steps<NR, SC, R0>(reg, bu, pre, buf, lc0, lane);
    else
      band_steps_sw<NR, SC, R0 + 1>(r0, reg, bu, pre, buf, lc0, lane);
  }
}

// One triangular sweep: virtual step t handles element e(t) = t (forward,
// L y = b with the columns of L, Mul = Lb) or p - 1 - t (backward, L^T z = b
// with the rows of L, Mul = LbT); Mul[e(t)*W + k] (1 <= k < W) multiplies the
// element k steps ahead, which sits in ring slot (t + k) mod 64 NR.  Whole
// workgroup of 256 threads; stage: kBandLds doubles of LDS.  Ends with a
// barrier.
template <int NR, int SC>
__device__ __forceinline__ void band_sweep_t(const double* __restrict__ b, double* __restrict__ out, const double* __restrict__ Mul,
                             const double* __restrict__ invd, int64_t p, int W, bool fwd, double* __restrict__ stage) {
  constexpr int RS = 64 * NR;
  constexpr int BUF = SC * NR * 64;
  static_assert(2 * BUF <= kBandLds, "stage buffers exceed the LDS budget");
  static_assert(64 % SC == 0, "sub-chunks must tile a chunk");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t nsub = (p + SC - 1) / SC;
  auto elem = [&](int64_t t) { return fwd ? t : p - 1 - t; };
  // Waves 1..3 stage sub-chunk s: staging thread u owns the ring distances
  // k = u + NL c (c < KC) and, for each of the SC steps, loads the multiplier
  // at distance k (zero outside 1 <= k < W or past the end) and stores it into
  // the LDS row of that step at slot (t + k) mod RS.  Every slot of a row is
  // written, so stale values never survive.  All PER loads of a thread are
  // issued before any is written to LDS, one sub-chunk early (into pend), so
  // their latency hides behind wave 0's steps.
  constexpr int NL = kWG - 64;
  constexpr int KC = (RS + NL - 1) / NL;
  constexpr int PER = KC * SC;
  const int u = tid - 64;
  const int64_t rstep = fwd ? (int64_t)W : -(int64_t)W;
  double pend[PER];
  auto stage_load = [&](int64_t s) {
    const int64_t t0 = s * SC;
    const int64_t rem = p - t0;
    const int lim = rem < SC ? (int)rem : SC;
    const double* row = Mul + elem(t0) * (int64_t)W;
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const int k = u + NL * c;
      const bool kin = k >= 1 && k < W;
#pragma unroll
      for (int l = 0; l < SC; ++l) pend[c * SC + l] = (kin && l < lim) ? row[l * rstep + k] : 0.0;
    }
  };
  auto stage_store = [&](double* buf, int64_t s) {
    const int rr0 = (int)((s * SC) % RS);
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const int k = u + NL * c;
      if (k < RS) {
        int slot = rr0 + k;
        if (slot >= RS) slot -= RS;
#pragma unroll
        for (int l = 0; l < SC; ++l) {
          buf[l * RS + slot] = pend[c * SC + l];
          slot = slot + 1 == RS ? 0 : slot + 1;
        }
      }
    }
  };
  double reg[NR];
  double idv = 0.0, nb = 0.0, idv_nx = 0.0, nb_nx = 0.0;
  // 1/L_jj of a chunk's 64 steps and the 64 elements that enter the ring at
  // its end, loaded one chunk ahead
  auto load_chunk = [&](int64_t tc0, double& iv, double& nv) {
    const int64_t tc = tc0 + lane, tn = tc0 + RS + lane;
    iv = tc < p ? invd[elem(tc)] : 0.0;
    nv = tn < p ? b[elem(tn)] : 0.0;
  };
  double bu = 0.0, pre = 0.0;  // b of the current element (final) and of the next (before this step)
  if (wave == 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int64_t t = r * 64 + lane;
      reg[r] = t < p ? b[elem(t)] : 0.0;
    }
    bu = readlane_f64(reg[0], 0);
    pre = readlane_f64(reg[0], 1);
    load_chunk(0, idv_nx, nb_nx);
  } else {
    stage_load(0);
    stage_store(stage, 0);
    if (nsub > 1) stage_load(1);
  }
  __syncthreads();
  for (int64_t s = 0; s < nsub; ++s) {
    double* cur = stage + (s & 1) * BUF;
    if (wave != 0) {
      if (s + 1 < nsub) stage_store(stage + ((s + 1) & 1) * BUF, s + 1);
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
      band_steps_sw<NR, SC, 0>(r0, reg, bu, pre, cur, lc0, lane);
      if (lc0 + SC == 64 || t0 + SC >= p) {
        // the chunk's slots hold their final right-hand sides: y = b / L_jj
        const int64_t tc = tc0 + lane;
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r == r0) {
            if (tc < p) out[elem(tc)] = reg[r] * idv;
            reg[r] = nb;
          }
      }
    }
    lds_barrier();  // the staging loads of the next sub-chunk stay in flight
  }
  __syncthreads();
}

template <int NR>
__device__ __forceinline__ void band_solve_nr(const double* r, double* tmp, double* z, const double* Lb,
                                              const double* LbT, const double* invd, int64_t p, int W, double* lds) {
  constexpr int SC = (2 * 32 * NR * 64 <= kBandLds) ? 32 : (2 * 16 * NR * 64 <= kBandLds) ? 16
                     : (2 * 8 * NR * 64 <= kBandLds) ? 8 : 4;
  band_sweep_t<NR, SC>(r, tmp, Lb, invd, p, W, true, lds);
  band_sweep_t<NR, SC>(tmp, z, LbT, invd, p, W, false, lds);
}

// z = M^-1 r = L^-T L^-1 r through tmp (p doubles).  Whole workgroup of 256
// threads; W <= kBandMaxW (checked on the host).  Ends with a barrier.
__device__ __forceinline__ void band_solve(const double* r, double* tmp, double* z, const double* Lb,
                                           const double* LbT, const double* invd, int64_t p, int W, double* lds) {
  switch (band_nr(W)) {
    case 2: band_solve_nr<2>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 3: band_solve_nr<3>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 5: band_solve_nr<5>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    case 8: band_solve_nr<8>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
    default: band_solve_nr<17>(r, tmp, z, Lb, LbT, invd, p, W, lds); break;
  }
}

}  // namespace flr
