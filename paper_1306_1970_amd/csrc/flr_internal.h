// Internal layout shared by the HIP kernels and the host engine.
//
// One solve is a device-resident state machine.  Every launch is one of three
// kernels that run in a fixed rotation A, B, C (a hipGraph holds S rounds);
// when M is banded with bandwidth >= 2 a fourth, K, applies M^-1 through its
// banded Cholesky factor after C:
//   A  row-panel GEMV   u = X v            (v = new CG direction, or the MM iterate)
//   B  column-panel GEMV q = X^T u (+ M v)  (plus, at an MM boundary: objective
//                                            partials, reweighting, factorization products)
//   C  per-block work   CG updates and the block-partitioned tridiagonal solve,
//                       or, at an MM boundary: objective test, factorization, new residual
// Each kernel reads the state written by the previous one and writes the next
// (double-buffered by launch parity), so the host only launches and polls.
// The last C workgroup to finish combines the per-block results (carries of
// the partitioned tridiagonal solve, r^T z, ||r||, the inner stopping test and
// gamma) once, so A only reads them.
#pragma once
#include <stdint.h>

namespace flr {

constexpr int kWG = 256;          // threads per workgroup (4 wave64)
constexpr int kBlk = 256;         // elements per solver block (one per thread)
constexpr int kMaxC1 = 2048;      // max columns of an A tile
constexpr int kMaxR2 = 1024;      // max rows of a B tile
constexpr int kMaxBlocks = 1024;  // max solver blocks -> p_pad <= 262144

// PH_BANDMM: an MM step goes on and M is banded (bandwidth >= 2): the fourth
// launch of the rotation factors M and solves with the new residual.
// PH_RES (mixed precision): the inner PCG with FP32 products has met its
// tolerance on its recursive residual; the next rotation recomputes the true
// residual c - Q x in FP64 at the same weights and either ends the MM step
// or restarts the PCG from it (iterative refinement).  PH_BANDRES: the same
// refreshed residual solved through the existing banded factor.
enum Phase : int32_t { PH_CG = 0, PH_END = 1, PH_DONE = 2, PH_BANDMM = 3, PH_RES = 4, PH_BANDRES = 5 };

// What a combine of the block scalars follows: a PCG step, the first residual
// of an MM step, or a residual refreshed in FP64 (refinement).
enum CombineMode : int32_t { CM_STEP = 0, CM_FIRST = 1, CM_REFRESH = 2 };
enum SolveStatus : int32_t { ST_OK = 0, ST_MAX_ITER = 1, ST_NUMERICAL = 2 };

// Block scalars of the partitioned tridiagonal solve (index into blk[]).
enum BlkField : int {
  BK_A = 0,    // forward gain of the block: prod(-L_j)
  BK_B = 1,    // zero-inflow forward value at the block end
  BK_SIGS = 2, // sigma at the block start
  BK_PSIS = 3, // psi at the block start
  BK_YS = 4,   // zero-inflow local solution at the block start
  BK_RY = 5,   // r . y over the block
  BK_RS = 6,   // r . sigma
  BK_RP = 7,   // r . psi
  BK_RR = 8,   // r . r
  BK_N = 9
};

struct Params {
  double lam1, lam2, eps, tol, inner_tol, cnorm;
  int32_t max_iter, max_cg, jacobi, mixed;
  int32_t band;  // W = bandwidth + 1 when M is applied through its banded Cholesky factor, else 0
  int32_t pad;
};

struct State {
  int32_t phase, status, first, first_cg;
  int32_t mm_iter, cg_iter;
  int64_t cg_total;
  double rz, f_old, f_new, rel_change, rel_res, nu, gamma;
  double rres;  // relative FP64 residual at the last MM boundary or refresh (mixed precision)
};

struct Dims {
  int64_t n, p, p_pad, ldx;
  int32_t dtype;          // 0 f64, 1 f32, 2 bf16
  int32_t c1, cb1, r1, rb1;
  int32_t c2, cb2, r2, rb2;
  int32_t nblk;
  int32_t gridB;          // max(cb2*rb2, nblk)
  int32_t flsa;           // 1: X = I (fused lasso signal approximation), no X is stored or read
  int32_t nloss;          // loss partials the block kernel sums (rb2, or cb2 when X = I)
};

struct Bufs {
  const void* X;
  const double* y;
  const int32_t* rowptr;
  const int32_t* col;
  const int32_t* prevpos;
  const double* c;
  const double* s;
  double* x;
  double* r;
  double* yv;
  double* pbuf;     // 2 * p_pad
  double* a;
  double* w;        // 2m CSR weights
  double* d;
  double* e;
  double* L;
  double* invD;
  double* sig;
  double* psi;
  double* upart;    // cb1 * n
  double* qpart;    // rb2 * p_pad
  double* pqpart;   // gridB
  double* losspart; // rb2
  double* penpart;  // nblk
  double* blk;      // BK_N * nblk
  double* carry;    // 2 * nblk: forward carries G, then backward carries Z
  double* Lb;       // banded Cholesky factor of M by columns, p x W (banded mode only)
  double* LbT;      // the same by rows
  double* invdb;    // 1 / L_jj
  double* btmp;     // intermediate of the two triangular sweeps
  unsigned* counter;// blocks of the current C launch that have finished
  State* st;        // 2
  const Params* prm;
};

// One problem of a grouped launch (the ragged batch): its sizes and buffers,
// the first workgroup of its share of the grouped A, B and C launches, and
// whether its M is applied through the banded factor (one workgroup of the
// grouped band launch; the other problems' workgroup only passes the state on).
struct GroupEntry {
  Dims D;
  Bufs B;
  int32_t wg_a, wg_b, wg_c;
  int32_t band;
};

}  // namespace flr
