/*
 * flr.h - C ABI of the MI355X (gfx950) majorization-minimization solver for
 * fused lasso regression (FLR).
 *
 * Problem (introduction, FLR objective): minimize over b in R^p
 *   f(b) = 1/2 ||y - X b||^2 + lambda1 sum_j |b_j| + lambda2 sum_{(j,k) in E} |b_j - b_k|
 * with X an n x p design matrix, y in R^n, lambda1, lambda2 >= 0 and E a set
 * of unordered index pairs (chain for the standard FLR, q x q lattice for the
 * two-dimensional FLR, all pairs for the clustered / pairwise fused lasso).
 *
 * Method (section 3.1, perturbed objective, majorizer and linear-system
 * equations; Algorithm 2): every |b_j| and |b_j - b_k| is replaced by
 * |t| - eps log(1 + |t|/eps) and majorized at the current iterate by a
 * quadratic; its minimizer solves
 *   (X^T X + lambda1 A + lambda2 B) b = X^T y,
 *   A = diag(1/(|b_j| + eps)),  B = Laplacian of E with w_jk = 1/(|b_j - b_k| + eps),
 * by conjugate gradients preconditioned with M = lambda1 A + lambda2 B,
 * warm-started at the current iterate (Algorithm 2).  Iteration stops when the
 * relative change of f falls to tol.  The whole loop runs on the GPU; the host
 * sees only launch and completion.
 *
 * Conventions
 *  - Every call returns flr_status; no C++ exception crosses this boundary.
 *  - Pointers named *_host must be host memory; pointers documented as
 *    "host or device" are classified with hipPointerGetAttributes.
 *  - The library copies what it needs at creation: the caller may free its
 *    buffers as soon as flr_create returns.  Handles are owned by the
 *    library until the matching *_destroy; output buffers are caller-owned.
 *  - Invalid arguments return FLR_ERR_INVALID_ARG and leave outputs untouched.
 *  - One thread at a time per problem handle; distinct handles may be used
 *    concurrently (each has its own device buffers, state and stream).
 *  - flr_last_error() returns a thread-local message for the last failure.
 */
#ifndef FLR_H
#define FLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct flr_ctx_s* flr_ctx;         /* one GPU: device id and default stream */
typedef struct flr_problem_s* flr_problem; /* resident X, y, CSR(E), X^T y, ||X_j||^2, warm start */
typedef struct flr_server_s* flr_server;   /* continuous-batching serving loop */

typedef enum {
  FLR_OK = 0,
  FLR_ERR_INVALID_ARG = 1,
  FLR_ERR_OUT_OF_MEMORY = 2,
  FLR_ERR_DEVICE = 3,
  FLR_ERR_NUMERICAL = 4, /* CG breakdown (p^T Q p <= 0) or a non-finite value inside the loop */
  FLR_ERR_MAX_ITER = 5,  /* iteration cap reached; outputs hold the last iterate */
  FLR_ERR_BUSY = 6,      /* handle in use by another thread, or no slot/memory (serving) */
  FLR_ERR_NOT_READY = 7  /* serving: the ticket has not completed yet */
} flr_status;

typedef enum { FLR_F64 = 0, FLR_F32 = 1, FLR_BF16 = 2 } flr_dtype;

/* Arithmetic of the inner products with X (the p-scale terms, dot products,
 * objective and stopping tests are always FP64).
 *   FP64        X widened exactly from its stored type, FP64 accumulation.
 *   MIXED_FP32  the PCG steps' products with X in FP32 (X read in its stored
 *               type, f32 or bf16 widened to f32), with the FP64 residual
 *               c - Q beta refreshed and the inner solve repeated until the
 *               true FP64 residual meets the inner tolerance.
 * There is no separate bf16-arithmetic mode: a bf16-stored X already halves
 * the bytes each pass streams, and the products are bound by those bytes,
 * so bf16 arithmetic would only lose accuracy. */
typedef enum { FLR_PREC_FP64 = 0, FLR_PREC_MIXED_FP32 = 1 } flr_precision;

/* Preconditioner of the PCG inner solve (Algorithm 2 uses M = lambda1 A +
 * lambda2 B itself).
 *   BAND    M exactly, through its banded Cholesky factor (bandwidth
 *           bw = max |j - k| over E; section 3.1): for bw >= 2, i.e. the 2-D
 *           lattice (bw = q) and all-pairs fusion; one factorization per MM
 *           iteration, two sequential triangular sweeps per PCG step.
 *           Needs lambda1 > 0 and bw + 1 <= 1025.
 *   TRIDIAG the tridiagonal part of M (edges (j-1, j) keep their coupling,
 *           every other edge adds only to the diagonal): exactly M for the
 *           chain; for other graphs a cheap but much weaker approximation.
 *   JACOBI  diag(Q), for lambda1 = 0, where M is singular.
 *   AUTO    BAND when bw >= 2 and the band fits, TRIDIAG otherwise;
 *           JACOBI when lambda1 = 0. */
typedef enum {
  FLR_PRECOND_AUTO = 0,
  FLR_PRECOND_TRIDIAG = 1,
  FLR_PRECOND_JACOBI = 2,
  FLR_PRECOND_BAND = 3
} flr_precond;

/* How each MM iteration solves its linear system (section 3.1).
 *   PCG       Algorithm 2: preconditioned conjugate gradients with M = lambda1 A
 *             + lambda2 B (the default; every entry point).
 *   CHOLESKY  Algorithm 1: the whole system Q = X^T X + lambda1 A + lambda2 B is
 *             formed (X^T X once per handle) and solved through its Cholesky
 *             factor; exact inner solves, cg_iters = 0.  The paper's route for a
 *             general edge set.  Needs p <= 8192 (two dense p x p FP64 matrices,
 *             allocated on first use and charged to the footprint); flr_solve,
 *             flr_solve_ex, flr_solve_path and the server only (the grid and
 *             the ragged batch reject it). */
typedef enum { FLR_METHOD_PCG = 0, FLR_METHOD_CHOLESKY = 1 } flr_method;

typedef struct {
  double eps;              /* perturbation; 0 -> 1e-8 (section 5) */
  double inner_tol;        /* PCG stop ||r|| / ||X^T y||; 0 -> tol (Algorithm 2 uses one delta) */
  int32_t max_iter;        /* MM iteration cap; 0 -> 10000 (section 5) */
  int32_t max_cg;          /* PCG steps per MM iteration; 0 -> p */
  int32_t precision;       /* flr_precision */
  int32_t preconditioner;  /* flr_precond */
  const double* warm_start;/* host or device, length p; NULL -> the handle's last beta if
                              use_last is set and a solve has run, else X_j^T y / X_j^T X_j */
  int32_t use_last;        /* 1: warm-start from the handle's previous solution */
  int32_t method;          /* flr_method: how each MM iteration solves its linear system */
} flr_solve_opts;

typedef struct {
  double objective;        /* f at the returned beta, FP64 on the stored instance */
  double rel_change;       /* last |f_new - f_old| / f_old */
  double rel_residual;     /* last PCG ||r|| / ||X^T y|| */
  double seconds;          /* wall time of the solve */
  int64_t cg_iters;        /* total PCG steps */
  int32_t mm_iters;        /* MM (outer) iterations */
  int32_t status;          /* flr_status of this solve */
} flr_result;

/* Fill opts with the defaults above. */
void flr_default_opts(flr_solve_opts* opts);

/* Bind a context to GPU `device`.  hip_stream: a hipStream_t to run on, or
 * NULL for a stream owned by the context. */
flr_status flr_ctx_create(int device, void* hip_stream, flr_ctx* out);
void flr_ctx_destroy(flr_ctx ctx);

/* Create a resident problem (problem statement of the introduction).
 * X: host or device, n x p row-major with row stride ldx >= p elements, in
 *    x_dtype (FLR_BF16 = uint16 bfloat16 bit patterns).
 * y: host, length n.  edges: host, 2*m int64 values (pairs (j, k), 0-based);
 *    stored as a set of unordered pairs (duplicates dropped).
 * Errors: n, p < 1, ldx < p, non-finite X or y, an edge out of range or a
 * self-loop -> FLR_ERR_INVALID_ARG; allocation failure -> FLR_ERR_OUT_OF_MEMORY. */
flr_status flr_create(flr_ctx ctx, const void* X, flr_dtype x_dtype, int64_t n, int64_t p, int64_t ldx,
                      const double* y, const int64_t* edges, int64_t m, flr_problem* out);
void flr_destroy(flr_problem h);

/* Create a resident fused lasso signal approximation problem (X = I, n = p;
 * the FLSA of the introduction, e.g. the 2-D image denoising of section 5.2):
 * minimize 1/2 ||y - b||^2 + lambda1 sum |b_j| + lambda2 sum_E |b_j - b_k|.
 * No X is stored or read: every solve runs the same MM / PCG iteration
 * (Algorithm 2) with X^T X p = p, c = y and ||X_j||^2 = 1.  y: host, length p.
 * edges as flr_create.  Every solve entry point accepts the handle (the grid
 * uses U = V = O in place of the products); flr_profile_grid rejects it.
 * Errors as flr_create. */
flr_status flr_create_flsa(flr_ctx ctx, const double* y, int64_t p, const int64_t* edges, int64_t m,
                           flr_problem* out);
/* 1 for a handle made by flr_create_flsa, 0 otherwise, -1 for NULL. */
int32_t flr_problem_is_flsa(flr_problem h);

/* Solve at (lambda1, lambda2) to relative objective change tol (Algorithm 2).
 * beta_out_host: length p.  objective_out, iterations_out: nullable.
 * Errors: lambda < 0 or non-finite, tol <= 0 -> FLR_ERR_INVALID_ARG;
 * FLR_ERR_MAX_ITER / FLR_ERR_NUMERICAL with beta_out holding the last iterate. */
flr_status flr_solve(flr_problem h, double lambda1, double lambda2, double tol, double* beta_out_host,
                     double* objective_out, int32_t* iterations_out);

/* As flr_solve with options.  beta_out: host or device, length p; res nullable. */
flr_status flr_solve_ex(flr_problem h, double lambda1, double lambda2, double tol, const flr_solve_opts* opts,
                        double* beta_out, flr_result* res);

/* Solve B (lambda1[i], lambda2[i]) settings on one problem in one launch
 * sequence: X P and X^T U become B-column products (MFMA), every column keeps
 * its own scalars, weights, preconditioner and convergence state.
 * lambda1, lambda2: host, length B.  beta_out: host or device, B x p row-major.
 * res: nullable host array of B results.  Returns FLR_OK when every column
 * converged, else the first failing column's status.
 * With the banded preconditioner, a column that reaches an MM boundary may
 * idle for up to 15 steps so that boundaries (one band factorization each)
 * share launches; its arithmetic, and so its result, does not change.  The
 * environment variable FLR_GRID_HOLD sets that period (1: no holding). */
flr_status flr_solve_grid(flr_problem h, const double* lambda1, const double* lambda2, int32_t B, double tol,
                          const flr_solve_opts* opts, double* beta_out, flr_result* res);

/* Warm-started sequence of solves on one problem: a regularization path over
 * (lambda1[k], lambda2[k]) and/or eps-continuation over eps[k] (section 3.2:
 * minimizers of the perturbed objective approach a minimizer of f as eps
 * decreases to 0, Lemma 1; section 5 fixes eps but notes that it could be
 * decreased).  Point k is solved as flr_solve_ex with its own lambdas and
 * eps, warm-started at point k-1's solution; point 0 starts from
 * opts->warm_start, or the initialization of Algorithms 1 and 2 when NULL.
 * eps: host, count values (> 0), or NULL for opts->eps at every point.
 * lambda1, lambda2: host, count values.  beta_out: nullable, host or device,
 * count x p row-major; res: nullable, count entries.  Stops at the first
 * point that fails validation or the device (its status is returned); points
 * that end in FLR_ERR_MAX_ITER / FLR_ERR_NUMERICAL are reported in res and
 * the path goes on from their last iterate.  Returns FLR_OK when every point
 * converged, else the first failing point's status. */
flr_status flr_solve_path(flr_problem h, const double* lambda1, const double* lambda2, const double* eps, int32_t count,
                          double tol, const flr_solve_opts* opts, double* beta_out, flr_result* res);

/* Static workspace of flr_solve_grid_static: bytes of the per-GPU array and
 * the most columns one call may solve. */
#define FLR_GRID_STATIC_BYTES (64u << 20)
#define FLR_GRID_STATIC_MAX_COLS 256

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the grid
 * solve of flr_solve_grid - same kernels, same arithmetic, same results -
 * with its whole device workspace (per-column vectors, batched products and
 * their split-K partials, column states, band factors) in one static device
 * array of FLR_GRID_STATIC_BYTES instead of memory the library allocates.
 * The call makes no device or pinned-host allocation.  The array belongs to
 * the loaded library: every GPU the library runs on holds it until the
 * process ends.  All calls on one GPU share that GPU's array, which keeps the
 * last call's contents (nothing in it has to start at zero); calls that
 * overlap on one GPU - from different threads or different handles - race
 * and must be serialized by the caller.  Limits: B <= FLR_GRID_STATIC_MAX_COLS
 * and a workspace of at most FLR_GRID_STATIC_BYTES (about
 * 8 B (13 p_pad + 9 ldu + nnz) bytes, plus 16 B p W with a banded M, where
 * p_pad is p rounded up to the row-panel width and ldu is n rounded up to
 * 64); beyond either it returns FLR_ERR_INVALID_ARG with the size in
 * flr_last_error().  Arguments, outputs and other errors as flr_solve_grid;
 * the handle's own grid workspace and footprint are not touched. */
flr_status flr_solve_grid_static(flr_problem h, const double* lambda1, const double* lambda2, int32_t B, double tol,
                                 const flr_solve_opts* opts, double* beta_out, flr_result* res);

/* Ragged batch: `count` solves on distinct, idle problem handles of any
 * sizes and graphs (n_i, p_i, E_i), each with its own (lambda1[i],
 * lambda2[i]), in one call.  One host thread keeps two captured rotations of
 * every solve in flight on that problem's own stream, so the solves' kernels
 * overlap on the device, and each result is the one the solo flr_solve_ex
 * gives (same kernels, same reduction trees).  beta_out: nullable array of
 * `count` pointers (host or device, length p_i each, each nullable); res:
 * nullable, `count` entries.  Returns FLR_OK when every solve converged, else
 * the first failing status; FLR_ERR_INVALID_ARG for a repeated handle,
 * FLR_ERR_BUSY when a handle is in use. */
flr_status flr_solve_batch(const flr_problem* problems, int32_t count, const double* lambda1,
                           const double* lambda2, double tol, const flr_solve_opts* opts, double* const* beta_out,
                           flr_result* res);

/* Device footprint of a problem in bytes (what serving admission charges). */
flr_status flr_problem_footprint(flr_problem h, size_t* bytes);
int64_t flr_problem_n(flr_problem h);
int64_t flr_problem_p(flr_problem h);
int64_t flr_problem_m(flr_problem h);

/* Serving: requests are admitted while the sum of the footprints of problems
 * in flight stays within hbm_budget_bytes and a slot is free; each slot runs
 * on its own stream, so solves that arrive while others run overlap on the
 * device.  Results do not depend on what else runs (fixed reduction trees,
 * no cross-request atomics). */
flr_status flr_server_create(flr_ctx ctx, size_t hbm_budget_bytes, int32_t max_slots, flr_server* out);
flr_status flr_server_submit(flr_server s, flr_problem h, double lambda1, double lambda2, double tol,
                             const flr_solve_opts* opts, uint64_t* ticket);
/* blocking = 0: FLR_ERR_NOT_READY until done.  beta_out_host: nullable, length p. */
flr_status flr_server_poll(flr_server s, uint64_t ticket, int blocking, double* beta_out_host, flr_result* res);
/* Queue depth, slots in use and bytes admitted. */
flr_status flr_server_stats(flr_server s, int32_t* queued, int32_t* running, size_t* bytes_in_use);
void flr_server_destroy(flr_server s);

/* Profiling: launch the rotation's row-panel kernel (X v), column-panel
 * kernel (X^T u + M v) and block kernel (PCG updates and the partitioned
 * tridiagonal solve) `reps` times each on the problem's stream, in the state
 * of a PCG step, and report their average durations in microseconds as
 * measured with HIP events on that stream.  avg_us: host, 3 entries (A, B, C).
 * The last solution is left intact.  Needs a completed solve on the handle. */
flr_status flr_profile_kernels(flr_problem h, int32_t reps, double* avg_us);

/* Profiling of the batched products of flr_solve_grid: run the two FP64 GEMMs
 * of one batched PCG step, U = X O (n x B) and V = X^T U (p x B), `reps` times
 * each for B right-hand sides on the problem's stream and report their average
 * durations in microseconds (HIP events; avg_us: host, 2 entries).  Uses the
 * grid workspace's scratch operand, so it needs a completed grid solve with at
 * least B columns on the handle; solver state is not touched. */
flr_status flr_profile_grid(flr_problem h, int32_t B, int32_t reps, double* avg_us);

/* Profiling of Algorithm 1 (section 3.1): at the handle's current iterate,
 * run `reps` times each (a) the reweighting and assembly of Q = X^T X +
 * lambda1 A + lambda2 B, (b) the blocked Cholesky factor Q = L L^T and (c) the
 * forward and backward triangular solves, on the problem's stream, and report
 * their average durations in microseconds (HIP events; avg_us: host, 3
 * entries).  Needs a completed FLR_METHOD_CHOLESKY solve on the handle (its
 * dense workspace); the iterate and the last result are left intact.
 * FLR_ERR_INVALID_ARG without that workspace or with negative lambdas. */
flr_status flr_profile_dense(flr_problem h, double lambda1, double lambda2, int32_t reps, double* avg_us);

const char* flr_status_string(flr_status st);
const char* flr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FLR_H */
