/*
 * FP64 CPU oracle for the majorization-minimization (MM) solver of fused
 * lasso regression.  TEST INFRASTRUCTURE ONLY: it is called by the tests,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by
 * the product path, and it shares no code with the HIP library.
 *
 * Problem (introduction, the FLR objective):
 *   f(b) = 1/2 ||y - X b||^2 + lambda1 sum_j |b_j| + lambda2 sum_{(j,k) in E} |b_j - b_k|
 * Method (section 3.1): each |t| is replaced by the perturbed
 * |t| - eps log(1 + |t|/eps) (perturbed objective), majorized at the
 * current iterate by a quadratic (majorizer equation); minimizing the
 * majorizer is the linear system (linear-system equation)
 *   (X^T X + lambda1 A + lambda2 B) b = X^T y,
 *   A = diag(1/(|b_j|+eps)),  B = weighted graph Laplacian, w = 1/(|b_j-b_k|+eps).
 * Algorithm 1 solves it by dense Cholesky, Algorithm 2 by preconditioned CG
 * with M = lambda1 A + lambda2 B as the preconditioner (banded Cholesky).
 */
#ifndef FLR_ORACLE_H
#define FLR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OFL_F64 = 0, OFL_F32 = 1, OFL_BF16 = 2 };
enum { OFL_ALG_AUTO = 0, OFL_ALG1_CHOLESKY = 1, OFL_ALG2_PCG = 2 };
enum { OFL_OK = 0, OFL_MAX_ITER = 1, OFL_NUMERICAL = 2, OFL_BAD_ARG = 3 };

typedef struct {
  int64_t n, p, ldx;       /* X is n x p, row-major, row stride ldx elements */
  int xdtype;              /* OFL_F64 / OFL_F32 / OFL_BF16 (uint16 bit patterns) */
  const void* X;
  const double* y;         /* length n */
  int64_t m;               /* number of edges */
  const int64_t* edges;    /* 2*m entries: pairs (j, k), 0-based, j != k */
} ofl_problem;

typedef struct {
  double eps;              /* perturbation, e.g. 1e-8 */
  double tol;              /* outer: relative objective change; 0 = run max_iter */
  double inner_tol;        /* PCG: ||r|| / ||X^T y||; <= 0 means tol */
  int32_t max_iter;        /* MM iteration cap; <= 0 means 10000 */
  int64_t max_cg;          /* PCG cap per MM step; <= 0 means p */
  int32_t method;          /* OFL_ALG_* */
  const double* beta0;     /* nullable warm start (length p) */
} ofl_opts;

typedef struct {
  double objective;        /* f at the returned iterate */
  double rel_change;       /* last relative objective change */
  double rel_residual;     /* last PCG relative residual (0 for Algorithm 1) */
  int32_t mm_iters;
  int32_t status;          /* OFL_OK / OFL_MAX_ITER / OFL_NUMERICAL / OFL_BAD_ARG */
  int64_t cg_iters;
  int32_t method_used;
  int32_t threads;
} ofl_result;

/* Per-MM-iteration trajectory record (traj has room for max_iter rows). */
typedef struct {
  double f, f_eps, rel_change, rel_residual;
  int64_t cg;
} ofl_traj;

int ofl_solve(const ofl_problem* P, double lambda1, double lambda2, const ofl_opts* o,
              double* beta_out, ofl_result* res, ofl_traj* traj);
double ofl_objective(const ofl_problem* P, double lambda1, double lambda2, const double* beta);
double ofl_objective_eps(const ofl_problem* P, double lambda1, double lambda2, double eps, const double* beta);
double ofl_surrogate(const ofl_problem* P, double lambda1, double lambda2, double eps,
                     const double* beta, const double* beta_ref);
void ofl_init_beta(const ofl_problem* P, double* beta0);
void ofl_gradient_eps(const ofl_problem* P, double lambda1, double lambda2, double eps,
                      const double* beta, double* grad);
void ofl_system(const ofl_problem* P, double lambda1, double lambda2, double eps,
                const double* beta_ref, double* Q, double* c);
int ofl_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
