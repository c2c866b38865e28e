/*
 * FP64 CPU oracle for the MM solver of fused lasso regression.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls
 * this file; it is the plain, slow reference that the HIP path is checked
 * against.  Every step follows the paper (section 3.1, Algorithms 1 and 2)
 * in its own order and notation; see flr_oracle.h for the problem.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *  - PCG residual update: the paper prints r_j = r_{j-1} + nu Q p_j while
 *    starting from r_0 = c - Q x_0; with that sign CG diverges.  The
 *    standard recurrence r_j = r_{j-1} - nu Q p_j is used.
 *  - The inner loop of Algorithm 2 is repeat-until: at least one PCG step
 *    runs in every MM iteration, and the test ||r||/||c|| <= delta_in is
 *    evaluated after each step.  The one exception is r_0 = 0 exactly (the
 *    warm start solves the system in floating point): then nu would be 0/0,
 *    and no step is taken.
 *  - Inner cap: p steps (the finite-termination bound of CG).
 *  - The outer test uses the true objective f (FLR objective), relative to
 *    the previous value: |f_new - f_old| / f_old <= delta.  delta = 0 runs
 *    exactly max_iter iterations (used by the closed-form pins, where f stops
 *    changing in floating point before the iterate does).
 *  - A zero column gives beta_j^(0) = 0 in the initialization.
 *  - lambda1 = 0 makes M = lambda2 B singular on a connected graph, so
 *    Algorithm 1 is used in that case.
 *  - The "dpotrf + dpotri" of Algorithm 1 is taken as factor + two
 *    triangular solves (same system, no explicit inverse).
 *  - E is a set of unordered pairs: each edge adds w to B_jj and B_kk and
 *    -w to B_jk = B_kj.
 */
#include "flr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int ofl_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* X widened to FP64 (exact for f32 and bf16 storage).                        */
/* ------------------------------------------------------------------------- */
static double* widen_x(const ofl_problem* P) {
  int64_t n = P->n, p = P->p;
  double* xd = (double*)malloc((size_t)n * (size_t)p * sizeof(double));
  if (!xd) return NULL;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < p; ++j) {
      double v;
      if (P->xdtype == OFL_F64) {
        v = ((const double*)P->X)[i * P->ldx + j];
      } else if (P->xdtype == OFL_F32) {
        v = (double)((const float*)P->X)[i * P->ldx + j];
      } else {
        uint32_t bits = ((uint32_t)((const uint16_t*)P->X)[i * P->ldx + j]) << 16;
        float f;
        memcpy(&f, &bits, sizeof f);
        v = (double)f;
      }
      xd[i * p + j] = v;
    }
  }
  return xd;
}

/* u = X v : one output per row, summed left to right. */
static void gemv_x(const double* xd, int64_t n, int64_t p, const double* v, double* u) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    const double* row = xd + i * p;
    for (int64_t j = 0; j < p; ++j) s += row[j] * v[j];
    u[i] = s;
  }
}

/* v = X^T u : each output summed over rows top to bottom (column blocks in
 * parallel, so the result does not depend on the thread count). */
static void gemv_xt(const double* xd, int64_t n, int64_t p, const double* u, double* v) {
  const int64_t B = 256;
  int64_t nb = (p + B - 1) / B;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    int64_t j0 = b * B, j1 = j0 + B < p ? j0 + B : p;
    for (int64_t j = j0; j < j1; ++j) v[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double* row = xd + i * p;
      double ui = u[i];
      for (int64_t j = j0; j < j1; ++j) v[j] += row[j] * ui;
    }
  }
}

static double dot(const double* a, const double* b, int64_t k) {
  double s = 0.0;
  for (int64_t i = 0; i < k; ++i) s += a[i] * b[i];
  return s;
}

/* ------------------------------------------------------------------------- */
/* Objectives (FLR objective; perturbed objective; majorizer).               */
/* ------------------------------------------------------------------------- */
static double pert_abs(double t, double eps) {
  double a = fabs(t);
  return a - eps * log1p(a / eps);
}

static double loss_from_xd(const ofl_problem* P, const double* xd, const double* beta) {
  double* u = (double*)malloc((size_t)P->n * sizeof(double));
  gemv_x(xd, P->n, P->p, beta, u);
  double s = 0.0;
  for (int64_t i = 0; i < P->n; ++i) {
    double d = P->y[i] - u[i];
    s += d * d;
  }
  free(u);
  return 0.5 * s;
}

static double objective_xd(const ofl_problem* P, const double* xd, double l1, double l2, const double* beta) {
  double f = loss_from_xd(P, xd, beta);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t j = 0; j < P->p; ++j) s1 += fabs(beta[j]);
  for (int64_t e = 0; e < P->m; ++e) s2 += fabs(beta[P->edges[2 * e]] - beta[P->edges[2 * e + 1]]);
  return f + l1 * s1 + l2 * s2;
}

double ofl_objective(const ofl_problem* P, double l1, double l2, const double* beta) {
  double* xd = widen_x(P);
  double f = objective_xd(P, xd, l1, l2, beta);
  free(xd);
  return f;
}

double ofl_objective_eps(const ofl_problem* P, double l1, double l2, double eps, const double* beta) {
  double* xd = widen_x(P);
  double f = loss_from_xd(P, xd, beta);
  free(xd);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t j = 0; j < P->p; ++j) s1 += pert_abs(beta[j], eps);
  for (int64_t e = 0; e < P->m; ++e) s2 += pert_abs(beta[P->edges[2 * e]] - beta[P->edges[2 * e + 1]], eps);
  return f + l1 * s1 + l2 * s2;
}

/* g_eps(beta | beta_ref): each perturbed term is replaced by its tangent
 * quadratic in t^2 at the reference point (majorizer equation). */
static double tangent_quad(double t, double t0, double eps) {
  double a0 = fabs(t0);
  return a0 - eps * log1p(a0 / eps) + (t * t - t0 * t0) / (2.0 * (a0 + eps));
}

double ofl_surrogate(const ofl_problem* P, double l1, double l2, double eps, const double* beta,
                     const double* beta_ref) {
  double* xd = widen_x(P);
  double f = loss_from_xd(P, xd, beta);
  free(xd);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t j = 0; j < P->p; ++j) s1 += tangent_quad(beta[j], beta_ref[j], eps);
  for (int64_t e = 0; e < P->m; ++e) {
    int64_t j = P->edges[2 * e], k = P->edges[2 * e + 1];
    s2 += tangent_quad(beta[j] - beta[k], beta_ref[j] - beta_ref[k], eps);
  }
  return f + l1 * s1 + l2 * s2;
}

/* gradient of f_eps: X^T(X b - y) + l1 b/(|b|+eps) + l2 sum_e +-(d_e/(|d_e|+eps)) */
static void gradient_xd(const ofl_problem* P, const double* xd, double l1, double l2, double eps,
                        const double* beta, double* g) {
  int64_t n = P->n, p = P->p;
  double* u = (double*)malloc((size_t)n * sizeof(double));
  gemv_x(xd, n, p, beta, u);
  for (int64_t i = 0; i < n; ++i) u[i] -= P->y[i];
  gemv_xt(xd, n, p, u, g);
  free(u);
  for (int64_t j = 0; j < p; ++j) g[j] += l1 * beta[j] / (fabs(beta[j]) + eps);
  for (int64_t e = 0; e < P->m; ++e) {
    int64_t j = P->edges[2 * e], k = P->edges[2 * e + 1];
    double d = beta[j] - beta[k];
    double t = l2 * d / (fabs(d) + eps);
    g[j] += t;
    g[k] -= t;
  }
}

void ofl_gradient_eps(const ofl_problem* P, double l1, double l2, double eps, const double* beta, double* grad) {
  double* xd = widen_x(P);
  gradient_xd(P, xd, l1, l2, eps, beta, grad);
  free(xd);
}

/* Initialization of Algorithms 1 and 2: b_j = X_j^T y / X_j^T X_j. */
static void init_xd(const ofl_problem* P, const double* xd, double* beta0) {
  int64_t n = P->n, p = P->p;
  double* c = (double*)malloc((size_t)p * sizeof(double));
  double* s = (double*)calloc((size_t)p, sizeof(double));
  gemv_xt(xd, n, p, P->y, c);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < p; ++j) s[j] += xd[i * p + j] * xd[i * p + j];
  for (int64_t j = 0; j < p; ++j) beta0[j] = s[j] > 0.0 ? c[j] / s[j] : 0.0;
  free(c);
  free(s);
}

void ofl_init_beta(const ofl_problem* P, double* beta0) {
  double* xd = widen_x(P);
  init_xd(P, xd, beta0);
  free(xd);
}

/* ------------------------------------------------------------------------- */
/* Reweighting (linear-system equation): a_j and per-edge w_e.               */
/* ------------------------------------------------------------------------- */
static void reweight(const ofl_problem* P, double eps, const double* beta, double* a, double* w) {
  for (int64_t j = 0; j < P->p; ++j) a[j] = 1.0 / (fabs(beta[j]) + eps);
  for (int64_t e = 0; e < P->m; ++e)
    w[e] = 1.0 / (fabs(beta[P->edges[2 * e]] - beta[P->edges[2 * e + 1]]) + eps);
}

/* M v = l1 A v + l2 B v with B the weighted Laplacian over E. */
static void apply_m(const ofl_problem* P, double l1, double l2, const double* a, const double* w,
                    const double* v, double* out) {
  for (int64_t j = 0; j < P->p; ++j) out[j] = l1 * a[j] * v[j];
  for (int64_t e = 0; e < P->m; ++e) {
    int64_t j = P->edges[2 * e], k = P->edges[2 * e + 1];
    double t = l2 * w[e] * (v[j] - v[k]);
    out[j] += t;
    out[k] -= t;
  }
}

/* Dense system of Algorithm 1: Q = X^T X + l1 A + l2 B, c = X^T y. */
static void form_q(const ofl_problem* P, const double* xtx, double l1, double l2, const double* a,
                   const double* w, double* Q) {
  int64_t p = P->p;
  memcpy(Q, xtx, (size_t)p * (size_t)p * sizeof(double));
  for (int64_t j = 0; j < p; ++j) Q[j * p + j] += l1 * a[j];
  for (int64_t e = 0; e < P->m; ++e) {
    int64_t j = P->edges[2 * e], k = P->edges[2 * e + 1];
    double t = l2 * w[e];
    Q[j * p + j] += t;
    Q[k * p + k] += t;
    Q[j * p + k] -= t;
    Q[k * p + j] -= t;
  }
}

static void gram(const double* xd, int64_t n, int64_t p, double* xtx) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t j = 0; j < p; ++j) {
    for (int64_t k = 0; k <= j; ++k) {
      double s = 0.0;
      for (int64_t i = 0; i < n; ++i) s += xd[i * p + j] * xd[i * p + k];
      xtx[j * p + k] = s;
      xtx[k * p + j] = s;
    }
  }
}

void ofl_system(const ofl_problem* P, double l1, double l2, double eps, const double* beta_ref, double* Q,
                double* c) {
  int64_t p = P->p;
  double* xd = widen_x(P);
  double* xtx = (double*)malloc((size_t)p * (size_t)p * sizeof(double));
  double* a = (double*)malloc((size_t)p * sizeof(double));
  double* w = (double*)malloc((size_t)(P->m > 0 ? P->m : 1) * sizeof(double));
  gram(xd, P->n, p, xtx);
  reweight(P, eps, beta_ref, a, w);
  form_q(P, xtx, l1, l2, a, w, Q);
  gemv_xt(xd, P->n, p, P->y, c);
  free(xd);
  free(xtx);
  free(a);
  free(w);
}

/* Dense Cholesky Q = L L^T in place (lower triangle); returns 0 on success. */
static int chol_dense(double* Q, int64_t p) {
  for (int64_t j = 0; j < p; ++j) {
    double s = Q[j * p + j];
    for (int64_t k = 0; k < j; ++k) s -= Q[j * p + k] * Q[j * p + k];
    if (!(s > 0.0)) return -1;
    double d = sqrt(s);
    Q[j * p + j] = d;
#pragma omp parallel for schedule(static) if (p - j > 256)
    for (int64_t i = j + 1; i < p; ++i) {
      double t = Q[i * p + j];
      for (int64_t k = 0; k < j; ++k) t -= Q[i * p + k] * Q[j * p + k];
      Q[i * p + j] = t / d;
    }
  }
  return 0;
}

static void chol_dense_solve(const double* L, int64_t p, const double* b, double* x) {
  for (int64_t i = 0; i < p; ++i) {
    double s = b[i];
    for (int64_t k = 0; k < i; ++k) s -= L[i * p + k] * x[k];
    x[i] = s / L[i * p + i];
  }
  for (int64_t i = p - 1; i >= 0; --i) {
    double s = x[i];
    for (int64_t k = i + 1; k < p; ++k) s -= L[k * p + i] * x[k];
    x[i] = s / L[i * p + i];
  }
}

/* ------------------------------------------------------------------------- */
/* Banded Cholesky of M = l1 A + l2 B (bandwidth bw = max |j - k| over E),   */
/* the preconditioner of Algorithm 2.  Lb[i*(bw+1) + d] holds L(i, i-d).      */
/* ------------------------------------------------------------------------- */
static int band_factor(const ofl_problem* P, double l1, double l2, const double* a, const double* w,
                       int64_t bw, double* Lb) {
  int64_t p = P->p, W = bw + 1;
  memset(Lb, 0, (size_t)p * (size_t)W * sizeof(double));
  for (int64_t j = 0; j < p; ++j) Lb[j * W] = l1 * a[j];
  for (int64_t e = 0; e < P->m; ++e) {
    int64_t j = P->edges[2 * e], k = P->edges[2 * e + 1];
    int64_t hi = j > k ? j : k, lo = j > k ? k : j;
    double t = l2 * w[e];
    Lb[j * W] += t;
    Lb[k * W] += t;
    Lb[hi * W + (hi - lo)] -= t;
  }
  for (int64_t j = 0; j < p; ++j) {
    int64_t k0 = j - bw > 0 ? j - bw : 0;
    double s = Lb[j * W];
    for (int64_t k = k0; k < j; ++k) s -= Lb[j * W + (j - k)] * Lb[j * W + (j - k)];
    if (!(s > 0.0)) return -1;
    double d = sqrt(s);
    Lb[j * W] = d;
    int64_t i1 = j + bw < p - 1 ? j + bw : p - 1;
    for (int64_t i = j + 1; i <= i1; ++i) {
      double t = Lb[i * W + (i - j)];
      int64_t kk0 = i - bw > k0 ? i - bw : k0;
      for (int64_t k = kk0; k < j; ++k) t -= Lb[i * W + (i - k)] * Lb[j * W + (j - k)];
      Lb[i * W + (i - j)] = t / d;
    }
  }
  return 0;
}

static void band_solve(const double* Lb, int64_t p, int64_t bw, const double* b, double* x) {
  int64_t W = bw + 1;
  for (int64_t i = 0; i < p; ++i) {
    double s = b[i];
    int64_t k0 = i - bw > 0 ? i - bw : 0;
    for (int64_t k = k0; k < i; ++k) s -= Lb[i * W + (i - k)] * x[k];
    x[i] = s / Lb[i * W];
  }
  for (int64_t i = p - 1; i >= 0; --i) {
    double s = x[i];
    int64_t k1 = i + bw < p - 1 ? i + bw : p - 1;
    for (int64_t k = i + 1; k <= k1; ++k) s -= Lb[k * W + (k - i)] * x[k];
    x[i] = s / Lb[i * W];
  }
}

/* ------------------------------------------------------------------------- */
/* Solver driver: Algorithm 1 or Algorithm 2.                                */
/* ------------------------------------------------------------------------- */
int ofl_solve(const ofl_problem* P, double l1, double l2, const ofl_opts* o, double* beta_out, ofl_result* res,
              ofl_traj* traj) {
  int64_t n = P->n, p = P->p, m = P->m;
  memset(res, 0, sizeof *res);
  res->threads = ofl_num_threads();
  if (n < 1 || p < 1 || P->ldx < p || !(l1 >= 0.0) || !(l2 >= 0.0) || !(o->eps > 0.0) || !(o->tol >= 0.0)) {
    res->status = OFL_BAD_ARG;
    return OFL_BAD_ARG;
  }
  double eps = o->eps, tol = o->tol;
  double itol = o->inner_tol > 0.0 ? o->inner_tol : tol;
  int32_t max_iter = o->max_iter > 0 ? o->max_iter : 10000;
  int64_t max_cg = o->max_cg > 0 ? o->max_cg : p;
  int64_t bw = 0;
  for (int64_t e = 0; e < m; ++e) {
    int64_t d = P->edges[2 * e] - P->edges[2 * e + 1];
    if (d < 0) d = -d;
    if (d > bw) bw = d;
  }
  int method = o->method;
  /* Algorithm 2 where M is banded (chain, lattice), Algorithm 1 otherwise
   * (the paper recommends the dense route for a general E). */
  if (method == OFL_ALG_AUTO) method = (bw * bw <= p) ? OFL_ALG2_PCG : OFL_ALG1_CHOLESKY;
  if (l1 == 0.0) method = OFL_ALG1_CHOLESKY;
  res->method_used = method;

  double* xd = widen_x(P);
  double* beta = (double*)malloc((size_t)p * sizeof(double));
  double* c = (double*)malloc((size_t)p * sizeof(double));
  double* a = (double*)malloc((size_t)p * sizeof(double));
  double* w = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
  double *xtx = NULL, *Q = NULL, *Lb = NULL, *u = NULL, *t = NULL;
  double *x = NULL, *r = NULL, *z = NULL, *pv = NULL, *q = NULL;
  if (method == OFL_ALG1_CHOLESKY) {
    xtx = (double*)malloc((size_t)p * (size_t)p * sizeof(double));
    Q = (double*)malloc((size_t)p * (size_t)p * sizeof(double));
    gram(xd, n, p, xtx);
  } else {
    Lb = (double*)malloc((size_t)p * (size_t)(bw + 1) * sizeof(double));
    u = (double*)malloc((size_t)n * sizeof(double));
    t = (double*)malloc((size_t)p * sizeof(double));
    x = (double*)malloc((size_t)p * sizeof(double));
    r = (double*)malloc((size_t)p * sizeof(double));
    z = (double*)malloc((size_t)p * sizeof(double));
    pv = (double*)malloc((size_t)p * sizeof(double));
    q = (double*)malloc((size_t)p * sizeof(double));
  }
  gemv_xt(xd, n, p, P->y, c);
  double cnorm = sqrt(dot(c, c, p));
  if (o->beta0)
    memcpy(beta, o->beta0, (size_t)p * sizeof(double));
  else
    init_xd(P, xd, beta);

  double f_old = objective_xd(P, xd, l1, l2, beta);
  int status = OFL_MAX_ITER;
  double re = 0.0, last_res = 0.0;
  int32_t it;
  for (it = 0; it < max_iter; ++it) {
    reweight(P, eps, beta, a, w);
    int64_t cg = 0;
    if (method == OFL_ALG1_CHOLESKY) {
      form_q(P, xtx, l1, l2, a, w, Q);
      if (chol_dense(Q, p) != 0) {
        status = OFL_NUMERICAL;
        break;
      }
      chol_dense_solve(Q, p, c, beta);
      last_res = 0.0;
    } else {
      if (band_factor(P, l1, l2, a, w, bw, Lb) != 0) {
        status = OFL_NUMERICAL;
        break;
      }
      /* x0 = beta; r0 = c - (X^T X + M) x0; z0 = M^-1 r0; p1 = z0 */
      memcpy(x, beta, (size_t)p * sizeof(double));
      gemv_x(xd, n, p, x, u);
      gemv_xt(xd, n, p, u, q);
      apply_m(P, l1, l2, a, w, x, t);
      for (int64_t j = 0; j < p; ++j) r[j] = c[j] - (q[j] + t[j]);
      band_solve(Lb, p, bw, r, z);
      memcpy(pv, z, (size_t)p * sizeof(double));
      double rz = dot(r, z, p);
      double rr0 = dot(r, r, p);
      double rn = sqrt(rr0) / cnorm;
      int bad = 0;
      /* repeat ... until ||r_j|| / ||X^T y|| <= delta_in (or the cap) */
      int more = rr0 > 0.0 && max_cg > 0;
      while (more) {
        gemv_x(xd, n, p, pv, u);
        gemv_xt(xd, n, p, u, q);
        apply_m(P, l1, l2, a, w, pv, t);
        for (int64_t j = 0; j < p; ++j) q[j] += t[j];
        double pq = dot(pv, q, p);
        if (!(pq > 0.0)) {
          bad = 1;
          break;
        }
        double nu = rz / pq;
        for (int64_t j = 0; j < p; ++j) {
          x[j] += nu * pv[j];
          r[j] -= nu * q[j];
        }
        band_solve(Lb, p, bw, r, z);
        double rz_new = dot(r, z, p);
        double gamma = rz_new / rz;
        rz = rz_new;
        for (int64_t j = 0; j < p; ++j) pv[j] = z[j] + gamma * pv[j];
        rn = sqrt(dot(r, r, p)) / cnorm;
        ++cg;
        more = rn > itol && cg < max_cg;
      }
      if (bad) {
        status = OFL_NUMERICAL;
        break;
      }
      memcpy(beta, x, (size_t)p * sizeof(double));
      last_res = rn;
    }
    res->cg_iters += cg;
    double f_new = objective_xd(P, xd, l1, l2, beta);
    double f_eps_new = NAN;
    if (traj) {
      f_eps_new = loss_from_xd(P, xd, beta);
      double s1 = 0.0, s2 = 0.0;
      for (int64_t j = 0; j < p; ++j) s1 += pert_abs(beta[j], eps);
      for (int64_t e = 0; e < m; ++e) s2 += pert_abs(beta[P->edges[2 * e]] - beta[P->edges[2 * e + 1]], eps);
      f_eps_new += l1 * s1 + l2 * s2;
    }
    re = f_old != 0.0 ? fabs(f_new - f_old) / fabs(f_old) : fabs(f_new - f_old);
    if (traj) {
      traj[it].f = f_new;
      traj[it].f_eps = f_eps_new;
      traj[it].rel_change = re;
      traj[it].rel_residual = last_res;
      traj[it].cg = cg;
    }
    f_old = f_new;
    if (!isfinite(f_new)) {
      status = OFL_NUMERICAL;
      ++it;
      break;
    }
    if (tol > 0.0 && re <= tol) {
      status = OFL_OK;
      ++it;
      break;
    }
  }
  res->mm_iters = it;
  res->objective = f_old;
  res->rel_change = re;
  res->rel_residual = last_res;
  res->status = status;
  memcpy(beta_out, beta, (size_t)p * sizeof(double));
  free(xd);
  free(beta);
  free(c);
  free(a);
  free(w);
  free(xtx);
  free(Q);
  free(Lb);
  free(u);
  free(t);
  free(x);
  free(r);
  free(z);
  free(pv);
  free(q);
  return status;
}
