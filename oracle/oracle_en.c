/*
 * FP64 CPU oracle for the SsNAL-EN elastic-net solver (test infrastructure).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  It is a plain, slow, literal transcription of the method in
 * the paper (Boschi, Reimherr, Chiaromonte, "An Efficient Semi-smooth Newton
 * Augmented Lagrangian Method for Elastic Net"):
 *   - no blocking, no fusion, no Sherman-Morrison-Woodbury branch: the Newton
 *     system is always the m x m one, solved by Cholesky or, on request, by
 *     plain conjugate gradients;
 *   - A^T y is recomputed from scratch every Newton iteration;
 *   - plain loops, left-to-right sums, no BLAS.
 * It is pinned by tests that do not use it (closed forms, brute force,
 * KKT certificates, duality gaps, a coordinate-descent cross-check).
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - grad h*(y) = y + b (Sec. 3.2, eq. grad_phy; the KKT display of Sec. 3
 *     writes y - b, which contradicts h*(y) = 1/2||y||^2 + b^T y).
 *   - a tie |t_i| = sigma*lambda1 is inactive (eq. Q_def uses ">").
 *   - inner stop: kkt1 <= tol; outer stop: kkt1 <= tol, kkt3 <= tol and the
 *     primal natural residual eta(x) <= tol.
 *   - line search: backtracking s = delta^k, delta = 0.5, at most 31 trials;
 *     if none passes, the inner loop ends (eq. line_search gives only mu).
 *   - the multiplier update x - sigma (A^T y + z) is evaluated as
 *     prox_{sigma p}(x - sigma A^T y), its value by the Moreau decomposition
 *     (Sec. 2.2); this keeps exact zeros in x.
 *   - conjugate gradients (the approximate solve for large m and r) start
 *     from d = 0 and stop at ||V d + g|| <= min(0.1, kkt1^0.5) ||g|| or after
 *     500 iterations (the paper fixes no rule; this is an inexact-Newton
 *     forcing term of order 1.5).
 *   - sigma0 defaults to 2.5 / mean_j ||a_j||^2 (= 5e-3 when the columns have
 *     squared norm m = 500, the setting of Sec. 4.1), factor 5, capped 1e8.
 */
#include "oracle_en.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define COL(A, lda, j) ((A) + (int64_t)(j) * (lda))

/* ---------------------------------------------------------------------- */
/* Proximal operators and conjugate (Sec. 2.1 Prop. 1; Sec. 2.2 eq. prox_elastic) */

/* prox_{sigma p}(t) = soft(t, sigma*lambda1) / (1 + sigma*lambda2)
 * (eq. prox_elastic, left).  Pinned: 1-D numeric argmin of eq. prox_op. */
double orc_prox_sp(double t, double sigma, double l1, double l2) {
  double thr = sigma * l1;
  double den = 1.0 + sigma * l2;
  if (t > thr) return (t - thr) / den;
  if (t < -thr) return (t + thr) / den;
  return 0.0;
}

/* prox_{p^* / sigma}(v / sigma) as a function of v (eq. prox_elastic, right).
 * Pinned: Moreau decomposition v = prox_{sigma p}(v) + sigma*prox_{p^* / sigma}(v/sigma)
 * and a 1-D numeric argmin of the conjugate's prox. */
double orc_prox_pstar(double v, double sigma, double l1, double l2) {
  double thr = sigma * l1;
  double den = 1.0 + sigma * l2;
  if (v >= thr) return (v * l2 + l1) / den;
  if (v <= -thr) return (v * l2 - l1) / den;
  return v / sigma;
}

/* p*(z) of the elastic-net penalty (Prop. 1, eq. p_star).
 * Pinned: numeric sup_x (z x - p(x)) in 1-D.  lambda2 = 0 (the Lasso): the
 * conjugate of lambda1 |.|_1 is the indicator of |z|_inf <= lambda1. */
double orc_pstar(const double* z, int64_t n, double l1, double l2) {
  if (l2 == 0.0) {
    for (int64_t i = 0; i < n; ++i)
      if (fabs(z[i]) > l1) return INFINITY;
    return 0.0;
  }
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double zi = z[i], e = 0.0;
    if (zi >= l1) e = (zi - l1) * (zi - l1);
    else if (zi <= -l1) e = (zi + l1) * (zi + l1);
    s += e;
  }
  return s / (2.0 * l2);
}

/* ---------------------------------------------------------------------- */
/* Dense products (plain dot products, left to right) */

/* Host threads for the loops below whose iterations are independent: each
 * output entry is one sum, evaluated in the same order whatever the thread
 * count, so every result is bit-for-bit the same with 1 or k threads (a pin
 * checks this).  Default 1. */
static int g_threads = 1;
void orc_set_threads(int k) { g_threads = k < 1 ? 1 : k; }
int orc_get_threads(void) { return g_threads; }

void orc_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* v, double* w) {
#pragma omp parallel for num_threads(g_threads) schedule(static) if (g_threads > 1 && n >= 256)
  for (int64_t j = 0; j < n; ++j) {
    const double* a = COL(A, lda, j);
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += a[i] * v[i];
    w[j] = s;
  }
}

/* out = A x; out_i accumulates a_ij x_j over j in increasing order.  Rows
 * are split into independent blocks of 256 for the threads. */
void orc_gemv_n(const double* A, int64_t lda, int64_t m, int64_t n, const double* x, double* out) {
  const int64_t nblk = (m + 255) / 256;
#pragma omp parallel for num_threads(g_threads) schedule(static) if (g_threads > 1 && nblk > 1)
  for (int64_t blk = 0; blk < nblk; ++blk) {
    const int64_t i0 = blk * 256, i1 = i0 + 256 < m ? i0 + 256 : m;
    for (int64_t i = i0; i < i1; ++i) out[i] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double xj = x[j];
      if (xj == 0.0) continue; /* adds +-0 only: skipping it changes no value */
      const double* a = COL(A, lda, j);
      for (int64_t i = i0; i < i1; ++i) out[i] += a[i] * xj;
    }
  }
}

static double dot(const double* a, const double* b, int64_t k) {
  double s = 0.0;
  for (int64_t i = 0; i < k; ++i) s += a[i] * b[i];
  return s;
}

static double nrm2(const double* a, int64_t k) { return sqrt(dot(a, a, k)); }

/* ---------------------------------------------------------------------- */
/* Objectives and certificates */

/* F(x), eq. objective_function.  Pinned jointly with the dual objective:
 * zero duality gap at closed-form / brute-force minimisers, weak duality
 * everywhere else. */
double orc_primal_obj(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                      const double* x, double l1, double l2) {
  double* r = (double*)malloc(sizeof(double) * (size_t)m);
  orc_gemv_n(A, lda, m, n, x, r);
  for (int64_t i = 0; i < m; ++i) r[i] -= b[i];
  double f = 0.5 * dot(r, r, m);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t j = 0; j < n; ++j) { s1 += fabs(x[j]); s2 += x[j] * x[j]; }
  free(r);
  return f + l1 * s1 + 0.5 * l2 * s2;
}

/* Dual objective of (D): -h*(y) - p*(z) with z = -A^T y (the constraint
 * A^T y + z = 0), h*(y) = 1/2||y||^2 + b^T y (Sec. 3).  Every y is feasible
 * for lambda2 > 0 because p* is finite (Prop. 1). */
/* lambda2 = 0: D is evaluated at theta*y, theta = min(1, lambda1/|A^T y|_inf),
 * the largest multiple of y inside the dual feasible set (p* is an
 * indicator), so that it stays a finite lower bound of F. */
double orc_dual_obj(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                    const double* y, double l1, double l2) {
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  orc_gemv_t(A, lda, m, n, y, z);
  for (int64_t j = 0; j < n; ++j) z[j] = -z[j];
  double theta = 1.0;
  if (l2 == 0.0) {
    double amax = 0.0;
    for (int64_t j = 0; j < n; ++j) amax = fabs(z[j]) > amax ? fabs(z[j]) : amax;
    if (amax > l1) theta = l1 / amax;
    for (int64_t j = 0; j < n; ++j) z[j] *= theta;
  }
  double hs = 0.5 * theta * theta * dot(y, y, m) + theta * dot(b, y, m);
  double ps = orc_pstar(z, n, l1, l2);
  free(z);
  return -hs - ps;
}

/* Relative primal natural residual
 *   eta(x) = ||x - prox_p(x - A^T(Ax - b))|| / (1 + ||x|| + ||Ax - b||),
 * prox_p(v) = soft(v, lambda1)/(1 + lambda2).  It is zero exactly at the
 * minimiser (fixed point of the proximal-gradient map); this is the relative
 * KKT residual the solver is gated on (the paper's own residuals are
 * eq. kkt_res, which the solve reports too). */
double orc_eta(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
               const double* x, double l1, double l2) {
  double* r = (double*)malloc(sizeof(double) * (size_t)m);
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
  orc_gemv_n(A, lda, m, n, x, r);
  for (int64_t i = 0; i < m; ++i) r[i] -= b[i];
  orc_gemv_t(A, lda, m, n, r, g);
  double num = 0.0, xx = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double p = orc_prox_sp(x[j] - g[j], 1.0, l1, l2);
    double e = x[j] - p;
    num += e * e;
    xx += x[j] * x[j];
  }
  double den = 1.0 + sqrt(xx) + nrm2(r, m);
  free(r);
  free(g);
  return sqrt(num) / den;
}

/* psi(y) of Prop. 2 (1):
 *   h*(y) + (1+sigma*lambda2)/(2 sigma) ||prox_{sigma p}(x - sigma A^T y)||^2 - ||x||^2/(2 sigma).
 * Pinned: equals min_z L_sigma(y, z, x) computed by 1-D minimisation. */
double orc_psi(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
               const double* x, const double* y, double sigma, double l1, double l2) {
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  orc_gemv_t(A, lda, m, n, y, w);
  double pp = 0.0, xx = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double p = orc_prox_sp(fma(-sigma, w[j], x[j]), sigma, l1, l2);
    pp += p * p;
    xx += x[j] * x[j];
  }
  free(w);
  return 0.5 * dot(y, y, m) + dot(b, y, m) + (1.0 + sigma * l2) / (2.0 * sigma) * pp -
         xx / (2.0 * sigma);
}

/* grad psi(y) = y + b - A prox_{sigma p}(x - sigma A^T y)  (eq. grad_phy).
 * Pinned: central differences of psi. */
void orc_grad_psi(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                  const double* x, const double* y, double sigma, double l1, double l2,
                  double* g) {
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  double* u = (double*)malloc(sizeof(double) * (size_t)m);
  orc_gemv_t(A, lda, m, n, y, w);
  for (int64_t j = 0; j < n; ++j) w[j] = orc_prox_sp(fma(-sigma, w[j], x[j]), sigma, l1, l2);
  orc_gemv_n(A, lda, m, n, w, u);
  for (int64_t i = 0; i < m; ++i) g[i] = y[i] + b[i] - u[i];
  free(w);
  free(u);
}

/* Active set and prox at t = x - sigma*w (w = A^T y):
 *   J = { i : |t_i| > sigma*lambda1 }   (eq. Q_def, strict; a tie is inactive)
 *   uJ = prox_{sigma p}(t)_J            (eq. prox_elastic)
 * t_i is fma(-sigma, w_i, x_i) (one rounding) and the threshold is the
 * rounded product sigma*lambda1; the GPU takes the same decisions the same
 * way, so J is compared bit for bit.  Returns r = |J| (indices ascending). */
int64_t orc_active_prox(const double* x, const double* w, int64_t n, double sigma, double l1,
                        double l2, int32_t* J, double* uJ) {
  double thr = sigma * l1;
  double den = 1.0 + sigma * l2;
  int64_t r = 0;
  for (int64_t i = 0; i < n; ++i) {
    double t = fma(-sigma, w[i], x[i]);
    if (t > thr) { J[r] = (int32_t)i; uJ[r] = (t - thr) / den; ++r; }
    else if (t < -thr) { J[r] = (int32_t)i; uJ[r] = (t + thr) / den; ++r; }
  }
  return r;
}

/* V = I_m + kappa A_J A_J^T  (eq. AJ_system), kappa = sigma/(1+sigma*lambda2).
 * V is m x m, row-major, both triangles filled. */
void orc_newton_matrix(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                       double kappa, double* V) {
  /* gather A_J as m rows of length r so each entry is one contiguous dot */
  double* AJ = (double*)malloc(sizeof(double) * (size_t)(m * (r > 0 ? r : 1)));
  for (int64_t k = 0; k < r; ++k) {
    const double* a = COL(A, lda, J[k]);
    for (int64_t i = 0; i < m; ++i) AJ[i * r + k] = a[i];
  }
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 4) if (g_threads > 1 && m >= 64)
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t l = 0; l <= i; ++l) {
      double s = dot(AJ + i * r, AJ + l * r, r);
      double v = kappa * s + (i == l ? 1.0 : 0.0);
      V[i * m + l] = v;
      V[l * m + i] = v;
    }
  }
  free(AJ);
}

/* W = I_r / kappa + A_J^T A_J (eq. smw_formula), r x r, row-major, both
 * triangles.  The oracle's own solve never uses it (it always takes the
 * m x m system); it is the reference for the r x r branch of the GPU path.
 * Pinned: the Woodbury identity against the m x m matrix. */
void orc_smw_matrix(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                    double kappa, double* W) {
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 4) if (g_threads > 1 && r >= 64)
  for (int64_t p = 0; p < r; ++p) {
    const double* ap = COL(A, lda, J[p]);
    for (int64_t q = 0; q <= p; ++q) {
      const double* aq = COL(A, lda, J[q]);
      double v = dot(ap, aq, m) + (p == q ? 1.0 / kappa : 0.0);
      W[p * r + q] = v;
      W[q * r + p] = v;
    }
  }
}

/* In-place Cholesky V = L L^T (row-major, L in the lower triangle, the
 * strict upper triangle zeroed).  Textbook Cholesky-Crout, one column at a
 * time:
 *   l_jj = sqrt(v_jj - sum_{k<j} l_jk^2),
 *   l_ij = (v_ij - sum_{k<j} l_ik l_jk) / l_jj   (i > j),
 * each sum taken in increasing k.  The entries below a pivot do not depend on
 * each other, so the threads share them.  Returns 0, or -(k+1) if the k-th
 * pivot is not positive. */
int orc_cholesky(double* V, int64_t m) {
  for (int64_t j = 0; j < m; ++j) {
    double s = V[j * m + j];
    for (int64_t k = 0; k < j; ++k) s -= V[j * m + k] * V[j * m + k];
    if (!(s > 0.0)) return -(int)(j + 1);
    const double p = sqrt(s);
    V[j * m + j] = p;
#pragma omp parallel for num_threads(g_threads) schedule(static) if (g_threads > 1 && m - j > 128)
    for (int64_t i = j + 1; i < m; ++i) {
      double t = V[i * m + j];
      for (int64_t k = 0; k < j; ++k) t -= V[i * m + k] * V[j * m + k];
      V[i * m + j] = t / p;
    }
  }
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = i + 1; j < m; ++j) V[i * m + j] = 0.0;
  return 0;
}

/* Newton direction d = -V^{-1} g with V = I + kappa A_J A_J^T (eq. AJ_system),
 * dense Cholesky and two triangular solves.  Returns 0 or the Cholesky error. */
int orc_newton_direction(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                         double kappa, const double* g, double* d) {
  double* V = (double*)malloc(sizeof(double) * (size_t)(m * m));
  orc_newton_matrix(A, lda, m, J, r, kappa, V);
  int rc = orc_cholesky(V, m);
  if (rc == 0) {
    /* L c = -g */
    for (int64_t i = 0; i < m; ++i) {
      double s = -g[i];
      for (int64_t k = 0; k < i; ++k) s -= V[i * m + k] * d[k];
      d[i] = s / V[i * m + i];
    }
    /* L^T d = c */
    for (int64_t i = m - 1; i >= 0; --i) {
      double s = d[i];
      for (int64_t k = i + 1; k < m; ++k) s -= V[k * m + i] * d[k];
      d[i] = s / V[i * m + i];
    }
  }
  free(V);
  return rc;
}

/* V p for V = I_m + kappa A_J A_J^T (eq. AJ_system) without forming V: the r
 * products A_J^T p, then p + kappa A_J (A_J^T p).  Pinned: equals the dense
 * matrix of orc_newton_matrix times p. */
void orc_newton_matvec(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                       double kappa, const double* p, double* q) {
  double* s = (double*)malloc(sizeof(double) * (size_t)(r > 0 ? r : 1));
  for (int64_t k = 0; k < r; ++k) s[k] = dot(COL(A, lda, J[k]), p, m);
  for (int64_t i = 0; i < m; ++i) q[i] = 0.0;
  for (int64_t k = 0; k < r; ++k) {
    const double* a = COL(A, lda, J[k]);
    for (int64_t i = 0; i < m; ++i) q[i] += a[i] * s[k];
  }
  for (int64_t i = 0; i < m; ++i) q[i] = p[i] + kappa * q[i];
  free(s);
}

/* Approximate Newton direction by conjugate gradients (Sec. 3.2: the
 * approximate solve of eq. newton_direction when m and r are large): textbook
 * CG on V d = -g from d = 0 with the product above, stopping once the
 * recursive residual satisfies ||res||^2 <= eps^2 ||g||^2 or after maxit
 * iterations.  Returns the number of iterations.  Pinned: finite
 * termination (V has at most r + 1 distinct eigenvalues), agreement with the
 * Cholesky direction, the V-norm error never growing, and the stopping point
 * being the first iterate that meets the test. */
int orc_newton_cg(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                  double kappa, const double* g, double eps, int32_t maxit, double* d) {
  double* res = (double*)malloc(sizeof(double) * (size_t)m);
  double* p = (double*)malloc(sizeof(double) * (size_t)m);
  double* q = (double*)malloc(sizeof(double) * (size_t)m);
  for (int64_t i = 0; i < m; ++i) {
    d[i] = 0.0;
    res[i] = -g[i];
    p[i] = res[i];
  }
  double rr = dot(res, res, m);
  const double stop = eps * eps * dot(g, g, m);
  int it = 0;
  while (it < maxit && rr > stop) {
    orc_newton_matvec(A, lda, m, J, r, kappa, p, q);
    const double alpha = rr / dot(p, q, m);
    for (int64_t i = 0; i < m; ++i) {
      d[i] += alpha * p[i];
      res[i] -= alpha * q[i];
    }
    const double rr_new = dot(res, res, m);
    const double beta = rr_new / rr;
    for (int64_t i = 0; i < m; ++i) p[i] = res[i] + beta * p[i];
    rr = rr_new;
    ++it;
  }
  free(res);
  free(p);
  free(q);
  return it;
}

/* Armijo quantity for eq. line_search:  psi(y + s d) - psi(y).
 * With t = x - sigma A^T y, wd = A^T d, u = prox(t), t(s) = t - s sigma wd,
 * gd = <grad psi(y), d>, dd = ||d||^2, the identity
 *   psi(y+sd) - psi(y) = s gd + s^2/2 dd
 *        + sum_i [ (1+sigma l2)/(2 sigma) (prox(t_i(s))^2 - u_i^2) + s wd_i u_i ]
 * holds exactly (expand Prop. 2 (1) and eq. grad_phy).  A summand whose
 * t_i and t_i(s) lie on the same active side equals s^2 kappa wd_i^2 / 2,
 * which is used in that case; it keeps the difference accurate when it is
 * far below the size of psi itself (near convergence). */
double orc_ls_delta(const double* t, const double* wd, int64_t n, double s, double sigma,
                    double l1, double l2, double gd, double dd) {
  double thr = sigma * l1;
  double den = 1.0 + sigma * l2;
  double kappa = sigma / den;
  double ss = s * sigma;
  double e = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t0 = t[i];
    double t1 = fma(-ss, wd[i], t0);
    double ei;
    if ((t0 > thr && t1 > thr) || (t0 < -thr && t1 < -thr)) {
      ei = 0.5 * s * s * kappa * wd[i] * wd[i];
    } else {
      double u0 = orc_prox_sp(t0, sigma, l1, l2);
      double u1 = orc_prox_sp(t1, sigma, l1, l2);
      ei = den / (2.0 * sigma) * (u1 * u1 - u0 * u0) + s * wd[i] * u0;
    }
    e += ei;
  }
  return s * gd + 0.5 * s * s * dd + e;
}

/* ---------------------------------------------------------------------- */
/* The solve: Algorithm 1 (augmented Lagrangian outer loop, semi-smooth
 * Newton inner loop), with Prop. 2, eq. grad_phy, eq. Q_def, eq. AJ_system,
 * eq. line_search, eq. kkt_res and the settings of Sec. 4.1. */
int orc_en_solve(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                 double l1, double l2, const double* x0, double tol, const orc_opts* o,
                 double* x_out, orc_info* info, double* trace, int32_t trace_cap,
                 int32_t* trace_rows) {
  if (m < 1 || n < 1 || lda < m || !(l1 >= 0.0) || !(l2 >= 0.0) || !(tol > 0.0)) return -1;
  orc_opts opt = {0};
  if (o) opt = *o;
  if (!(opt.sigma_factor > 0.0)) opt.sigma_factor = 5.0;
  if (!(opt.sigma_max > 0.0)) opt.sigma_max = 1e8;
  if (!(opt.mu > 0.0)) opt.mu = 0.2;
  if (!(opt.delta > 0.0)) opt.delta = 0.5;
  if (opt.max_outer <= 0) opt.max_outer = 100;
  if (opt.max_inner <= 0) opt.max_inner = 50;
  if (opt.max_backtrack <= 0) opt.max_backtrack = 30;
  if (opt.cg_maxit <= 0) opt.cg_maxit = 500;
  if (!(opt.cg_eta > 0.0)) opt.cg_eta = 0.1;
  if (!(opt.cg_tau > 0.0)) opt.cg_tau = 0.5;
  if (!(opt.sigma0 > 0.0)) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) { const double* a = COL(A, lda, j); s += dot(a, a, m); }
    double mean = s / (double)n;
    opt.sigma0 = 2.5 / (mean > 0.0 ? mean : 1.0);
  }

  double* x = x_out;
  double* y = (double*)calloc((size_t)m, sizeof(double));
  double* g = (double*)calloc((size_t)m, sizeof(double));
  double* d = (double*)calloc((size_t)m, sizeof(double));
  double* Au = (double*)calloc((size_t)m, sizeof(double));
  double* w = (double*)calloc((size_t)n, sizeof(double));
  double* t = (double*)calloc((size_t)n, sizeof(double));
  double* u = (double*)calloc((size_t)n, sizeof(double));
  double* wd = (double*)calloc((size_t)n, sizeof(double));
  int32_t* J = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  double* uJ = (double*)calloc((size_t)n, sizeof(double));

  /* x0 (or 0); y0 = A x0 - b, the KKT-consistent dual start */
  for (int64_t j = 0; j < n; ++j) x[j] = x0 ? x0[j] : 0.0;
  orc_gemv_n(A, lda, m, n, x, y);
  for (int64_t i = 0; i < m; ++i) y[i] -= b[i];

  double normb = nrm2(b, m);
  double sigma = opt.sigma0;
  double kkt1 = INFINITY, kkt3 = INFINITY, eta = INFINITY;
  /* Inner tolerance: tol, divided by 10 (down to tol/1000) after an outer
   * iteration that met kkt1 and kkt3 but not eta; the decreasing inner
   * tolerances of the criteria the paper refers to for the inner stop. */
  double eps_in = tol;
  int status = 1, stalled = 0, newton = 0, outer = 0, outer_done = 0, rows = 0, cg_iters = 0;
  int64_t r = 0;

  for (outer = 0; outer < opt.max_outer; ++outer) {
    double den = 1.0 + sigma * l2;
    double kappa = sigma / den;
    /* ---- semi-smooth Newton on psi (Algorithm 1, lower half) ---- */
    for (int inner = 0;; ++inner) {
      orc_gemv_t(A, lda, m, n, y, w); /* fresh A^T y */
      r = orc_active_prox(x, w, n, sigma, l1, l2, J, uJ);
      for (int64_t i = 0; i < n; ++i) { t[i] = fma(-sigma, w[i], x[i]); u[i] = 0.0; }
      for (int64_t k = 0; k < r; ++k) u[J[k]] = uJ[k];
      orc_gemv_n(A, lda, m, n, u, Au);
      for (int64_t i = 0; i < m; ++i) g[i] = y[i] + b[i] - Au[i]; /* eq. grad_phy */
      kkt1 = nrm2(g, m) / (1.0 + normb);                          /* eq. kkt_res */
      if (kkt1 <= eps_in || inner >= opt.max_inner) break;
      if (opt.newton_cg && r > 0) {
        /* CG to the relative residual min(cg_eta, kkt1^cg_tau) */
        double eps = pow(kkt1, opt.cg_tau);
        if (eps > opt.cg_eta) eps = opt.cg_eta;
        cg_iters += orc_newton_cg(A, lda, m, J, r, kappa, g, eps, opt.cg_maxit, d);
      } else if (orc_newton_direction(A, lda, m, J, r, kappa, g, d) != 0) {
        stalled = 1;
        break;
      }
      orc_gemv_t(A, lda, m, n, d, wd);
      double gd = dot(g, d, m), dd = dot(d, d, m);
      double s = 1.0;
      int ok = 0;
      for (int k = 0; k <= opt.max_backtrack; ++k) {
        if (orc_ls_delta(t, wd, n, s, sigma, l1, l2, gd, dd) <= opt.mu * s * gd) { ok = 1; break; }
        s *= opt.delta;
      }
      if (trace && rows < trace_cap) {
        double* row = trace + (int64_t)rows * ORC_TRACE_COLS;
        row[0] = outer; row[1] = inner; row[2] = (double)r; row[3] = sigma;
        row[4] = ok ? s : 0.0; row[5] = kkt1;
        ++rows;
      }
      if (!ok) { stalled = 1; break; }
      for (int64_t i = 0; i < m; ++i) y[i] += s * d[i];
      ++newton;
    }
    /* ---- multiplier update (Algorithm 1, step (2)) ---- */
    /* z = prox_{p^* / sigma}(x/sigma - A^T y) (Prop. 2 (2)), from the final inner iterate */
    double zz = 0.0, xu = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double zi = orc_prox_pstar(t[i], sigma, l1, l2);
      zz += zi * zi;
      double e = x[i] - u[i];
      xu += e * e;
    }
    /* A^T y + z = (x - u)/sigma by the Moreau decomposition */
    kkt3 = sqrt(xu) / sigma / (1.0 + nrm2(y, m) + sqrt(zz)); /* eq. kkt_res */
    for (int64_t i = 0; i < n; ++i) x[i] = u[i];           /* x - sigma(A^T y + z) */
    ++outer_done;
    if (kkt1 <= tol && kkt3 <= tol) {
      eta = orc_eta(A, lda, b, m, n, x, l1, l2);
      if (eta <= tol) { status = 0; break; }
      eps_in = eps_in * 0.1 > tol * 1e-3 ? eps_in * 0.1 : tol * 1e-3;
    }
    if (stalled) break;
    sigma = sigma * opt.sigma_factor;
    if (sigma > opt.sigma_max) sigma = opt.sigma_max;
  }
  if (status != 0) {
    eta = orc_eta(A, lda, b, m, n, x, l1, l2);
    if (stalled) status = 2;
  }
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = status;
    info->outer_iters = outer_done;
    info->newton_iters = newton;
    info->cg_iters = cg_iters;
    info->r_final = (int32_t)r;
    int64_t nnz = 0;
    for (int64_t j = 0; j < n; ++j) nnz += (x[j] != 0.0);
    info->nnz = nnz;
    info->eta = eta;
    info->kkt1 = kkt1;
    info->kkt3 = kkt3;
    info->primal_obj = orc_primal_obj(A, lda, b, m, n, x, l1, l2);
    double* res = (double*)malloc(sizeof(double) * (size_t)m);
    orc_gemv_n(A, lda, m, n, x, res);
    for (int64_t i = 0; i < m; ++i) res[i] -= b[i];
    info->dual_obj = orc_dual_obj(A, lda, b, m, n, res, l1, l2);
    free(res);
    info->rel_gap = (info->primal_obj - info->dual_obj) / (1.0 + fabs(info->primal_obj));
    info->sigma_final = sigma;
  }
  if (trace_rows) *trace_rows = rows;
  free(y); free(g); free(d); free(Au); free(w); free(t); free(u); free(wd); free(J); free(uJ);
  return status;
}

/* Model selection at a solution x (Sec. "Parameter tuning", eq. gcv_bic).
 * J = {i : x_i != 0}, r = |J|.
 *   nu   = tr( A_J (A_J^T A_J + lambda2 I_r)^{-1} A_J^T )   (EN degrees of freedom)
 *   beta = argmin ||A_J beta - b||^2                        (least squares on the
 *          selected features: the de-biased estimate; normal equations by
 *          Cholesky, which needs r < m and A_J of full column rank)
 *   rss  = ||A_J beta - b||^2, rss_en = ||A x - b||^2
 *   gcv  = (rss / m) / (1 - nu/m)^2
 *   ebic = log(rss / m) + (nu / m) (log m + log n)
 * out[0..6] = r, nu, rss_en, rss, gcv, ebic, status (0 ok; 1: r >= m, the
 * least-squares fit is not determined and rss/gcv/ebic are NaN; 2: A_J^T A_J
 * not positive definite, likewise).  beta_out (n, nullable) gets beta
 * scattered to J (zeros elsewhere).  nu follows its definition directly:
 * Z = (A_J^T A_J + lambda2 I)^{-1} A_J^T by Cholesky and m right-hand sides,
 * then the trace of A_J Z. */
void orc_model_select(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                      double lambda2, const double* x, double* out, double* beta_out) {
  int64_t r = 0;
  for (int64_t i = 0; i < n; ++i) r += x[i] != 0.0;
  int32_t* J = (int32_t*)malloc(sizeof(int32_t) * (size_t)(r > 0 ? r : 1));
  r = 0;
  for (int64_t i = 0; i < n; ++i)
    if (x[i] != 0.0) J[r++] = (int32_t)i;
  const double NaN = 0.0 / 0.0;
  /* rss of the EN estimate */
  double* res = (double*)malloc(sizeof(double) * (size_t)m);
  orc_gemv_n(A, lda, m, n, x, res);
  double rss_en = 0.0;
  for (int64_t i = 0; i < m; ++i) {
    res[i] -= b[i];
    rss_en += res[i] * res[i];
  }
  /* G = A_J^T A_J */
  double* G = (double*)malloc(sizeof(double) * (size_t)(r * r > 0 ? r * r : 1));
  for (int64_t p = 0; p < r; ++p)
    for (int64_t q = 0; q < r; ++q) {
      double s = 0.0;
      for (int64_t i = 0; i < m; ++i) s += A[J[p] * lda + i] * A[J[q] * lda + i];
      G[p * r + q] = s;
    }
  /* nu: L L^T = G + lambda2 I, Z = L^{-T} L^{-1} A_J^T column by column */
  double nu = 0.0;
  if (r > 0) {
    double* M = (double*)malloc(sizeof(double) * (size_t)(r * r));
    for (int64_t k = 0; k < r * r; ++k) M[k] = G[k];
    for (int64_t p = 0; p < r; ++p) M[p * r + p] += lambda2;
    if (orc_cholesky(M, r) != 0) {
      nu = NaN;
    } else {
      double* z = (double*)malloc(sizeof(double) * (size_t)r);
      for (int64_t i = 0; i < m; ++i) {
        /* z = M^{-1} (row i of A_J)^T; nu += (row i of A_J) . z */
        for (int64_t p = 0; p < r; ++p) {
          double s = A[J[p] * lda + i];
          for (int64_t k = 0; k < p; ++k) s -= M[p * r + k] * z[k];
          z[p] = s / M[p * r + p];
        }
        for (int64_t p = r - 1; p >= 0; --p) {
          double s = z[p];
          for (int64_t k = p + 1; k < r; ++k) s -= M[k * r + p] * z[k];
          z[p] = s / M[p * r + p];
        }
        for (int64_t p = 0; p < r; ++p) nu += A[J[p] * lda + i] * z[p];
      }
      free(z);
    }
    free(M);
  }
  /* least squares on J */
  double rss = NaN, gcv = NaN, ebic = NaN, status = 0.0;
  double* beta = (double*)malloc(sizeof(double) * (size_t)(r > 0 ? r : 1));
  if (r >= m) {
    status = 1.0;
  } else {
    int ok = 1;
    if (r > 0) {
      double* M = (double*)malloc(sizeof(double) * (size_t)(r * r));
      for (int64_t k = 0; k < r * r; ++k) M[k] = G[k];
      if (orc_cholesky(M, r) != 0) {
        ok = 0;
      } else {
        for (int64_t p = 0; p < r; ++p) {
          double s = 0.0;
          for (int64_t i = 0; i < m; ++i) s += A[J[p] * lda + i] * b[i];
          for (int64_t k = 0; k < p; ++k) s -= M[p * r + k] * beta[k];
          beta[p] = s / M[p * r + p];
        }
        for (int64_t p = r - 1; p >= 0; --p) {
          double s = beta[p];
          for (int64_t k = p + 1; k < r; ++k) s -= M[k * r + p] * beta[k];
          beta[p] = s / M[p * r + p];
        }
      }
      free(M);
    }
    if (!ok) {
      status = 2.0;
    } else {
      rss = 0.0;
      for (int64_t i = 0; i < m; ++i) {
        double s = -b[i];
        for (int64_t p = 0; p < r; ++p) s += A[J[p] * lda + i] * beta[p];
        rss += s * s;
      }
      const double md = (double)m;
      gcv = (rss / md) / ((1.0 - nu / md) * (1.0 - nu / md));
      ebic = log(rss / md) + (nu / md) * (log(md) + log((double)n));
    }
  }
  if (beta_out) {
    for (int64_t i = 0; i < n; ++i) beta_out[i] = 0.0;
    if (status == 0.0)
      for (int64_t p = 0; p < r; ++p) beta_out[J[p]] = beta[p];
  }
  out[0] = (double)r;
  out[1] = nu;
  out[2] = rss_en;
  out[3] = rss;
  out[4] = gcv;
  out[5] = ebic;
  out[6] = status;
  free(beta);
  free(G);
  free(res);
  free(J);
}

/* k-fold cross validation on a lambda grid (Sec. "Parameter tuning": the
 * k-fold criterion costs k extra solves per (lambda1, lambda2)).
 * fold[i] in [0, k) assigns row i to a validation fold.  The grid is the
 * full data's: lam_q = c_lambda[q] * ||A^T b||_inf / alpha, lambda1 = alpha
 * lam_q, lambda2 = (1 - alpha) lam_q.  For each fold f: the rows with
 * fold != f form the training problem, solved along the grid in order, each
 * point warm-started from the previous one (tol as given, default options);
 * err[f*nlam + q] = mean over the rows of fold f of (A x_q - b)^2.
 * Returns 0, or the first failing solve's status. */
int orc_cv(const double* A, int64_t lda, const double* b, int64_t m, int64_t n, const int32_t* fold,
           int k, double alpha, const double* c_lambda, int nlam, double tol, double* err) {
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  orc_gemv_t(A, lda, m, n, b, w);
  double amax = 0.0;
  for (int64_t j = 0; j < n; ++j) amax = fabs(w[j]) > amax ? fabs(w[j]) : amax;
  free(w);
  const double lam_max = amax / alpha;
  int worst = 0;
  double* At = (double*)malloc(sizeof(double) * (size_t)(m * n));
  double* bt = (double*)malloc(sizeof(double) * (size_t)m);
  double* x = (double*)malloc(sizeof(double) * (size_t)n);
  double* xprev = (double*)malloc(sizeof(double) * (size_t)n);
  double* res = (double*)malloc(sizeof(double) * (size_t)m);
  for (int f = 0; f < k; ++f) {
    int64_t mt = 0, mv = 0;
    for (int64_t i = 0; i < m; ++i) {
      if (fold[i] == f) { ++mv; continue; }
      bt[mt++] = b[i];
    }
    for (int64_t j = 0; j < n; ++j) {
      int64_t r = 0;
      for (int64_t i = 0; i < m; ++i)
        if (fold[i] != f) At[j * mt + r++] = A[j * lda + i];
    }
    for (int q = 0; q < nlam; ++q) {
      const double lam = c_lambda[q] * lam_max;
      orc_info info;
      const int rc = orc_en_solve(At, mt, bt, mt, n, alpha * lam, (1.0 - alpha) * lam,
                                  q > 0 ? xprev : NULL, tol, NULL, x, &info, NULL, 0, NULL);
      if (rc != 0 && worst == 0) worst = rc;
      orc_gemv_n(A, lda, m, n, x, res);
      double s = 0.0;
      for (int64_t i = 0; i < m; ++i)
        if (fold[i] == f) s += (res[i] - b[i]) * (res[i] - b[i]);
      err[(int64_t)f * nlam + q] = mv > 0 ? s / (double)mv : NAN;
      memcpy(xprev, x, sizeof(double) * (size_t)n);
    }
  }
  free(At); free(bt); free(x); free(xprev); free(res);
  return worst;
}
