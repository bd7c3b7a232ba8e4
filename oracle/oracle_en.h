/*
 * FP64 CPU oracle for the SsNAL-EN elastic-net solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU solver shares
 * no code with it and never calls it.
 *
 * Problem (Sec. 1, eq. objective_function):
 *     min_x F(x) = 1/2 ||A x - b||^2 + lambda1 ||x||_1 + lambda2/2 ||x||^2
 * with A (m x n) column-major, leading dimension lda >= m.
 *
 * Everything is IEEE binary64, round to nearest even, built without
 * floating-point contraction; sums run left to right.  The one fused
 * operation is t = x - sigma*w, written fma(-sigma, w, x) on purpose (it
 * decides the active set; see orc_active_prox).
 *
 * Parity status of each entry point is stated at its definition in
 * oracle_en.c.
 */
#ifndef ORACLE_EN_H
#define ORACLE_EN_H
#include <stdint.h>

typedef struct {
  double sigma0;       /* <= 0: 2.5 / mean_j ||a_j||^2 */
  double sigma_factor; /* <= 0: 5 */
  double sigma_max;    /* <= 0: 1e8 */
  double mu;           /* <= 0: 0.2 */
  double delta;        /* <= 0: 0.5 */
  int32_t max_outer;   /* <= 0: 100 */
  int32_t max_inner;   /* <= 0: 50 */
  int32_t max_backtrack; /* <= 0: 30 */
  int32_t newton_cg;   /* 0: Cholesky of the m x m system; 1: conjugate gradients */
  int32_t cg_maxit;    /* <= 0: 500 */
  double cg_eta;       /* <= 0: 0.1; CG stops at ||V d + g|| <= min(cg_eta, kkt1^cg_tau) ||g|| */
  double cg_tau;       /* <= 0: 0.5 */
} orc_opts;

typedef struct {
  int32_t status;      /* 0 converged, 1 not converged, 2 line search stalled */
  int32_t outer_iters;
  int32_t newton_iters;
  int32_t r_final;
  int64_t nnz;
  double eta, kkt1, kkt3, primal_obj, dual_obj, rel_gap, sigma_final;
  int32_t cg_iters;    /* conjugate-gradient iterations over all Newton steps */
} orc_info;

/* One row per Newton iteration: outer, inner, r, sigma, step, kkt1 */
#define ORC_TRACE_COLS 6

/* Host threads for the loops whose outputs are independent sums (A^T v, A x,
 * the Newton matrices, the entries below each Cholesky pivot).  Results do
 * not depend on the count.  Default 1. */
void orc_set_threads(int k);
int orc_get_threads(void);

/* primitives */
double orc_prox_sp(double t, double sigma, double l1, double l2);
double orc_prox_pstar(double v, double sigma, double l1, double l2);
double orc_pstar(const double* z, int64_t n, double l1, double l2);
void orc_gemv_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* v, double* w);
void orc_gemv_n(const double* A, int64_t lda, int64_t m, int64_t n, const double* x, double* out);
double orc_primal_obj(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                      const double* x, double l1, double l2);
double orc_dual_obj(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                    const double* y, double l1, double l2);
double orc_eta(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
               const double* x, double l1, double l2);
double orc_psi(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
               const double* x, const double* y, double sigma, double l1, double l2);
void orc_grad_psi(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                  const double* x, const double* y, double sigma, double l1, double l2, double* g);
int64_t orc_active_prox(const double* x, const double* w, int64_t n, double sigma, double l1,
                        double l2, int32_t* J, double* uJ);
void orc_newton_matrix(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                       double kappa, double* V);
void orc_smw_matrix(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                    double kappa, double* W);
int orc_cholesky(double* V, int64_t m);
int orc_newton_direction(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                         double kappa, const double* g, double* d);
void orc_newton_matvec(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                       double kappa, const double* p, double* q);
int orc_newton_cg(const double* A, int64_t lda, int64_t m, const int32_t* J, int64_t r,
                  double kappa, const double* g, double eps, int32_t maxit, double* d);
double orc_ls_delta(const double* t, const double* wd, int64_t n, double s, double sigma,
                    double l1, double l2, double gd, double dd);

/* whole solve; trace may be NULL (trace_cap rows of ORC_TRACE_COLS doubles) */
int orc_en_solve(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                 double l1, double l2, const double* x0, double tol, const orc_opts* opts,
                 double* x_out, orc_info* info, double* trace, int32_t trace_cap,
                 int32_t* trace_rows);

/* Model selection at a solution x (Sec. "Parameter tuning", eq. gcv_bic):
 * out[0..6] = r, nu, rss_en, rss (de-biased), gcv, ebic, status. */
void orc_model_select(const double* A, int64_t lda, const double* b, int64_t m, int64_t n,
                      double lambda2, const double* x, double* out, double* beta_out);

/* k-fold cross validation on the full data's lambda grid: err (k x nlam) =
 * mean squared validation error per fold and point. */
int orc_cv(const double* A, int64_t lda, const double* b, int64_t m, int64_t n, const int32_t* fold,
           int k, double alpha, const double* c_lambda, int nlam, double tol, double* err);

#endif
