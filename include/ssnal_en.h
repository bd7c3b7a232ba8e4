/*
 * ssnal_en.h -- C ABI of the MI355X (gfx950) SsNAL-EN elastic-net solver.
 *
 * Problem (Sec. 1, eq. objective_function):
 *     min_x  1/2 ||A x - b||^2 + lambda1 ||x||_1 + lambda2/2 ||x||^2,
 * A in R^{m x n} with n >> m, solved by the semi-smooth Newton augmented
 * Lagrangian method of Sec. 3 (Algorithm 1): an augmented-Lagrangian outer
 * loop on the dual (D) whose sub-problem, min_y psi(y) of Prop. 2, is solved
 * by a semi-smooth Newton method with the reduced system eq. AJ_system (or its
 * r x r form eq. smw_formula) and the line search eq. line_search.
 *
 * Conventions shared by every entry point
 *   - Arrays are DEVICE pointers owned by the caller (e.g. torch tensors),
 *     unless a parameter says "host".
 *   - A is column-major with leading dimension lda >= m, stored as
 *     ssnal_dtype: FP64, FP32 or BF16 (bfloat16 bit patterns, uint16).
 *     Offsets are 64-bit: m*n may exceed 2^31.  The streaming kernels read
 *     16 bytes per lane when A is 16-byte aligned and lda*sizeof(elem) is a
 *     multiple of 16; other layouts take a slower element-wise path.
 *     Entries of A in rows m..lda-1 are never used.
 *   - b, x0, x_out, and every other vector are FP64, contiguous.
 *   - Work is enqueued on `stream` (a hipStream_t; 0 = null stream).  Calls
 *     that report results to the host return after their work completes.
 *   - One ssnal_ctx per device and per host thread; a context is not
 *     thread-safe.  Calls on one context serialise.
 *   - Return value: 0 success; > 0 a result with a warning; < 0 an error, with
 *     a message available from ssnal_last_error() (per calling thread).  The
 *     library never aborts the process.
 */
#ifndef SSNAL_EN_H
#define SSNAL_EN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* storage type of A */
typedef enum { SSNAL_F64 = 0, SSNAL_F32 = 1, SSNAL_BF16 = 2 } ssnal_dtype;

/* status codes */
#define SSNAL_OK 0
#define SSNAL_NOT_CONVERGED 1     /* max_outer reached; x_out holds the last iterate */
#define SSNAL_LINESEARCH_STALL 2  /* no trial step passed eq. line_search and eta > tol */
#define SSNAL_PATH_TRUNCATED 3    /* ssnal_en_path stopped early at max_active nonzeros */
#define SSNAL_EINVAL (-1)         /* invalid argument (message says which) */
#define SSNAL_ENONFINITE (-2)     /* NaN or Inf in b, x0 or A^T b */
#define SSNAL_ENOMEM (-3)         /* device workspace allocation failed */
#define SSNAL_EHIP (-4)           /* a HIP runtime call failed */
#define SSNAL_ENUMERIC (-5)       /* Cholesky met a non-positive pivot */

typedef struct ssnal_ctx ssnal_ctx;

/*
 * Solver options.  Zero (or negative) fields take the defaults, so a
 * zero-initialised struct is the default configuration.  The defaults are
 * the settings of Sec. 4.1 (mu = 0.2, sigma multiplied by 5 per outer
 * iteration) with sigma0 scaled to the column norms (5e-3 at squared norm
 * 500, the setting of Sec. 4.1).
 */
typedef struct {
  double sigma0;         /* <= 0: 2.5 / mean_j ||a_j||^2 */
  double sigma_factor;   /* <= 0: 5 */
  double sigma_max;      /* <= 0: 1e8 */
  double mu;             /* <= 0: 0.2, Armijo constant of eq. line_search */
  double delta;          /* <= 0: 0.5, backtracking factor */
  int32_t max_outer;     /* <= 0: 100 augmented-Lagrangian iterations */
  int32_t max_inner;     /* <= 0: 50 Newton iterations per sub-problem */
  int32_t max_backtrack; /* <= 0: 30 (trial steps 1, delta, ..., delta^30; at most 31) */
  int32_t no_refine;     /* FP32/BF16 storage: 0 = refresh A^T y with FP64 accumulation
                            before each multiplier update (default); 1 = never */
  int32_t no_smw;        /* 0 = r < m uses the r x r system of eq. smw_formula (default);
                            1 = always the m x m system of eq. AJ_system */
  int32_t timing;        /* 1 = time every A^T v launch with HIP events (info->gemv_ms) */
  int32_t trace_cap;     /* rows available in `trace` (0 = no trace) */
  double* trace;         /* HOST, nullable: one row per Newton iteration:
                            outer, inner, r, sigma, step, kkt1 (6 doubles) */
  int32_t newton_cg;     /* 0 = factor the Newton system while it fits (m <= 4096, or
                            r < m and r <= 4096 for the Woodbury form), conjugate
                            gradients beyond (default); 1 = conjugate gradients always */
  int32_t cg_maxit;      /* <= 0: 500 conjugate-gradient iterations per Newton step */
  double cg_eta;         /* <= 0: 0.1; < 1; CG stops at ||V d + g|| <= min(cg_eta, kkt1^cg_tau) ||g|| */
  double cg_tau;         /* <= 0: 0.5 */
  int32_t workers;       /* ssnal_en_solve_batch: <= 0: 8 concurrent workers (own context and
                            stream each, kept by the context); 1 = every problem in turn on
                            the caller's stream */
  int32_t no_small;      /* 0 = a problem with A in FP64, m <= 120 and either m n <= 2^17
                            or n <= (150112 - 16 ceil(m (m + 1) / 4)) / 36 (its n-vectors
                            fit in LDS: n <= 3047 at m = 100) runs its whole solve
                            (Algorithm 1: both loops, the stopping tests, the certificates)
                            in one workgroup, one launch and one host wait, unless trace,
                            timing or newton_cg is asked for; a batch runs its such
                            problems (m n <= 2^21) as one launch, one workgroup each
                            (default); 1 = never */
} ssnal_en_opts;

typedef struct {
  int32_t status;        /* same code as the return value */
  int32_t outer_iters;   /* multiplier updates performed */
  int32_t newton_iters;  /* Newton steps taken */
  int32_t r_final;       /* |J| at the last iterate = nonzeros of x */
  int64_t nnz;
  double kkt_rel;        /* eta(x) = ||x - prox_p(x - A^T(Ax-b))|| / (1+||x||+||Ax-b||),
                            FP64 accumulation over the stored A; the gated residual */
  double kkt1;           /* eq. kkt_res, first residual, at the last iterate */
  double kkt3;           /* eq. kkt_res, third residual, at the last multiplier update */
  double primal_obj;     /* F(x) */
  double dual_obj;       /* D(Ax - b), Prop. 1 conjugate */
  double rel_gap;        /* (F - D) / (1 + |F|) */
  double sigma_final;
  int32_t gemv_calls;    /* full A^T v passes over the n columns */
  int32_t syncs;         /* device-to-host synchronisations */
  double gemv_ms;        /* with opts.timing: summed durations of the A^T v launches */
  double solve_ms;       /* host wall time of the call */
  int32_t atd_launches;  /* with opts.timing: launches of the Newton pass w_d = A^T d ... */
  double atd_ms;         /* ... and their summed durations (HIP events on the solve's stream) */
  int32_t cg_iters;      /* conjugate-gradient iterations over all Newton steps */
  double sigma0;         /* the initial penalty the solve used (a warm-started path point
                            that continues from this one passes min(sigma_final, cap)) */
  double queue_ms;       /* serving: submission -> admission to a slot (host clock) */
  double upload_ms;      /* serving, host-resident request: the upload of A, b and x0
                            (HIP events on the slot's stream); 0 otherwise */
  int32_t chol_calls;    /* with opts.timing: Cholesky factor + solve calls of the Newton
                            directions ... */
  double chol_ms;        /* ... their summed durations (HIP events on the solve's stream) ... */
  double chol_gflop;     /* ... and their summed N^3/3 flops, in GFLOP */
  int32_t one_workgroup; /* 1 when the solve ran in one workgroup (see opts.no_small) */
} ssnal_en_info;

/* Fill *opts with the defaults listed above. */
void ssnal_en_opts_init(ssnal_en_opts* opts);

/*
 * Create a context on `device` (HIP ordinal).  The context owns the device
 * workspace, sized lazily to the largest problem seen; it holds O(n) FP64
 * vectors, an N x N FP64 matrix (N = min(m, 4096)), split-K partial sums
 * (bounded by (2048 + (N/64)^2) * 32 KiB) and up to 1025 m-vectors of gathered
 * partial sums.  Returns 0 or an error code.
 */
int ssnal_ctx_create(int device, ssnal_ctx** out);
void ssnal_ctx_destroy(ssnal_ctx* ctx);

/* Message of the last error on the calling thread ("" if none). */
const char* ssnal_last_error(void);

/*
 * One elastic-net solve (Algorithm 1).
 *   A, a_dtype, lda, m, n : the design (see conventions); 1 <= m <= 2^20, n >= 1.
 *                           The Newton system (eq. newton_direction) is factored
 *                           while it fits 4096 x 4096 (m x m, or r x r by eq.
 *                           smw_formula when r < m) and solved by conjugate
 *                           gradients beyond (Sec. 3.2), see opts.newton_cg.
 *   b                     : m responses.
 *   lambda1 >= 0, lambda2 >= 0: the penalty of eq. objective_function (unscaled;
 *                           callers using a 1/m-scaled loss multiply by m);
 *                           lambda2 = 0 is the Lasso limit, whose certificate
 *                           takes the dual objective at theta*(A x - b), theta =
 *                           min(1, lambda1/|A^T(A x - b)|_inf) (p* is then the
 *                           indicator of |z|_inf <= lambda1).
 *   x0                    : n starting coefficients (warm start) or NULL for 0.
 *   tol > 0               : stop when kkt1 <= tol, kkt3 <= tol and eta <= tol.
 *   x_out                 : n coefficients on return (may alias x0).
 *   opts                  : NULL for defaults.   info: HOST, nullable.
 * FP32/BF16 storage runs the A^T v passes and the Newton matrix with FP32
 * accumulation and refreshes A^T y with FP64 accumulation before each
 * multiplier update; the KKT residual, the objectives, the Cholesky factor and
 * the line-search sums are FP64 in every mode.
 */
int ssnal_en_solve(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda,
                   const double* b, int64_t m, int64_t n, double lambda1, double lambda2,
                   const double* x0, double tol, hipStream_t stream, double* x_out,
                   const ssnal_en_opts* opts, ssnal_en_info* info);

/*
 * ssnal_en_solve without allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, semantics and results as
 * ssnal_en_solve; the device workspace lives in one static device array of
 * 48 MiB per device (held from the library's load until the process ends)
 * instead of the context's buffers, so the call makes no hipMalloc, hipFree
 * or other allocation.  The context still supplies its scalar slots and
 * pinned read-back memory (allocated when it was created).
 * Limits: m <= 512 and n <= 131072 (sizes beyond: SSNAL_EINVAL), opts->timing
 * and opts->newton_cg must be 0 (SSNAL_EINVAL).  Every call on a device shares
 * that device's array: calls that overlap on one device (several host threads
 * or streams) race and must be serialised by the caller.
 */
int ssnal_en_solve_noalloc(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda,
                           const double* b, int64_t m, int64_t n, double lambda1, double lambda2,
                           const double* x0, double tol, hipStream_t stream, double* x_out,
                           const ssnal_en_opts* opts, ssnal_en_info* info);

/*
 * Regularisation path with warm starts (Sec. 3.3: each solve starts from the
 * solution at the previous, larger lambda).
 *   alpha in (0, 1]       : mixing weight (1: the Lasso); point k solves lambda1 = alpha*lam_k,
 *                           lambda2 = (1 - alpha)*lam_k with lam_k = c_lambda[k]*lam_max,
 *                           lam_max = ||A^T b||_inf / alpha (the smallest lam with
 *                           solution 0), computed with FP64 accumulation over the
 *                           stored A.
 *   c_lambda              : HOST, nlam factors > 0, normally decreasing.
 *   max_active            : 0 = off; else the path stops after the first point with
 *                           more than max_active nonzeros (later columns of X_out are
 *                           zero and their infos carry SSNAL_PATH_TRUNCATED).
 *   X_out                 : n x nlam, column-major (column k = point k); the state
 *                           never leaves the device between points.
 *   opts                  : as for ssnal_en_solve; when opts->sigma0 is not set,
 *                           point k > 0 starts from the final sigma of point k-1,
 *                           capped at sigma0 * sigma_factor^4 of the cold default.
 *   infos                 : HOST, nullable, nlam entries.
 * Returns the most severe status over the points (an error stops the path).
 */
int ssnal_en_path(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, const double* b,
                  int64_t m, int64_t n, double alpha, const double* c_lambda, int nlam,
                  int64_t max_active, double tol, hipStream_t stream, double* X_out,
                  const ssnal_en_opts* opts, ssnal_en_info* infos);

/*
 * k-fold cross validation on a lambda grid (Sec. "Parameter tuning": k extra
 * solves per (lambda1, lambda2) and fold), as k warm-started paths over the
 * full data's grid lam_q = c_lambda[q] * ||A^T b||_inf / alpha (lambda1 = alpha
 * lam_q, lambda2 = (1 - alpha) lam_q):
 *   fold     : device, m int32 labels in [0, k); fold f validates its rows and
 *              trains on the others (each fold needs both).
 *   err_out  : HOST, k x nlam (row f = fold f): mean over the rows of fold f of
 *              (A x_q - b)^2, x_q the fold's solution at point q.
 *   infos    : HOST, nullable, k x nlam.
 *   slots    : folds run concurrently on min(slots, k) workers (1..64), each
 *              with its own context and stream, created on first use and kept
 *              by ctx (1: every fold in turn on `stream`).  Each fold's work is
 *              independent of the others, so the results do not depend on slots.
 * The training rows of a fold are copied into a buffer of its worker ((m-1) x n
 * elements of A's storage type, plus the path: nlam x n doubles); alpha in
 * (0, 1].  `stream` orders the call after the caller's earlier work
 * (the call synchronises it before the workers start).  Returns the most
 * severe status over the solves (an error stops).
 */
int ssnal_en_cv(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, const double* b,
                int64_t m, int64_t n, const int32_t* fold, int k, double alpha,
                const double* c_lambda, int nlam, double tol, int slots, hipStream_t stream,
                const ssnal_en_opts* opts, double* err_out, ssnal_en_info* infos);

/* where the arrays of a problem live */
#define SSNAL_ON_DEVICE 0
#define SSNAL_ON_HOST 1

/* One problem of a batch or of the serving loop (fields as in ssnal_en_solve). */
typedef struct {
  const void* A;
  ssnal_dtype a_dtype;
  int64_t lda, m, n;
  const double* b;
  double lambda1, lambda2;
  const double* x0;  /* nullable */
  double tol;
  double* x_out;
  double sigma0;       /* > 0: this problem's initial penalty, overriding opts->sigma0 (a
                          warm-started path point passes the sigma its predecessor ended
                          with, as ssnal_en_path does); <= 0: opts / default */
  int32_t location;    /* SSNAL_ON_DEVICE: A, b, x0, x_out are device pointers.
                          SSNAL_ON_HOST (serving only): they are host memory (pinned for
                          asynchronous uploads); the server uploads A, b and x0 into
                          device buffers of the slot on admission and copies x back */
  hipEvent_t ready;    /* nullable, device-resident problems: the solve's stream waits for
                          this event before reading A, b and x0 (record it on the stream
                          that wrote them); without it the caller must have completed
                          those writes before submitting */
} ssnal_en_problem;

/*
 * Model selection at a solution (Sec. "Parameter tuning", eq. gcv_bic), for
 * choosing (lambda1, lambda2) along a path:
 *   J = {i : x_i != 0}, r = |J|;
 *   nu   = tr(A_J (A_J^T A_J + lambda2 I_r)^{-1} A_J^T), the elastic-net degrees
 *          of freedom, computed as r - lambda2 ||L^{-1}||_F^2 with L L^T =
 *          A_J^T A_J + lambda2 I_r (r < m), or as m - lambda2 ||L^{-1}||_F^2 with
 *          L L^T = A_J A_J^T + lambda2 I_m (r >= m);
 *   beta = the least-squares fit of b on the columns J (the de-biased
 *          estimate), by Cholesky of A_J^T A_J (needs 0 < r < m and A_J of full
 *          column rank);
 *   rss  = ||A_J beta - b||^2 (||b||^2 when r = 0), rss_en = ||A x - b||^2;
 *   gcv  = (rss/m) / (1 - nu/m)^2,  ebic = log(rss/m) + (nu/m)(log m + log n).
 * The Gram matrices read A with the storage's accumulation (FP32 for F32/BF16
 * storage, as in the Newton matrix); the factorisations, solves and
 * reductions are FP64.  x, b: device, n and m doubles; beta_out: device, n
 * doubles (nullable; beta scattered to J, zero elsewhere); out: HOST.
 * status in out: 0 ok; 1 r >= m (the least-squares fit is not determined:
 * rss, gcv, ebic are NaN, beta_out zero); 2 A_J^T A_J not positive definite
 * (likewise).  Needs lambda2 >= 0 and min(r, m) <= 4096 (any m when the support
 * has at most 4096 features); with lambda2 = 0 a singular
 * Gram matrix returns SSNAL_ENUMERIC.
 */
typedef struct {
  int32_t status;
  int32_t r;
  double nu, rss_en, rss, gcv, ebic;
} ssnal_en_select;
int ssnal_en_model_select(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda,
                          const double* b, int64_t m, int64_t n, double lambda2, const double* x,
                          hipStream_t stream, double* beta_out, ssnal_en_select* out);

/* Independent solves (k-fold or grid-search style) of device-resident
 * problems.  Problems with A in FP64, m <= 120 and m n <= 2^21 (unless
 * opts->no_small, trace, timing or newton_cg) run as one launch on `stream`,
 * one workgroup each; the others run on opts->workers concurrent workers
 * (default 8; each a context and stream of its own, created on first use and
 * kept by ctx) that start after the caller's earlier work on `stream` and
 * each problem's `ready` event; with opts->workers = 1, one after the other
 * on `stream` with ctx's workspace.  Every solve's result is the same bits
 * under any worker count, and the bits of the same problem solved alone when
 * both take the same path (the limits of a single solve in one workgroup
 * are at opts->no_small; see info->one_workgroup); otherwise the two agree
 * to rounding.
 * Returns after every solve has completed.  infos: HOST, nullable, count
 * entries.  Returns the most severe status; an error stops handing out
 * problems. */
int ssnal_en_solve_batch(ssnal_ctx* ctx, const ssnal_en_problem* problems, int count,
                         const ssnal_en_opts* opts, hipStream_t stream, ssnal_en_info* infos);

/*
 * Serving loop (continuous batching of independent solves): a slot table of
 * up to max_slots concurrent solves on one device.  Each slot owns a context
 * and a HIP stream (default priority) and is driven by its own host thread,
 * so the latency-bound phases of different requests overlap on the GPU.
 *
 * Admission by HBM footprint: a request is admitted to an idle slot when its
 * footprint, ssnal_srv_footprint (the context workspace for its (m, n), plus
 * for a host-resident request the device copies of A, b and x), fits in
 * hbm_budget bytes next to what the other slots hold.  Among the queued
 * requests that fit, the one with the smallest estimated work (its passes
 * over A and its Newton factorisations) goes first, so small requests do not
 * wait behind multi-gigabyte ones; a request that has been passed over
 * 4*max_slots times is admitted next, before any other (no starvation).  When
 * nothing runs and the oldest request does not fit, idle slots release their
 * buffers.  A host-resident request is uploaded on its slot's stream on
 * admission (info->upload_ms) and its x copied back before completion.
 *
 * A request's reductions have a fixed tiling that depends only on its (m, n),
 * so its result is bitwise the same alone or in the mix.  Pointers in a
 * submitted problem (and its ready event) must stay valid until its ticket
 * completes.
 */
typedef struct ssnal_srv ssnal_srv;
int ssnal_srv_create(int device, size_t hbm_budget, int max_slots, const ssnal_en_opts* opts,
                     ssnal_srv** out);
/* Non-blocking; *ticket identifies the request. */
int ssnal_srv_submit(ssnal_srv* srv, const ssnal_en_problem* problem, uint64_t* ticket);
/* 1 = pending; otherwise the request's status (its result is in problem->x_out)
 * and *info (HOST, nullable) is filled; a ticket can be collected once. */
int ssnal_srv_poll(ssnal_srv* srv, uint64_t ticket, ssnal_en_info* info);
/* Blocks until the ticket completes; returns its status. */
int ssnal_srv_wait(ssnal_srv* srv, uint64_t ticket, ssnal_en_info* info);
/* Finishes every admitted and queued request, then frees the slots. */
void ssnal_srv_destroy(ssnal_srv* srv);
/* Workspace bytes a context holds for an (m, n) problem. */
size_t ssnal_workspace_bytes(int64_t m, int64_t n);
/* Device bytes a served problem occupies while it runs (the admission
 * footprint): ssnal_workspace_bytes(m, n), plus m*n*sizeof(elem) + (m + n)*8
 * for a host-resident problem.  0 for an invalid problem. */
size_t ssnal_srv_footprint(const ssnal_en_problem* problem);

/* ---------------------------------------------------------------------
 * Building blocks of the solve, exported for verification and benchmarking.
 * Each runs the same kernels the solve runs.
 * --------------------------------------------------------------------- */

/* w = A^T v over all n columns (the HBM pass of every Newton iteration).
 * acc64 != 0: FP64 accumulation; else the storage's own (FP64 for F64,
 * FP32 for F32/BF16).  v: m doubles, w: n doubles. */
int ssnal_gemv_t(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, int64_t m,
                 int64_t n, const double* v, double* w, int acc64, hipStream_t stream);

/* Active set and prox at t = fma(-sigma, w, x) (eq. Q_def, eq. prox_elastic):
 * J = {i : |t_i| > sigma*lambda1} ascending (int32, capacity n), uJ = prox_{sigma p}(t)_J.
 * *r_out (HOST) receives |J|. */
int ssnal_active_prox(ssnal_ctx* ctx, const double* x, const double* w, int64_t n, double sigma,
                      double lambda1, double lambda2, int32_t* J, double* uJ, int64_t* r_out,
                      hipStream_t stream);

/* Newton matrix (eq. AJ_system / eq. smw_formula) for the active columns J (r entries):
 * form 0: out = I_m + kappa A_J A_J^T (m x m); form 1: out = I_r / kappa + A_J^T A_J (r x r).
 * out: N x N row-major FP64 (N = m or r), both triangles written; N <= 4096
 * (SSNAL_EINVAL beyond). */
int ssnal_newton_matrix(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda,
                        int64_t m, const int32_t* J, int64_t r, double kappa, int form,
                        double* out, hipStream_t stream);

/* In-place FP64 Cholesky of an SPD N x N row-major matrix: on return the lower
 * triangle holds L (V = L L^T) and the strict upper triangle is zero.
 * 1 <= N <= 4096.  Returns SSNAL_ENUMERIC for a non-positive pivot. */
int ssnal_cholesky(ssnal_ctx* ctx, double* V, int64_t N, hipStream_t stream);

/* Newton direction d = -(I + kappa A_J A_J^T)^{-1} g (eq. AJ_system), by the
 * m x m system (form 0), the r x r system of eq. smw_formula (form 1), or the
 * solver's own choice (form -1: r x r when 0 < r < m). g, d: m doubles.  The
 * factored system must fit 4096 x 4096 (SSNAL_EINVAL otherwise; larger systems
 * take ssnal_newton_cg). */
int ssnal_newton_direction(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda,
                           int64_t m, const int32_t* J, int64_t r, double kappa, const double* g,
                           double* d, int form, hipStream_t stream);

/* Approximate Newton direction by conjugate gradients (Sec. 3.2, the
 * approximate solve of eq. newton_direction for large m and r): CG on
 * (I + kappa A_J A_J^T) d = -g from d = 0, with the product applied as
 * p + kappa A_J (A_J^T p) (never formed), stopping once the recursive residual
 * has ||res|| <= eps ||g|| or after maxit iterations.  Any m <= 2^20, any r.
 * J: device, r ascending column indices; g, d: device, m doubles;
 * iters: HOST, nullable, the iterations taken.  Synchronises the stream. */
int ssnal_newton_cg(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, int64_t m,
                    const int32_t* J, int64_t r, double kappa, const double* g, double eps,
                    int32_t maxit, hipStream_t stream, double* d, int32_t* iters);

/* Line-search increments psi(y + s_k d) - psi(y) (Prop. 2 (1), eq. line_search)
 * for K <= 32 trial steps s (HOST), from x, w = A^T y, wd = A^T d (n doubles
 * each), gd = <grad psi(y), d>, dd = |d|^2.  delta_out: HOST, K doubles. */
int ssnal_ls_delta(ssnal_ctx* ctx, const double* x, const double* w, const double* wd, int64_t n,
                   double sigma, double lambda1, double lambda2, double gd, double dd, int K,
                   const double* s, double* delta_out, hipStream_t stream);

/* Certificates of a point x: out4 (HOST) = {eta, F(x), D(Ax-b), (F-D)/(1+|F|)},
 * all FP64 accumulation over the stored A. */
int ssnal_kkt(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, const double* b,
              int64_t m, int64_t n, const double* x, double lambda1, double lambda2, double* out4,
              hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SSNAL_EN_H */
