// Host-side launchers of the SsNAL-EN kernels.  All pointers are device
// pointers; every launcher enqueues on `st` and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssnal {

// A request to publish the scalar slots to the host at the end of a kernel:
// copy them to coherent pinned memory (dst, device address), then set *flag
// = seq.  flag == nullptr: no request.
struct Pub {
  double* dst = nullptr;
  unsigned long long* flag = nullptr;
  unsigned long long seq = 0;
};

enum DType : int { kF64 = 0, kF32 = 1, kBF16 = 2 };

inline int dtype_size(int dt) { return dt == kF64 ? 8 : (dt == kF32 ? 4 : 2); }

// ---- A^T v  (k_gemv.hip) -------------------------------------------------
// w[k] = sum_i A[i, col(k)] v[i], col(k) = J ? J[k] : k, k < ncols.
// acc64: accumulate in FP64 (always for F64 storage); else FP32.
// ev0/ev1 (nullable): timing events, stamped by the kernel dispatch itself
// (hipExtLaunchKernel) so that their interval is the kernel's duration.
// Columns longer than one register-resident slice of v (4096 FP32, 2048 FP64,
// 8192 BF16 rows) and gathered columns go through row panels.  skip
// (nullable, honoured by the gathered and long-column forms): nothing is done
// while *skip != 0.
hipError_t gemv_t(const void* A, int dtype, int64_t lda, int m, int64_t ncols, const int32_t* J,
                  const double* v, double* w, bool acc64, hipStream_t st,
                  hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, const double* skip = nullptr);
// Same pass also accumulating sum_j ||a_j||^2 into colsq (FP64, one value).
hipError_t gemv_t_colsq(const void* A, int dtype, int64_t lda, int m, int64_t n,
                        const double* v, double* w, double* colsq_part, int* nparts,
                        hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// ---- vector passes over n  (k_vec.hip) -----------------------------------
struct ProxArgs {
  double sigma, thr, den;  // t = fma(-sigma, w, x); active iff |t| > thr; u = soft(t,thr)/den
};
// Number of blocks the prox passes use for n elements.
int prox_blocks(int64_t n);
// Pass 1: optional w += s*wd (s read from s_dev; skipped when s_dev == null),
// then per-block active counts.
hipError_t prox_count(const double* x, double* w, const double* wd, const double* s_dev, int64_t n,
                      ProxArgs pa, int* counts, hipStream_t st);
// Pass 2: order-preserving compaction J (ascending), uJ; r written to *r_out (as double).
hipError_t prox_write(const double* x, const double* w, int64_t n, ProxArgs pa, const int* counts,
                      int32_t* J, double* uJ, double* r_out, hipStream_t st);
// Support of x0 (x0 != 0) compacted the same way (J, uJ = x0_J); r to *r_out.
hipError_t support_count(const double* x, int64_t n, int* counts, hipStream_t st);
hipError_t support_write(const double* x, int64_t n, const int* counts, int32_t* J, double* uJ,
                         double* r_out, hipStream_t st);

// A_J c as per-chunk partial m-vectors: part[chunk*m + i].  r is read from
// r_dev when non-null (the grid is sized for r_bound >= r), else r = r_bound.
// gather_chunks(r_bound, m) bounds the chunk count of every r <= r_bound over
// m rows; the partial buffer holds that many m-vectors.  gather_nchunks(r, m) is the
// chunk count of exactly r columns of m rows.  skip (nullable): nothing is
// done while *skip != 0.
int gather_chunks(int64_t r_bound, int m);
int gather_nchunks(int64_t r, int m);
hipError_t gather_gemv_partial(const void* A, int dtype, int64_t lda, int m, const int32_t* J,
                               const double* c, const double* r_dev, int64_t r_bound, double* part,
                               hipStream_t st, const double* skip = nullptr);
// Finishers over the partial sums S = sum_chunks part:
//  mode 0 (gradient): g = y + b - S, out2 = rho = S - b; |g|^2, |rho|^2, b^T rho into scal
//  mode 1 (Woodbury): out2 = d = -g + S
//  mode 2 (residual): out2 = y = S - b
// blk (mode 0, nullable): 3 * ceil(m/256) doubles for the block partials; null
// uses the scalar block, which holds them for m <= 4096 only.
hipError_t gather_finish(const double* part, const double* r_dev, int64_t r_host, int m, int mode,
                         const double* y, const double* b, double* g, double* out2, double* scal,
                         hipStream_t st, Pub pub = Pub{}, double* blk = nullptr);

// ---- conjugate gradients on V d = -g, V = I + kappa A_J A_J^T  (k_cg.hip) --
// State on the device: d, res (residual -g - V d), p (search direction), q
// (V p), s (A_J^T p, r entries); scalars in scal: SC_CG_RR (two slots,
// alternating by iteration parity), SC_CG_STOP, SC_CG_DONE, SC_CG_IT.
// cg_init: d = 0, res = p = -g, rr = |g|^2, stop = eps2 * rr,
// done = (rr <= stop), it = 0.
// blk: 2 * cg_blocks(m) doubles (block partials).
hipError_t cg_init(const double* g, double* d, double* res, double* p, int m, double eps2,
                   double* blk, double* scal, hipStream_t st);
// One iteration (a no-op once done is set): s = A_J^T p, q = p + kappa A_J s,
// alpha = rr/(p^T q), d += alpha p, res -= alpha q, beta = rr_new/rr,
// p = res + beta p; done once rr_new <= stop.  par = iteration parity.
// gpart: gather_chunks(r, m) m-vectors; blk: ceil(m/256) + cg_blocks(m) doubles.
int cg_blocks(int m);
hipError_t cg_iteration(const void* A, int dtype, int64_t lda, int m, const int32_t* J, int64_t r,
                        double kappa, bool acc64, double* d, double* res, double* p, double* q,
                        double* s, double* gpart, double* blk, int par, double* scal,
                        hipStream_t st);

// Line search: for the K trial steps s_k, Delta_k = psi(y + s_k d) - psi(y);
// a one-block follow-up kernel picks the first k with Delta_k <= mu s_k g^T d,
// updates y += s d and writes s (0 if none) to scal.
constexpr int kMaxTrials = 32;
struct LsArgs {
  double sigma, thr, den, kappa, mu;
  int K;
  double s[kMaxTrials];
};
// Doubles of partial sums the line-search pass writes for n features.
size_t ls_part_doubles(int64_t n);
hipError_t linesearch(const double* x, const double* w, const double* wd, int64_t n, LsArgs la,
                      const double* g, const double* d, double* y, int m, double* part,
                      double* scal, hipStream_t st);
// Line-search increments only (no selection): scal[SC_DELTA + k] = Delta_k, k < K.
hipError_t ls_delta(const double* x, const double* w, const double* wd, int64_t n, LsArgs la,
                    double gd, double dd, double* part, double* scal, hipStream_t st);

// Multiplier update x <- prox(t), with |x - u|^2, |z|^2 (z the conjugate
// prox of Prop. 2 (2)) and |y|^2 reduced into scal.
hipError_t outer_update(double* x, const double* w, int64_t n, ProxArgs pa, double l1, double l2,
                        const double* y, int m, double* part, double* scal, hipStream_t st,
                        Pub pub = Pub{});
// eta pass over q = A^T rho: sums of (x - prox_p(x - q))^2, x^2, |x|, and
// (|q| - l1)_+^2 into scal.
hipError_t eta_pass(const double* x, const double* q, int64_t n, double l1, double l2,
                    double* part, double* scal, hipStream_t st);

// Small helpers
hipError_t vec_scale_copy(const double* src, double alpha, double* dst, int64_t n, hipStream_t st);
hipError_t vec_fill(double* dst, double v, int64_t n, hipStream_t st);
// k-fold: rows = the rows with fold != f in ascending order; scal
// slots get their count, the count of fold f, and the labels outside [0, k).
hipError_t fold_rows(const int32_t* fold, int m, int k, int f, int32_t* rows, double* scal,
                     hipStream_t st);
// At (mt x n, leading dimension mt, same storage type as A) = A[rows, :], bt = b[rows].
hipError_t gather_rows(const void* A, int dtype, int64_t lda, int64_t n, const int32_t* rows, int mt,
                       const double* b, void* At, double* bt, hipStream_t st);
// *out = sum of res_i^2 over the rows of fold f.
hipError_t fold_sq(const double* res, const int32_t* fold, int m, int f, double* out, hipStream_t st);
// out[J[k]] = v[k] for k < r (r read from r_dev; r_bound >= r).
hipError_t scatter(const int32_t* J, const double* v, const double* r_dev, int64_t r_bound,
                   double* out, hipStream_t st);
hipError_t nonfinite_count(const double* v, int64_t n, double* scal_slot, double* part,
                           hipStream_t st);

// ---- Newton matrix (k_syrk.hip) ------------------------------------------
// form 0: out = shift*I_m + scale * A_J A_J^T   (m x m, K = r)
// form 1: out = shift*I_r + scale * A_J^T A_J   (r x r, K = m)
// out is N x N row-major, both triangles written.  Workspace: partial sums.
size_t syrk_workspace_bytes(int form, int m, int64_t r);
hipError_t syrk(const void* A, int dtype, int64_t lda, int m, const int32_t* J, int64_t r, int form,
                double shift, double scale, double* out, void* work, hipStream_t st);

// *out = sum_b part[b], b < nb; with y non-null also *yy_out = |y|^2 (m entries).
// Copy n scalars from the device to coherent pinned host memory (host_dst,
// host_flag: mapped host pointers) and then set *host_flag = seq; a host
// thread that sees the new seq may read host_dst.
hipError_t publish_scalars(const double* scal, int n, double* host_dst, unsigned long long* host_flag,
                           unsigned long long seq, hipStream_t st);
hipError_t sum_parts(const double* part, int nb, double* out, const double* y, int m,
                     double* yy_out, hipStream_t st);
// *out = max_i |v_i| (part: 1024 doubles of scratch).
hipError_t absmax(const double* v, int64_t n, double* part, double* out, hipStream_t st);

// ---- one-workgroup solves of small problems (k_small.hip) ----------------
// FP64 storage, m <= kSmallMaxM; the whole solve (outer and inner loops,
// stopping tests, certificates) in one workgroup, one workgroup per problem.
constexpr int kSmallMaxM = 120;
struct SmallOpts {
  double sigma_factor, sigma_max, mu;
  int max_outer, max_inner, K, no_smw;
  double s[kMaxTrials];  // trial steps delta^k, k < K
  int64_t nl, vec_off;   // set by solve_small: n-vectors in LDS for n <= nl, at this offset (doubles)
};
struct SmallOut {
  int status;  // 0 converged, 1 not converged, 2 line-search stall, -1 sigma0 not a positive
               // number, -2 non-finite, -5 non-positive pivot
  int outer, newton, passes;
  int chol_row;  // status -5: row + 1 of the pivot
  int64_t r;
  double eta, kkt1, kkt3, F, D, sigma, sigma0;
};
struct SmallArgs {
  const double* A;
  int64_t lda;
  int m;
  int64_t n;
  const double* b;
  const double* x0;  // null: cold start
  double* x;
  double l1, l2, tol, sigma0;  // sigma0 <= 0: 2.5 / mean |a_j|^2
  double* wy;  // n doubles each
  double* wd;
  double* uJ;
  int32_t* J;  // n entries
  SmallOut* out;
};
// Raise the dynamic LDS limit of the one-workgroup solve (once per device).
hipError_t small_init();
size_t small_lds_bytes(int mmax, int64_t nl);
// Features whose n-vectors (36 bytes each) fit in LDS beside the Newton
// matrix of mmax rows.
int64_t small_lds_cap(int mmax);
// count problems whose descriptors probs[] the device reads (device or mapped
// pinned memory), or one problem passed by value in *one (probs ignored);
// mmax, nmax = max m and n over them (problems whose n-vectors fit beside
// the Newton matrix keep them in LDS).  With pub.flag set (single problem),
// the result record is published with that sequence number once written.
hipError_t solve_small(const SmallArgs* probs, const SmallArgs* one, int count, int mmax, int64_t nmax,
                       const SmallOpts& o, Pub pub, hipStream_t st);

// ---- Cholesky and triangular solves (k_chol.hip) --------------------------
// Raise the dynamic LDS limits of the Cholesky kernels (once per device).
hipError_t chol_init();
// Factor the SPD N x N row-major V (the blocks below the 64 x 64 diagonal
// blocks of V become those of L; the diagonal blocks of L go to Ld, T =
// ceil(N/64) blocks of 64 x 64 doubles, while V's diagonal blocks keep stale
// values) and, when rhs is non-null, solve L L^T x = alpha*rhs (z: N doubles
// of scratch for L^{-1} alpha rhs; x may alias rhs; Ld then holds 2T blocks,
// the second T for the inverses of the diagonal blocks).  info_dev (int)
// receives row+1 of a non-positive pivot.
hipError_t chol_factor_solve(double* V, int N, const double* rhs, double alpha, double* z,
                             double* x, double* Ld, int* info_dev, hipStream_t st);
// Factor only, with the diagonal blocks of L copied back into V (lower
// triangle = L; the strict upper triangle keeps stale values).
hipError_t cholesky(double* V, int N, double* Ld, int* info_dev, hipStream_t st);
// After chol_factor_solve with a right-hand side (Ld: 2T blocks, then room for
// T(T+1)/2 more): part[j] = the squares of block column j of L^{-1}, j < T,
// so that their sum is ||L^{-1}||_F^2 = tr((L L^T)^{-1}).
hipError_t chol_inv_frob(const double* V, int N, double* Ld, double* part, hipStream_t st);
// Zero the strict upper triangle (for callers that want L alone).
hipError_t zero_upper(double* V, int N, hipStream_t st);

}  // namespace ssnal
