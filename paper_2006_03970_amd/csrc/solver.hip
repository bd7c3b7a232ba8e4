// Host orchestration of the SsNAL-EN solve (Algorithm 1) and the C ABI.
//
// Per Newton iteration the device runs: compaction of the active set (with
// the pending w_y += s w_d folded in), the gradient A_J u_J, one read-back of
// a few scalars (r, |grad psi|^2, the previous line-search outcome), the
// Newton matrix and its Cholesky solve (m x m, or r x r when r < m), the
// A^T d pass, and the line search, which also updates y on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ssnal_en.h"
#include "kernels.hpp"
#include "scal.hpp"

using namespace ssnal;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(SSNAL_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                 \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct ssnal_ctx {
  int device = 0;
  DevBuf wy, wd, uJ, J, counts, part, gpart, V, syrk, mvec, scal;
  DevBuf cv_a, cv_x, cv_m;  // k-fold: a fold's training design, its path, rows / b / errors
  DevBuf sm_ws;             // batch: the n-vectors of the problems solved in one workgroup each
  SmallArgs* h_small = nullptr;  // batch: coherent pinned descriptors, then the result records
  int small_cap = 0;             // problems h_small holds
  std::vector<ssnal_ctx*> cv_sub;      // k-fold worker contexts (created on first use)
  std::vector<hipStream_t> cv_streams;  // their streams (default priority)
  double* h_scal = nullptr;  // coherent pinned: SC_SIZE doubles, then the publish flag
  double* d_scal = nullptr;  // the same memory as the device addresses it
  unsigned long long pub_seq = 0;
  std::vector<hipEvent_t> ev;
  hipEvent_t ev_order = nullptr;  // orders worker streams after the caller's stream
  bool chol_ready = false;
  double last_sigma0 = 0.0;  // sigma0 of the last solve (after defaults)
};

namespace {

// Grow-only allocation; contents are not preserved.
int ensure(DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes) return 0;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (e != hipSuccess) return fail(SSNAL_EHIP, "hipFree: %s", hipGetErrorString(e));
  }
  size_t want = bytes < 256 ? 256 : bytes;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(SSNAL_ENOMEM, "device allocation of %zu bytes failed", want);
  }
  b.bytes = want;
  return 0;
}

// m-vector slots inside ctx->mvec
enum MV : int { MV_Y = 0, MV_G, MV_D, MV_RHO, MV_T1, MV_T2, MV_T3, MV_COUNT };

struct Workspace {
  double *wy, *wd, *uJ, *part, *gpart, *V, *scal;
  double *y, *g, *d, *rho, *t1, *t2, *t3;
  int32_t* J;
  int* counts;
  void* syrk;
  int* info;
};

// Bytes of each workspace buffer an (m, n) problem needs, in the order of
// WsPlan::bufs (the admission footprint of the serving loop is their sum).
struct WsPlan {
  size_t bytes[10];
};
// Largest dense Newton system (m x m, or r x r in the Woodbury form) that is
// factored; beyond it on both sides the direction comes from conjugate
// gradients.
constexpr int64_t kDenseMax = 4096;
// Largest m a solve accepts (the m-vectors and the gathered partial sums grow
// with m; the finishers that sweep them are single-block).
constexpr int64_t kMaxRows = 1 << 20;

WsPlan plan_ws(int64_t m, int64_t n) {
  const int nb = prox_blocks(n);
  const int64_t md = std::min<int64_t>(m, kDenseMax);  // dense systems stay within kDenseMax
  const int64_t T = (md + 63) / 64;
  const size_t m_part = std::max<size_t>(3 * (size_t)((m + 255) / 256), 2 * (size_t)cg_blocks((int)m));
  WsPlan p;
  p.bytes[0] = (size_t)n * 8;  // wy
  p.bytes[1] = (size_t)n * 8;  // wd
  p.bytes[2] = (size_t)n * 8;  // uJ
  p.bytes[3] = (size_t)n * 4;  // J
  p.bytes[4] = (size_t)nb * 4;  // counts
  p.bytes[5] = (std::max({ls_part_doubles(n), (size_t)(2048 + nb) + 4 * (size_t)nb, m_part}) + 64) * 8;  // part
  p.bytes[6] = (size_t)(gather_chunks(n, (int)m) + 1) * m * 8;  // gpart
  p.bytes[7] = (size_t)md * md * 8;  // V
  p.bytes[8] = (size_t)(2048 + T * (T + 1) / 2 + 1) * 64 * 64 * sizeof(double);  // syrk split-K
  p.bytes[9] = (size_t)MV_COUNT * m * 8;  // m-vectors
  for (size_t& b : p.bytes) b = b < 256 ? 256 : b;
  return p;
}
DevBuf* ws_bufs(ssnal_ctx* c, int i) {
  DevBuf* b[10] = {&c->wy, &c->wd, &c->uJ, &c->J, &c->counts, &c->part, &c->gpart, &c->V, &c->syrk, &c->mvec};
  return b[i];
}
// Bytes the context would hold after preparing for plan p (buffers only grow).
size_t held_after(ssnal_ctx* c, const WsPlan& p) {
  size_t t = SC_SIZE * sizeof(double);
  for (int i = 0; i < 10; ++i) t += std::max(ws_bufs(c, i)->bytes, p.bytes[i]);
  return t;
}
// Free the workspace buffers (the context stays usable; they regrow on demand).
// The caller guarantees that no work of this context is in flight.
void ctx_trim(ssnal_ctx* c) {
  (void)hipSetDevice(c->device);
  for (int i = 0; i < 10; ++i) {
    DevBuf* b = ws_bufs(c, i);
    if (b->p) (void)hipFree(b->p);
    b->p = nullptr;
    b->bytes = 0;
  }
}

int prepare(ssnal_ctx* c, int64_t m, int64_t n, Workspace& w) {
  const WsPlan plan = plan_ws(m, n);
  for (int i = 0; i < 10; ++i)
    if (int rc = ensure(*ws_bufs(c, i), plan.bytes[i])) return rc;
  w.wy = (double*)c->wy.p;
  w.wd = (double*)c->wd.p;
  w.uJ = (double*)c->uJ.p;
  w.J = (int32_t*)c->J.p;
  w.counts = (int*)c->counts.p;
  w.part = (double*)c->part.p;
  w.gpart = (double*)c->gpart.p;
  w.V = (double*)c->V.p;
  w.syrk = c->syrk.p;
  double* mv = (double*)c->mvec.p;
  w.y = mv + MV_Y * m;
  w.g = mv + MV_G * m;
  w.d = mv + MV_D * m;
  w.rho = mv + MV_RHO * m;
  w.t1 = mv + MV_T1 * m;
  w.t2 = mv + MV_T2 * m;
  w.t3 = mv + MV_T3 * m;
  w.scal = (double*)c->scal.p;
  w.info = (int*)(w.scal + SC_CHOL);  // Cholesky status, read back with the scalars
  return 0;
}

// Bring the scalar slots to the host once the stream has produced them.  A
// one-workgroup kernel writes them into coherent pinned memory and raises a
// sequence flag; the host spins on the flag (the stream's work before it is
// then complete), which avoids a copy launch and the wake-up latency of a
// stream synchronisation.  After kSpinLimit the host falls back to
// hipStreamSynchronize; errors of the stream are picked up by hipStreamQuery
// while spinning.
// The next publish request (the last kernel of a phase may carry it).
Pub next_pub(ssnal_ctx* c) {
  Pub p;
  p.dst = c->d_scal;
  p.flag = reinterpret_cast<unsigned long long*>(c->d_scal + SC_SIZE);
  p.seq = ++c->pub_seq;
  return p;
}

// Wait until the stream has published the scalar slots with sequence seq.
int wait_pub(ssnal_ctx* c, hipStream_t st, unsigned long long seq, int* syncs) {
  constexpr auto kSpinLimit = std::chrono::microseconds(2000);
  constexpr auto kQueryEvery = std::chrono::microseconds(100);
  unsigned long long* flag = reinterpret_cast<unsigned long long*>(c->h_scal + SC_SIZE);
  if (syncs) ++*syncs;
  const auto t0 = std::chrono::steady_clock::now();
  auto tq = t0;
  for (;;) {
    if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == seq) return 0;
    const auto t = std::chrono::steady_clock::now();
    if (t - t0 > kSpinLimit) break;
    if (t - tq > kQueryEvery) {
      tq = t;
      const hipError_t e = hipStreamQuery(st);
      if (e != hipSuccess && e != hipErrorNotReady)
        return fail(SSNAL_EHIP, "stream error: %s", hipGetErrorString(e));
    }
    __builtin_ia32_pause();
  }
  HIPCHK(hipStreamSynchronize(st));
  if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) != seq)
    return fail(SSNAL_EHIP, "scalar readback: flag %llu after the stream finished, expected %llu",
                (unsigned long long)*flag, seq);
  return 0;
}

int readback(ssnal_ctx* c, const Workspace& w, hipStream_t st, int* syncs) {
  const Pub p = next_pub(c);
  HIPCHK(publish_scalars(w.scal, SC_SIZE, p.dst, p.flag, p.seq, st));
  return wait_pub(c, st, p.seq, syncs);
}

// Error of a non-zero Cholesky status word: row + 1 of a non-positive pivot,
// or -1 when a wait inside a factorisation step ran out (an internal error).
int chol_fail(int info) {
  if (info < 0) return fail(SSNAL_EHIP, "Cholesky: an internal wait of a factorisation step timed out");
  return fail(SSNAL_ENUMERIC, "Cholesky: non-positive pivot at row %d", info - 1);
}

int check_args(const void* A, int dt, int64_t lda, const double* b, int64_t m, int64_t n) {
  if (!A || !b) return fail(SSNAL_EINVAL, "A and b must be non-null device pointers");
  if (dt < 0 || dt > 2) return fail(SSNAL_EINVAL, "a_dtype %d is not SSNAL_F64/F32/BF16", dt);
  if (m < 1 || n < 1) return fail(SSNAL_EINVAL, "m=%lld and n=%lld must be >= 1", (long long)m, (long long)n);
  if (m > kMaxRows) return fail(SSNAL_EINVAL, "m=%lld exceeds %lld", (long long)m, (long long)kMaxRows);
  if (n > 2147483647LL) return fail(SSNAL_EINVAL, "n=%lld exceeds 2^31-1", (long long)n);
  if (lda < m) return fail(SSNAL_EINVAL, "lda=%lld < m=%lld", (long long)lda, (long long)m);
  return 0;
}

struct Timer {
  ssnal_ctx* c;
  hipStream_t st;
  bool on;
  int used = 0;
  std::vector<char> tags;  // 1 = the Newton A^T d pass, 2 = a Cholesky factor + solve, 0 = any other A^T v pass
  double chol_flops = 0.0;  // N^3/3 summed over the timed factorisations
  hipEvent_t e0 = nullptr, e1 = nullptr;  // the pair for the next timed launch
  // Hand out the next event pair (nulls when timing is off); the launch
  // stamps them around the kernel.
  int next(int tag = 0) {
    e0 = e1 = nullptr;
    if (!on) return 0;
    if ((size_t)(2 * used + 2) > c->ev.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->ev.push_back(e);
      }
    }
    e0 = c->ev[2 * used];
    e1 = c->ev[2 * used + 1];
    tags.push_back((char)tag);
    ++used;
    return 0;
  }
  // Summed durations of the timed A^T v passes (tags 0 and 1), of the tag-1
  // passes alone, and of the tag-2 factorisations.
  int total_ms(double* out, double* out1, int* n1, double* out2, int* n2) {
    double t = 0.0, t1 = 0.0, t2 = 0.0;
    int c1 = 0, c2 = 0;
    for (int k = 0; k < used; ++k) {
      float ms = 0.0f;
      HIPCHK(hipEventSynchronize(c->ev[2 * k + 1]));  // readbacks do not wait for events
      HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
      if (tags[k] == 2) {
        t2 += ms;
        ++c2;
        continue;
      }
      t += ms;
      if (tags[k] == 1) {
        t1 += ms;
        ++c1;
      }
    }
    *out = t;
    *out1 = t1;
    *n1 = c1;
    *out2 = t2;
    *n2 = c2;
    return 0;
  }
};

// ---------------------------------------------------------------- direction
// d = -(I + kappa A_J A_J^T)^{-1} g  (eq. AJ_system), with the r x r form of
// eq. smw_formula when 0 < r < m and smw is allowed.
int newton_direction(const void* A, int dt, int64_t lda, int m, const int32_t* J, int64_t r,
                     double kappa, const double* g, double* d, int form, const Workspace& w,
                     hipStream_t st, Timer* tm = nullptr) {
  // factor + solve of an N x N system, timed as tag 2 when timing is on
  auto factor_solve = [&](int N, const double* rhs, double alpha, double* out) -> int {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm && tm->on) {
      if (int rc = tm->next(2)) return rc;
      e0 = tm->e0;
      e1 = tm->e1;
      tm->chol_flops += (double)N * N * N / 3.0;
      HIPCHK(hipEventRecord(e0, st));
    }
    HIPCHK(chol_factor_solve(w.V, N, rhs, alpha, w.t3, out, (double*)w.syrk, w.info, st));
    if (e1) HIPCHK(hipEventRecord(e1, st));
    return 0;
  };
  if (r == 0) {
    HIPCHK(vec_scale_copy(g, -1.0, d, m, st));
    return 0;
  }
  if (form < 0) form = (r < m) ? 1 : 0;
  if (form == 0) {
    HIPCHK(syrk(A, dt, lda, m, J, r, 0, 1.0, kappa, w.V, w.syrk, st));
    // the SYRK partials are dead once V is formed: their buffer holds the
    // diagonal blocks of L
    return factor_solve(m, g, -1.0, d);
  }
  // (I + kappa A_J A_J^T)^{-1} = I - A_J (I/kappa + A_J^T A_J)^{-1} A_J^T
  // d = -g + A_J q,  (I/kappa + A_J^T A_J) q = A_J^T g
  const int N = (int)r;
  double* v = w.t1;  // r <= m entries
  double* q = w.t2;
  HIPCHK(gemv_t(A, dt, lda, m, r, J, g, v, true, st));
  HIPCHK(syrk(A, dt, lda, m, J, r, 1, 1.0 / kappa, 1.0, w.V, w.syrk, st));
  if (int rc = factor_solve(N, v, 1.0, q)) return rc;
  HIPCHK(gather_gemv_partial(A, dt, lda, m, J, q, nullptr, r, w.gpart, st));
  HIPCHK(gather_finish(w.gpart, nullptr, r, m, 1, nullptr, nullptr, const_cast<double*>(g), d, w.scal,
                       st));
  return 0;
}

// d ~ -(I + kappa A_J A_J^T)^{-1} g by conjugate gradients (Sec. 3.2, the
// approximate solve for large m and r), to ||V d + g|| <= eps ||g|| or maxit
// iterations.  The iterations are queued in growing chunks between
// read-backs of the done flag (kernels of an iteration after the flag is set
// return at once).  Iterations taken go to *iters.
int newton_cg(ssnal_ctx* c, const void* A, int dt, int64_t lda, int m, const int32_t* J, int64_t r,
              double kappa, const double* g, double* d, double eps, int maxit, const Workspace& w,
              hipStream_t st, int* syncs, int* iters) {
  *iters = 0;
  if (r == 0) {
    HIPCHK(vec_scale_copy(g, -1.0, d, m, st));
    return 0;
  }
  double* res = w.t1;
  double* p = w.t2;
  double* q = w.t3;
  double* s = w.wd;  // r entries; the A^T d pass rewrites it after the direction
  HIPCHK(cg_init(g, d, res, p, m, eps * eps, w.part, w.scal, st));
  int launched = 0, chunk = 4;
  for (;;) {
    const int k = std::min(chunk, maxit - launched);
    for (int i = 0; i < k; ++i, ++launched)
      HIPCHK(cg_iteration(A, dt, lda, m, J, r, kappa, true, d, res, p, q, s, w.gpart, w.part,
                          launched & 1, w.scal, st));
    if (int rc = readback(c, w, st, syncs)) return rc;
    if (c->h_scal[SC_CG_DONE] != 0.0 || launched >= maxit) break;
    chunk = std::min(2 * chunk, 32);
  }
  *iters = (int)c->h_scal[SC_CG_IT];
  return 0;
}

#pragma clang fp contract(off)
ProxArgs prox_args(double sigma, double l1, double l2) {
  ProxArgs pa;
  pa.sigma = sigma;
  const double p1 = sigma * l1;
  const double p2 = sigma * l2;
  pa.thr = p1;
  pa.den = 1.0 + p2;
  return pa;
}
#pragma clang fp contract(on)

// Prox + gradient: J, uJ, r (device), g, rho, |g|^2 ...  (pending step folded in)
int prox_grad(const void* A, int dt, int64_t lda, const double* b, int m, int64_t n, const double* x,
              const ProxArgs& pa, bool pending, const Workspace& w, hipStream_t st, Pub pub) {
  HIPCHK(prox_count(x, w.wy, w.wd, pending ? w.scal + SC_S : nullptr, n, pa, w.counts, st));
  HIPCHK(prox_write(x, w.wy, n, pa, w.counts, w.J, w.uJ, w.scal + SC_R, st));
  HIPCHK(gather_gemv_partial(A, dt, lda, m, w.J, w.uJ, w.scal + SC_R, n, w.gpart, st));
  HIPCHK(gather_finish(w.gpart, w.scal + SC_R, 0, m, 0, w.y, b, w.g, w.rho, w.scal, st, pub,
                       m > kDenseMax ? w.part : nullptr));
  return 0;
}

// eta, F, D from rho = A x - b (already in w.rho); q = A^T rho into w.wd.
int certify(const void* A, int dt, int64_t lda, int m, int64_t n, const double* x, double l1,
            double l2, const Workspace& w, hipStream_t st, Timer& tm, int* gemv_calls) {
  if (int rc = tm.next()) return rc;
  HIPCHK(gemv_t(A, dt, lda, m, n, nullptr, w.rho, w.wd, true, st, tm.e0, tm.e1));
  ++*gemv_calls;
  HIPCHK(eta_pass(x, w.wd, n, l1, l2, w.part, w.scal, st));
  // the Lasso (lambda2 = 0) bounds D at a scaled feasible point: |A^T rho|_inf
  if (l2 == 0.0) HIPCHK(absmax(w.wd, n, w.part, w.scal + SC_AMAX, st));
  return 0;
}

// D(rho) with p* of Prop. 1; for the Lasso (lambda2 = 0) p* is the indicator
// of |z|_inf <= lambda1 and D is taken at theta*rho, theta = min(1,
// lambda1/|A^T rho|_inf), the largest feasible multiple of rho.
void certificate_values(const double* hs, double l1, double l2, double* eta, double* F, double* D) {
  const double RR = hs[SC_RR], BR = hs[SC_BR];
  *eta = std::sqrt(hs[SC_ETA_E]) / (1.0 + std::sqrt(hs[SC_ETA_XX]) + std::sqrt(RR));
  *F = 0.5 * RR + l1 * hs[SC_ETA_X1] + 0.5 * l2 * hs[SC_ETA_XX];
  if (l2 == 0.0) {
    const double amax = hs[SC_AMAX];
    const double th = amax > l1 ? l1 / amax : 1.0;
    *D = -(0.5 * th * th * RR + th * BR);
  } else {
    *D = -0.5 * RR - BR - hs[SC_ETA_PS] / (2.0 * l2);
  }
}

// ---- one-workgroup solves of small problems (k_small.hip)
// At m <= 120 and small m n the multi-kernel path is bound by its launches
// and its host read-back per Newton step; one workgroup runs the whole solve
// there, streaming A at one CU's rate.  A single solve takes that path when
// m n <= kSmallMaxMN or when its n-vectors fit in LDS beside the Newton
// matrix (n <= 3047 at m = 100): past both, the per-step passes of one CU
// over A and over the n-vectors in global memory cost more than the launches
// they replace (measured at m = 100 to 120: n = 3000 0.65 against 0.96 ms a
// solve, n = 4000 0.83 against 0.74, n = 5000 1.40 against 0.92).  A batch,
// whose problems fill the CUs side by side, takes it up to kSmallBatchMaxMN.
constexpr int64_t kSmallMaxMN = (int64_t)1 << 17;
constexpr int64_t kSmallBatchMaxMN = (int64_t)1 << 21;

bool small_ok(int dt, int64_t m, int64_t n, const ssnal_en_opts& o, bool single) {
  if (o.no_small || dt != kF64 || m > kSmallMaxM || o.newton_cg || o.timing || (o.trace && o.trace_cap > 0))
    return false;
  if (single) return m * n <= kSmallMaxMN || n <= small_lds_cap((int)m);
  return m * n <= kSmallBatchMaxMN;
}

SmallOpts small_opts(const ssnal_en_opts& o) {
  SmallOpts so{};
  so.sigma_factor = o.sigma_factor;
  so.sigma_max = o.sigma_max;
  so.mu = o.mu;
  so.max_outer = o.max_outer;
  so.max_inner = o.max_inner;
  so.K = o.max_backtrack + 1;
  so.no_smw = o.no_smw;
  double t = 1.0;
  for (int k = 0; k < kMaxTrials; ++k) {
    so.s[k] = k < so.K ? t : 0.0;
    t *= o.delta;
  }
  return so;
}

// Options of one solve: the defaults, overridden by the caller's positive
// fields, validated.
int parse_opts(const ssnal_en_opts* user_opts, ssnal_en_opts& o) {
  ssnal_en_opts_init(&o);
  if (user_opts) {
    if (user_opts->sigma0 > 0) o.sigma0 = user_opts->sigma0;
    if (user_opts->sigma_factor > 0) o.sigma_factor = user_opts->sigma_factor;
    if (user_opts->sigma_max > 0) o.sigma_max = user_opts->sigma_max;
    if (user_opts->mu > 0) o.mu = user_opts->mu;
    if (user_opts->delta > 0) o.delta = user_opts->delta;
    if (user_opts->max_outer > 0) o.max_outer = user_opts->max_outer;
    if (user_opts->max_inner > 0) o.max_inner = user_opts->max_inner;
    if (user_opts->max_backtrack > 0) o.max_backtrack = user_opts->max_backtrack;
    o.no_refine = user_opts->no_refine;
    o.no_smw = user_opts->no_smw;
    o.newton_cg = user_opts->newton_cg;
    if (user_opts->cg_maxit > 0) o.cg_maxit = user_opts->cg_maxit;
    if (user_opts->cg_eta > 0) o.cg_eta = user_opts->cg_eta;
    if (user_opts->cg_tau > 0) o.cg_tau = user_opts->cg_tau;
    o.timing = user_opts->timing;
    o.trace = user_opts->trace;
    o.trace_cap = user_opts->trace_cap;
    o.workers = user_opts->workers;
    o.no_small = user_opts->no_small;
  }
  if (o.max_backtrack > kMaxTrials - 1) o.max_backtrack = kMaxTrials - 1;
  if (!(o.mu < 0.5)) return fail(SSNAL_EINVAL, "mu must lie in (0, 1/2)");
  if (!(o.delta < 1.0)) return fail(SSNAL_EINVAL, "delta must lie in (0, 1)");
  if (!(o.cg_eta < 1.0)) return fail(SSNAL_EINVAL, "cg_eta must lie in (0, 1)");
  if (user_opts && user_opts->sigma0 > 0 && !std::isfinite(user_opts->sigma0))
    return fail(SSNAL_EINVAL, "sigma0 = %g is not a positive number", user_opts->sigma0);
  return 0;
}

int check_scalars(const double* x, double l1, double l2, double tol) {
  if (!x) return fail(SSNAL_EINVAL, "x_out must be a non-null device pointer");
  if (!(l1 >= 0.0) || !std::isfinite(l1)) return fail(SSNAL_EINVAL, "lambda1 must be finite and >= 0");
  if (!(l2 >= 0.0) || !std::isfinite(l2)) return fail(SSNAL_EINVAL, "lambda2 must be finite and >= 0");
  if (!(tol > 0.0)) return fail(SSNAL_EINVAL, "tol must be > 0");
  return 0;
}

SmallArgs small_args(const void* A, int64_t lda, const double* b, int64_t m, int64_t n, double l1, double l2,
                     const double* x0, double tol, double* x, const ssnal_en_opts* user_opts, double* wy,
                     double* wd, double* uJ, int32_t* J, SmallOut* out) {
  SmallArgs a{};
  a.A = static_cast<const double*>(A);
  a.lda = lda;
  a.m = (int)m;
  a.n = n;
  a.b = b;
  a.x0 = x0;
  a.x = x;
  a.l1 = l1;
  a.l2 = l2;
  a.tol = tol;
  a.sigma0 = user_opts && user_opts->sigma0 > 0 ? user_opts->sigma0 : 0.0;
  a.wy = wy;
  a.wd = wd;
  a.uJ = uJ;
  a.J = J;
  a.out = out;
  return a;
}

// The outcome of a one-workgroup solve as the multi-kernel path reports it:
// errors as their codes, info filled, the status returned.
int small_result(ssnal_ctx* c, const SmallOut& so, double tol, double solve_ms, ssnal_en_info* info) {
  if (so.status == -2)
    return fail(SSNAL_ENONFINITE, "non-finite values in b, x0, A or the iterates");
  if (so.status == -1) return fail(SSNAL_EINVAL, "sigma0 = %g is not a positive number", so.sigma0);
  if (so.status == -5) return chol_fail(so.chol_row);
  c->last_sigma0 = so.sigma0;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = so.status;
    info->outer_iters = so.outer;
    info->newton_iters = so.newton;
    info->r_final = (int32_t)so.r;
    info->nnz = so.r;
    info->kkt_rel = so.eta;
    info->kkt1 = so.kkt1;
    info->kkt3 = so.kkt3;
    info->primal_obj = so.F;
    info->dual_obj = so.D;
    info->rel_gap = (so.F - so.D) / (1.0 + std::fabs(so.F));
    info->sigma_final = so.sigma;
    info->gemv_calls = so.passes;
    info->syncs = 1;
    info->sigma0 = so.sigma0;
    info->solve_ms = solve_ms;
    info->one_workgroup = 1;
  }
  if (so.status != SSNAL_OK) {
    snprintf(g_err, sizeof(g_err), "%s after %d outer iterations (eta=%.3e, tol=%.3e)",
             so.status == SSNAL_NOT_CONVERGED ? "not converged" : "line search stalled", so.outer, so.eta,
             tol);
  }
  return so.status;
}
static_assert(sizeof(SmallOut) <= SC_SIZE * sizeof(double), "the result record fits the scalar slots");

// preset (nullable): a workspace the caller laid out (the no-allocation entry
// point); otherwise the context's workspace, grown as needed.
int solve_impl(ssnal_ctx* c, const void* A, int dt, int64_t lda, const double* b, int64_t m64,
               int64_t n, double l1, double l2, const double* x0, double tol, hipStream_t st,
               double* x, const ssnal_en_opts* user_opts, ssnal_en_info* info,
               const Workspace* preset = nullptr) {
  const auto t_start = std::chrono::steady_clock::now();
  if (int rc = check_args(A, dt, lda, b, m64, n)) return rc;
  if (int rc = check_scalars(x, l1, l2, tol)) return rc;
  const int m = (int)m64;
  ssnal_en_opts o;
  if (int rc = parse_opts(user_opts, o)) return rc;
  HIPCHK(hipSetDevice(c->device));
  Workspace w;
  if (preset) {
    w = *preset;
  } else if (int rc = prepare(c, m, n, w)) {
    return rc;
  }
  int gemv_calls = 0, syncs = 0;
  double* hs = c->h_scal;
  if (small_ok(dt, m, n, o, true)) {
    // the whole solve in one workgroup; its result record lands in the
    // pinned scalar slots with the publish flag
    const Pub pub = next_pub(c);
    const SmallArgs a = small_args(A, lda, b, m, n, l1, l2, x0, tol, x, user_opts, w.wy, w.wd, w.uJ, w.J,
                                   reinterpret_cast<SmallOut*>(pub.dst));
    HIPCHK(solve_small(nullptr, &a, 1, m, n, small_opts(o), pub, st));
    if (int rc = wait_pub(c, st, pub.seq, &syncs)) return rc;
    SmallOut so;
    std::memcpy(&so, hs, sizeof(so));
    return small_result(c, so, tol,
                        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count(),
                        info);
  }
  const bool mixed = dt != kF64;
  Timer tm{c, st, o.timing != 0};
  HIPCHK(hipMemsetAsync(w.info, 0, sizeof(double), st));

  // ---- start: x = x0 (or 0), y = A x0 - b, w_y = A^T y
  if (x0) {
    if (x0 != x) HIPCHK(hipMemcpyAsync(x, x0, n * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(nonfinite_count(x, n, w.scal + SC_NONFIN, w.part, st));
    if (int rc = readback(c, w, st, &syncs)) return rc;
    if (hs[SC_NONFIN] != 0.0) return fail(SSNAL_ENONFINITE, "x0 holds %g non-finite entries", hs[SC_NONFIN]);
    HIPCHK(support_count(x, n, w.counts, st));
    HIPCHK(support_write(x, n, w.counts, w.J, w.uJ, w.scal + SC_R, st));
    HIPCHK(gather_gemv_partial(A, dt, lda, m, w.J, w.uJ, w.scal + SC_R, n, w.gpart, st));
    HIPCHK(gather_finish(w.gpart, w.scal + SC_R, 0, m, 2, nullptr, b, nullptr, w.y, w.scal, st));
  } else {
    HIPCHK(hipMemsetAsync(x, 0, n * 8, st));
    HIPCHK(vec_scale_copy(b, -1.0, w.y, m, st));
  }
  int nparts = 0;
  if (int rc = tm.next()) return rc;
  HIPCHK(gemv_t_colsq(A, dt, lda, m, n, w.y, w.wy, w.part, &nparts, st, tm.e0, tm.e1));
  ++gemv_calls;
  // sum_j |a_j|^2 (for the default sigma0) and |b|^2, reduced on the device
  // and read back with the scalar slots (no pageable host copies)
  HIPCHK(sum_parts(w.part, nparts, w.scal + SC_COLSQ, b, m, w.scal + SC_BB, st));
  HIPCHK(nonfinite_count(w.wy, n, w.scal + SC_NONFIN, w.part + 2048, st));
  if (int rc = readback(c, w, st, &syncs)) return rc;
  const double normb2 = hs[SC_BB], colsq = hs[SC_COLSQ];
  if (!std::isfinite(normb2)) return fail(SSNAL_ENONFINITE, "b holds non-finite entries");
  if (hs[SC_NONFIN] != 0.0)
    return fail(SSNAL_ENONFINITE, "A^T (A x0 - b) holds %g non-finite entries (non-finite A?)",
                hs[SC_NONFIN]);
  const double normb = std::sqrt(normb2);
  double sigma = o.sigma0;
  if (!(user_opts && user_opts->sigma0 > 0)) {
    const double mean = colsq / (double)n;
    sigma = 2.5 / (mean > 0.0 ? mean : 1.0);
  }
  if (!(sigma > 0.0) || !std::isfinite(sigma))
    return fail(SSNAL_EINVAL, "sigma0 = %g is not a positive number", sigma);
  c->last_sigma0 = sigma;

  double kkt1 = INFINITY, kkt3 = INFINITY, eta = INFINITY, F = NAN, D = NAN;
  // Inner tolerance: tol, divided by 10 (down to tol/1000) after an outer
  // iteration that met kkt1 and kkt3 but not eta (decreasing inner
  // tolerances, as in the inner stopping criteria the method refers to).
  double eps_in = tol;
  int status = SSNAL_NOT_CONVERGED, newton = 0, outer_done = 0, rows = 0, cg_iters = 0;
  int64_t r = 0;
  bool stalled = false, pending = false, converged = false;
  int pending_row = -1;

  for (int outer = 0; outer < o.max_outer; ++outer) {
    const ProxArgs pa = prox_args(sigma, l1, l2);
    const double kappa = sigma / pa.den;
    LsArgs la;
    la.sigma = sigma;
    la.thr = pa.thr;
    la.den = pa.den;
    la.kappa = kappa;
    la.mu = o.mu;
    la.K = o.max_backtrack + 1;
    {
      double s = 1.0;
      for (int k = 0; k < la.K; ++k) {
        la.s[k] = s;
        s *= o.delta;
      }
    }
    bool refreshed = false;
    int inner = 0;
    for (;;) {
      const Pub pub = next_pub(c);
      if (int rc = prox_grad(A, dt, lda, b, m, n, x, pa, pending, w, st, pub)) return rc;
      pending = false;
      if (int rc = wait_pub(c, st, pub.seq, &syncs)) return rc;
      {
        int cinfo = 0;
        std::memcpy(&cinfo, &hs[SC_CHOL], sizeof(int));
        if (cinfo != 0) return chol_fail(cinfo);
      }
      if (pending_row >= 0) {
        if (o.trace && pending_row < o.trace_cap) o.trace[pending_row * 6 + 4] = hs[SC_S];
        pending_row = -1;
        if (hs[SC_LSK] < 0.0) {
          stalled = true;
        } else {
          ++newton;
        }
      }
      r = (int64_t)hs[SC_R];
      kkt1 = std::sqrt(hs[SC_GG]) / (1.0 + normb);
      if (!std::isfinite(kkt1)) return fail(SSNAL_ENONFINITE, "non-finite gradient");
      if (stalled) break;
      if (kkt1 <= eps_in) {
        if (mixed && !o.no_refine && !refreshed) {
          // refresh A^T y with FP64 accumulation over the stored A, then re-test
          if (int rc = tm.next()) return rc;
          HIPCHK(gemv_t(A, dt, lda, m, n, nullptr, w.y, w.wy, true, st, tm.e0, tm.e1));
          ++gemv_calls;
          refreshed = true;
          continue;
        }
        break;
      }
      if (inner >= o.max_inner) break;
      refreshed = false;
      // Newton direction: a dense factorisation (m x m, or r x r in the
      // Woodbury form when r < m) while one fits kDenseMax, else conjugate
      // gradients (always with opts.newton_cg)
      const bool dense_m = m <= kDenseMax;
      const bool dense_r = !o.no_smw && r < m && r <= kDenseMax;
      int rc;
      if (r > 0 && (o.newton_cg || !(dense_m || dense_r))) {
        const double eps = std::min(o.cg_eta, std::pow(kkt1, o.cg_tau));
        int it = 0;
        rc = newton_cg(c, A, dt, lda, m, w.J, r, kappa, w.g, w.d, eps, o.cg_maxit, w, st, &syncs, &it);
        cg_iters += it;
      } else {
        rc = newton_direction(A, dt, lda, m, w.J, r, kappa, w.g, w.d, dense_r ? 1 : 0, w, st, &tm);
      }
      if (rc) return rc;
      // w_d = A^T d, the HBM pass
      if ((rc = tm.next(1))) return rc;
      HIPCHK(gemv_t(A, dt, lda, m, n, nullptr, w.d, w.wd, !mixed, st, tm.e0, tm.e1));
      ++gemv_calls;
      HIPCHK(linesearch(x, w.wy, w.wd, n, la, w.g, w.d, w.y, m, w.part, w.scal, st));
      pending = true;
      if (o.trace && rows < o.trace_cap) {
        double* row = o.trace + rows * 6;
        row[0] = outer;
        row[1] = inner;
        row[2] = (double)r;
        row[3] = sigma;
        row[4] = 0.0;
        row[5] = kkt1;
      }
      pending_row = rows;
      ++rows;
      ++inner;
    }
    // multiplier update x <- prox(x - sigma A^T y)
    const Pub pub = next_pub(c);
    HIPCHK(outer_update(x, w.wy, n, pa, l1, l2, w.y, m, w.part, w.scal, st, pub));
    ++outer_done;
    bool need_eta = false;
    if (int rc = wait_pub(c, st, pub.seq, &syncs)) return rc;
    kkt3 = std::sqrt(hs[SC_XU]) / sigma / (1.0 + std::sqrt(hs[SC_YY]) + std::sqrt(hs[SC_ZZ]));
    need_eta = (kkt1 <= tol && kkt3 <= tol);
    if (need_eta) {
      if (int rc = certify(A, dt, lda, m, n, x, l1, l2, w, st, tm, &gemv_calls)) return rc;
      if (int rc = readback(c, w, st, &syncs)) return rc;
      certificate_values(hs, l1, l2, &eta, &F, &D);
      if (eta <= tol) {
        converged = true;
        status = SSNAL_OK;
        break;
      }
      eps_in = std::max(eps_in * 0.1, tol * 1e-3);
    }
    if (stalled) break;
    sigma *= o.sigma_factor;
    if (sigma > o.sigma_max) sigma = o.sigma_max;
  }
  if (!converged) {
    // certificates of the returned point; rho = A x - b from the last gradient
    if (int rc = certify(A, dt, lda, m, n, x, l1, l2, w, st, tm, &gemv_calls)) return rc;
    if (int rc = readback(c, w, st, &syncs)) return rc;
    certificate_values(hs, l1, l2, &eta, &F, &D);
    status = stalled ? SSNAL_LINESEARCH_STALL : SSNAL_NOT_CONVERGED;
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = status;
    info->outer_iters = outer_done;
    info->newton_iters = newton;
    info->r_final = (int32_t)r;
    info->nnz = r;
    info->kkt_rel = eta;
    info->kkt1 = kkt1;
    info->kkt3 = kkt3;
    info->primal_obj = F;
    info->dual_obj = D;
    info->rel_gap = (F - D) / (1.0 + std::fabs(F));
    info->sigma_final = sigma;
    info->gemv_calls = gemv_calls;
    info->syncs = syncs;
    info->cg_iters = cg_iters;
    info->sigma0 = c->last_sigma0;
    double gms = 0.0, dms = 0.0, cms = 0.0;
    int dn = 0, cn = 0;
    if (int rc = tm.total_ms(&gms, &dms, &dn, &cms, &cn)) return rc;
    info->gemv_ms = gms;
    info->atd_ms = dms;
    info->atd_launches = dn;
    info->chol_ms = cms;
    info->chol_calls = cn;
    info->chol_gflop = tm.chol_flops * 1e-9;
    info->solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  if (status != SSNAL_OK) {
    snprintf(g_err, sizeof(g_err), "%s after %d outer iterations (eta=%.3e, tol=%.3e)",
             status == SSNAL_NOT_CONVERGED ? "not converged" : "line search stalled", outer_done,
             eta, tol);
  }
  return status;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

void ssnal_en_opts_init(ssnal_en_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sigma0 = 0.0;
  o->sigma_factor = 5.0;
  o->sigma_max = 1e8;
  o->mu = 0.2;
  o->delta = 0.5;
  o->max_outer = 100;
  o->max_inner = 50;
  o->max_backtrack = 30;
  o->cg_maxit = 500;
  o->cg_eta = 0.1;
  o->cg_tau = 0.5;
}

const char* ssnal_last_error(void) { return g_err; }

int ssnal_ctx_create(int device, ssnal_ctx** out) {
  g_err[0] = 0;
  if (!out) return fail(SSNAL_EINVAL, "out must be non-null");
  *out = nullptr;
  int count = 0;
  HIPCHK(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(SSNAL_EINVAL, "device %d not in [0, %d)", device, count);
  HIPCHK(hipSetDevice(device));
  ssnal_ctx* c = new (std::nothrow) ssnal_ctx();
  if (!c) return fail(SSNAL_ENOMEM, "host allocation failed");
  c->device = device;
  int rc;
  if ((rc = ensure(c->scal, SC_SIZE * sizeof(double)))) {
    ssnal_ctx_destroy(c);
    return rc;
  }
  if (hipMemset(c->scal.p, 0, c->scal.bytes) != hipSuccess ||
      hipHostMalloc((void**)&c->h_scal, (SC_SIZE + 1) * sizeof(double),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&c->d_scal, c->h_scal, 0) != hipSuccess ||
      chol_init() != hipSuccess || small_init() != hipSuccess) {
    ssnal_ctx_destroy(c);
    return fail(SSNAL_EHIP, "context initialisation failed");
  }
  std::memset(c->h_scal, 0, (SC_SIZE + 1) * sizeof(double));  // publish flag 0: nothing yet
  *out = c;
  return 0;
}

void ssnal_ctx_destroy(ssnal_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&c->wy, &c->wd, &c->uJ, &c->J, &c->counts, &c->part, &c->gpart, &c->V,
                    &c->syrk, &c->mvec, &c->scal, &c->cv_a, &c->cv_x, &c->cv_m, &c->sm_ws};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (c->h_scal) (void)hipHostFree(c->h_scal);
  if (c->h_small) (void)hipHostFree(c->h_small);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->ev_order) (void)hipEventDestroy(c->ev_order);
  for (ssnal_ctx* s : c->cv_sub) ssnal_ctx_destroy(s);
  for (hipStream_t s : c->cv_streams) (void)hipStreamDestroy(s);
  delete c;
}

int ssnal_en_solve(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, const double* b,
                   int64_t m, int64_t n, double lambda1, double lambda2, const double* x0,
                   double tol, hipStream_t stream, double* x_out, const ssnal_en_opts* opts,
                   ssnal_en_info* info) {
  g_err[0] = 0;
  if (!ctx) return fail(SSNAL_EINVAL, "ctx is null");
  return solve_impl(ctx, A, (int)a_dtype, lda, b, m, n, lambda1, lambda2, x0, tol, stream, x_out,
                    opts, info);
}

static int path_impl(ssnal_ctx* ctx, const void* A, int dt, int64_t lda, const double* b, int64_t m,
                     int64_t n, double alpha, double lam_max, const double* c_lambda, int nlam,
                     int64_t max_active, double tol, hipStream_t stream, double* X_out,
                     const ssnal_en_opts* opts, ssnal_en_info* infos);

int ssnal_en_path(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, const double* b,
                  int64_t m, int64_t n, double alpha, const double* c_lambda, int nlam,
                  int64_t max_active, double tol, hipStream_t stream, double* X_out,
                  const ssnal_en_opts* opts, ssnal_en_info* infos) {
  g_err[0] = 0;
  if (!ctx) return fail(SSNAL_EINVAL, "ctx is null");
  if (int rc = check_args(A, (int)a_dtype, lda, b, m, n)) return rc;
  if (!X_out || !c_lambda) return fail(SSNAL_EINVAL, "X_out and c_lambda must be non-null");
  if (nlam < 1) return fail(SSNAL_EINVAL, "nlam must be >= 1");
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(SSNAL_EINVAL, "alpha must lie in (0, 1] (1: the Lasso)");
  if (!(tol > 0.0)) return fail(SSNAL_EINVAL, "tol must be > 0");
  if (max_active < 0) return fail(SSNAL_EINVAL, "max_active must be >= 0");
  for (int k = 0; k < nlam; ++k)
    if (!(c_lambda[k] > 0.0) || !std::isfinite(c_lambda[k]))
      return fail(SSNAL_EINVAL, "c_lambda[%d] must be finite and > 0", k);
  HIPCHK(hipSetDevice(ctx->device));
  const int dt = (int)a_dtype;
  double amax = 0.0;
  {
    // lam_max = ||A^T b||_inf / alpha: the smallest lam whose solution is 0
    Workspace ws;
    if (int rc = prepare(ctx, m, n, ws)) return rc;
    HIPCHK(gemv_t(A, dt, lda, (int)m, n, nullptr, b, ws.wd, true, stream));
    HIPCHK(absmax(ws.wd, n, ws.part, ws.scal + SC_AMAX, stream));
    HIPCHK(nonfinite_count(ws.wd, n, ws.scal + SC_NONFIN, ws.part + 2048, stream));
    if (int rc = readback(ctx, ws, stream, nullptr)) return rc;
    if (ctx->h_scal[SC_NONFIN] != 0.0) return fail(SSNAL_ENONFINITE, "A^T b holds non-finite entries");
    amax = ctx->h_scal[SC_AMAX];
  }
  return path_impl(ctx, A, dt, lda, b, m, n, alpha, amax / alpha, c_lambda, nlam, max_active, tol,
                   stream, X_out, opts, infos);
}

// The path at lam_k = c_lambda[k] * lam_max (lam_max given; 0: x = 0 throughout).
static int path_impl(ssnal_ctx* ctx, const void* A, int dt, int64_t lda, const double* b, int64_t m,
                     int64_t n, double alpha, double lam_max, const double* c_lambda, int nlam,
                     int64_t max_active, double tol, hipStream_t stream, double* X_out,
                     const ssnal_en_opts* opts, ssnal_en_info* infos) {
  const double amax = lam_max;
  // Each point starts from the previous point's x and, unless the caller fixes
  // sigma0, from its final penalty sigma: the warm start then usually ends
  // after one multiplier update.  The carried sigma is capped at the value a
  // cold solve reaches in its fifth outer iteration (sigma0 * factor^4):
  // sigma only grows along a path, and far past that, t = x - sigma A^T y
  // loses the digits of x, so x stops moving while the KKT residual stays
  // above tol.
  ssnal_en_opts o;
  if (opts) o = *opts;
  else ssnal_en_opts_init(&o);
  o.trace = nullptr;
  o.trace_cap = 0;
  const bool carry_sigma = !(o.sigma0 > 0.0);
  const double factor = o.sigma_factor > 0.0 ? o.sigma_factor : 5.0;
  double sigma_cap = 0.0;  // set from the first cold solve
  int worst = 0;
  for (int k = 0; k < nlam; ++k) {
    double* xk = X_out + (int64_t)k * n;
    ssnal_en_info info_k;
    std::memset(&info_k, 0, sizeof(info_k));
    if (amax == 0.0) {
      // A^T b = 0: x = 0 at every lambda
      HIPCHK(hipMemsetAsync(xk, 0, (size_t)n * 8, stream));
    } else {
      const double lam = c_lambda[k] * lam_max;
      const double* x0 = k > 0 ? X_out + (int64_t)(k - 1) * n : nullptr;
      const int rc = solve_impl(ctx, A, dt, lda, b, m, n, alpha * lam, (1.0 - alpha) * lam, x0, tol,
                                stream, xk, &o, &info_k);
      if (rc < 0) return rc;
      worst = std::max(worst, rc);
      if (carry_sigma) {
        if (sigma_cap == 0.0) sigma_cap = ctx->last_sigma0 * factor * factor * factor * factor;
        o.sigma0 = std::min(info_k.sigma_final, sigma_cap);
      }
    }
    if (infos) infos[k] = info_k;
    if (max_active > 0 && info_k.nnz > max_active && k + 1 < nlam) {
      HIPCHK(hipMemsetAsync(xk + n, 0, (size_t)(nlam - k - 1) * n * 8, stream));
      if (infos)
        for (int q = k + 1; q < nlam; ++q) {
          std::memset(&infos[q], 0, sizeof(infos[q]));
          infos[q].status = SSNAL_PATH_TRUNCATED;
        }
      worst = std::max(worst, SSNAL_PATH_TRUNCATED);
      break;
    }
  }
  HIPCHK(hipStreamSynchronize(stream));
  if (worst == SSNAL_PATH_TRUNCATED) snprintf(g_err, sizeof(g_err), "path truncated at max_active");
  return worst;
}

// Worker contexts of ctx (k-fold folds, batch problems), each with its own
// stream of default priority; created on first use and kept by ctx.
static int ensure_workers(ssnal_ctx* ctx, int nw) {
  while ((int)ctx->cv_sub.size() < nw) {
    ssnal_ctx* sub = nullptr;
    if (int rc = ssnal_ctx_create(ctx->device, &sub)) return rc;
    hipStream_t s = nullptr;
    if (hipStreamCreate(&s) != hipSuccess) {
      ssnal_ctx_destroy(sub);
      return fail(SSNAL_EHIP, "stream creation failed");
    }
    ctx->cv_sub.push_back(sub);
    ctx->cv_streams.push_back(s);
  }
  return 0;
}

// Options of one problem of a batch or of the serving loop: the shared
// options with the problem's own sigma0 when it sets one.
static const ssnal_en_opts* problem_opts(const ssnal_en_problem& p, const ssnal_en_opts* shared,
                                         ssnal_en_opts& local) {
  if (!(p.sigma0 > 0.0)) return shared;
  if (shared) local = *shared;
  else ssnal_en_opts_init(&local);
  local.sigma0 = p.sigma0;
  return &local;
}

// Fold f of k-fold cross validation on context c and stream st: the
// training rows (fold != f, in order) copied into c's buffer, the path over
// the full data's grid on them, then the mean squared error over the rows of
// fold f at every point into err_row (HOST, nlam).
static int cv_fold(ssnal_ctx* c, const void* A, int dt, int64_t lda, const double* b, int m, int64_t n,
                   const int32_t* fold, int k, int f, double alpha, double lam_max,
                   const double* c_lambda, int nlam, double tol, hipStream_t st,
                   const ssnal_en_opts* opts, double* err_row, ssnal_en_info* inf) {
  HIPCHK(hipSetDevice(c->device));
  double* hs = c->h_scal;
  const size_t sa = (size_t)dtype_size(dt);
  if (int rc = ensure(c->cv_a, (size_t)(m - 1) * (size_t)n * sa)) return rc;
  if (int rc = ensure(c->cv_x, (size_t)nlam * (size_t)n * 8)) return rc;
  if (int rc = ensure(c->cv_m, (size_t)m * 4 + (size_t)(m + nlam + 2) * 8)) return rc;
  int32_t* rows = (int32_t*)c->cv_m.p;
  double* bt = (double*)((char*)c->cv_m.p + ((size_t)m * 4 + 7) / 8 * 8);
  double* errd = bt + m;
  double* X = (double*)c->cv_x.p;
  Workspace w;
  if (int rc = prepare(c, m, n, w)) return rc;
  HIPCHK(fold_rows(fold, m, k, f, rows, w.scal, st));
  if (int rc = readback(c, w, st, nullptr)) return rc;
  if (hs[SC_CV_BAD] != 0.0) return fail(SSNAL_EINVAL, "%g fold labels outside [0, %d)", hs[SC_CV_BAD], k);
  const int mt = (int)hs[SC_CV_MT];
  const double mv = hs[SC_CV_MV];
  if (mt < 1 || mv < 1) return fail(SSNAL_EINVAL, "fold %d leaves no training or no validation rows", f);
  HIPCHK(gather_rows(A, dt, lda, n, rows, mt, b, c->cv_a.p, bt, st));
  const int rc = path_impl(c, c->cv_a.p, dt, mt, bt, mt, n, alpha, lam_max, c_lambda, nlam, 0, tol, st,
                           X, opts, inf);
  if (rc < 0) return rc;
  // validation errors: residual of the full design, summed over fold f
  if (int rc2 = prepare(c, m, n, w)) return rc2;
  for (int q = 0; q < nlam; ++q) {
    const double* xq = X + (int64_t)q * n;
    HIPCHK(support_count(xq, n, w.counts, st));
    HIPCHK(support_write(xq, n, w.counts, w.J, w.uJ, w.scal + SC_R, st));
    HIPCHK(gather_gemv_partial(A, dt, lda, m, w.J, w.uJ, w.scal + SC_R, n, w.gpart, st));
    HIPCHK(gather_finish(w.gpart, w.scal + SC_R, 0, m, 2, nullptr, b, nullptr, w.t1, w.scal, st));
    HIPCHK(fold_sq(w.t1, fold, m, f, errd + q, st));
  }
  HIPCHK(hipMemcpyAsync(err_row, errd, (size_t)nlam * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int q = 0; q < nlam; ++q) err_row[q] /= mv;
  return rc;
}

int ssnal_en_cv(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, const double* b,
                int64_t m, int64_t n, const int32_t* fold, int k, double alpha,
                const double* c_lambda, int nlam, double tol, int slots, hipStream_t stream,
                const ssnal_en_opts* opts, double* err_out, ssnal_en_info* infos) {
  g_err[0] = 0;
  if (!ctx || !fold || !err_out || !c_lambda) return fail(SSNAL_EINVAL, "null argument");
  if (int rc = check_args(A, (int)a_dtype, lda, b, m, n)) return rc;
  if (k < 2 || k > m) return fail(SSNAL_EINVAL, "need 2 <= k <= m folds");
  if (nlam < 1) return fail(SSNAL_EINVAL, "nlam must be >= 1");
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(SSNAL_EINVAL, "alpha must lie in (0, 1]");
  if (!(tol > 0.0)) return fail(SSNAL_EINVAL, "tol must be > 0");
  if (slots < 1 || slots > 64) return fail(SSNAL_EINVAL, "slots must lie in [1, 64]");
  for (int q = 0; q < nlam; ++q)
    if (!(c_lambda[q] > 0.0) || !std::isfinite(c_lambda[q]))
      return fail(SSNAL_EINVAL, "c_lambda[%d] must be finite and > 0", q);
  HIPCHK(hipSetDevice(ctx->device));
  const int dt = (int)a_dtype;
  const int mi = (int)m;
  // the full data's grid: lam_max = ||A^T b||_inf / alpha.  The read-back
  // also means the caller's stream has finished all earlier work, so the
  // workers' streams may read A, b and fold.
  double amax = 0.0;
  {
    Workspace w;
    if (int rc = prepare(ctx, m, n, w)) return rc;
    HIPCHK(gemv_t(A, dt, lda, mi, n, nullptr, b, w.wd, true, stream));
    HIPCHK(absmax(w.wd, n, w.part, w.scal + SC_AMAX, stream));
    if (int rc = readback(ctx, w, stream, nullptr)) return rc;
    amax = ctx->h_scal[SC_AMAX];
  }
  const double lam_max = amax / alpha;
  const int nw = std::min(slots, k);
  if (nw == 1) {
    int worst = 0;
    for (int f = 0; f < k; ++f) {
      const int rc = cv_fold(ctx, A, dt, lda, b, mi, n, fold, k, f, alpha, lam_max, c_lambda, nlam, tol,
                             stream, opts, err_out + (int64_t)f * nlam,
                             infos ? infos + (int64_t)f * nlam : nullptr);
      if (rc < 0) return rc;
      worst = std::max(worst, rc);
    }
    return worst;
  }
  // folds run concurrently: worker i has its own context and stream; each
  // fold's work is independent of the others, so the results do not depend
  // on the schedule
  if (int rc = ensure_workers(ctx, nw)) return rc;
  std::vector<int> rcs(k, 0);
  std::vector<std::string> msgs(k);
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int i = 0; i < nw; ++i) {
    th.emplace_back([&, i]() {
      for (int f = next++; f < k; f = next++) {
        g_err[0] = 0;
        rcs[f] = cv_fold(ctx->cv_sub[i], A, dt, lda, b, mi, n, fold, k, f, alpha, lam_max, c_lambda, nlam,
                         tol, ctx->cv_streams[i], opts, err_out + (int64_t)f * nlam,
                         infos ? infos + (int64_t)f * nlam : nullptr);
        msgs[f] = g_err;
        if (rcs[f] < 0) next = k;  // stop handing out folds
      }
    });
  }
  for (std::thread& t : th) t.join();
  int worst = 0;
  for (int f = 0; f < k; ++f) {
    if (rcs[f] < 0) {
      snprintf(g_err, sizeof(g_err), "%s", msgs[f].c_str());
      return rcs[f];
    }
    worst = std::max(worst, rcs[f]);
  }
  return worst;
}

int ssnal_en_solve_batch(ssnal_ctx* ctx, const ssnal_en_problem* problems, int count,
                         const ssnal_en_opts* opts, hipStream_t stream, ssnal_en_info* infos) {
  g_err[0] = 0;
  if (!ctx) return fail(SSNAL_EINVAL, "ctx is null");
  if (count < 0 || (count > 0 && !problems)) return fail(SSNAL_EINVAL, "invalid problem list");
  for (int i = 0; i < count; ++i)
    if (problems[i].location != SSNAL_ON_DEVICE)
      return fail(SSNAL_EINVAL, "problem %d: a batch takes device-resident problems only", i);
  if (count == 0) return 0;
  HIPCHK(hipSetDevice(ctx->device));
  const int want = opts && opts->workers > 0 ? opts->workers : 8;
  if (want > 64) return fail(SSNAL_EINVAL, "opts->workers must lie in [1, 64]");
  ssnal_en_opts shared;
  if (int rc = parse_opts(opts, shared)) return rc;
  // the problems solved in one workgroup each (one launch on `stream`), and the rest
  std::vector<int> small, rest;
  for (int i = 0; i < count; ++i) {
    const ssnal_en_problem& p = problems[i];
    if (check_args(p.A, (int)p.a_dtype, p.lda, p.b, p.m, p.n) == 0 &&
        small_ok((int)p.a_dtype, p.m, p.n, shared, false))
      small.push_back(i);
    else
      rest.push_back(i);
  }
  g_err[0] = 0;
  const int nsmall = (int)small.size(), nrest = (int)rest.size();
  const auto t_small = std::chrono::steady_clock::now();
  SmallOut* h_out = nullptr;
  int worst = 0;
  if (nsmall > 0) {
    size_t ws = 0;
    int mmax = 1;
    int64_t nmax = 1;
    for (int i : small) {
      const ssnal_en_problem& p = problems[i];
      if (int rc = check_scalars((double*)p.x_out, p.lambda1, p.lambda2, p.tol))
        return fail(rc, "problem %d: %s", i, std::string(g_err).c_str());
      if (p.sigma0 > 0.0 && !std::isfinite(p.sigma0))
        return fail(SSNAL_EINVAL, "problem %d: sigma0 = %g is not a positive number", i, p.sigma0);
      ws += ((size_t)p.n * 28 + 255) / 256 * 256;
      mmax = std::max(mmax, (int)p.m);
      nmax = std::max(nmax, (int64_t)p.n);
    }
    if (int rc = ensure(ctx->sm_ws, ws)) return rc;
    if (ctx->small_cap < nsmall) {
      if (ctx->h_small) HIPCHK(hipHostFree(ctx->h_small));
      ctx->h_small = nullptr;
      ctx->small_cap = 0;
      HIPCHK(hipHostMalloc((void**)&ctx->h_small, (size_t)nsmall * (sizeof(SmallArgs) + sizeof(SmallOut)),
                           hipHostMallocMapped | hipHostMallocCoherent));
      ctx->small_cap = nsmall;
    }
    SmallArgs* d_args = nullptr;
    HIPCHK(hipHostGetDevicePointer((void**)&d_args, ctx->h_small, 0));
    h_out = reinterpret_cast<SmallOut*>(ctx->h_small + ctx->small_cap);
    SmallOut* d_out = reinterpret_cast<SmallOut*>(d_args + ctx->small_cap);
    char* base = static_cast<char*>(ctx->sm_ws.p);
    for (int k = 0; k < nsmall; ++k) {
      const ssnal_en_problem& p = problems[small[k]];
      const int64_t n = p.n;
      double* wy = reinterpret_cast<double*>(base);
      ssnal_en_opts local;
      ctx->h_small[k] = small_args(p.A, p.lda, p.b, p.m, n, p.lambda1, p.lambda2, (const double*)p.x0, p.tol,
                                   (double*)p.x_out, problem_opts(p, opts, local), wy, wy + n, wy + 2 * n,
                                   reinterpret_cast<int32_t*>(wy + 3 * n), d_out + k);
      base += ((size_t)n * 28 + 255) / 256 * 256;
      if (p.ready) HIPCHK(hipStreamWaitEvent(stream, p.ready, 0));
    }
    // the other problems' workers start after the caller's earlier work, not after this launch
    if (nrest > 0 && want > 1) {
      if (!ctx->ev_order) HIPCHK(hipEventCreateWithFlags(&ctx->ev_order, hipEventDisableTiming));
      HIPCHK(hipEventRecord(ctx->ev_order, stream));
    }
    HIPCHK(solve_small(d_args, nullptr, nsmall, mmax, nmax, small_opts(shared), Pub{}, stream));
  }
  // the results of the one-workgroup solves, once the launch has finished
  auto small_results = [&]() -> int {
    if (nsmall == 0) return 0;
    HIPCHK(hipStreamSynchronize(stream));
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_small).count();
    for (int k = 0; k < nsmall; ++k) {
      const int i = small[k];
      SmallOut so;
      std::memcpy(&so, h_out + k, sizeof(so));
      ssnal_en_info info_i;
      const int rc = small_result(ctx, so, problems[i].tol, ms, &info_i);
      if (rc < 0) return fail(rc, "problem %d: %s", i, std::string(g_err).c_str());
      if (infos) infos[i] = info_i;
      worst = std::max(worst, rc);
    }
    return 0;
  };
  const int nw = std::min(want, nrest);
  if (nw <= 1) {
    for (int i : rest) {
      const ssnal_en_problem& p = problems[i];
      if (p.ready) HIPCHK(hipStreamWaitEvent(stream, p.ready, 0));
      ssnal_en_opts local;
      ssnal_en_info info_i;
      const int rc = solve_impl(ctx, p.A, (int)p.a_dtype, p.lda, p.b, p.m, p.n, p.lambda1, p.lambda2,
                                p.x0, p.tol, stream, p.x_out, problem_opts(p, opts, local), &info_i);
      if (rc < 0) {
        if (nsmall > 0) (void)hipStreamSynchronize(stream);
        return rc;
      }
      if (infos) infos[i] = info_i;
      worst = std::max(worst, rc);
    }
    if (int rc = small_results()) return rc;
    return worst;
  }
  if (int rc = ensure_workers(ctx, nw)) return rc;
  // the workers' streams start after the caller's earlier work on `stream`
  if (nsmall == 0) {
    if (!ctx->ev_order) HIPCHK(hipEventCreateWithFlags(&ctx->ev_order, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ctx->ev_order, stream));
  }
  hipEvent_t start = ctx->ev_order;
  for (int i = 0; i < nw; ++i) HIPCHK(hipStreamWaitEvent(ctx->cv_streams[i], start, 0));
  std::vector<int> rcs(count, 0);
  std::vector<std::string> msgs(count);
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int w = 0; w < nw; ++w) {
    th.emplace_back([&, w]() {
      for (int k = next++; k < nrest; k = next++) {
        const int i = rest[k];
        g_err[0] = 0;
        const ssnal_en_problem& p = problems[i];
        hipStream_t st = ctx->cv_streams[w];
        if (p.ready && hipStreamWaitEvent(st, p.ready, 0) != hipSuccess) {
          rcs[i] = fail(SSNAL_EHIP, "problem %d: waiting for its ready event failed", i);
        } else {
          ssnal_en_opts local;
          ssnal_en_info info_i;
          rcs[i] = solve_impl(ctx->cv_sub[w], p.A, (int)p.a_dtype, p.lda, p.b, p.m, p.n, p.lambda1,
                              p.lambda2, p.x0, p.tol, st, p.x_out, problem_opts(p, opts, local),
                              &info_i);
          if (infos && rcs[i] >= 0) infos[i] = info_i;
        }
        msgs[i] = g_err;
        if (rcs[i] < 0) next = nrest;  // stop handing out problems
      }
    });
  }
  for (std::thread& t : th) t.join();
  for (int i : rest) {
    if (rcs[i] < 0) {
      if (nsmall > 0) (void)hipStreamSynchronize(stream);
      snprintf(g_err, sizeof(g_err), "problem %d: %s", i, msgs[i].c_str());
      return rcs[i];
    }
    worst = std::max(worst, rcs[i]);
  }
  if (int rc = small_results()) return rc;
  return worst;
}

size_t ssnal_workspace_bytes(int64_t m, int64_t n) {
  if (m < 1 || n < 1) return 0;
  const WsPlan p = plan_ws(m, n);
  size_t t = SC_SIZE * sizeof(double);
  for (size_t b : p.bytes) t += b;
  return t;
}

}  // extern "C"

// ====================================================================== no-allocation solve
// ssnal_en_solve_noalloc lays the solve's device workspace out in one
// file-scope device array instead of the context's grow-only buffers, for
// callers that cannot allocate.  Each device holds its own copy of the array
// for the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (taken once per device).
namespace {

constexpr size_t kScratchBytes = (size_t)48 << 20;
constexpr int64_t kScratchMaxM = 512;
constexpr int64_t kScratchMaxN = 131072;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (current), looked up on first use.
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(SSNAL_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SSNAL_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return 0;
}

// Bytes of the split-K Newton-matrix partials (and, after them, the
// Cholesky's diagonal blocks and their inverses) of any dense system of an
// m-row solve: split-K keeps ntiles * nsplit <= 1024 + ntiles - 1 tiles of
// 64 x 64 doubles, ntiles <= T (T + 1) / 2, T = ceil(min(m, 4096) / 64).
size_t scratch_syrk_bytes(int64_t m) {
  const int64_t T = (std::min<int64_t>(m, kDenseMax) + 63) / 64;
  const int64_t tiles = std::max<int64_t>(1024 + T * (T + 1) / 2, 2 * T);
  return (size_t)tiles * 64 * 64 * sizeof(double);
}

// Lay an (m, n) workspace out in [base, base + bytes): the buffers of plan_ws
// in its order (the Newton-matrix partials at their exact bound), 256-byte
// aligned; the scalar slots stay the context's.  Returns the bytes used, or 0
// if they do not fit.
size_t layout_scratch(ssnal_ctx* c, unsigned char* base, size_t bytes, int64_t m, int64_t n, Workspace& w) {
  WsPlan p = plan_ws(m, n);
  p.bytes[8] = scratch_syrk_bytes(m);
  size_t off[10], used = 0;
  for (int i = 0; i < 10; ++i) {
    off[i] = used;
    used += (p.bytes[i] + 255) / 256 * 256;
  }
  if (used > bytes) return 0;
  w.wy = (double*)(base + off[0]);
  w.wd = (double*)(base + off[1]);
  w.uJ = (double*)(base + off[2]);
  w.J = (int32_t*)(base + off[3]);
  w.counts = (int*)(base + off[4]);
  w.part = (double*)(base + off[5]);
  w.gpart = (double*)(base + off[6]);
  w.V = (double*)(base + off[7]);
  w.syrk = base + off[8];
  double* mv = (double*)(base + off[9]);
  w.y = mv + MV_Y * m;
  w.g = mv + MV_G * m;
  w.d = mv + MV_D * m;
  w.rho = mv + MV_RHO * m;
  w.t1 = mv + MV_T1 * m;
  w.t2 = mv + MV_T2 * m;
  w.t3 = mv + MV_T3 * m;
  w.scal = (double*)c->scal.p;
  w.info = (int*)(w.scal + SC_CHOL);
  return used;
}

}  // namespace

extern "C" {

int ssnal_en_solve_noalloc(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, const double* b,
                           int64_t m, int64_t n, double lambda1, double lambda2, const double* x0, double tol,
                           hipStream_t stream, double* x_out, const ssnal_en_opts* opts, ssnal_en_info* info) {
  g_err[0] = 0;
  if (!ctx) return fail(SSNAL_EINVAL, "ctx is null");
  if (int rc = check_args(A, (int)a_dtype, lda, b, m, n)) return rc;
  if (m > kScratchMaxM || n > kScratchMaxN)
    return fail(SSNAL_EINVAL, "m=%lld, n=%lld: the no-allocation solve takes m <= %lld and n <= %lld",
                (long long)m, (long long)n, (long long)kScratchMaxM, (long long)kScratchMaxN);
  if (opts && opts->timing)
    return fail(SSNAL_EINVAL, "opts->timing creates events: not available without allocation");
  if (opts && opts->newton_cg)
    return fail(SSNAL_EINVAL, "opts->newton_cg: the no-allocation solve factors the Newton systems");
  HIPCHK(hipSetDevice(ctx->device));
  void* base = nullptr;
  if (int rc = scratch_address(ctx->device, &base)) return rc;
  Workspace w;
  if (!layout_scratch(ctx, (unsigned char*)base, kScratchBytes, m, n, w))
    return fail(SSNAL_EINVAL, "m=%lld, n=%lld needs more than the %zu scratch bytes", (long long)m,
                (long long)n, kScratchBytes);
  return solve_impl(ctx, A, (int)a_dtype, lda, b, m, n, lambda1, lambda2, x0, tol, stream, x_out, opts,
                    info, &w);
}

}  // extern "C"

// ====================================================================== serving loop
// Slot i is a host thread with its own context, stream and (for host-resident
// requests) device buffers for the uploaded A, b and x.  Admission: among the
// queued requests whose footprint fits the budget next to what the other
// slots hold, the one with the least estimated work goes to an idle slot; the
// oldest request goes first once it has been passed over kBypassPerSlot *
// slots times.  When nothing is running and the oldest request still does
// not fit, idle slots release their buffers (no work is in flight, so freeing
// is safe) and it is admitted.
namespace {

constexpr int kBypassPerSlot = 4;

using Clock = std::chrono::steady_clock;

// Staging bytes a host-resident problem needs on the device: A packed with
// lda = m, then b and x.
size_t stage_a_bytes(const ssnal_en_problem& p) {
  return p.location == SSNAL_ON_HOST ? (size_t)p.m * (size_t)p.n * (size_t)dtype_size((int)p.a_dtype) : 0;
}
size_t stage_v_bytes(const ssnal_en_problem& p) {
  return p.location == SSNAL_ON_HOST ? (size_t)(p.m + p.n) * 8 : 0;
}

// Estimated device time of a solve in milliseconds, for ordering only: about
// 15 passes over A at 6 TB/s, 10 factorisations of ceil(N/64) block steps of
// 20 us each (N = min(m, 4096)), and 1 ms of fixed costs.
double est_ms(const ssnal_en_problem& p) {
  const double pass = (double)p.m * (double)p.n * dtype_size((int)p.a_dtype) / 6e9;
  const double steps = (double)((std::min<int64_t>(p.m, 4096) + 63) / 64);
  return 15.0 * pass + 10.0 * steps * 0.02 + 1.0;
}

}  // namespace

struct ssnal_srv {
  struct Req {
    uint64_t ticket;
    ssnal_en_problem p;
    Clock::time_point t_submit;
    double cost;
    int bypassed;
  };
  struct Done {
    int status;
    ssnal_en_info info;
    char err[256];
  };
  int device = 0;
  size_t budget = 0;
  int max_bypass = 0;
  ssnal_en_opts opts;
  bool has_opts = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req> queue;
  std::unordered_map<uint64_t, Done> done;
  std::unordered_map<uint64_t, int> live;  // queued or running tickets
  std::vector<ssnal_ctx*> ctx;
  std::vector<DevBuf> stage_a, stage_v;  // per slot: uploaded A; b then x
  std::vector<size_t> held;  // bytes held by each slot (context + staging)
  std::vector<char> busy;
  std::vector<std::thread> workers;
  int running = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  int init_rc = 0;
  char init_err[512] = "";
};

namespace {

size_t ctx_held(ssnal_ctx* c) {
  size_t t = SC_SIZE * sizeof(double);
  for (int i = 0; i < 10; ++i) t += ws_bufs(c, i)->bytes;
  return t;
}
size_t slot_held(ssnal_srv* s, int slot) {
  return ctx_held(s->ctx[slot]) + s->stage_a[slot].bytes + s->stage_v[slot].bytes;
}
// Bytes slot would hold while serving p (every buffer only grows).
size_t slot_held_after(ssnal_srv* s, int slot, const ssnal_en_problem& p) {
  return held_after(s->ctx[slot], plan_ws(p.m, p.n)) + std::max(s->stage_a[slot].bytes, stage_a_bytes(p)) +
         std::max(s->stage_v[slot].bytes, stage_v_bytes(p));
}
void slot_trim(ssnal_srv* s, int slot) {
  ctx_trim(s->ctx[slot]);
  for (DevBuf* b : {&s->stage_a[slot], &s->stage_v[slot]}) {
    if (b->p) (void)hipFree(b->p);
    b->p = nullptr;
    b->bytes = 0;
  }
  s->held[slot] = slot_held(s, slot);
}

// Index in s->queue of the request slot should take now, or -1 (caller holds
// the lock).  Passed-over requests older than the one taken count a bypass.
int srv_pick(ssnal_srv* s, int slot) {
  size_t others = 0;
  for (size_t j = 0; j < s->held.size(); ++j)
    if ((int)j != slot) others += s->held[j];
  auto fits = [&](const ssnal_en_problem& p) { return others + slot_held_after(s, slot, p) <= s->budget; };
  const int nq = (int)s->queue.size();
  if (nq == 0) return -1;
  if (s->queue.front().bypassed >= s->max_bypass) {
    // the oldest request has waited long enough: it goes next, as soon as it fits
    if (fits(s->queue.front().p)) return 0;
    if (s->running == 0) {
      for (size_t j = 0; j < s->ctx.size(); ++j) slot_trim(s, (int)j);
      return 0;
    }
    return -1;
  }
  int best = -1;
  for (int i = 0; i < nq; ++i) {
    const ssnal_srv::Req& q = s->queue[i];
    if (!fits(q.p)) continue;
    if (best < 0 || q.cost < s->queue[best].cost) best = i;
  }
  if (best < 0) {
    if (s->running != 0) return -1;
    for (size_t j = 0; j < s->ctx.size(); ++j) slot_trim(s, (int)j);
    best = 0;
  }
  for (int i = 0; i < best; ++i) ++s->queue[i].bypassed;
  return best;
}

// Run one admitted request on slot's context and stream.
int srv_run(ssnal_srv* s, int slot, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
            const ssnal_en_problem& p, ssnal_en_info* info) {
  ssnal_ctx* c = s->ctx[slot];
  ssnal_en_opts local;
  const ssnal_en_opts* o = problem_opts(p, s->has_opts ? &s->opts : nullptr, local);
  if (p.location != SSNAL_ON_HOST) {
    if (p.ready) HIPCHK(hipStreamWaitEvent(st, p.ready, 0));
    return solve_impl(c, p.A, (int)p.a_dtype, p.lda, p.b, p.m, p.n, p.lambda1, p.lambda2, p.x0, p.tol, st,
                      p.x_out, o, info);
  }
  // host-resident: upload A (packed, lda = m), b and x0 into the slot's buffers
  if (int rc = ensure(s->stage_a[slot], stage_a_bytes(p))) return rc;
  if (int rc = ensure(s->stage_v[slot], stage_v_bytes(p))) return rc;
  const size_t es = (size_t)dtype_size((int)p.a_dtype);
  void* dA = s->stage_a[slot].p;
  double* db = (double*)s->stage_v[slot].p;
  double* dx = db + p.m;
  HIPCHK(hipEventRecord(ev0, st));
  if (p.lda == p.m)
    HIPCHK(hipMemcpyAsync(dA, p.A, (size_t)p.m * (size_t)p.n * es, hipMemcpyHostToDevice, st));
  else
    HIPCHK(hipMemcpy2DAsync(dA, (size_t)p.m * es, p.A, (size_t)p.lda * es, (size_t)p.m * es, (size_t)p.n,
                            hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(db, p.b, (size_t)p.m * 8, hipMemcpyHostToDevice, st));
  if (p.x0) HIPCHK(hipMemcpyAsync(dx, p.x0, (size_t)p.n * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(ev1, st));
  const int rc = solve_impl(c, dA, (int)p.a_dtype, p.m, db, p.m, p.n, p.lambda1, p.lambda2,
                            p.x0 ? dx : nullptr, p.tol, st, dx, o, info);
  if (rc < 0) return rc;
  HIPCHK(hipMemcpyAsync(p.x_out, dx, (size_t)p.n * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
  if (info) info->upload_ms = ms;
  return rc;
}

void srv_worker(ssnal_srv* s, int slot) {
  hipStream_t st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (hipSetDevice(s->device) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) {
      s->init_rc = SSNAL_EHIP;
      snprintf(s->init_err, sizeof(s->init_err), "slot %d: stream creation failed", slot);
      st = nullptr;
    }
    s->cv_done.notify_all();
  }
  for (;;) {
    ssnal_srv::Req req;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      int pick = -1;
      for (;;) {
        if (s->queue.empty() && s->stop) {
          lk.unlock();
          if (ev0) (void)hipEventDestroy(ev0);
          if (ev1) (void)hipEventDestroy(ev1);
          if (st) (void)hipStreamDestroy(st);
          return;
        }
        if ((pick = srv_pick(s, slot)) >= 0) break;
        s->cv_work.wait(lk);
      }
      req = s->queue[pick];
      s->queue.erase(s->queue.begin() + pick);
      s->held[slot] = slot_held_after(s, slot, req.p);
      s->busy[slot] = 1;
      ++s->running;
      s->cv_work.notify_all();  // another queued request may fit another idle slot
    }
    ssnal_srv::Done d;
    std::memset(&d.info, 0, sizeof(d.info));
    const double queue_ms = std::chrono::duration<double, std::milli>(Clock::now() - req.t_submit).count();
    g_err[0] = 0;
    d.status = st ? srv_run(s, slot, st, ev0, ev1, req.p, &d.info) : SSNAL_EHIP;
    if (d.status < 0) d.info.status = d.status;
    d.info.queue_ms = queue_ms;
    snprintf(d.err, sizeof(d.err), "%s", g_err);
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->held[slot] = slot_held(s, slot);
      s->busy[slot] = 0;
      --s->running;
      s->live.erase(req.ticket);
      s->done[req.ticket] = d;
      s->cv_done.notify_all();
      s->cv_work.notify_all();
    }
  }
}

int check_problem(const ssnal_en_problem* p) {
  if (int rc = check_args(p->A, (int)p->a_dtype, p->lda, p->b, p->m, p->n)) return rc;
  if (!p->x_out) return fail(SSNAL_EINVAL, "x_out must be non-null");
  if (!(p->lambda1 >= 0.0) || !(p->lambda2 >= 0.0) || !(p->tol > 0.0))
    return fail(SSNAL_EINVAL, "need lambda1 >= 0, lambda2 >= 0, tol > 0");
  if (p->location != SSNAL_ON_DEVICE && p->location != SSNAL_ON_HOST)
    return fail(SSNAL_EINVAL, "location %d is not SSNAL_ON_DEVICE or SSNAL_ON_HOST", (int)p->location);
  if (p->location == SSNAL_ON_HOST && p->ready)
    return fail(SSNAL_EINVAL, "a host-resident problem takes no ready event");
  return 0;
}

}  // namespace

extern "C" {

size_t ssnal_srv_footprint(const ssnal_en_problem* p) {
  if (!p || p->m < 1 || p->n < 1) return 0;
  return ssnal_workspace_bytes(p->m, p->n) + stage_a_bytes(*p) + stage_v_bytes(*p);
}

int ssnal_srv_create(int device, size_t hbm_budget, int max_slots, const ssnal_en_opts* opts,
                     ssnal_srv** out) {
  g_err[0] = 0;
  if (!out) return fail(SSNAL_EINVAL, "out must be non-null");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 64) return fail(SSNAL_EINVAL, "max_slots must lie in [1, 64]");
  if (hbm_budget == 0) return fail(SSNAL_EINVAL, "hbm_budget must be > 0");
  ssnal_srv* s = new (std::nothrow) ssnal_srv();
  if (!s) return fail(SSNAL_ENOMEM, "host allocation failed");
  s->device = device;
  s->budget = hbm_budget;
  s->max_bypass = kBypassPerSlot * max_slots;
  if (opts) {
    s->opts = *opts;
    s->opts.trace = nullptr;
    s->opts.trace_cap = 0;
    s->has_opts = true;
  }
  for (int i = 0; i < max_slots; ++i) {
    ssnal_ctx* c = nullptr;
    if (int rc = ssnal_ctx_create(device, &c)) {
      for (ssnal_ctx* q : s->ctx) ssnal_ctx_destroy(q);
      delete s;
      return rc;
    }
    s->ctx.push_back(c);
    s->stage_a.emplace_back();
    s->stage_v.emplace_back();
    s->held.push_back(ctx_held(c));
    s->busy.push_back(0);
  }
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(srv_worker, s, i);
  *out = s;
  return 0;
}

int ssnal_srv_submit(ssnal_srv* s, const ssnal_en_problem* p, uint64_t* ticket) {
  g_err[0] = 0;
  if (!s || !p || !ticket) return fail(SSNAL_EINVAL, "null argument");
  if (int rc = check_problem(p)) return rc;
  const size_t need = ssnal_srv_footprint(p);
  if (need > s->budget)
    return fail(SSNAL_ENOMEM, "request needs %zu device bytes, budget is %zu", need, s->budget);
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->init_rc) return fail(s->init_rc, "%s", s->init_err);
  if (s->stop) return fail(SSNAL_EINVAL, "server is shutting down");
  const uint64_t t = s->next_ticket++;
  s->queue.push_back({t, *p, Clock::now(), est_ms(*p), 0});
  s->live[t] = 1;
  *ticket = t;
  s->cv_work.notify_all();
  return 0;
}

static int srv_collect(ssnal_srv* s, uint64_t ticket, ssnal_en_info* info, bool block) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    auto it = s->done.find(ticket);
    if (it != s->done.end()) {
      const int st = it->second.status;
      if (info) *info = it->second.info;
      if (st != 0) snprintf(g_err, sizeof(g_err), "%s", it->second.err);
      s->done.erase(it);
      return st;
    }
    if (!s->live.count(ticket)) return fail(SSNAL_EINVAL, "unknown or already collected ticket %llu",
                                            (unsigned long long)ticket);
    if (!block) return 1;
    s->cv_done.wait(lk);
  }
}

int ssnal_srv_poll(ssnal_srv* s, uint64_t ticket, ssnal_en_info* info) {
  g_err[0] = 0;
  if (!s) return fail(SSNAL_EINVAL, "null server");
  return srv_collect(s, ticket, info, false);
}

int ssnal_srv_wait(ssnal_srv* s, uint64_t ticket, ssnal_en_info* info) {
  g_err[0] = 0;
  if (!s) return fail(SSNAL_EINVAL, "null server");
  return srv_collect(s, ticket, info, true);
}

void ssnal_srv_destroy(ssnal_srv* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  for (std::thread& t : s->workers) t.join();
  (void)hipSetDevice(s->device);
  for (size_t j = 0; j < s->ctx.size(); ++j) {
    for (DevBuf* b : {&s->stage_a[j], &s->stage_v[j]})
      if (b->p) (void)hipFree(b->p);
    ssnal_ctx_destroy(s->ctx[j]);
  }
  delete s;
}

int ssnal_gemv_t(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, int64_t m,
                 int64_t n, const double* v, double* w, int acc64, hipStream_t stream) {
  g_err[0] = 0;
  if (!ctx) return fail(SSNAL_EINVAL, "ctx is null");
  if (int rc = check_args(A, (int)a_dtype, lda, v, m, n)) return rc;
  if (!w) return fail(SSNAL_EINVAL, "w is null");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(gemv_t(A, (int)a_dtype, lda, (int)m, n, nullptr, v, w, acc64 != 0 || a_dtype == SSNAL_F64,
                stream));
  HIPCHK(hipStreamSynchronize(stream));
  return 0;
}

int ssnal_active_prox(ssnal_ctx* ctx, const double* x, const double* w, int64_t n, double sigma,
                      double lambda1, double lambda2, int32_t* J, double* uJ, int64_t* r_out,
                      hipStream_t stream) {
  g_err[0] = 0;
  if (!ctx || !x || !w || !J || !uJ || !r_out) return fail(SSNAL_EINVAL, "null argument");
  if (n < 1) return fail(SSNAL_EINVAL, "n must be >= 1");
  HIPCHK(hipSetDevice(ctx->device));
  Workspace ws;
  if (int rc = prepare(ctx, 1, n, ws)) return rc;
  const ProxArgs pa = prox_args(sigma, lambda1, lambda2);
  HIPCHK(prox_count(x, const_cast<double*>(w), nullptr, nullptr, n, pa, ws.counts, stream));
  HIPCHK(prox_write(x, w, n, pa, ws.counts, J, uJ, ws.scal + SC_R, stream));
  if (int rc = readback(ctx, ws, stream, nullptr)) return rc;
  *r_out = (int64_t)ctx->h_scal[SC_R];
  return 0;
}

int ssnal_newton_matrix(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, int64_t m,
                        const int32_t* J, int64_t r, double kappa, int form, double* out,
                        hipStream_t stream) {
  g_err[0] = 0;
  if (!ctx || !out || (r > 0 && !J)) return fail(SSNAL_EINVAL, "null argument");
  if (int rc = check_args(A, (int)a_dtype, lda, out, m, 1)) return rc;
  if (form != 0 && form != 1) return fail(SSNAL_EINVAL, "form must be 0 or 1");
  if (form == 0 && m > kDenseMax) return fail(SSNAL_EINVAL, "form 0 needs m <= 4096");
  if (form == 1 && (r < 1 || r > kDenseMax)) return fail(SSNAL_EINVAL, "form 1 needs 1 <= r <= 4096");
  if (!(kappa > 0)) return fail(SSNAL_EINVAL, "kappa must be > 0");
  HIPCHK(hipSetDevice(ctx->device));
  Workspace ws;
  const int64_t Nmax = form == 0 ? m : (r > m ? r : m);
  if (int rc = prepare(ctx, Nmax, 1, ws)) return rc;
  if (form == 0)
    HIPCHK(syrk(A, (int)a_dtype, lda, (int)m, J, r, 0, 1.0, kappa, out, ws.syrk, stream));
  else
    HIPCHK(syrk(A, (int)a_dtype, lda, (int)m, J, r, 1, 1.0 / kappa, 1.0, out, ws.syrk, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return 0;
}

int ssnal_cholesky(ssnal_ctx* ctx, double* V, int64_t N, hipStream_t stream) {
  g_err[0] = 0;
  if (!ctx || !V) return fail(SSNAL_EINVAL, "null argument");
  if (N < 1 || N > 4096) return fail(SSNAL_EINVAL, "N must lie in [1, 4096]");
  HIPCHK(hipSetDevice(ctx->device));
  Workspace ws;
  if (int rc = prepare(ctx, N, 1, ws)) return rc;
  HIPCHK(hipMemsetAsync(ws.info, 0, sizeof(int), stream));
  HIPCHK(cholesky(V, (int)N, (double*)ws.syrk, ws.info, stream));
  HIPCHK(zero_upper(V, (int)N, stream));
  if (int rc = readback(ctx, ws, stream, nullptr)) return rc;
  int hinfo = 0;
  std::memcpy(&hinfo, &ctx->h_scal[SC_CHOL], sizeof(int));
  if (hinfo != 0) return chol_fail(hinfo);
  return 0;
}

int ssnal_newton_direction(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda,
                           int64_t m, const int32_t* J, int64_t r, double kappa, const double* g,
                           double* d, int form, hipStream_t stream) {
  g_err[0] = 0;
  if (!ctx || !g || !d || (r > 0 && !J)) return fail(SSNAL_EINVAL, "null argument");
  if (int rc = check_args(A, (int)a_dtype, lda, g, m, 1)) return rc;
  if (!(kappa > 0)) return fail(SSNAL_EINVAL, "kappa must be > 0");
  if (form == 1 && r >= m) return fail(SSNAL_EINVAL, "form 1 needs r < m");
  if (form < 0) form = r < m ? 1 : 0;
  if (r > 0 && form == 0 && m > kDenseMax) return fail(SSNAL_EINVAL, "the m x m system needs m <= 4096");
  if (r > 0 && form == 1 && r > kDenseMax) return fail(SSNAL_EINVAL, "the r x r system needs r <= 4096");
  HIPCHK(hipSetDevice(ctx->device));
  Workspace ws;
  if (int rc = prepare(ctx, m, r > 0 ? r : 1, ws)) return rc;
  HIPCHK(hipMemsetAsync(ws.info, 0, sizeof(int), stream));
  if (int rc = newton_direction(A, (int)a_dtype, lda, (int)m, J, r, kappa, g, d, form, ws, stream))
    return rc;
  if (int rc = readback(ctx, ws, stream, nullptr)) return rc;
  int hinfo = 0;
  std::memcpy(&hinfo, &ctx->h_scal[SC_CHOL], sizeof(int));
  if (hinfo != 0) return chol_fail(hinfo);
  return 0;
}

int ssnal_newton_cg(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, int64_t m,
                    const int32_t* J, int64_t r, double kappa, const double* g, double eps,
                    int32_t maxit, hipStream_t stream, double* d, int32_t* iters) {
  g_err[0] = 0;
  if (!ctx || !g || !d || (r > 0 && !J)) return fail(SSNAL_EINVAL, "null argument");
  if (int rc = check_args(A, (int)a_dtype, lda, g, m, 1)) return rc;
  if (!(kappa > 0)) return fail(SSNAL_EINVAL, "kappa must be > 0");
  if (!(eps >= 0.0)) return fail(SSNAL_EINVAL, "eps must be >= 0");
  if (maxit < 0) return fail(SSNAL_EINVAL, "maxit must be >= 0");
  if (r < 0) return fail(SSNAL_EINVAL, "r must be >= 0");
  HIPCHK(hipSetDevice(ctx->device));
  Workspace ws;
  if (int rc = prepare(ctx, m, r > 0 ? r : 1, ws)) return rc;
  int it = 0;
  if (int rc = newton_cg(ctx, A, (int)a_dtype, lda, (int)m, J, r, kappa, g, d, eps, maxit, ws, stream,
                         nullptr, &it))
    return rc;
  HIPCHK(hipStreamSynchronize(stream));
  if (iters) *iters = it;
  return 0;
}

int ssnal_en_model_select(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda,
                          const double* b, int64_t m, int64_t n, double lambda2, const double* x,
                          hipStream_t stream, double* beta_out, ssnal_en_select* out) {
  g_err[0] = 0;
  if (!ctx || !x || !out) return fail(SSNAL_EINVAL, "null argument");
  if (int rc = check_args(A, (int)a_dtype, lda, b, m, n)) return rc;
  if (!(lambda2 >= 0.0) || !std::isfinite(lambda2)) return fail(SSNAL_EINVAL, "lambda2 must be >= 0");
  HIPCHK(hipSetDevice(ctx->device));
  Workspace w;
  if (int rc = prepare(ctx, m, n, w)) return rc;
  const int dt = (int)a_dtype;
  const int mi = (int)m;
  hipStream_t st = stream;
  double* hs = ctx->h_scal;
  std::memset(out, 0, sizeof(*out));
  // support of x and the residual of the elastic-net fit
  HIPCHK(support_count(x, n, w.counts, st));
  HIPCHK(support_write(x, n, w.counts, w.J, w.uJ, w.scal + SC_R, st));
  HIPCHK(gather_gemv_partial(A, dt, lda, mi, w.J, w.uJ, w.scal + SC_R, n, w.gpart, st));
  HIPCHK(gather_finish(w.gpart, w.scal + SC_R, 0, mi, 2, nullptr, b, nullptr, w.t1, w.scal, st));
  HIPCHK(sum_parts(w.part, 0, w.scal + SC_MS_NONE, w.t1, mi, w.scal + SC_MS_RSSEN, st));
  HIPCHK(sum_parts(w.part, 0, w.scal + SC_MS_NONE, b, mi, w.scal + SC_BB, st));
  if (int rc = readback(ctx, w, st, nullptr)) return rc;
  const int64_t r = (int64_t)hs[SC_R];
  if (std::min<int64_t>(r, m) > kDenseMax)
    return fail(SSNAL_EINVAL, "model selection needs min(r, m) <= 4096 (r=%lld, m=%lld): its systems are dense",
                (long long)r, (long long)m);
  out->r = (int32_t)r;
  out->rss_en = hs[SC_MS_RSSEN];
  const double bb = hs[SC_BB];
  const double md = (double)m;
  auto criteria = [&](double rss) {
    out->rss = rss;
    out->gcv = (rss / md) / ((1.0 - out->nu / md) * (1.0 - out->nu / md));
    out->ebic = std::log(rss / md) + (out->nu / md) * (std::log(md) + std::log((double)n));
  };
  if (beta_out) HIPCHK(vec_fill(beta_out, 0.0, n, st));
  if (r == 0) {
    out->nu = 0.0;
    criteria(bb);
    HIPCHK(hipStreamSynchronize(st));
    return 0;
  }
  // degrees of freedom: N - lambda2 ||L^{-1}||_F^2, L L^T = lambda2 I_N + Gram
  const int form = r < m ? 1 : 0;
  const int N = (int)(r < m ? r : m);
  HIPCHK(syrk(A, dt, lda, mi, w.J, r, form, lambda2, 1.0, w.V, w.syrk, st));
  HIPCHK(vec_fill(w.t2, 0.0, N, st));
  HIPCHK(hipMemsetAsync(w.info, 0, sizeof(double), st));
  HIPCHK(chol_factor_solve(w.V, N, w.t2, 1.0, w.t3, w.d, (double*)w.syrk, w.info, st));
  HIPCHK(chol_inv_frob(w.V, N, (double*)w.syrk, w.part, st));
  HIPCHK(sum_parts(w.part, (N + 63) / 64, w.scal + SC_MS_FROB, nullptr, 0, nullptr, st));
  if (int rc = readback(ctx, w, st, nullptr)) return rc;
  {
    int cinfo = 0;
    std::memcpy(&cinfo, &hs[SC_CHOL], sizeof(int));
    if (cinfo < 0) return chol_fail(cinfo);
    if (cinfo != 0) return fail(SSNAL_ENUMERIC, "lambda2 I + Gram: non-positive pivot at row %d", cinfo - 1);
  }
  out->nu = (double)N - lambda2 * hs[SC_MS_FROB];
  const double nan = std::nan("");
  if (r >= m) {
    out->status = 1;
    out->rss = out->gcv = out->ebic = nan;
    HIPCHK(hipStreamSynchronize(st));
    return 0;
  }
  // least squares on the selected features: A_J^T A_J beta = A_J^T b
  HIPCHK(syrk(A, dt, lda, mi, w.J, r, 1, 0.0, 1.0, w.V, w.syrk, st));
  HIPCHK(gemv_t(A, dt, lda, mi, r, w.J, b, w.wd, true, st));
  HIPCHK(hipMemsetAsync(w.info, 0, sizeof(double), st));
  HIPCHK(chol_factor_solve(w.V, (int)r, w.wd, 1.0, w.t3, w.wy, (double*)w.syrk, w.info, st));
  HIPCHK(gather_gemv_partial(A, dt, lda, mi, w.J, w.wy, w.scal + SC_R, n, w.gpart, st));
  HIPCHK(gather_finish(w.gpart, w.scal + SC_R, 0, mi, 2, nullptr, b, nullptr, w.t1, w.scal, st));
  HIPCHK(sum_parts(w.part, 0, w.scal + SC_MS_NONE, w.t1, mi, w.scal + SC_MS_RSS, st));
  if (int rc = readback(ctx, w, st, nullptr)) return rc;
  {
    int cinfo = 0;
    std::memcpy(&cinfo, &hs[SC_CHOL], sizeof(int));
    if (cinfo < 0) return chol_fail(cinfo);
    if (cinfo != 0) {
      out->status = 2;
      out->rss = out->gcv = out->ebic = nan;
      HIPCHK(hipStreamSynchronize(st));
      return 0;
    }
  }
  criteria(hs[SC_MS_RSS]);
  if (beta_out) HIPCHK(scatter(w.J, w.wy, w.scal + SC_R, n, beta_out, st));
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}

int ssnal_ls_delta(ssnal_ctx* ctx, const double* x, const double* w, const double* wd, int64_t n,
                   double sigma, double lambda1, double lambda2, double gd, double dd, int K,
                   const double* s, double* delta_out, hipStream_t stream) {
  g_err[0] = 0;
  if (!ctx || !x || !w || !wd || !s || !delta_out) return fail(SSNAL_EINVAL, "null argument");
  if (n < 1 || K < 1 || K > kMaxTrials) return fail(SSNAL_EINVAL, "need n >= 1 and 1 <= K <= 32");
  for (int k = 1; k < K; ++k)
    if (!(s[k] <= s[k - 1])) return fail(SSNAL_EINVAL, "trial steps must be non-increasing");
  HIPCHK(hipSetDevice(ctx->device));
  Workspace ws;
  if (int rc = prepare(ctx, 1, n, ws)) return rc;
  const ProxArgs pa = prox_args(sigma, lambda1, lambda2);
  LsArgs la;
  la.sigma = sigma;
  la.thr = pa.thr;
  la.den = pa.den;
  la.kappa = sigma / pa.den;
  la.mu = 0.2;
  la.K = K;
  for (int k = 0; k < kMaxTrials; ++k) la.s[k] = k < K ? s[k] : 0.0;
  HIPCHK(ls_delta(x, w, wd, n, la, gd, dd, ws.part, ws.scal, stream));
  if (int rc = readback(ctx, ws, stream, nullptr)) return rc;
  for (int k = 0; k < K; ++k) delta_out[k] = ctx->h_scal[SC_DELTA + k];
  return 0;
}

int ssnal_kkt(ssnal_ctx* ctx, const void* A, ssnal_dtype a_dtype, int64_t lda, const double* b,
              int64_t m, int64_t n, const double* x, double lambda1, double lambda2, double* out4,
              hipStream_t stream) {
  g_err[0] = 0;
  if (!ctx || !x || !out4) return fail(SSNAL_EINVAL, "null argument");
  if (int rc = check_args(A, (int)a_dtype, lda, b, m, n)) return rc;
  if (!(lambda2 >= 0)) return fail(SSNAL_EINVAL, "lambda2 must be >= 0");
  HIPCHK(hipSetDevice(ctx->device));
  Workspace ws;
  if (int rc = prepare(ctx, m, n, ws)) return rc;
  const int dt = (int)a_dtype;
  HIPCHK(support_count(x, n, ws.counts, stream));
  HIPCHK(support_write(x, n, ws.counts, ws.J, ws.uJ, ws.scal + SC_R, stream));
  HIPCHK(gather_gemv_partial(A, dt, lda, (int)m, ws.J, ws.uJ, ws.scal + SC_R, n, ws.gpart, stream));
  // mode 0 with y = 0 gives rho = A x - b and its norms
  HIPCHK(vec_fill(ws.y, 0.0, m, stream));
  HIPCHK(gather_finish(ws.gpart, ws.scal + SC_R, 0, (int)m, 0, ws.y, b, ws.g, ws.rho, ws.scal, stream,
                       Pub{}, m > kDenseMax ? ws.part : nullptr));
  Timer tm{ctx, stream, false};
  int calls = 0;
  if (int rc = certify(A, dt, lda, (int)m, n, x, lambda1, lambda2, ws, stream, tm, &calls)) return rc;
  if (int rc = readback(ctx, ws, stream, nullptr)) return rc;
  double eta, F, D;
  certificate_values(ctx->h_scal, lambda1, lambda2, &eta, &F, &D);
  out4[0] = eta;
  out4[1] = F;
  out4[2] = D;
  out4[3] = (F - D) / (1.0 + std::fabs(F));
  return 0;
}

}  // extern "C"
