// The whole SsNAL-EN solve of a small problem in one workgroup (Algorithm 1:
// the augmented-Lagrangian loop of Sec. 3.1 around the semi-smooth Newton
// inner loop of Sec. 3.2), with no host synchronisation: the outer and inner
// loops, the stopping tests and the certificates all run on the device, and
// a batch of problems is one launch with one workgroup per problem.
//
// For m <= 120 rows and small m n, the multi-kernel path is bound by its
// launches (about 25 kernels and one host read-back per Newton step) rather
// than by any pass over A; here a Newton step costs its passes over A at one
// CU's rate plus a Cholesky of at most 120 x 120 in LDS.
//
// One workgroup of 256 threads per problem, single or batched (the same
// summation orders, so a batched problem gives its single solve's bits);
// at most 256 registers a lane.  A (FP64, column-major, lda >= m) stays in
// global memory (cache-resident at these sizes); the m-vectors (y, g, d,
// rho, b), the Newton matrix (packed as a lower triangle: 58 KB at m = 120)
// and its Cholesky factor live in LDS, and so do the n-vectors (x,
// w_y = A^T y, w_d = A^T d, the active set J and u_J: 36 bytes a feature)
// when they fit beside them, else they stay in global memory (two problems
// can then share a CU).  Per Newton step, in the order of the
// multi-kernel path (and of eq. grad_phy, eq. AJ_system / eq. smw_formula,
// eq. line_search):
//   t = x - sigma w_y, J = {|t| > sigma lambda1} in index order, u_J =
//   prox(t)_J (eq. prox_elastic); g = y + b - A_J u_J; kkt1 (eq. kkt_res);
//   the Newton matrix I + kappa A_J A_J^T (r >= m) or I/kappa + A_J^T A_J
//   (r < m) on FP64 MFMA straight from A; its Cholesky in LDS (8-column
//   panels, the trailing updates on FP64 MFMA); the triangular solves in
//   one wave; d; w_d = A^T d; the trial steps of the line search;
//   y += s d, w_y += s w_d.
// The multiplier update, kkt3 and the certificate eta (with F and D of
// Prop. 1) follow each inner loop as in the multi-kernel path.  Every sum is
// taken in a fixed order, so a solve's result does not depend on which CU
// or batch runs it.
//
// The phases are separate (non-inlined) functions; each reaches LDS through
// the kernel's dynamic LDS array and global memory through address-space-1
// pointers, so the compiler emits LDS and global instructions rather than
// generic ones.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace ssnal {

namespace {

typedef const double __attribute__((address_space(1)))* GCD;
typedef double __attribute__((address_space(1)))* GD;
typedef const int32_t __attribute__((address_space(1)))* GCI;
typedef int32_t __attribute__((address_space(1)))* GI;
typedef const double __attribute__((address_space(3)))* LCD;
typedef double __attribute__((address_space(3)))* LD;
typedef const int32_t __attribute__((address_space(3)))* LCI;
typedef int32_t __attribute__((address_space(3)))* LI;
typedef double d2v __attribute__((ext_vector_type(2)));
typedef const d2v __attribute__((address_space(1)))* GCD2;

// Where the n-vectors of a solve (x, w_y, w_d, u_J, J) live: in global
// memory, or in LDS after the Newton matrix when they fit (36 bytes a
// feature), which takes the global round trips out of every phase but the
// passes over A.
struct InGlobal {
  typedef GD D;
  typedef GCD CD;
  typedef GI I;
  typedef GCI CI;
};
struct InLds {
  typedef LD D;
  typedef LCD CD;
  typedef LI I;
  typedef LCI CI;
};

constexpr int kSmNT = 256;                        // threads a problem
constexpr int kSmWaves = kSmNT / kWave;
constexpr int kSmVec = 128;                       // LDS m-vector length (m <= kSmallMaxM < 128)
constexpr int kSmRows = (kSmallMaxM + 15) / 16;   // rows a lane takes in the 16-lane column layout
constexpr int kSmLsChunk = 8;                     // trial steps summed per pass of the line search

// LDS: these fixed parts, then the lower triangle of the Newton matrix M,
// packed by rows (row i at offset i (i + 1) / 2).
struct SmallLds {
  double y[kSmVec], g[kSmVec], d[kSmVec], rho[kSmVec], b[kSmVec], q[kSmVec];
  double idg[kSmVec];             // 1 / L_kk of the last factorisation
  double part[kSmWaves][kSmVec];  // per-wave partial m-vectors of the gathers
  double red[kSmWaves * 36];      // per-wave partials of the block reductions
  double ts[kMaxTrials];          // the trial steps of the line search
  int cnt[kSmWaves];              // compaction: per-wave counts
  int pad_[kSmWaves];
};
static_assert(sizeof(SmallLds) % 16 == 0, "M starts 16-byte aligned");
// offsets (in doubles) of the m-vectors an A^T v pass reads or writes
constexpr int kOffY = 0, kOffG = kSmVec, kOffD = 2 * kSmVec, kOffRho = 3 * kSmVec, kOffQ = 5 * kSmVec;

extern __shared__ __align__(16) double sm_dyn[];
__device__ __forceinline__ SmallLds& sl() { return *reinterpret_cast<SmallLds*>(sm_dyn); }
__device__ __forceinline__ double* sm_mat() { return sm_dyn + sizeof(SmallLds) / sizeof(double); }
__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }  // start of row i of M

struct SmallCtx {
  int tid, lane, wid;
  int nt, nw;  // threads and waves of the workgroup
  int m;
};

// Sum over the 16 lanes of each row; every lane of the row gets the same bits.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<kQuadXor1>(v);
  v += dpp_d<kQuadXor2>(v);
  v += dpp_d<kRowHalfMirror>(v);
  v += dpp_d<kRowMirror>(v);
  return v;
}

// Sum of K values over the block (every thread receives the K sums): each
// 16-lane row sums with DPP, the first lane of every row stores its row's
// K sums, lane k of every wave adds value k's 16 row sums in (wave, row)
// order, and readlane hands value k from lane k to the wave.  A broadcast
// through a scalar register costs about 70 cycles before its first use;
// this takes K of them in one batch, against 4 K for a wave-wide sum per
// value.
template <int K>
__device__ __forceinline__ void bsum(double (&v)[K], const SmallCtx& c) {
  constexpr int kRows = kSmWaves * 4;
  static_assert(K * kRows <= kSmWaves * 36 && K <= kWave, "row sums fit the reduction buffer");
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = row16_sum(v[k]);
  __syncthreads();
  if ((c.lane & 15) == 0) {
    const int row = c.wid * 4 + (c.lane >> 4);
#pragma unroll
    for (int k = 0; k < K; ++k) sl().red[row * K + k] = v[k];
  }
  __syncthreads();
  const int kk = c.lane < K ? c.lane : K - 1;
  double t = sl().red[kk];
#pragma unroll
  for (int i = 1; i < kRows; ++i) t += sl().red[i * K + kk];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = readlane_d(t, k);
}

// Sum over the 8 lanes of each half-row; every lane of the half gets the same
// bits.
__device__ __forceinline__ double row8_sum(double v) {
  v += dpp_d<kQuadXor1>(v);
  v += dpp_d<kQuadXor2>(v);
  v += dpp_d<kRowHalfMirror>(v);
  return v;
}

// out[j] = sum_{i<m} A[i, col(j)] v[i] for j < n, col(j) = J[j] (GATHER) or
// j; v at LDS offset voff; out to global (ldsout < 0) or to LDS offset
// ldsout.  With colsq, the sum of |a_j|^2 over the n columns (every thread
// receives it).
//
// One CU streams A at the rate its loads in flight allow, and that counts
// instructions rather than bytes (measured at m = 100: 22 bytes a cycle
// with 8-byte loads, 43 with 16-byte loads), so when every column starts
// 16-byte aligned (A aligned, lda even) lane 8 q + s of a wave takes
// column 8 g + q of a group g and the row pairs (2 s, 2 s + 1) + 16 k,
// k < R, with one 16-byte load each; an 8-lane sum finishes each column.
// A pair that straddles m reads row m inside the padded leading dimension
// (lda > m when m is odd and lda even) and masks it.  Other layouts take
// 8-byte loads: lane 16 q + s takes column 4 g + q and rows s + 16 k, a
// 16-lane sum.  Wave w takes groups w U .. w U + U - 1, then every
// (waves * U)-th, with two rounds of loads in flight.
template <int R, bool GATHER, class V>
__device__ __noinline__ void sm_atv_r2(GCD A, int64_t lda, int64_t n, typename V::CI J, int voff,
                                       typename V::D out, int ldsout, double* colsq, SmallCtx c) {
  const int m = c.m;
  const int q = c.lane >> 3, s = c.lane & 7;
  double v0[R], v1[R];
  int rr[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int row = 2 * s + 16 * k;
    v0[k] = row < m ? sm_dyn[voff + row] : 0.0;
    v1[k] = row + 1 < m ? sm_dyn[voff + row + 1] : 0.0;
    rr[k] = row < m ? row : 0;  // a pair past m reads rows 0 and 1
  }
  // rows 2 s + 16 k + 1 < m for every k < R - 1 (16 (R - 1) < m): only the
  // last pair can reach row m, which may hold anything
  const bool hi_ok = 2 * s + 16 * (R - 1) + 1 < m;
  double sq = 0.0;
  constexpr int U = 16 / R > 8 ? 8 : (16 / R < 1 ? 1 : 16 / R);  // about 16 loads a round
  const int64_t ngroups = (n + 7) / 8;
  const int64_t stride = (int64_t)c.nw * U;
  auto load = [&](d2v (&a)[U][R], int64_t g0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = 8 * (g0 + u) + q;
      const int64_t jc = j < n ? j : n - 1;
      const int64_t col = GATHER ? (int64_t)J[jc] : jc;
      GCD p = A + col * lda;
#pragma unroll
      for (int k = 0; k < R; ++k) a[u][k] = *reinterpret_cast<GCD2>(p + rr[k]);
    }
  };
  auto finish = [&](d2v (&a)[U][R], int64_t g0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = 8 * (g0 + u) + q;
      a[u][R - 1][1] = hi_ok ? a[u][R - 1][1] : 0.0;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < R; ++k) acc = fma(a[u][k][1], v1[k], fma(a[u][k][0], v0[k], acc));
      if (colsq) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const bool ok = j < n && 2 * s + 16 * k < m;
          sq += ok ? a[u][k][0] * a[u][k][0] + a[u][k][1] * a[u][k][1] : 0.0;
        }
      }
      acc = row8_sum(acc);
      if (s == 0 && j < n) {
        if (ldsout >= 0)
          sm_dyn[ldsout + j] = acc;
        else
          out[j] = acc;
      }
    }
  };
  d2v a0[U][R], a1[U][R];
  int64_t g0 = (int64_t)c.wid * U;
  if (g0 < ngroups) load(a0, g0);
  for (; g0 < ngroups; g0 += 2 * stride) {
    load(a1, g0 + stride);
    finish(a0, g0);
    if (g0 + stride >= ngroups) break;
    load(a0, g0 + 2 * stride);
    finish(a1, g0 + stride);
  }
  if (colsq) {
    double t[1] = {sq};
    bsum<1>(t, c);
    *colsq = t[0];
  }
  __syncthreads();  // out complete for every thread
}

template <int R, bool GATHER, class V>
__device__ __noinline__ void sm_atv_r(GCD A, int64_t lda, int64_t n, typename V::CI J, int voff,
                                      typename V::D out, int ldsout, double* colsq, SmallCtx c) {
  const int m = c.m;
  const int q = c.lane >> 4, s = c.lane & 15;
  double vv[R];
  int rr[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int row = s + 16 * k;
    vv[k] = row < m ? sm_dyn[voff + row] : 0.0;
    rr[k] = row < m ? row : 0;  // a masked lane reads row 0 (never a padding row)
  }
  double sq = 0.0;
  constexpr int U = 32 / R > 8 ? 8 : 32 / R;  // groups per round (about 32 loads)
  const int64_t ngroups = (n + 3) / 4;
  const int64_t stride = (int64_t)c.nw * U;
  // loads of a round (columns clamped to n - 1: a round past the end reads
  // in bounds and stores nothing)
  auto load = [&](double (&a)[U][R], int64_t g0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = 4 * (g0 + u) + q;
      const int64_t jc = j < n ? j : n - 1;
      const int64_t col = GATHER ? (int64_t)J[jc] : jc;
      GCD p = A + col * lda;
#pragma unroll
      for (int k = 0; k < R; ++k) a[u][k] = p[rr[k]];
    }
  };
  auto finish = [&](const double (&a)[U][R], int64_t g0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = 4 * (g0 + u) + q;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < R; ++k) acc = fma(a[u][k], vv[k], acc);
      if (colsq) {
#pragma unroll
        for (int k = 0; k < R; ++k) sq += (j < n && s + 16 * k < m) ? a[u][k] * a[u][k] : 0.0;
      }
      acc = row16_sum(acc);
      if (s == 0 && j < n) {
        if (ldsout >= 0)
          sm_dyn[ldsout + j] = acc;
        else
          out[j] = acc;
      }
    }
  };
  // two rounds in flight: the next round's loads are issued before this
  // round's sums
  double a0[U][R], a1[U][R];
  int64_t g0 = (int64_t)c.wid * U;
  if (g0 < ngroups) load(a0, g0);
  for (; g0 < ngroups; g0 += 2 * stride) {
    load(a1, g0 + stride);
    finish(a0, g0);
    if (g0 + stride >= ngroups) break;
    load(a0, g0 + 2 * stride);
    finish(a1, g0 + stride);
  }
  if (colsq) {
    double t[1] = {sq};
    bsum<1>(t, c);
    *colsq = t[0];
  }
  __syncthreads();  // out complete for every thread
}

template <bool GATHER, class V>
__device__ __forceinline__ void sm_atv(GCD A, int64_t lda, int64_t n, typename V::CI J, int voff,
                                       typename V::D out, int ldsout, double* colsq, const SmallCtx& c) {
  if ((reinterpret_cast<uintptr_t>(A) & 15) != 0 || (lda & 1) != 0) {
    switch ((c.m + 15) / 16) {
      case 1: sm_atv_r<1, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
      case 2: sm_atv_r<2, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
      case 3: sm_atv_r<3, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
      case 4: sm_atv_r<4, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
      case 5: sm_atv_r<5, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
      case 6: sm_atv_r<6, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
      case 7: sm_atv_r<7, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
      default: sm_atv_r<kSmRows, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
    }
    return;
  }
  switch ((c.m + 15) / 16) {
    case 1: sm_atv_r2<1, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
    case 2: sm_atv_r2<2, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
    case 3: sm_atv_r2<3, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
    case 4: sm_atv_r2<4, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
    case 5: sm_atv_r2<5, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
    case 6: sm_atv_r2<6, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
    case 7: sm_atv_r2<7, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
    default: sm_atv_r2<kSmRows, GATHER, V>(A, lda, n, J, voff, out, ldsout, colsq, c); break;
  }
}

// out[i] = sum_{k<r} A[i, J[k]] coef[k] for i < m (coef an n-vector), into LDS at
// offset ooff.  Lane l takes rows 2 l and 2 l + 1 (16-byte loads, when
// every column starts 16-byte aligned) or rows l and l + 64; wave w takes
// k = w, w + waves, ... (eight at a time); the per-wave partial m-vectors
// are added in wave order.
template <class V>
__device__ __noinline__ void sm_gather(GCD A, int64_t lda, typename V::CI J, typename V::CD coef, int64_t r,
                                       int ooff, SmallCtx c) {
  const int m = c.m;
  constexpr int U = 8;
  if ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda & 1) == 0) {
    // 16-byte loads: lane l takes rows 2 l and 2 l + 1 (one load a column;
    // a pair that straddles m reads row m inside the padded leading
    // dimension and masks it), each row summed in the same order as below
    const int l2 = 2 * c.lane;
    const int rp = l2 < m ? l2 : 0;
    const bool ok0 = l2 < m, ok1 = l2 + 1 < m;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t k0 = c.wid; k0 < r; k0 += (int64_t)c.nw * U) {
      d2v a[U];
      double cf[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = k0 + (int64_t)c.nw * u;
        const int64_t kc = k < r ? k : r - 1;
        a[u] = *reinterpret_cast<GCD2>(A + (int64_t)J[kc] * lda + rp);
        cf[u] = coef[kc];
        cf[u] = k < r ? cf[u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        s0 = fma(ok0 ? a[u][0] : 0.0, cf[u], s0);
        s1 = fma(ok1 ? a[u][1] : 0.0, cf[u], s1);
      }
    }
    sl().part[c.wid][l2] = s0;
    sl().part[c.wid][l2 + 1] = s1;
  } else {
    const int l0 = c.lane, l1 = c.lane + kWave;
    const int r0 = l0 < m ? l0 : 0, r1 = l1 < m ? l1 : 0;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t k0 = c.wid; k0 < r; k0 += (int64_t)c.nw * U) {
      double a0[U], a1[U], cf[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = k0 + (int64_t)c.nw * u;
        const int64_t kc = k < r ? k : r - 1;
        GCD col = A + (int64_t)J[kc] * lda;
        a0[u] = col[r0];
        a1[u] = col[r1];  // unconditional (row clamped): a load in a branch would wait at the join
        cf[u] = coef[kc];
        cf[u] = k < r ? cf[u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        s0 = fma(l0 < m ? a0[u] : 0.0, cf[u], s0);
        s1 = fma(l1 < m ? a1[u] : 0.0, cf[u], s1);
      }
    }
    sl().part[c.wid][l0] = s0;
    sl().part[c.wid][l1] = s1;
  }
  __syncthreads();
  if (c.tid < m) {
    double t = sl().part[0][c.tid];
    for (int w = 1; w < c.nw; ++w) t += sl().part[w][c.tid];
    sm_dyn[ooff + c.tid] = t;
  }
  __syncthreads();
}

// Newton matrix into M (lower triangle), FP64 MFMA 16x16x4 straight from A:
//   form 0: M = I_m + kappa A_J A_J^T      (N = m, contraction over the r columns)
//   form 1: M = I_r / kappa + A_J^T A_J    (N = r, contraction over the m rows)
// 16 x 16 blocks of the lower triangle round-robin over the waves.  In form
// 1 with every column 16-byte aligned (A aligned, lda even), a lane loads
// the row pair (8 t + 2 q, 8 t + 2 q + 1), q = lane / 16, of its column
// with one 16-byte load and feeds the two rows to two 16x16x4 steps (the
// contraction taken in that fixed order, the same for both operands): half
// the load instructions, which bound one CU's rate from the caches.  A
// pair that straddles an odd m reads row m inside the padded leading
// dimension and masks it.
template <class V>
__device__ __noinline__ void sm_gram(GCD A, int64_t lda, typename V::CI J, int64_t r, int form, double kappa,
                                     SmallCtx c) {
  double* M = sm_mat();
  const int m = c.m;
  const int N = form ? (int)r : m;
  const int64_t K = form ? (int64_t)m : r;
  const int nbk = (N + 15) / 16;
  const int nblk = nbk * (nbk + 1) / 2;
  const bool pairs = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda & 1) == 0;
  for (int blk = c.wid; blk < nblk; blk += c.nw) {
    int bi = (int)((sqrtf(8.0f * (float)blk + 1.0f) - 1.0f) * 0.5f);
    while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
    while (bi * (bi + 1) / 2 > blk) --bi;
    const int bj = blk - bi * (bi + 1) / 2;
    const int pa = 16 * bi + (c.lane & 15), pb = 16 * bj + (c.lane & 15);
    const bool oka = pa < N, okb = pb < N;
    const int pac = oka ? pa : N - 1, pbc = okb ? pb : N - 1;
    // form 1: the gathered columns of this block's rows and columns
    GCD ca = A + (int64_t)(form ? J[pac] : 0) * lda;
    GCD cb = A + (int64_t)(form ? J[pbc] : 0) * lda;
    dbl4 acc = dbl4{0, 0, 0, 0};
    constexpr int U = 16;
    // the form is decided outside the load loops: a load in a branch would
    // wait at the join, serialising the U loads
    auto contract = [&](auto gathered_rows) {
      for (int64_t k0 = 0; k0 < K; k0 += 4 * U) {
        double av[U], bv[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t kk = k0 + 4 * u + c.lane / 16;
          ok[u] = kk < K;
          const int64_t kc = ok[u] ? kk : K - 1;
          if constexpr (decltype(gathered_rows)::value) {
            GCD col = A + (int64_t)J[kc] * lda;
            av[u] = col[pac];
            bv[u] = col[pbc];
          } else {
            av[u] = ca[kc];
            bv[u] = cb[kc];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double a = (ok[u] & oka) ? av[u] : 0.0;
          const double b = (ok[u] & okb) ? bv[u] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
      }
    };
    // form 1, aligned columns: row pairs by 16-byte loads
    auto contract_pairs = [&]() {
      constexpr int U2 = 8;
      const int q2 = 2 * (c.lane / 16);
      // the second row of each pair goes to a second accumulator, added at
      // the end: two dependent MFMA chains of half the length
      dbl4 acc2 = dbl4{0, 0, 0, 0};
      for (int64_t k0 = 0; k0 < K; k0 += 8 * U2) {
        d2v av[U2], bv[U2];
#pragma unroll
        for (int u = 0; u < U2; ++u) {
          const int64_t row = k0 + 8 * u + q2;
          const int64_t rc = row < K ? row : 0;
          av[u] = *reinterpret_cast<GCD2>(ca + rc);
          bv[u] = *reinterpret_cast<GCD2>(cb + rc);
        }
#pragma unroll
        for (int u = 0; u < U2; ++u) {
          const int64_t row = k0 + 8 * u + q2;
          const bool ok0 = row < K, ok1 = row + 1 < K;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64((ok0 & oka) ? av[u][0] : 0.0, (ok0 & okb) ? bv[u][0] : 0.0,
                                                     acc, 0, 0, 0);
          acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64((ok1 & oka) ? av[u][1] : 0.0, (ok1 & okb) ? bv[u][1] : 0.0,
                                                      acc2, 0, 0, 0);
        }
      }
      acc += acc2;
    };
    if (form && pairs)
      contract_pairs();
    else if (form)
      contract(std::false_type{});
    else
      contract(std::true_type{});
    // accumulator v holds row lane/16 + 4v, column lane%16 of the block
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * bi + c.lane / 16 + 4 * v, col = 16 * bj + (c.lane & 15);
      if (row < N && col <= row) {
        const double e = form ? acc[v] + (row == col ? 1.0 / kappa : 0.0)
                              : fma(kappa, acc[v], row == col ? 1.0 : 0.0);
        M[tri(row) + col] = e;
      }
    }
  }
  __syncthreads();
}

// 1/sqrt(t) for a positive normal t: hardware estimate, two Newton steps.
__device__ __forceinline__ double sm_rsqrt(double t) {
  double y = __builtin_amdgcn_rsq(t);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-(t * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Smallest pivot accepted (the smallest normal double).
constexpr double kSmMinPivot = 2.2250738585072014e-308;

// Cholesky of the N x N lower triangle of M in place (L below and on the
// diagonal; 1 / L_kk into idg), right-looking in 8-column panels: every
// thread factors the 8 x 8 pivot block itself (same bits everywhere) and the
// rows below solve against it; after one barrier the trailing lower triangle
// takes the rank-8 update while the pivot block's L is written (no thread
// reads that block after its factorisation), then a second barrier.
// Returns the first non-positive pivot's row + 1, or 0.
__device__ __noinline__ int sm_cholesky(int N, SmallCtx c) {
  double* M = sm_mat();
  for (int j0 = 0; j0 < N; j0 += 8) {
    const int w = N - j0 < 8 ? N - j0 : 8;
    double l[8][8], rl[8];
    // unconditional loads (rows and columns clamped into the block), then
    // the identity past its w rows: a load in a branch would wait at the join
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int k = 0; k <= i; ++k) {
        const int ic = i < w ? i : w - 1, kc = k <= ic ? k : ic;
        l[i][k] = M[tri(j0 + ic) + j0 + kc];
      }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int k = 0; k <= i; ++k) l[i][k] = (i < w) ? l[i][k] : (i == k ? 1.0 : 0.0);
    int bad = -1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      double t = l[k][k];
#pragma unroll
      for (int q = 0; q < k; ++q) t = fma(-l[k][q], l[k][q], t);
      if (!(t >= kSmMinPivot) && bad < 0 && k < w) bad = k;
      const double y = sm_rsqrt(t >= kSmMinPivot ? t : 1.0);
      rl[k] = y;
      l[k][k] = t * y;
#pragma unroll
      for (int i = k + 1; i < 8; ++i) {
        double u = l[i][k];
#pragma unroll
        for (int q = 0; q < k; ++q) u = fma(-l[i][q], l[k][q], u);
        l[i][k] = u * y;
      }
    }
    if (bad >= 0) {
      __syncthreads();  // every thread has read the pivot block (the caller reuses LDS)
      return j0 + bad + 1;  // the same in every thread
    }
    // the rows below the pivot block: x L^T = (their 8 entries)
    for (int R = j0 + w + c.tid; R < N; R += c.nt) {
      double x[8], raw[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) raw[k] = M[tri(R) + j0 + (k < w ? k : w - 1)];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        double u = k < w ? raw[k] : 0.0;
#pragma unroll
        for (int q = 0; q < k; ++q) u = fma(-x[q], l[k][q], u);
        x[k] = u * rl[k];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < w) M[tri(R) + j0 + k] = x[k];
    }
    __syncthreads();
    // the pivot block's L and 1 / L_kk (compile-time row index: l stays in
    // registers), by the first lanes of the last wave, which takes the
    // fewest trailing blocks below
    const int pl = c.tid - (c.nt - kWave);
    if (pl >= 0 && pl < w) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (pl == i) {
          sl().idg[j0 + i] = rl[i];
#pragma unroll
          for (int k = 0; k <= i; ++k) M[tri(j0 + i) + j0 + k] = l[i][k];
        }
    }
    // trailing update M[i][j] -= sum_k L[i][j0+k] L[j][j0+k], j0+w <= j <= i < N
    // (w = 8: only the last panel is narrower, and nothing trails it), on
    // the FP64 matrix cores: one 16 x 16 block of the lower triangle per
    // wave at a time, two 16x16x4 steps over the panel's 8 columns (the
    // panel's columns are read, columns >= j0 + 8 written: no overlap)
    const int b = j0 + w, nt = N - b;
    const int nbk = (nt + 15) / 16;
    const int nblk = nt > 0 ? nbk * (nbk + 1) / 2 : 0;
    for (int blk = c.wid; blk < nblk; blk += c.nw) {
      int bi = (int)((sqrtf(8.0f * (float)blk + 1.0f) - 1.0f) * 0.5f);
      while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
      while (bi * (bi + 1) / 2 > blk) --bi;
      const int bj = blk - bi * (bi + 1) / 2;
      const int kq = c.lane >> 4, l16 = c.lane & 15;
      // operands: A[i][k] = L[b + 16 bi + i][j0 + k], B[k][j] = L[b + 16 bj + j][j0 + k]
      // (rows past nt clamped: they feed only outputs that are not stored)
      const int ia = 16 * bi + l16, ja = 16 * bj + l16;
      const double* La = M + tri(b + (ia < nt ? ia : nt - 1)) + j0;
      const double* Lb = M + tri(b + (ja < nt ? ja : nt - 1)) + j0;
      const double a0 = La[kq], a1 = La[kq + 4], b0 = Lb[kq], b1 = Lb[kq + 4];
      // accumulator v: row 16 bi + kq + 4 v, column 16 bj + l16 of the trailing block
      dbl4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * bi + kq + 4 * v, j = 16 * bj + l16;
        const int ic = i < nt ? i : nt - 1;
        acc[v] = M[tri(b + ic) + b + (j < ic ? j : ic)];
      }
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a0, b0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a1, b1, acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * bi + kq + 4 * v, j = 16 * bj + l16;
        if (i < nt && j <= i) M[tri(b + i) + b + j] = acc[v];
      }
    }
    __syncthreads();
  }
  return 0;
}

// x = (L L^T)^{-1} rhs with the factor in M (rows packed) and 1 / L_kk in
// idg (N <= kSmVec); rhs and x at LDS offsets (may alias; rhs is consumed).
// One wave sweeps the columns with no barrier: lane l holds rows l and (TWO)
// l + 64 of the right-hand side; at column k the lane holding row k scales
// it, readlane hands the value to every lane, and each lane takes its
// row's term.  The entries of L a lane needs are loaded eight columns ahead
// (unconditional, indices clamped into the row) and zeroed where the row
// takes no term, so a step is a multiply, a broadcast and an FMA; a row's
// value stops changing once its column has passed, so the values handed
// out are recomputed at the end with the same operation.  Forward,
// each row adds its terms in column order; backward (L^T x = y, row k of
// L^T is column k of L, a contiguous row slice across the lanes), in
// descending column order.  The other waves wait at the closing barrier.
// Measured at N = 43: 15.4k cycles for both sweeps against 26.0k for
// 8-row blocks solved by all four waves with a barrier per block (a
// column's broadcast through a scalar register costs about 70 cycles;
// blocks of 8 columns per broadcast in one wave measured 30.8k).
template <bool TWO>
__device__ __forceinline__ void chol_solve_wave(int N, int rhs_off, int x_off, int lane) {
  const double* M = sm_mat();
  const double* idg = sl().idg;
  const int r0 = lane, r1 = lane + kWave;
  // rows past N (no result) address row N - 1
  const int q0 = r0 < N ? r0 : N - 1, q1 = r1 < N ? r1 : N - 1;
  const int b0 = tri(q0), b1 = tri(q1);
  double z0 = r0 < N ? sm_dyn[rhs_off + r0] : 0.0;
  double z1 = TWO && r1 < N ? sm_dyn[rhs_off + r1] : 0.0;
  // each lane scales its own rows (1 / L_ii in a register), so the lane
  // that owns column k hands out z_k / L_kk with no broadcast load
  const double d0 = idg[q0], d1 = TWO ? idg[q1] : 0.0;
  // forward: L y = rhs; row i takes -L_ik y_k for k < i
  {
    auto load = [&](double (&a0)[8], double (&a1)[8], int k0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + u;
        const double v0 = M[b0 + (k < q0 ? k : 0)];
        a0[u] = k < r0 ? v0 : 0.0;  // zero where the row takes no term: -0 y leaves it as it is
        if (TWO) {
          const double v1 = M[b1 + (k < q1 ? k : 0)];
          a1[u] = k < r1 ? v1 : 0.0;
        }
      }
    };
    auto step = [&](const double (&a0)[8], const double (&a1)[8], int k0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + u;  // k >= N: no row takes a term
        const double t = TWO && k >= kWave ? z1 * d1 : z0 * d0;
        const double y = readlane_d(t, k & (kWave - 1));
        z0 = fma(-a0[u], y, z0);
        if (TWO) z1 = fma(-a1[u], y, z1);
      }
    };
    double a0[8], a1[8], c0[8], c1[8];
    load(a0, a1, 0);
    for (int k0 = 0; k0 < N; k0 += 16) {
      load(c0, c1, k0 + 8);
      step(a0, a1, k0);
      if (k0 + 8 >= N) break;
      load(a0, a1, k0 + 16);
      step(c0, c1, k0 + 8);
    }
  }
  // y_i = z_i / L_ii (the value the sweep handed out at column i)
  z0 *= d0;
  if (TWO) z1 *= d1;
  // backward: L^T x = y; row i takes -L_ki x_k for k > i, k descending
  {
    auto load = [&](double (&a0)[8], double (&a1)[8], int k0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 - u < 0 ? 0 : k0 - u;
        const double v0 = M[tri(k) + (r0 < k ? r0 : k)];
        a0[u] = r0 < k0 - u ? v0 : 0.0;  // k0 - u < 0: no row takes a term
        if (TWO) {
          const double v1 = M[tri(k) + (r1 < k ? r1 : k)];
          a1[u] = r1 < k0 - u ? v1 : 0.0;
        }
      }
    };
    auto step = [&](const double (&a0)[8], const double (&a1)[8], int k0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 - u;  // k < 0: no row takes a term
        const double t = TWO && k >= kWave ? z1 * d1 : z0 * d0;
        const double x = readlane_d(t, k & (kWave - 1));
        z0 = fma(-a0[u], x, z0);
        if (TWO) z1 = fma(-a1[u], x, z1);
      }
    };
    double a0[8], a1[8], c0[8], c1[8];
    const int top = N - 1;
    load(a0, a1, top);
    for (int k0 = top; k0 >= 0; k0 -= 16) {
      load(c0, c1, k0 - 8);
      step(a0, a1, k0);
      if (k0 - 8 < 0) break;
      load(a0, a1, k0 - 16);
      step(c0, c1, k0 - 8);
    }
    // a row's value stops changing once its column has passed: x_i is the
    // value the sweep handed out at column i, recomputed here
    if (r0 < N) sm_dyn[x_off + r0] = z0 * d0;
    if (TWO && r1 < N) sm_dyn[x_off + r1] = z1 * d1;
  }
}

__device__ __noinline__ void sm_chol_solve(int N, int rhs_off, int x_off, SmallCtx c) {
  if (c.wid == 0) {
    if (N > kWave)
      chol_solve_wave<true>(N, rhs_off, x_off, c.lane);
    else
      chol_solve_wave<false>(N, rhs_off, x_off, c.lane);
  }
  __syncthreads();
}

// The active set of t = x - sigma w_y (after w_y += s w_d when s != 0):
// J in index order, u_J = prox(t)_J.  Wave w owns the slab [w S, (w+1) S)
// of the features (S a multiple of 64): it counts its actives with wave
// ballots, the counts are scanned once in LDS, and a second walk writes J
// and u_J at the wave's offset.  Returns r.
template <class V>
__device__ __noinline__ int64_t sm_prox(typename V::D x, typename V::D wy, typename V::CD wd, int64_t n, double s,
                                        double sigma, double thr, double den, typename V::I J, typename V::D uJ,
                                        SmallCtx c) {
  const int64_t S = ((n + c.nt - 1) / c.nt) * kWave;
  const int64_t lo = (int64_t)c.wid * S;
  const int64_t hi = lo + S < n ? lo + S : n;
  // both passes take four chunks of 64 at a time, their loads issued
  // together (indices clamped into the slab)
  constexpr int Q = 4;
  int cnt = 0;
  for (int64_t i0 = lo; i0 < hi; i0 += Q * kWave) {
    double w[Q], dw[Q], xi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = i0 + q * kWave + c.lane;
      const int64_t ic = i < hi ? i : hi - 1;
      w[q] = wy[ic];
      dw[q] = wd[ic];  // unconditional: a load in a branch would wait at the join
      xi[q] = x[ic];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = i0 + q * kWave + c.lane;
      const bool in = i < hi;
      if (s != 0.0) {
        w[q] = fma(s, dw[q], w[q]);
        if (in) wy[i] = w[q];
      }
      const double t = fma(-sigma, w[q], xi[q]);
      const bool act = in & ((t > thr) | (t < -thr));
      cnt += __builtin_popcountll(__builtin_amdgcn_ballot_w64(act));
    }
  }
  if (c.lane == 0) sl().cnt[c.wid] = cnt;
  __syncthreads();
  int base = 0, r = 0;
  for (int w2 = 0; w2 < c.nw; ++w2) {
    const int v = sl().cnt[w2];
    base += w2 < c.wid ? v : 0;
    r += v;
  }
  for (int64_t i0 = lo; i0 < hi; i0 += Q * kWave) {
    double w[Q], xi[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = i0 + q * kWave + c.lane;
      const int64_t ic = i < hi ? i : hi - 1;
      w[q] = wy[ic];
      xi[q] = x[ic];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = i0 + q * kWave + c.lane;
      const bool in = i < hi;
      const double t = fma(-sigma, w[q], xi[q]);
      const bool act = in & ((t > thr) | (t < -thr));
      const uint64_t bal = __builtin_amdgcn_ballot_w64(act);
      if (act) {
        const int pos = base + __builtin_popcountll(bal & ((1ull << c.lane) - 1ull));
        J[pos] = (int32_t)i;
        uJ[pos] = prox_en(t, thr, den);
      }
      base += __builtin_popcountll(bal);
    }
  }
  __syncthreads();  // J and u_J complete for every thread; cnt read
  return r;
}

// The line search of eq. line_search: Delta(s) = s g^T d + s^2/2 |d|^2 +
// sum_i e_i(s) with e_i as in the multi-kernel path's pass (a feature that
// stays inactive contributes nothing; one that stays on its active side,
// s^2 kappa wd_i^2 / 2), the trial steps in chunks of 8 in order: the index
// of the first step with Delta(s) <= mu s g^T d, or -1.
template <class V>
__device__ __noinline__ int sm_linesearch(typename V::CD x, typename V::CD wy, typename V::CD wd, int64_t n,
                                          double sigma, double thr, double den,
                                          double kappa, double gd, double dd, int K, double mu, SmallCtx c) {
  const double* ts = sl().ts;
  const double rden = 1.0 / den, h = den / (2.0 * sigma);
  const double smax = ts[0];
  double common = 0.0;  // sum of kappa/2 w_i^2 over features active on one side for every step
  for (int k0 = 0; k0 < K; k0 += kSmLsChunk) {
    double e[kSmLsChunk + 1];
#pragma unroll
    for (int k = 0; k <= kSmLsChunk; ++k) e[k] = 0.0;
    double sk[kSmLsChunk];
#pragma unroll
    for (int k = 0; k < kSmLsChunk; ++k) sk[k] = k0 + k < K ? ts[k0 + k] : 0.0;
    // each iteration loads the next feature's values first (index clamped),
    // so the loads overlap the current feature's work
    int64_t ic = c.tid < n ? c.tid : n - 1;
    double xn = x[ic], yn = wy[ic], dn = wd[ic];
#pragma unroll 1
    for (int64_t i = c.tid; i < n; i += c.nt) {
      const double t0 = fma(-sigma, yn, xn);
      const double wi = dn;
      ic = i + c.nt < n ? i + c.nt : n - 1;
      xn = x[ic];
      yn = wy[ic];
      dn = wd[ic];
      const double a0 = fabs(t0);
      const double reach = smax * sigma * fabs(wi) * (1.0 + 1e-12);
      if (a0 + reach < thr) continue;  // inactive for every trial step
      const double hk = 0.5 * kappa * wi * wi;
      if (((t0 > thr) & (t0 - reach > thr)) | ((t0 < -thr) & (t0 + reach < -thr))) {
        e[kSmLsChunk] += hk;  // same active side for every trial step
        continue;
      }
      const double u0 = prox_en(t0, thr, den);
#pragma unroll
      for (int k = 0; k < kSmLsChunk; ++k) {
        const double t1 = fma(-(sk[k] * sigma), wi, t0);
        const bool same = ((t0 > thr) & (t1 > thr)) | ((t0 < -thr) & (t1 < -thr));
        const double num = t1 > thr ? t1 - thr : (t1 < -thr ? t1 + thr : 0.0);
        const double u1 = num * rden;
        const double other = h * (u1 * u1 - u0 * u0) + sk[k] * wi * u0;
        e[k] += same ? sk[k] * sk[k] * hk : other;
      }
    }
    bsum<kSmLsChunk + 1>(e, c);
    if (k0 == 0) common = e[kSmLsChunk];
#pragma unroll
    for (int k = 0; k < kSmLsChunk; ++k) {
      const double delta = sk[k] * gd + 0.5 * sk[k] * sk[k] * dd + sk[k] * sk[k] * common + e[k];
      if (k0 + k < K && delta <= mu * sk[k] * gd) return k0 + k;  // the same in every thread
    }
  }
  return -1;
}

// The solve of one problem with its n-vectors in V's memory (x, wy, wd, uJ,
// J); in LDS, x is written back to the problem's x at the end.
template <class V>
__device__ __forceinline__ void solve_body(const SmallArgs& pr, const SmallOpts& o, const Pub& pub, SmallCtx c,
                                           typename V::D x, typename V::D wy, typename V::D wd,
                                           typename V::D uJ, typename V::I J) {
  GCD A = (GCD)pr.A;
  GCD bvec = (GCD)pr.b;
  GCD x0 = (GCD)pr.x0;
  const int64_t lda = pr.lda, n = pr.n;
  const int m = pr.m;
  c.m = m;
  SmallLds& L = sl();
  const double l1 = pr.l1, l2 = pr.l2, tol = pr.tol;

  // ---- start: x = x0 (or 0), y = A x0 - b, w_y = A^T y, sum |a_j|^2, |b|^2
  if (c.tid < m) L.b[c.tid] = bvec[c.tid];
  if (c.tid < kMaxTrials) L.ts[c.tid] = o.s[c.tid];
  int64_t r = 0;
  bool x0_nonfinite = false;  // a NaN would drop out of the support compaction below
  if (pr.x0) {
    // support of x0 (as a compaction with threshold 0), then y = A_S x0_S - b
    int bad_x0 = 0;
    for (int64_t i = c.tid; i < n; i += c.nt) {
      const double xi = x0[i];
      bad_x0 |= !(fabs(xi) < INFINITY);
      x[i] = xi;
      wy[i] = 0.0;
    }
    x0_nonfinite = __syncthreads_or(bad_x0) != 0;
    // u_J = prox(t) with thr 0, den 1: t = x (w_y = 0), so u_J = x_J
    r = sm_prox<V>(x, wy, wd, n, 0.0, 1.0, 0.0, 1.0, J, uJ, c);
    sm_gather<V>(A, lda, J, uJ, r, kOffY, c);
    if (c.tid < m) L.y[c.tid] -= L.b[c.tid];
  } else {
    for (int64_t i = c.tid; i < n; i += c.nt) x[i] = 0.0;
    if (c.tid < m) L.y[c.tid] = -L.b[c.tid];
  }
  __syncthreads();
  double colsq = 0.0;
  sm_atv<false, V>(A, lda, n, nullptr, kOffY, wy, -1, &colsq, c);
  double nb2[1] = {c.tid < m ? L.b[c.tid] * L.b[c.tid] : 0.0};
  bsum<1>(nb2, c);
  const double normb = sqrt(nb2[0]);
  double sigma = pr.sigma0;
  if (!(sigma > 0.0)) {
    const double mean = colsq / (double)n;
    sigma = 2.5 / (mean > 0.0 ? mean : 1.0);
  }
  const double sigma0 = sigma;
  const bool bad_sigma = !(sigma > 0.0 && sigma < INFINITY);  // a subnormal mean column norm
  int passes = 1;  // full A^T v passes over the n columns

  double kkt1 = INFINITY, kkt3 = INFINITY, eta = INFINITY, F = NAN, D = NAN;
  double eps_in = tol;
  int status = 1, newton = 0, outer_done = 0;
  bool stalled = false, converged = false, chol_bad = false;
  bool nonfinite = x0_nonfinite || !(normb < INFINITY && colsq < INFINITY);
  double pend = 0.0;  // the pending line-search step (w_y += pend w_d)
  double RR = 0.0, BR = 0.0;

  int chol_row = 0;  // row + 1 of a non-positive pivot
  for (int outer = 0; outer < o.max_outer && !nonfinite && !bad_sigma; ++outer) {
    const double den = fma(sigma, l2, 1.0);
    const double thr = sigma * l1;
    const double kappa = sigma / den;
    int inner = 0;
    for (;;) {
      // ---- prox, active set, gradient (eq. grad_phy), kkt1 (eq. kkt_res)
      r = sm_prox<V>(x, wy, wd, n, pend, sigma, thr, den, J, uJ, c);
      pend = 0.0;
      sm_gather<V>(A, lda, J, uJ, r, kOffRho, c);  // A_J u_J
      double s3[3] = {0.0, 0.0, 0.0};
      if (c.tid < m) {
        const double au = L.rho[c.tid];
        const double gi = L.y[c.tid] + L.b[c.tid] - au;
        const double rh = au - L.b[c.tid];
        L.g[c.tid] = gi;
        L.rho[c.tid] = rh;
        s3[0] = gi * gi;
        s3[1] = rh * rh;
        s3[2] = L.b[c.tid] * rh;
      }
      bsum<3>(s3, c);
      RR = s3[1];
      BR = s3[2];
      kkt1 = sqrt(s3[0]) / (1.0 + normb);
      if (!(kkt1 < INFINITY)) {  // a non-finite A, b, x0 or iterate
        nonfinite = true;
        break;
      }
      if (kkt1 <= eps_in || inner >= o.max_inner) break;
      // ---- Newton direction: (I + kappa A_J A_J^T) d = -g (eq. AJ_system),
      // via the r x r system of eq. smw_formula when 0 < r < m
      if (r == 0) {
        if (c.tid < m) L.d[c.tid] = -L.g[c.tid];
        __syncthreads();
      } else if (r < m && !o.no_smw) {
        // q: W q = A_J^T g, W = I/kappa + A_J^T A_J; d = -g + A_J q
        const int N = (int)r;
        sm_atv<true, V>(A, lda, r, J, kOffG, nullptr, kOffQ, nullptr, c);  // A_J^T g into q
        sm_gram<V>(A, lda, J, r, 1, kappa, c);
        const int bad = sm_cholesky(N, c);
        if (bad) {
          chol_bad = true;
          chol_row = bad;
          break;
        }
        sm_chol_solve(N, kOffQ, kOffQ, c);
        // d = -g + A_J q (q staged in w_d, which the pass below rewrites)
        for (int k = c.tid; k < N; k += c.nt) wd[k] = L.q[k];
        __syncthreads();
        sm_gather<V>(A, lda, J, wd, r, kOffD, c);
        if (c.tid < m) L.d[c.tid] -= L.g[c.tid];
        __syncthreads();
      } else {
        sm_gram<V>(A, lda, J, r, 0, kappa, c);
        const int bad = sm_cholesky(m, c);
        if (bad) {
          chol_bad = true;
          chol_row = bad;
          break;
        }
        if (c.tid < m) L.q[c.tid] = -L.g[c.tid];
        __syncthreads();
        sm_chol_solve(m, kOffQ, kOffD, c);
      }
      // ---- w_d = A^T d, the pass over A
      sm_atv<false, V>(A, lda, n, nullptr, kOffD, wd, -1, nullptr, c);
      ++passes;
      // ---- line search (eq. line_search)
      double gd2[2] = {c.tid < m ? L.g[c.tid] * L.d[c.tid] : 0.0, c.tid < m ? L.d[c.tid] * L.d[c.tid] : 0.0};
      bsum<2>(gd2, c);
      const double gd = gd2[0], dd = gd2[1];
      const int ks = sm_linesearch<V>(x, wy, wd, n, sigma, thr, den, kappa, gd, dd, o.K, o.mu, c);
      if (ks < 0) {
        stalled = true;
        break;
      }
      const double s = L.ts[ks];
      if (c.tid < m) L.y[c.tid] = fma(s, L.d[c.tid], L.y[c.tid]);
      __syncthreads();
      pend = s;  // w_y += s w_d at the next prox
      ++newton;
      ++inner;
    }
    if (chol_bad || nonfinite) break;
    // ---- multiplier update x <- prox(x - sigma w_y), kkt3
    double s3[3] = {0.0, 0.0, 0.0};
    for (int64_t i = c.tid; i < n; i += c.nt) {
      const double xi = x[i];
      const double t = fma(-sigma, wy[i], xi);
      const double u = prox_en(t, thr, den);
      const double z = t >= thr ? (t * l2 + l1) / den : (t <= -thr ? (t * l2 - l1) / den : t / sigma);
      const double ex = xi - u;
      s3[0] = fma(ex, ex, s3[0]);
      s3[1] = fma(z, z, s3[1]);
      x[i] = u;
    }
    if (c.tid < m) s3[2] = L.y[c.tid] * L.y[c.tid];
    bsum<3>(s3, c);
    ++outer_done;
    kkt3 = sqrt(s3[0]) / sigma / (1.0 + sqrt(s3[2]) + sqrt(s3[1]));
    bool need_eta = kkt1 <= tol && kkt3 <= tol;
    if (need_eta || stalled || outer + 1 >= o.max_outer) {
      // ---- certificates at x (eq. kkt_res, Prop. 1): rho = A x - b is the
      // last gradient's (x = u of the last prox), q = A^T rho
      sm_atv<false, V>(A, lda, n, nullptr, kOffRho, wd, -1, nullptr, c);
      ++passes;
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      double mx = 0.0;  // |A^T rho|_inf, for the Lasso's scaled dual point
      const double den1 = 1.0 + l2;
      for (int64_t i = c.tid; i < n; i += c.nt) {
        const double xi = x[i], qi = wd[i];
        const double p = prox_en(xi - qi, l1, den1);
        const double ee = xi - p;
        s4[0] = fma(ee, ee, s4[0]);
        s4[1] = fma(xi, xi, s4[1]);
        s4[2] += fabs(xi);
        const double a = fabs(qi) - l1;
        s4[3] += a > 0.0 ? a * a : 0.0;
        mx = fmax(mx, fabs(qi));
      }
      bsum<4>(s4, c);
      mx = wave_max(mx);
      __syncthreads();
      if (c.lane == 0) L.red[c.wid] = mx;
      __syncthreads();
      double am = L.red[0];
      for (int w2 = 1; w2 < c.nw; ++w2) am = fmax(am, L.red[w2]);
      __syncthreads();
      eta = sqrt(s4[0]) / (1.0 + sqrt(s4[1]) + sqrt(RR));
      F = 0.5 * RR + l1 * s4[2] + 0.5 * l2 * s4[1];
      if (l2 == 0.0) {
        const double th = am > l1 ? l1 / am : 1.0;
        D = -(0.5 * th * th * RR + th * BR);
      } else {
        D = -0.5 * RR - BR - s4[3] / (2.0 * l2);
      }
      if (need_eta && eta <= tol) {
        converged = true;
        status = 0;
        break;
      }
      if (need_eta) eps_in = fmax(eps_in * 0.1, tol * 1e-3);
    }
    if (stalled) break;
    sigma *= o.sigma_factor;
    if (sigma > o.sigma_max) sigma = o.sigma_max;
  }
  if (!converged) status = nonfinite ? -2 : (bad_sigma ? -1 : (chol_bad ? -5 : (stalled ? 2 : 1)));
  if constexpr (std::is_same<V, InLds>::value) {
    __syncthreads();
    GD xo = (GD)pr.x;
    for (int64_t i = c.tid; i < n; i += c.nt) xo[i] = x[i];
  }
  __syncthreads();  // every thread's stores of x are issued
  if (c.tid == 0) {
    SmallOut* out = pr.out;
    out->status = status;
    out->chol_row = chol_row;
    out->passes = passes;
    out->outer = outer_done;
    out->newton = newton;
    out->r = r;
    out->eta = eta;
    out->kkt1 = kkt1;
    out->kkt3 = kkt3;
    out->F = F;
    out->D = D;
    out->sigma = sigma;
    out->sigma0 = sigma0;
    if (pub.flag) {
      // the record and x visible to the host, then the sequence flag
      __threadfence_system();
      __hip_atomic_store(pub.flag, pub.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

}  // namespace

__global__ __launch_bounds__(kSmNT, 2) void k_solve_small(const SmallArgs* __restrict__ probs, SmallArgs one,
                                                       SmallOpts o, Pub pub) {
  SmallCtx c;
  c.tid = threadIdx.x;
  c.lane = c.tid & (kWave - 1);
  c.wid = __builtin_amdgcn_readfirstlane(c.tid / kWave);
  c.nt = blockDim.x;
  c.nw = c.nt / kWave;
  const SmallArgs pr = probs ? probs[blockIdx.x] : one;
  if (pr.n <= o.nl) {
    // the n-vectors in LDS after the Newton matrix: x, w_y, w_d, u_J (nl
    // doubles each), then J (nl ints)
    double* v = sm_dyn + o.vec_off;
    const int64_t nl = o.nl;
    solve_body<InLds>(pr, o, pub, c, (LD)v, (LD)(v + nl), (LD)(v + 2 * nl), (LD)(v + 3 * nl), (LI)(v + 4 * nl));
  } else {
    solve_body<InGlobal>(pr, o, pub, c, (GD)pr.x, (GD)pr.wy, (GD)pr.wd, (GD)pr.uJ, (GI)pr.J);
  }
}

// LDS of a launch: the fixed parts and the packed Newton matrix of the
// largest m (rounded to 16 bytes), then 36 bytes a feature for the
// problems whose n-vectors fit (at most kSmallLdsMax in all).
constexpr size_t kSmallLdsMax = 160 * 1024 - 1024;  // leaves room for the static LDS
size_t small_matrix_bytes(int mmax) {
  const size_t b = sizeof(SmallLds) + sizeof(double) * (size_t)mmax * (size_t)(mmax + 1) / 2;
  return (b + 15) / 16 * 16;
}
size_t small_lds_bytes(int mmax, int64_t nl) { return small_matrix_bytes(mmax) + (size_t)nl * 36; }
int64_t small_lds_cap(int mmax) { return (int64_t)((kSmallLdsMax - small_matrix_bytes(mmax)) / 36); }

hipError_t small_init() {
  return hipFuncSetAttribute((const void*)k_solve_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kSmallLdsMax);
}

hipError_t solve_small(const SmallArgs* probs, const SmallArgs* one, int count, int mmax, int64_t nmax,
                       const SmallOpts& o, Pub pub, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (mmax < 1 || mmax > kSmallMaxM || nmax < 1 || (!probs && (!one || count != 1))) return hipErrorInvalidValue;
  const SmallArgs a = one ? *one : SmallArgs{};
  SmallOpts oo = o;
  const int64_t cap = small_lds_cap(mmax);
  oo.vec_off = (int64_t)(small_matrix_bytes(mmax) / sizeof(double));
  oo.nl = nmax <= cap ? nmax : cap;  // problems with n <= nl keep their n-vectors in LDS
  hipLaunchKernelGGL(k_solve_small, dim3((unsigned)count), dim3(kSmNT), small_lds_bytes(mmax, oo.nl), st,
                     one ? nullptr : probs, a, oo, pub);
  return hipGetLastError();
}

}  // namespace ssnal
