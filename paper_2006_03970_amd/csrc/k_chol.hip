// FP64 Cholesky factorisation and solve of the Newton system
// (eq. AJ_system: (I + kappa A_J A_J^T) d = -grad psi, or the r x r matrix of
// eq. smw_formula).  The matrix is N x N, row-major, lower triangle used; on
// exit it holds L (V = L L^T).
//
// Right-looking, 64 x 64 blocks, ONE launch per block column s:
//   * panel workgroups p = 0 .. T-s-1 own row block s+p of column s.  Each
//     applies the previous step's rank-64 update to its own tile and to the
//     diagonal tile (FP64 matrix cores), then eliminates the stacked
//     [diagonal tile; own tile] held in the MFMA accumulators, eight columns at
//     a time.  Every panel workgroup factors the diagonal tile itself, so no
//     workgroup waits for another inside a launch.  The diagonal tile of V is
//     therefore read by every panel workgroup and written by none: the
//     diagonal workgroup stores L_ss in a separate buffer of diagonal blocks
//     (a workgroup may start after another has finished, for instance when
//     other streams' kernels hold the CUs).
//   * the launch's remaining workgroups apply the previous step's update to
//     the trailing tiles of columns s+1 .. T-1.
//   * the forward substitution L z = alpha*rhs rides along: workgroup p
//     subtracts L_{s+p,s-1} z_{s-1} from its block of the right-hand side, and
//     an otherwise idle wave of the diagonal workgroup solves block s while
//     the columns are eliminated.
// A single workgroup then runs the backward substitution L^T x = z.
//
// Every chain here is latency-bound (N <= 4096, one 64-column block per
// launch), so the kernels issue all global loads of a phase before the first
// use (unconditional loads at clamped addresses, masked with non-short-
// circuit conditions: a guarded load becomes a branch that waits for it), and
// pivots use the hardware reciprocal-square-root estimate refined by Newton
// steps instead of a correctly rounded sqrt and divide.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace ssnal {

constexpr int kNB = 64;
constexpr int kBP = kNB + 1;  // LDS pitch of a 64 x 64 tile
constexpr double kMinPivot = 2.2250738585072014e-308;  // smallest positive normal double

// 1/sqrt(t) for a positive normal t: hardware estimate, then two Newton steps
// y <- y + y (1 - t y^2) / 2 (quadratic convergence: a 2^-22 estimate reaches
// rounding level after the second step).
__device__ __forceinline__ double rsqrt_pos(double t) {
  double y = __builtin_amdgcn_rsq(t);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-(t * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// 1/d for a normal d: hardware estimate, then two Newton steps r <- r + r(1 - d r).
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
  }
  return r;
}

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

__device__ __forceinline__ void tri_of(int t, int& i, int& j) {
  // t enumerates lower-triangle pairs (i >= j) row by row: t = i(i+1)/2 + j
  int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  i = r;
  j = t - r * (r + 1) / 2;
}

// Cholesky step workgroups have 512 threads: four "VALU" waves (0..3) and
// four "MFMA" waves (4..7), one of each per SIMD, so the matrix-core updates
// of the MFMA waves run while the VALU waves factor and solve (an MFMA holds
// up the issue of its own wave, not of the other wave on its SIMD).
constexpr int kStepNT = 512;

// Load the 64 x 64 block of V at rows i0, cols k0 with NT threads (thread t
// holds entry e = t + NT q as (e / 64, e % 64)).  Addresses are clamped into
// the matrix, so every load is issued unconditionally; entries outside the
// matrix are zeroed by mask_tile once every load of the phase is in flight (a
// select right after its load would wait for it).
template <int NT>
__device__ __forceinline__ void load_tile(const double* __restrict__ V, int N, int i0, int k0, int t,
                                          double (&v)[kNB * kNB / NT]) {
#pragma unroll
  for (int q = 0; q < kNB * kNB / NT; ++q) {
    const int e = t + q * NT;
    const int i = i0 + e / kNB, k = k0 + e % kNB;
    v[q] = V[(int64_t)min(i, N - 1) * N + min(k, N - 1)];
  }
}
template <int NT>
__device__ __forceinline__ void mask_tile(int N, int i0, int k0, int t, double (&v)[kNB * kNB / NT]) {
#pragma unroll
  for (int q = 0; q < kNB * kNB / NT; ++q) {
    const int e = t + q * NT;
    const int i = i0 + e / kNB, k = k0 + e % kNB;
    v[q] = ((i < N) & (k < N)) ? v[q] : 0.0;
  }
}
// Store a block loaded by load_tile transposed: dst[k][i].
template <int NT>
__device__ __forceinline__ void store_t(const double (&v)[kNB * kNB / NT], int t, double (*dst)[kBP]) {
#pragma unroll
  for (int q = 0; q < kNB * kNB / NT; ++q) {
    const int e = t + q * NT;
    dst[e % kNB][e / kNB] = v[q];
  }
}

// C[i][j] = sum_k P[k][i] Q[k][j] for the 64 x 64 tile, with P, Q staged by
// store_t.  Wave w < 4 owns rows 32*(w>>1).., columns 32*(w&1)..; FP64 MFMA
// 16x16x4, whose accumulator v holds row lane/16 + 4*v, column lane%16.
__device__ __forceinline__ void mfma_64(double (*P)[kBP], double (*Q)[kBP], dbl4 acc[2][2], int w) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wi = w >> 1, wj = w & 1;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = dbl4{0, 0, 0, 0};
#pragma unroll 4
  for (int ks = 0; ks < kNB; ks += 4) {
    const int kr = ks + lane / 16;
    double a[2], b[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) a[p] = P[kr][wi * 32 + p * 16 + (lane & 15)];
#pragma unroll
    for (int q = 0; q < 2; ++q) b[q] = Q[kr][wj * 32 + q * 16 + (lane & 15)];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p][q], 0, 0, 0);
  }
}

struct StepLds {
  union {
    struct {
      double P[kNB][kBP];  // L_{s,s-1}, transposed (previous step's update)
      double Q[kNB][kBP];  // L_{s+p,s-1}, transposed
      double D[kNB][kBP];  // diagonal tile of column s (masked, identity padding)
      double B[kNB][kBP];  // own tile of column s (masked)
    } st;
    double LF[2 * kNB][kBP];  // factor of the stacked [diagonal tile; own tile]
  } u;
  double PN[2 * kNB][9];      // current 8-column panel
  double zprev[kNB];          // z_{s-1}
  int bad;                    // first non-positive pivot of the current panel, or -1
  double zrow[kNB];           // right-hand side of block s after the previous updates
};

// 16 x 16 FP64 MFMA accumulator blocks: acc[rb][cb][v] holds row lane/16 + 4v,
// column lane%16 of block (rb, cb).
typedef dbl4 Acc[2][4];

// Trailing update of step s-1 on tile (i, l): V_il -= L_{i,s-1} L_{l,s-1}^T
// (all waves load, waves 0..3 multiply).
__device__ __forceinline__ void trailing_tile(double* __restrict__ V, int N, int s, int i, int l,
                                              StepLds& L) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = wave_id();
  const int wi = (wid & 3) >> 1, wj = wid & 1;
  const int k0 = (s - 1) * kNB;
  double pv[kNB * kNB / kStepNT], qv[kNB * kNB / kStepNT], ov[2][2][4];
  load_tile<kStepNT>(V, N, i * kNB, k0, tid, pv);
  load_tile<kStepNT>(V, N, l * kNB, k0, tid, qv);
  if (wid < 4) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = i * kNB + wi * 32 + p * 16 + (lane / 16) + 4 * v;
          const int c = l * kNB + wj * 32 + q * 16 + (lane & 15);
          ov[p][q][v] = V[(int64_t)min(r, N - 1) * N + min(c, N - 1)];
        }
  }
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before any use
  mask_tile<kStepNT>(N, i * kNB, k0, tid, pv);
  mask_tile<kStepNT>(N, l * kNB, k0, tid, qv);
  store_t<kStepNT>(pv, tid, L.u.st.P);
  store_t<kStepNT>(qv, tid, L.u.st.Q);
  __syncthreads();
  if (wid >= 4) return;
  dbl4 acc[2][2];
  mfma_64(L.u.st.P, L.u.st.Q, acc, wid);
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = i * kNB + wi * 32 + p * 16 + (lane / 16) + 4 * v;
        const int c = l * kNB + wj * 32 + q * 16 + (lane & 15);
        if (r < N && c < N && (i != l || c <= r)) V[(int64_t)r * N + c] = ov[p][q][v] - acc[p][q][v];
      }
}

// W = L^{-1} for a full 64 x 64 lower-triangular block (row-major, zero
// strict upper triangle), written row-major with zeros above the diagonal,
// by 2 x 2 blocks of 32: W11 = L11^{-1} and W22 = L22^{-1} by waves 0 and 1
// at once (lane j holds column j and eliminates right-looking: the unknown of
// row k is final once the rows above have updated it, then it updates the
// rows below with column k of L, broadcast from LDS), then
// W21 = -W22 (L21 W11) by all waves, two entries a thread per product.
// A partial block (nk < 64: the last block of L, zero outside its nk x nk
// lower triangle) is inverted with identity padding and written with zeros
// outside nk x nk.
__device__ __forceinline__ void invert_block(const double* __restrict__ Ls, double* __restrict__ Ws,
                                             StepLds& L, int nk = kNB) {
  constexpr int kH = kNB / 2;
  const int tid = threadIdx.x;
  const int wid = wave_id();
  double(*A)[kBP] = L.u.LF;             // L
  double(*WI)[kBP] = L.u.LF + kNB;      // W
  double(*Tm)[kH + 1] = reinterpret_cast<double(*)[kH + 1]>(&L.PN[0][0]);  // L21 W11
#pragma unroll
  for (int q = 0; q < kNB * kNB / kStepNT; ++q) {
    const int e = tid + kStepNT * q;
    const int r = e / kNB, c = e % kNB;
    const double v = Ls[e];
    A[r][c] = r < nk ? v : (r == c ? 1.0 : 0.0);
    WI[r][c] = 0.0;
  }
  __syncthreads();
  if (wid < 2) {
    const int o = kH * wid;                    // diagonal block of this wave
    const int j = threadIdx.x & (kH - 1);      // column within it (lanes 32..63 repeat 0..31)
    double w[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) w[i] = i == j ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < kH; ++k) {
      w[k] *= rcp_nr(A[o + k][o + k]);
#pragma unroll
      for (int i = k + 1; i < kH; ++i) w[i] = fma(-A[o + i][o + k], w[k], w[i]);
    }
    if ((threadIdx.x & (kWave - 1)) < kH) {
#pragma unroll
      for (int i = 0; i < kH; ++i) WI[o + i][o + j] = w[i];
    }
  }
  __syncthreads();
  const int ti = tid / (kH / 2), tj = 2 * (tid % (kH / 2));  // row, first of two columns
  {
    // Tm = L21 W11 (W11 lower: only k >= column contributes)
    double t0 = 0.0, t1 = 0.0;
#pragma unroll 8
    for (int k = 0; k < kH; ++k) {
      const double a = A[kH + ti][k];
      t0 = fma(a, WI[k][tj], t0);
      t1 = fma(a, WI[k][tj + 1], t1);
    }
    Tm[ti][tj] = t0;
    Tm[ti][tj + 1] = t1;
  }
  __syncthreads();
  {
    // W21 = -W22 Tm (W22 lower: only k <= row contributes)
    double t0 = 0.0, t1 = 0.0;
#pragma unroll 8
    for (int k = 0; k < kH; ++k) {
      const double a = WI[kH + ti][kH + k];
      t0 = fma(a, Tm[k][tj], t0);
      t1 = fma(a, Tm[k][tj + 1], t1);
    }
    WI[kH + ti][tj] = -t0;
    WI[kH + ti][tj + 1] = -t1;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kNB * kNB / kStepNT; ++q) {
    const int e = tid + kStepNT * q;
    const int r = e / kNB, c = e % kNB;
    Ws[e] = ((r < nk) & (c < nk)) ? WI[r][c] : 0.0;
  }
}

// Ld: T diagonal blocks of L, 64 x 64 row-major each (block s at Ld + s*4096).
// Wd (null: none): inverses of the diagonal blocks; launch s >= 1 inverts
// block s-1 (finished by the previous launch) in one extra workgroup.
__global__ __launch_bounds__(kStepNT) void k_chol_step(double* __restrict__ V, int N, int T, int s,
                                                       const double* __restrict__ rhs, double alpha,
                                                       double* __restrict__ z, double* __restrict__ Ld,
                                                       double* __restrict__ Wd,
                                                       int* __restrict__ info) {
  extern __shared__ double smem[];
  StepLds& L = *reinterpret_cast<StepLds*>(smem);
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = wave_id();
  const int npanel = T - s;
  const int s0 = s * kNB;

  if ((int)blockIdx.x >= npanel) {
    const int q = (int)blockIdx.x - npanel;
    if (q == (T - s - 1) * (T - s) / 2) {  // past the trailing tiles: the inverse
      invert_block(Ld + (int64_t)(s - 1) * kNB * kNB, Wd + (int64_t)(s - 1) * kNB * kNB, L);
      return;
    }
    int ii, ll;
    tri_of(q, ii, ll);
    trailing_tile(V, N, s, s + 1 + ii, s + 1 + ll, L);
    return;
  }

  // ---- panel workgroup p: row block s+p of column s.  The stacked matrix
  // S = [diagonal tile; own tile] (128 x 64) lives in the accumulators of the
  // MFMA waves: MFMA wave mw = wid - 4 owns row blocks 2mw, 2mw+1 (rows
  // 32mw..32mw+31 of S) x 4 column blocks.  MFMA waves 0, 1 hold the
  // diagonal tile ("D"), 2, 3 the own tile ("B"); of D only the blocks on or
  // below the diagonal are kept up to date.  VALU wave 0 solves the rows of
  // D, VALU wave 1 those of B, VALU wave 2 of the diagonal workgroup carries
  // the forward substitution.
  const int p = blockIdx.x;
  const int b0 = (s + p) * kNB;
  const int nk = N - s0 < kNB ? N - s0 : kNB;  // width of column s
  const int nbr = p == 0 ? 0 : (N - b0 < kNB ? N - b0 : kNB);
  const bool vw = wid < 4;
  const int mw = wid - 4;
  const bool in_b = mw >= 2;
  const bool live = !vw && (!in_b || p > 0);
  const bool fwd = rhs != nullptr && p == 0;  // VALU wave 2 solves block s of L z = rhs

  // ---- every global load first, by all 512 threads, 16 bytes a load when
  // the row pitch allows: previous-step factors P = L_{s,s-1} and
  // Q = L_{s+p,s-1}, the diagonal tile D and the own tile B of column s
  // (entry pair e = tid + 512 q of a tile: row e / 32, columns 2(e % 32)..),
  // and the right-hand side (VALU wave 0).  Addresses are clamped into the
  // matrix; masks are applied when the tiles are staged in LDS.
  constexpr int kTQ = kNB * kNB / 2 / kStepNT;  // entry pairs of a tile per thread
  const bool v2 = (N & 1) == 0 && ((uintptr_t)V & 15) == 0;
  auto ld2 = [&](int i, int k) -> double2 {
    const int64_t row = (int64_t)min(i, N - 1) * N;
    if (v2) return *reinterpret_cast<const double2*>(V + row + min(k, N - 2));
    return double2{V[row + min(k, N - 1)], V[row + min(k + 1, N - 1)]};
  };
  double2 pv[kTQ], qv[kTQ], dv[kTQ], bv[kTQ];
#pragma unroll
  for (int q = 0; q < kTQ; ++q) {
    const int e = tid + kStepNT * q;
    const int r = e / (kNB / 2), c = 2 * (e % (kNB / 2));
    if (s > 0) {
      pv[q] = ld2(s0 + r, s0 - kNB + c);
      if (p > 0) qv[q] = ld2(b0 + r, s0 - kNB + c);
    }
    dv[q] = ld2(s0 + r, s0 + c);
    if (p > 0) bv[q] = ld2(b0 + r, s0 + c);
  }
  double zp = 0.0, zc = 0.0;
  if (rhs && tid < kNB) {
    const int g = b0 + tid;
    if (s > 0) zp = z[s0 - kNB + tid];  // block s-1 is always full
    const double r0 = s == 0 ? alpha * rhs[min(g, N - 1)] : z[min(g, N - 1)];
    zc = g < N ? r0 : 0.0;
  }
  __builtin_amdgcn_sched_barrier(0);  // every load above is issued before any use
#pragma unroll
  for (int q = 0; q < kTQ; ++q) {
    const int e = tid + kStepNT * q;
    const int r = e / (kNB / 2), c = 2 * (e % (kNB / 2));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int C = c + h;
      if (s > 0) {
        // P, Q transposed, zero outside the matrix (column block s-1 is full)
        L.u.st.P[C][r] = s0 + r < N ? (h ? pv[q].y : pv[q].x) : 0.0;
        if (p > 0) L.u.st.Q[C][r] = b0 + r < N ? (h ? qv[q].y : qv[q].x) : 0.0;
      }
      // the diagonal tile keeps its lower triangle and gets identity padding;
      // the own tile is zero outside the matrix
      const double d = h ? dv[q].y : dv[q].x;
      L.u.st.D[r][C] = ((r < nk) & (C <= r)) ? d : (r == C ? 1.0 : 0.0);
      if (p > 0) L.u.st.B[r][C] = ((r < nbr) & (C < nk)) ? (h ? bv[q].y : bv[q].x) : 0.0;
    }
  }
  if (rhs && tid < kNB && s > 0) L.zprev[tid] = zp;
  __syncthreads();
  Acc acc;
  if (live) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int R = 32 * mw + 16 * rb + lane / 16 + 4 * v;
          const int C = 16 * cb + (lane & 15);
          acc[rb][cb][v] = in_b ? L.u.st.B[R - kNB][C] : L.u.st.D[R][C];
        }
  }

  if (s > 0) {
    // previous step's rank-64 update: S -= [L_{s,s-1}; L_{s+p,s-1}] L_{s,s-1}^T
    if (live) {
      double(*Ls)[kBP] = in_b ? L.u.st.Q : L.u.st.P;
      const int rbase = in_b ? 32 * mw - kNB : 32 * mw;
#pragma unroll 4
      for (int ks = 0; ks < kNB; ks += 4) {
        const int kr = ks + lane / 16;
        double a[2], b[4];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) a[rb] = -Ls[kr][rbase + 16 * rb + (lane & 15)];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) b[cb] = L.u.st.P[kr][16 * cb + (lane & 15)];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            if (in_b || cb <= 2 * mw + rb)
              acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
      }
    }
    if (rhs && tid < kNB) {
      // rhs block s+p loses L_{s+p,s-1} z_{s-1} (VALU wave 0, beside the MFMAs)
      double(*Lp)[kBP] = p > 0 ? L.u.st.Q : L.u.st.P;
      double t = 0.0;
#pragma unroll 8
      for (int k = 0; k < kNB; ++k) t = fma(Lp[k][tid], L.zprev[k], t);
      zc -= t;
    }
    __syncthreads();  // P and Q are reused as LF below
  }
  if (rhs && tid < kNB) {
    if (p > 0) {
      if (b0 + tid < N) z[b0 + tid] = zc;
    } else {
      L.zrow[tid] = zc;
    }
  }
  double zv = 0.0;  // VALU wave 2 of the diagonal workgroup: residual rhs of row `lane` of block s
  if (fwd) {
    __syncthreads();
    if (wid == 2) zv = L.zrow[lane];
  }

  // ---- elimination, eight columns at a time.  Per panel: the MFMA waves
  // write their rows of the eight columns to PN; the row-solving VALU waves
  // (0, 1 of a workgroup with an own tile, 2 for the forward substitution)
  // factor the 8 x 8 pivot block themselves, wave 0 solves the 64 rows of D
  // and wave 1 the 64 of B against it into LF; then the MFMA waves apply the
  // rank-8 update right of the panel.  Rows of the diagonal tile above the
  // pivot block get zeros in LF, so the strict upper triangle never feeds a
  // later column.  Look-ahead: after a panel only the column block of the
  // next panel is updated at once; the panel's updates of the blocks beyond
  // are issued after the next panel's first barrier, on the matrix cores
  // while the VALU waves factor.
  constexpr int kPW = 8;  // panel width
  const bool factors = wid == 0 || (wid == 1 && p > 0) || (fwd && wid == 2);
  int prev_j0 = -1, prev_cbn = 4;  // the previous panel's blocks > prev_cbn are still to update
  auto panel_update = [&](int pj0, int cb_lo, int cb_hi) {
    // S[rows of this wave][blocks cb_lo..cb_hi] -= L_panel(rows) L_panel(block rows)^T
#pragma unroll
    for (int kh = 0; kh < kPW; kh += 4) {
      const int kr = pj0 + kh + lane / 16;
      double a[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) a[rb] = -L.u.LF[32 * mw + 16 * rb + (lane & 15)][kr];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        if (cb < cb_lo || cb > cb_hi) continue;
        const double bv = L.u.LF[16 * cb + (lane & 15)][kr];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          if (in_b || cb <= 2 * mw + rb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], bv, acc[rb][cb], 0, 0, 0);
      }
    }
  };
#pragma unroll
  for (int cbp = 0; cbp < 4; ++cbp) {
    for (int sub = 0; sub < 16; sub += kPW) {
      const int j0 = 16 * cbp + sub;
      const int cc = (lane & 15) - sub;
      if (live && cc >= 0 && cc < kPW) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) L.PN[32 * mw + 16 * rb + lane / 16 + 4 * v][cc] = acc[rb][cbp][v];
      }
      __syncthreads();
      // deferred updates of the previous panel (blocks this panel's extract did not need)
      if (live && prev_j0 >= 0 && prev_cbn < 3) panel_update(prev_j0, prev_cbn + 1, 3);
      double zz[kPW];
      if (factors) {
        // 8 x 8 pivot block, factored redundantly by each factoring thread
        // (same bits everywhere).  Every LDS value the panel needs -- the
        // pivot block and the thread's own row -- is read first, in one round
        // trip; l[i][k] replaces the entry it came from.
        const int R = kNB * (wid & 1) + lane;  // row of S this lane solves (wave 2: rows of D)
        double l[kPW][kPW], rl[kPW], a[kPW];
#pragma unroll
        for (int i = 0; i < kPW; ++i)
#pragma unroll
          for (int k = 0; k <= i; ++k) l[i][k] = L.PN[j0 + i][k];
#pragma unroll
        for (int k = 0; k < kPW; ++k) a[k] = L.PN[R][k];
        __builtin_amdgcn_sched_barrier(0);
        uint64_t badk = 0;  // bit k: pivot k not positive (wave-uniform)
#pragma unroll
        for (int k = 0; k < kPW; ++k) {
          double t = l[k][k];
#pragma unroll
          for (int q = 0; q < k; ++q) t = fma(-l[k][q], l[k][q], t);
          badk |= (uint64_t)(__builtin_amdgcn_ballot_w64(!(t >= kMinPivot)) != 0) << k;
          const double y = rsqrt_pos(t);
          rl[k] = y;
          l[k][k] = t * y;
#pragma unroll
          for (int i = k + 1; i < kPW; ++i) {
            double u = l[i][k];
#pragma unroll
            for (int q = 0; q < k; ++q) u = fma(-l[i][q], l[k][q], u);
            l[i][k] = u * y;
          }
        }
        const int bad = badk ? __builtin_ctzll(badk) : -1;
        if (tid == 0) L.bad = bad;
        if (wid < 2 && bad < 0) {
          // x L^T = a.  For a row of the pivot block this recomputes its L row
          // with the same operations in the same order, so the entries on or
          // left of the diagonal equal l bit for bit; the entries right of it
          // (and whole rows above the pivot block) are zeroed.
          const int r = R >= kNB ? kPW : R - j0;  // last kept column (>= kPW: all)
          double x[kPW];
#pragma unroll
          for (int k = 0; k < kPW; ++k) {
            double u = a[k];
#pragma unroll
            for (int q = 0; q < k; ++q) u = fma(-x[q], l[k][q], u);
            x[k] = u * rl[k];
          }
#pragma unroll
          for (int k = 0; k < kPW; ++k) L.u.LF[R][j0 + k] = k <= r ? x[k] : 0.0;
        }
        if (fwd && wid == 2) {
          // z entries of the pivot rows: L_pivot zz = (residual rhs of rows j0..j0+7)
#pragma unroll
          for (int k = 0; k < kPW; ++k) {
            double u = readlane_d(zv, j0 + k);
#pragma unroll
            for (int q = 0; q < k; ++q) u = fma(-l[k][q], zz[q], u);
            zz[k] = u * rl[k];
          }
        }
      }
      __syncthreads();
      {
        const int bad = L.bad;
        if (bad >= 0) {  // a uniform exit: every thread read the same flag
          if (tid == 0 && p == 0) atomicCAS(info, 0, s0 + j0 + bad + 1);  // the first bad pivot wins
          return;
        }
      }
      // the column block of the next panel at once; the blocks beyond later
      const int cbn = sub + kPW < 16 ? cbp : cbp + 1;
      if (live && cbn < 4) panel_update(j0, cbn, cbn);
      prev_j0 = j0;
      prev_cbn = cbn;
      if (fwd && wid == 2) {
        // rows below the pivot rows lose L[row][j0..j0+7] zz; pivot rows take zz
        const int rel = lane - j0;
        if (rel >= kPW) {
          double u = zv;
#pragma unroll
          for (int k = 0; k < kPW; ++k) u = fma(-L.u.LF[lane][j0 + k], zz[k], u);
          zv = u;
        } else if (rel >= 0) {
          double e = zz[0];
#pragma unroll
          for (int k = 1; k < kPW; ++k) e = rel == k ? zz[k] : e;
          zv = e;
        }
      }
    }
  }
  // ---- write back (LF is complete after the last panel's second barrier):
  // the diagonal workgroup writes L_ss to its block of Ld (zero outside the
  // lower triangle of the nk x nk block), the others their L_{s+p,s} to V
  {
    constexpr int kWB = kNB * kWave / kStepNT;  // rows per thread
    const int C = tid & (kNB - 1);
    const int base = p == 0 ? 0 : kNB;
    double wv[kWB];
#pragma unroll
    for (int i = 0; i < kWB; ++i) wv[i] = L.u.LF[base + wid + 8 * i][C];
    if (p == 0) {
      double* Ls = Ld + (int64_t)s * kNB * kNB;
#pragma unroll
      for (int i = 0; i < kWB; ++i) {
        const int R = wid + 8 * i;
        Ls[R * kNB + C] = ((R < nk) & (C <= R)) ? wv[i] : 0.0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kWB; ++i) {
        const int R = wid + 8 * i;
        if (R < nbr && C < nk) V[(int64_t)(b0 + R) * N + s0 + C] = wv[i];
      }
    }
  }
  if (fwd && wid == 2 && lane < nk) z[s0 + lane] = zv;
}

// Inverse of the last diagonal block of L (which the step launches leave
// out), for the Frobenius norm of L^{-1}.
__global__ __launch_bounds__(kStepNT) void k_invert_last(const double* __restrict__ Ld,
                                                         double* __restrict__ Wd, int N) {
  extern __shared__ double smem[];
  StepLds& L = *reinterpret_cast<StepLds*>(smem);
  const int T = (N + kNB - 1) / kNB;
  const int nk = N - (T - 1) * kNB;
  invert_block(Ld + (int64_t)(T - 1) * kNB * kNB, Wd + (int64_t)(T - 1) * kNB * kNB, L, nk);
}

// ||L^{-1}||_F^2 (= tr((L L^T)^{-1})) by block columns of X = L^{-1}: X_jj = W_jj
// (the diagonal-block inverses) and, down the column, X_ij = -W_ii sum_{k=j}^{i-1}
// L_ik X_kj on FP64 MFMA.  One workgroup (4 waves) per block column j writes
// its partial sum to part[j]; X_kj, k > j, are kept in Xs (triangular block
// index) for the later rows of the same column.  V holds L below the diagonal
// blocks (row-major N x N), Wd the T inverses.
struct InvLds {
  double P[kNB][kBP];
  double Q[kNB][kBP];
};
__device__ __forceinline__ int64_t tri_block(int i, int j, int T) {
  return (int64_t)j * T - (int64_t)j * (j - 1) / 2 + (i - j);  // i >= j
}
__global__ __launch_bounds__(256) void k_inv_frob(const double* __restrict__ V, int N,
                                                  const double* __restrict__ Wd,
                                                  double* __restrict__ Xs, double* __restrict__ part) {
  extern __shared__ double smem[];
  InvLds& S = *reinterpret_cast<InvLds*>(smem);
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = wave_id();
  const int wi = wid >> 1, wj = wid & 1;
  const int T = (N + kNB - 1) / kNB;
  const int j = blockIdx.x;
  constexpr int kE = kNB * kNB / 256;
  double frob = 0.0;
  {
    const double* W = Wd + (int64_t)j * kNB * kNB;
#pragma unroll
    for (int q = 0; q < kE; ++q) {
      const double v = W[tid + 256 * q];
      frob = fma(v, v, frob);
    }
  }
  for (int i = j + 1; i < T; ++i) {
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[a][c] = dbl4{0, 0, 0, 0};
    for (int k = j; k < i; ++k) {
      // P = L_ik transposed (zero past N), Q = X_kj
      double lv[kE], xv[kE];
      load_tile<256>(V, N, i * kNB, k * kNB, tid, lv);
      const double* X = k == j ? Wd + (int64_t)j * kNB * kNB : Xs + tri_block(k, j, T) * kNB * kNB;
#pragma unroll
      for (int q = 0; q < kE; ++q) xv[q] = X[tid + 256 * q];
      __builtin_amdgcn_sched_barrier(0);
      mask_tile<256>(N, i * kNB, k * kNB, tid, lv);
      __syncthreads();  // the previous product's reads of P, Q are done
      store_t<256>(lv, tid, S.P);
#pragma unroll
      for (int q = 0; q < kE; ++q) {
        const int e = tid + 256 * q;
        S.Q[e / kNB][e % kNB] = xv[q];
      }
      __syncthreads();
#pragma unroll 4
      for (int ks = 0; ks < kNB; ks += 4) {
        const int kr = ks + lane / 16;
        double a[2], b[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) a[p] = S.P[kr][wi * 32 + p * 16 + (lane & 15)];
#pragma unroll
        for (int q = 0; q < 2; ++q) b[q] = S.Q[kr][wj * 32 + q * 16 + (lane & 15)];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q)
            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p][q], 0, 0, 0);
      }
    }
    // X_ij = -W_ii acc: P = W_ii transposed, Q = acc
    {
      const double* W = Wd + (int64_t)i * kNB * kNB;
      double wv[kE];
#pragma unroll
      for (int q = 0; q < kE; ++q) wv[q] = W[tid + 256 * q];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kE; ++q) {
        const int e = tid + 256 * q;
        S.P[e % kNB][e / kNB] = wv[q];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            S.Q[wi * 32 + p * 16 + lane / 16 + 4 * v][wj * 32 + q * 16 + (lane & 15)] = acc[p][q][v];
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = dbl4{0, 0, 0, 0};
#pragma unroll 4
      for (int ks = 0; ks < kNB; ks += 4) {
        const int kr = ks + lane / 16;
        double a[2], b[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) a[p] = S.P[kr][wi * 32 + p * 16 + (lane & 15)];
#pragma unroll
        for (int q = 0; q < 2; ++q) b[q] = S.Q[kr][wj * 32 + q * 16 + (lane & 15)];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q)
            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p][q], 0, 0, 0);
      }
      double* X = Xs + tri_block(i, j, T) * kNB * kNB;
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double x = -acc[p][q][v];
            X[(wi * 32 + p * 16 + lane / 16 + 4 * v) * kNB + wj * 32 + q * 16 + (lane & 15)] = x;
            frob = fma(x, x, frob);
          }
      __syncthreads();  // X_ij in place before the next row reads it
    }
  }
  __shared__ double red[256 / kWave];
  frob = block_sum<256>(frob, red);
  if (tid == 0) part[j] = frob;
}

// Backward substitution L^T x = z by one workgroup of 1024 threads, left-
// looking by blocks of 64 rows from the last: block s needs
// c_s = sum_{r below} L[r][s0 + j] x_r, then solves L_ss^T x_s = z_s - c_s.
// The waves split into two roles with the same barriers:
//   * waves 1..15 ("loaders") hold the rows below block s in registers (each
//     load instruction covers W rows of 64/W lanes, W doubles a lane: W = 2
//     for 16-byte loads when the row pitch allows), form the partial sums of
//     c_s, then issue the loads of block s-1 (rows and diagonal block) so they
//     travel while block s is solved, and stage the diagonal block in the
//     second LDS buffer;
//   * wave 0 ("solver") sums the partials and solves the 64 x 64 triangle in
//     eight 8 x 8 steps: the eight unknowns of a step come from a short
//     chain on broadcast values, then one rank-8 update of the remaining
//     right-hand sides (lanes = rows of L^T).
// Disjoint roles keep each role's registers to itself.
constexpr int kBackNT = 1024;
constexpr int kBackWaves = kBackNT / kWave;
constexpr int kBackLW = kBackWaves - 1;  // loader waves
constexpr int kBackRegs = 32;             // doubles of L a loader thread holds (480 rows)

template <int W>
__global__ __launch_bounds__(1024) void k_chol_back(const double* __restrict__ Lm, int N,
                                                    const double* __restrict__ Ldg,
                                                    const double* __restrict__ Wdg,
                                                    const double* __restrict__ z,
                                                    double* __restrict__ x) {
  extern __shared__ double sm[];
  const int T = (N + kNB - 1) / kNB;
  const int xsz = kNB * T + 2;  // x, then zeros: rows past N read x = 0
  double* xs = sm;
  double(*Ld)[kNB][kBP] = reinterpret_cast<double(*)[kNB][kBP]>(sm + xsz);      // 2 x 64 x 65
  double(*cp)[kNB] = reinterpret_cast<double(*)[kNB]>(sm + xsz + 2 * kNB * kBP);  // 16 x 64
  double* rs = sm + xsz + 2 * kNB * kBP + kBackWaves * kNB;  // 64 reciprocal pivots
  const int tid = threadIdx.x;
  const int wid = wave_id();
  const int lane = tid & (kWave - 1);
  for (int i = tid; i < xsz; i += kBackNT) {
    const double zi = z[min(i, N - 1)];
    xs[i] = i < N ? zi : 0.0;
  }

  if (wid > 0) {
    // ------------------------------------------------------------ loaders
    constexpr int kLPR = kNB / W;          // lanes per row
    constexpr int kR = kBackRegs / W;      // rounds held in registers
    constexpr int kDiag = (kNB * kNB / W + kBackLW * kWave - 1) / (kBackLW * kWave);
    typedef typename std::conditional<W == 2, double2, double>::type VT;
    const int lt = tid - kWave;            // 0 .. 959
    const int wv = wid - 1;
    const int grp = lane / kLPR, cc = lane % kLPR;
    // row of round i of block s: rb + W * kBackLW * i, rb = first row of this
    // thread below block s (kept opaque so the rounds' offsets stay constants)
    auto first_row = [&](int s) {
      int rb = s * kNB + kNB + W * wv + grp;
      asm volatile("" : "+v"(rb));
      return rb;
    };
    // row r, columns of block s (clamped into the matrix: rows past N and the
    // columns of a partial last block are loaded but never used)
    auto ld = [&](int r, int s) -> VT {
      return *reinterpret_cast<const VT*>(Lm + (int64_t)min(r, N - 1) * N + min(s * kNB + W * cc, N - W));
    };
    VT bv[kR], dg[kDiag];
    auto load_diag = [&](int s) {  // L_ss for the last block, W_s = L_ss^{-1} for the others
      const VT* Ls = reinterpret_cast<const VT*>((s == T - 1 ? Ldg : Wdg) + (int64_t)s * kNB * kNB);
#pragma unroll
      for (int q = 0; q < kDiag; ++q) dg[q] = Ls[min(lt + q * kBackLW * kWave, kNB * kNB / W - 1)];
    };
    auto store_diag = [&](int s) {
      double(*D)[kBP] = Ld[s & 1];
#pragma unroll
      for (int q = 0; q < kDiag; ++q) {
        const int e = lt + q * kBackLW * kWave;  // element group: row e / kLPR, columns W (e % kLPR)..
        if (e < kNB * kNB / W) {
          const double* d = reinterpret_cast<const double*>(&dg[q]);
#pragma unroll
          for (int w = 0; w < W; ++w) D[e / kLPR][W * (e % kLPR) + w] = d[w];
        }
      }
    };
    // rounds of block s holding rows of the matrix for this wave (uniform)
    auto rounds = [&](int s) {
      const int left = N - (s * kNB + kNB + W * wv);
      return left > 0 ? (left + W * kBackLW - 1) / (W * kBackLW) : 0;
    };
    load_diag(T - 1);
    store_diag(T - 1);
    for (int s = T - 1; s >= 0; --s) {
      __syncthreads();  // A: x of every block below s is in xs
      const int rb = first_row(s);
      const int nr = rounds(s);
      double t[2][W];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int w = 0; w < W; ++w) t[h][w] = 0.0;
#pragma unroll
      for (int i = 0; i < kR; ++i) {
        if (i < nr) {
          const double xr = xs[min(rb + W * kBackLW * i, N)];
          const double* b = reinterpret_cast<const double*>(&bv[i]);
#pragma unroll
          for (int w = 0; w < W; ++w) t[i & 1][w] = fma(b[w], xr, t[i & 1][w]);
        }
      }
      // rows past the registers (N > 544): four loads in flight at a time
      for (int i = kR; i < nr; i += 4) {
        VT b4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) b4[u] = ld(rb + W * kBackLW * (i + u), s);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double xr = xs[min(rb + W * kBackLW * (i + u), N)];
          const double* b = reinterpret_cast<const double*>(&b4[u]);
#pragma unroll
          for (int w = 0; w < W; ++w) t[u & 1][w] = fma(b[w], xr, t[u & 1][w]);
        }
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        double v = t[0][w] + t[1][w];
        if (W == 2) v += __shfl_xor(v, 32);
        if (grp == 0) cp[wid][W * cc + w] = v;
      }
      __syncthreads();  // B: partials in cp
      if (s > 0) {
        // block s-1 travels while block s is solved
        const int rb1 = first_row(s - 1);
        const int nr1 = min(rounds(s - 1), kR);
#pragma unroll
        for (int i = 0; i < kR; ++i)
          if (i < nr1) bv[i] = ld(rb1 + W * kBackLW * i, s - 1);
        __builtin_amdgcn_sched_barrier(0);  // the rows go out first
        load_diag(s - 1);
        store_diag(s - 1);
      }
    }
  } else {
    // ------------------------------------------------------------ solver
    for (int s = T - 1; s >= 0; --s) {
      __syncthreads();  // A: L_ss in Ld[s & 1], x of every block below s in xs
      const int s0 = s * kNB;
      const int nk = N - s0 < kNB ? N - s0 : kNB;
      double(*D)[kBP] = Ld[s & 1];
      const bool last = s == T - 1;
      if (last) rs[lane] = lane < nk ? rcp_nr(D[lane][lane]) : 0.0;  // read back by this wave only
      const double zs = xs[s0 + lane];
      __syncthreads();  // B: partials in cp
      double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int w = 1; w < kBackWaves; ++w) c[w & 3] += cp[w][lane];
      double v = lane < nk ? zs - ((c[0] + c[1]) + (c[2] + c[3])) : 0.0;
      if (!last) {
        // full block below the last: x_s = W_s^T r with W_s = L_ss^{-1} in D
        rs[lane] = v;  // r, broadcast through LDS (this wave only)
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < kNB; ++i) a[i & 3] = fma(D[i][lane], rs[i], a[i & 3]);
        xs[s0 + lane] = (a[0] + a[1]) + (a[2] + a[3]);
        continue;
      }
#pragma unroll
      for (int j0 = kNB - 8; j0 >= 0; j0 -= 8) {
        // every LDS value of the step first (one round trip), then the chain
        double uu[8][8], col[8], ri[8];
#pragma unroll
        for (int q = 1; q < 8; ++q)
#pragma unroll
          for (int k = 0; k < q; ++k) uu[q][k] = D[j0 + q][j0 + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) ri[k] = rs[j0 + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) col[k] = D[j0 + k][lane];
        double u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = readlane_d(v, j0 + k);
        __builtin_amdgcn_sched_barrier(0);
        // right-looking: each new unknown updates the ones before it and the
        // rows above the step (lane = row of L^T), so only one FMA and one
        // multiply separate consecutive unknowns
        double xx[8];
#pragma unroll
        for (int q = 7; q >= 0; --q) {
          xx[q] = u[q] * ri[q];
#pragma unroll
          for (int k = q - 1; k >= 0; --k) u[k] = fma(-uu[q][k], xx[q], u[k]);
          v = fma(-col[q], xx[q], v);
        }
        if (lane == 0) {  // past nk these are zeros, which xs keeps past N
#pragma unroll
          for (int k = 0; k < 8; ++k) xs[s0 + j0 + k] = xx[k];
        }
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < N; i += kBackNT) x[i] = xs[i];
}

// Diagonal blocks of L from the block buffer into V (lower triangles).
__global__ __launch_bounds__(256) void k_copy_diag(double* __restrict__ V, int N,
                                                   const double* __restrict__ Ld) {
  const int s = blockIdx.x;
  const int s0 = s * kNB;
  const int nk = N - s0 < kNB ? N - s0 : kNB;
  const double* Ls = Ld + (int64_t)s * kNB * kNB;
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    if (r < nk && c <= r) V[(int64_t)(s0 + r) * N + s0 + c] = Ls[e];
  }
}

__global__ void k_zero_upper(double* __restrict__ V, int N) {
  const int64_t tot = (int64_t)N * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / N, j = e - i * N;
    if (j > i) V[e] = 0.0;
  }
}

// ---------------------------------------------------------------- launchers
static size_t back_lds(int N) {
  return sizeof(double) *
         ((size_t)kNB * ((N + kNB - 1) / kNB) + 2 + 2 * kNB * kBP + kBackWaves * kNB + kNB);
}

hipError_t chol_init() {
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_step,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, sizeof(StepLds));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_chol_back<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)back_lds(4096));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_invert_last, hipFuncAttributeMaxDynamicSharedMemorySize,
                          sizeof(StepLds));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_inv_frob, hipFuncAttributeMaxDynamicSharedMemorySize,
                          sizeof(InvLds));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_chol_back<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)back_lds(4096));
}

hipError_t chol_factor_solve(double* V, int N, const double* rhs, double alpha, double* z,
                             double* x, double* Ld, int* info_dev, hipStream_t st) {
  if (N < 1 || N > 4096) return hipErrorInvalidValue;
  const int T = (N + kNB - 1) / kNB;
  double* Wd = rhs ? Ld + (int64_t)T * kNB * kNB : nullptr;
  for (int s = 0; s < T; ++s) {
    const int npanel = T - s;
    const int U = s >= 1 ? (T - s - 1) * (T - s) / 2 : 0;
    const int inv = rhs && s >= 1 ? 1 : 0;  // inverse of diagonal block s-1
    hipLaunchKernelGGL(k_chol_step, dim3(npanel + U + inv), dim3(kStepNT), sizeof(StepLds), st, V, N,
                       T, s, rhs, alpha, z, Ld, Wd, info_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!rhs) return hipSuccess;
  // 16-byte loads need even rows and 16-byte aligned bases
  const bool v2 = N % 2 == 0 && ((uintptr_t)V & 15) == 0 && ((uintptr_t)Ld & 15) == 0;
  if (v2)
    hipLaunchKernelGGL(k_chol_back<2>, dim3(1), dim3(kBackNT), back_lds(N), st, V, N, Ld, Wd, z, x);
  else
    hipLaunchKernelGGL(k_chol_back<1>, dim3(1), dim3(kBackNT), back_lds(N), st, V, N, Ld, Wd, z, x);
  return hipGetLastError();
}

hipError_t cholesky(double* V, int N, double* Ld, int* info_dev, hipStream_t st) {
  hipError_t e = chol_factor_solve(V, N, nullptr, 1.0, nullptr, nullptr, Ld, info_dev, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_diag, dim3((N + kNB - 1) / kNB), dim3(256), 0, st, V, N, Ld);
  return hipGetLastError();
}

hipError_t chol_inv_frob(const double* V, int N, double* Ld, double* part, hipStream_t st) {
  if (N < 1 || N > 4096) return hipErrorInvalidValue;
  const int T = (N + kNB - 1) / kNB;
  double* Wd = Ld + (int64_t)T * kNB * kNB;
  double* Xs = Wd + (int64_t)T * kNB * kNB;
  hipLaunchKernelGGL(k_invert_last, dim3(1), dim3(kStepNT), sizeof(StepLds), st, Ld, Wd, N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_inv_frob, dim3(T), dim3(256), sizeof(InvLds), st, V, N, Wd, Xs, part);
  return hipGetLastError();
}

hipError_t zero_upper(double* V, int N, hipStream_t st) {
  int64_t nb = ((int64_t)N * N + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)nb), dim3(256), 0, st, V, N);
  return hipGetLastError();
}

}  // namespace ssnal
