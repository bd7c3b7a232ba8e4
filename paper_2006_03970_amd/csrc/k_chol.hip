// FP64 Cholesky factorisation and solve of the Newton system
// (eq. AJ_system: (I + kappa A_J A_J^T) d = -grad psi, or the r x r matrix of
// eq. smw_formula).  The matrix is N x N, row-major, lower triangle used; on
// exit it holds L (V = L L^T).
//
// Right-looking, 64 x 64 blocks, ONE launch per block column s:
//   * panel workgroups p = 0 .. T-s-1 own row block s+p of column s.  Each
//     first applies the rank-64 update of the previous step to its own tile
//     and to the diagonal tile (matrix cores, FP64 MFMA), then runs the
//     elimination of the stacked [diagonal tile; own tile] on registers
//     (256 threads x 8 x 4 entries, one barrier per column), in unscaled
//     form: a_il -= a_ij a_lj / a_jj, then L_il = a_il / sqrt(a_ll).
//     Every panel workgroup factors the diagonal tile itself, so no
//     workgroup waits for another inside a launch.
//   * the same launch's remaining workgroups apply the previous step's
//     update to the trailing tiles of columns s+1 .. T-1.
//   * the forward substitution L z = alpha*rhs rides along: workgroup p
//     subtracts L_{s+p,s-1} z_{s-1} from its block of the right-hand side,
//     and the diagonal workgroup solves its block for z_s.
// A single workgroup then runs the backward substitution L^T x = z.
#include "common.hpp"
#include "kernels.hpp"

namespace ssnal {

constexpr int kNB = 64;
constexpr int kBP = kNB + 1;  // LDS pitch of a 64 x 64 tile

__device__ __forceinline__ void tri_of(int t, int& i, int& j) {
  // t enumerates lower-triangle pairs (i >= j) row by row: t = i(i+1)/2 + j
  int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  i = r;
  j = t - r * (r + 1) / 2;
}

// Stage a 64 x 64 block of V (rows i0.., cols k0..) transposed into LDS:
// dst[k][i] = V[i0+i][k0+k], zero outside the matrix.
// All 16 loads of a thread are issued before the first store to LDS.
__device__ __forceinline__ void stage_t(const double* __restrict__ V, int N, int i0, int k0,
                                        double (*dst)[kBP]) {
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + q * 256;
    const int i = e / kNB, k = e % kNB;
    v[q] = (i0 + i < N && k0 + k < N) ? V[(int64_t)(i0 + i) * N + k0 + k] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + q * 256;
    dst[e % kNB][e / kNB] = v[q];
  }
}

// C[i][j] = sum_k P[k][i] Q[k][j] for the 64 x 64 tile, with P, Q staged by
// stage_t.  Wave w owns rows 32*(w>>1).., columns 32*(w&1)..; FP64 MFMA
// 16x16x4, whose accumulator v holds row lane/16 + 4*v, column lane%16.
__device__ __forceinline__ void mfma_64(double (*P)[kBP], double (*Q)[kBP], dbl4 acc[2][2]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int wi = wid >> 1, wj = wid & 1;
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

// tile[r][c] -= C  (r, c local to the 64 x 64 tile)
__device__ __forceinline__ void sub_acc(double (*tile)[kBP], dbl4 acc[2][2]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int wi = wid >> 1, wj = wid & 1;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wi * 32 + p * 16 + (lane / 16) + 4 * v;
        const int c = wj * 32 + q * 16 + (lane & 15);
        tile[r][c] -= acc[p][q][v];
      }
}

struct StepLds {
  double P[kNB][kBP];  // L_{s,s-1}, transposed
  double Q[kNB][kBP];  // L_{s+p,s-1}, transposed
  double D[kNB][kBP];  // diagonal tile
  double B[kNB][kBP];  // own tile
  double col[2][2 * kNB];
  double piv[kNB];
  double rs[kNB];
  double zprev[kNB];
};

__global__ __launch_bounds__(256) void k_chol_step(double* __restrict__ V, int N, int T, int s,
                                                   const double* __restrict__ rhs, double alpha,
                                                   double* __restrict__ z, int* __restrict__ info) {
  extern __shared__ double smem[];
  StepLds& L = *reinterpret_cast<StepLds*>(smem);
  const int tid = threadIdx.x;
  const int npanel = T - s;
  const int s0 = s * kNB;

  if ((int)blockIdx.x >= npanel) {
    // ---- trailing update of step s-1 on tiles (i, l), s+1 <= l <= i < T
    int ii, ll;
    tri_of((int)blockIdx.x - npanel, ii, ll);
    const int i = s + 1 + ii, l = s + 1 + ll;
    const int k0 = (s - 1) * kNB;
    stage_t(V, N, i * kNB, k0, L.P);
    stage_t(V, N, l * kNB, k0, L.Q);
    __syncthreads();
    dbl4 acc[2][2];
    mfma_64(L.P, L.Q, acc);
    const int lane = tid & (kWave - 1), wid = tid / kWave;
    const int wi = wid >> 1, wj = wid & 1;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = i * kNB + wi * 32 + p * 16 + (lane / 16) + 4 * v;
          const int c = l * kNB + wj * 32 + q * 16 + (lane & 15);
          if (r < N && c < N && (i != l || c <= r)) V[(int64_t)r * N + c] -= acc[p][q][v];
        }
    return;
  }

  // ---- panel workgroup p: row block s+p of column s
  for (int e = tid; e < 4 * kNB; e += blockDim.x) (&L.col[0][0])[e] = 0.0;
  const int p = blockIdx.x;
  const int b0 = (s + p) * kNB;
  const int nk = N - s0 < kNB ? N - s0 : kNB;  // width of column s
  const int nbr = p == 0 ? 0 : (N - b0 < kNB ? N - b0 : kNB);

  {
    double vd[16], vb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + q * 256;
      const int r = e / kNB, c = e % kNB;
      vd[q] = (r < nk && c <= r) ? V[(int64_t)(s0 + r) * N + s0 + c] : (r == c ? 1.0 : 0.0);
      vb[q] = (p > 0 && r < nbr && c < nk) ? V[(int64_t)(b0 + r) * N + s0 + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + q * 256;
      L.D[e / kNB][e % kNB] = vd[q];
      L.B[e / kNB][e % kNB] = vb[q];
    }
  }
  if (rhs && tid < kNB) {
    const int g = b0 + tid;
    if (s == 0) {
      if (g < N) z[g] = alpha * rhs[g];
    } else {
      L.zprev[tid] = z[s0 - kNB + tid];  // block s-1 is always full
    }
  }
  if (s > 0) {
    // previous step's rank-64 update of the diagonal tile and of the own tile
    stage_t(V, N, s0, s0 - kNB, L.P);
    if (p > 0) stage_t(V, N, b0, s0 - kNB, L.Q);
    __syncthreads();
    dbl4 acc[2][2];
    mfma_64(L.P, L.P, acc);
    sub_acc(L.D, acc);
    if (p > 0) {
      mfma_64(L.Q, L.P, acc);
      sub_acc(L.B, acc);
    }
    if (rhs && tid < kNB && b0 + tid < N) {
      // rhs block s+p loses L_{s+p,s-1} z_{s-1}
      double(*Lp)[kBP] = p > 0 ? L.Q : L.P;
      double t = 0.0;
      for (int k = 0; k < kNB; ++k) t += Lp[k][tid] * L.zprev[k];
      z[b0 + tid] -= t;
    }
  }
  __syncthreads();

  // ---- elimination on registers: thread (tr, tc) owns rows 8tr..8tr+7 of
  // the stacked [D; B] (128 rows) and columns 4tc..4tc+3
  const int tr = tid / 16, tc = tid % 16;
  const bool in_b = tr >= 8;
  const bool live = !in_b || p > 0;
  double a[8][4];
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int r = 8 * tr + q, col = 4 * tc + c;
      a[q][c] = live ? (in_b ? L.B[r - kNB][col] : L.D[r][col]) : 0.0;
    }
  // Four columns per iteration, so the column a thread publishes is a
  // compile-time register index (a runtime pick serialises the LDS writes).
  for (int j0 = 0; j0 < kNB; j0 += 4) {
    const bool owner = (tc == (j0 >> 2)) && live;
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      const int j = j0 + c4;
      double* cb = L.col[j & 1];
      if (owner) {
#pragma unroll
        for (int q = 0; q < 8; ++q) cb[8 * tr + q] = a[q][c4];
      }
      __syncthreads();
      const double pv = cb[j];
      if (!(pv > 0.0)) {  // every thread reads the same pivot: a uniform exit
        if (tid == 0 && p == 0) *info = s0 + j + 1;
        return;
      }
      if (tid == 0) L.piv[j] = pv;
      // Branch-free update of every column > j.  In the diagonal tile this
      // also touches entries above the diagonal: they start at zero, stay
      // finite, and are never read back (only columns j' >= j of rows > j
      // feed later steps, and the write-back keeps the lower triangle).
      const double inv = 1.0 / pv;
      double ci[8], cl[4];
#pragma unroll
      for (int q = 0; q < 8; ++q) ci[q] = cb[8 * tr + q] * inv;
#pragma unroll
      for (int c = 0; c < 4; ++c) cl[c] = (4 * tc + c > j) ? cb[4 * tc + c] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) a[q][c] = fma(-ci[q], cl[c], a[q][c]);
    }
  }
  __syncthreads();
  if (tid < kNB) L.rs[tid] = 1.0 / sqrt(L.piv[tid]);
  __syncthreads();
  // scale and write back: L_rc = a_rc / sqrt(d_c), L_cc = sqrt(d_c)
  if (live) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int r = 8 * tr + q, col = 4 * tc + c;
        if (in_b) {
          const int rr = r - kNB;
          if (rr < nbr && col < nk) V[(int64_t)(b0 + rr) * N + s0 + col] = a[q][c] * L.rs[col];
        } else if (col <= r) {
          const double v = col == r ? L.piv[col] * L.rs[col] : a[q][c] * L.rs[col];
          L.D[r][col] = v;
          if (p == 0 && r < nk) V[(int64_t)(s0 + r) * N + s0 + col] = v;
        }
      }
  }
  if (p != 0 || !rhs) return;
  __syncthreads();
  // forward substitution of this block: L_ss z_s = (updated) rhs_s
  if (tid < kWave) {
    const int lane = tid;
    double v = lane < nk ? z[s0 + lane] : 0.0;
    for (int j = 0; j < nk; ++j) {
      const double zj = readlane_d(v, j) * L.rs[j];
      const double upd = fma(-L.D[lane][j], zj, v);
      v = lane == j ? zj : (lane > j ? upd : v);
    }
    if (lane < nk) z[s0 + lane] = v;
  }
}

// Backward substitution L^T x = z by one workgroup (1024 threads).
__global__ __launch_bounds__(1024) void k_chol_back(const double* __restrict__ Lm, int N,
                                                    const double* __restrict__ z,
                                                    double* __restrict__ x) {
  extern __shared__ double sm[];
  double* xs = sm;                                                          // N
  double(*Ld)[kBP] = reinterpret_cast<double(*)[kBP]>(sm + ((N + 1) & ~1));  // 64 x 65
  double* rinv = sm + ((N + 1) & ~1) + kNB * kBP;                           // 64
  for (int i = threadIdx.x; i < N; i += blockDim.x) xs[i] = z[i];
  const int T = (N + kNB - 1) / kNB;
  for (int s = T - 1; s >= 0; --s) {
    const int s0 = s * kNB;
    const int nk = N - s0 < kNB ? N - s0 : kNB;
    __syncthreads();
    {
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + q * 1024;
        const int r = e / kNB, c = e % kNB;
        v[q] = (r < nk && c <= r) ? Lm[(int64_t)(s0 + r) * N + s0 + c] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + q * 1024;
        Ld[e / kNB][e % kNB] = v[q];
      }
    }
    __syncthreads();
    if (threadIdx.x < kNB) rinv[threadIdx.x] = threadIdx.x < nk ? 1.0 / Ld[threadIdx.x][threadIdx.x] : 0.0;
    __syncthreads();
    if (threadIdx.x < kWave) {
      const int lane = threadIdx.x;
      double v = lane < nk ? xs[s0 + lane] : 0.0;
      for (int b = nk - 1; b >= 0; --b) {
        const double xb = readlane_d(v, b) * rinv[b];
        const double upd = fma(-Ld[b][lane], xb, v);
        v = lane == b ? xb : (lane < b ? upd : v);
      }
      if (lane < nk) xs[s0 + lane] = v;
    }
    __syncthreads();
    // entries above the block: x_i -= sum_b L[s0+b][i] x_{s0+b}.  Eight
    // threads share a column i (rows b = 8*part .. 8*part+7 < nk, loads
    // issued together) and combine with lane shuffles; a group of eight
    // lanes enters and leaves the loop together.
    for (int idx = threadIdx.x; idx < s0 * 8; idx += blockDim.x) {
      const int i = idx >> 3, part = idx & 7;
      double lv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int b = 8 * part + q;
        lv[q] = b < nk ? Lm[(int64_t)(s0 + b) * N + i] : 0.0;
      }
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int b = 8 * part + q;
        if (b < nk) t += lv[q] * xs[s0 + b];
      }
      t = group8_sum(t);
      if (part == 0) xs[i] -= t;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) x[i] = xs[i];
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
static size_t back_lds(int N) { return sizeof(double) * ((size_t)((N + 1) & ~1) + kNB * kBP + kNB); }

hipError_t chol_init() {
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_step,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, sizeof(StepLds));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_chol_back, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)back_lds(4096));
}

hipError_t chol_factor_solve(double* V, int N, const double* rhs, double alpha, double* z,
                             double* x, int* info_dev, hipStream_t st) {
  if (N < 1 || N > 4096) return hipErrorInvalidValue;
  const int T = (N + kNB - 1) / kNB;
  for (int s = 0; s < T; ++s) {
    const int npanel = T - s;
    const int U = s >= 1 ? (T - s - 1) * (T - s) / 2 : 0;
    hipLaunchKernelGGL(k_chol_step, dim3(npanel + U), dim3(256), sizeof(StepLds), st, V, N, T, s,
                       rhs, alpha, z, info_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!rhs) return hipSuccess;
  hipLaunchKernelGGL(k_chol_back, dim3(1), dim3(1024), back_lds(N), st, V, N, z, x);
  return hipGetLastError();
}

hipError_t cholesky(double* V, int N, int* info_dev, hipStream_t st) {
  return chol_factor_solve(V, N, nullptr, 1.0, nullptr, nullptr, info_dev, st);
}

hipError_t zero_upper(double* V, int N, hipStream_t st) {
  int64_t nb = ((int64_t)N * N + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)nb), dim3(256), 0, st, V, N);
  return hipGetLastError();
}

}  // namespace ssnal
