// FP64 Cholesky factorisation and solves for the Newton system
// (eq. AJ_system: (I + kappa A_J A_J^T) d = -grad psi, or the r x r matrix of
// eq. smw_formula).  The matrix is N x N, row-major, lower triangle used.
//
// Elimination is written in its unscaled form: at step k every trailing
// entry a_ij (k < j <= i) loses a_ik a_jk / a_kk, so only column k has to be
// final before step k; afterwards L_ik = a_ik / sqrt(a_kk).
//
//   N <= 128: one workgroup holds the whole matrix in LDS, factors it and
//             solves for the right-hand side (one launch).
//   N  > 128: right-looking blocked factorisation with 64 x 64 blocks: one
//             launch factors the diagonal block (redundantly in every
//             workgroup) and solves the panel below it, one launch applies
//             the rank-64 trailing update on the matrix cores (FP64 MFMA);
//             then one workgroup runs both triangular solves.
#include "common.hpp"
#include "kernels.hpp"

namespace ssnal {

constexpr int kNB = 64;
constexpr int kBP = kNB + 1;  // LDS pitch of a 64 x 64 block

// Unscaled in-LDS factorisation of an n x n block (pitch P); on exit
// a[i][j] (j < i) = L_ij, a[j][j] = L_jj, rinv[j] = 1 / L_jj.
// Returns the first non-positive pivot + 1, or 0.
template <int NT>
__device__ int lds_factor(double* a, int P, int n, double* rinv) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double akk = a[k * P + k];
    if (!(akk > 0.0)) {  // uniform: every thread reads the same value
      if (threadIdx.x == 0) bad = k + 1;
      __syncthreads();
      return bad;
    }
    const double inv = 1.0 / akk;
    const int M = n - k - 1;
    for (int e = threadIdx.x; e < M * M; e += NT) {
      const int ii = e / M, jj = e - ii * M;
      if (jj <= ii) {
        const int i = k + 1 + ii, j = k + 1 + jj;
        a[i * P + j] -= a[i * P + k] * a[j * P + k] * inv;
      }
    }
    __syncthreads();
  }
  // scale: L_ij = a_ij / sqrt(a_jj)
  for (int j = threadIdx.x; j < n; j += NT) rinv[j] = 1.0 / sqrt(a[j * P + j]);
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e - i * n;
    if (j < i) a[i * P + j] *= rinv[j];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += NT) a[j * P + j] = sqrt(a[j * P + j]);
  __syncthreads();
  return 0;
}

// Forward and backward substitution by one wave: L L^T x = c, c held in LDS.
// Lane l keeps entries l, l+64, ... of c in registers (NS slots).
template <int NS>
__device__ void wave_solve(const double* a, int P, int n, const double* rinv, double* c) {
  const int lane = threadIdx.x & (kWave - 1);
  double v[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + s * kWave;
    v[s] = i < n ? c[i] : 0.0;
  }
  // L z = c  (column-oriented)
  for (int k = 0; k < n; ++k) {
    const int sk = k / kWave;
    double own = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (s == sk) own = v[s];
    const double zk = __shfl(own, k & (kWave - 1), kWave) * rinv[k];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + s * kWave;
      if (i == k) v[s] = zk;
      else if (i > k && i < n) v[s] -= a[i * P + k] * zk;
    }
  }
  // L^T x = z  (row k of L updates the entries above it)
  for (int k = n - 1; k >= 0; --k) {
    const int sk = k / kWave;
    double own = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (s == sk) own = v[s];
    const double xk = __shfl(own, k & (kWave - 1), kWave) * rinv[k];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + s * kWave;
      if (i == k) v[s] = xk;
      else if (i < k) v[s] -= a[k * P + i] * xk;
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + s * kWave;
    if (i < n) c[i] = v[s];
  }
}

// ---------------------------------------------------------------- N <= 128
__global__ __launch_bounds__(256) void k_chol_small(double* __restrict__ V, int N,
                                                    const double* __restrict__ rhs, double alpha,
                                                    double* __restrict__ x, int* __restrict__ info,
                                                    int write_l) {
  extern __shared__ double sm[];
  const int P = N + 1;
  double* a = sm;
  double* c = sm + N * P;
  double* rinv = c + N;
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int i = e / N, j = e - i * N;
    if (j <= i) a[i * P + j] = V[e];
  }
  if (rhs)
    for (int i = threadIdx.x; i < N; i += blockDim.x) c[i] = alpha * rhs[i];
  __syncthreads();
  const int bad = lds_factor<256>(a, P, N, rinv);
  if (threadIdx.x == 0) *info = bad;
  if (bad) return;
  if (write_l) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
      const int i = e / N, j = e - i * N;
      V[e] = j <= i ? a[i * P + j] : 0.0;
    }
  }
  if (!rhs) return;
  if (threadIdx.x < kWave) wave_solve<2>(a, P, N, rinv, c);
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) x[i] = c[i];
}

// ---------------------------------------------------------------- blocked, N > 128
// Block kb: every workgroup factors the diagonal block; workgroup 0 writes it
// back, workgroup p >= 1 solves X L_kk^T = B for row block kb + p.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ V, int N, int kb,
                                                    int* __restrict__ info) {
  __shared__ double d[kNB * kBP];
  __shared__ double b[kNB * kBP];
  __shared__ double rinv[kNB];
  const int r0 = kb * kNB;
  const int nk = N - r0 < kNB ? N - r0 : kNB;
  for (int e = threadIdx.x; e < nk * nk; e += blockDim.x) {
    const int i = e / nk, j = e - i * nk;
    if (j <= i) d[i * kBP + j] = V[(int64_t)(r0 + i) * N + r0 + j];
  }
  __syncthreads();
  const int bad = lds_factor<256>(d, kBP, nk, rinv);
  if (bad) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *info = r0 + bad;
    return;
  }
  if (blockIdx.x == 0) {
    for (int e = threadIdx.x; e < nk * nk; e += blockDim.x) {
      const int i = e / nk, j = e - i * nk;
      if (j <= i) V[(int64_t)(r0 + i) * N + r0 + j] = d[i * kBP + j];
    }
    return;
  }
  const int p0 = r0 + (int)blockIdx.x * kNB;  // first row of this panel block
  const int np = N - p0 < kNB ? N - p0 : kNB;
  for (int e = threadIdx.x; e < np * nk; e += blockDim.x) {
    const int i = e / nk, j = e - i * nk;
    b[i * kBP + j] = V[(int64_t)(p0 + i) * N + r0 + j];
  }
  __syncthreads();
  // X L^T = B, column by column: x_j = b_j / L_jj, then b_l -= x_j L_lj (l > j)
  for (int j = 0; j < nk; ++j) {
    for (int i = threadIdx.x; i < np; i += blockDim.x) b[i * kBP + j] *= rinv[j];
    __syncthreads();
    const int M = nk - j - 1;
    for (int e = threadIdx.x; e < np * M; e += blockDim.x) {
      const int i = e / M, l = j + 1 + (e - (e / M) * M);
      b[i * kBP + l] -= b[i * kBP + j] * d[l * kBP + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < np * nk; e += blockDim.x) {
    const int i = e / nk, j = e - i * nk;
    V[(int64_t)(p0 + i) * N + r0 + j] = b[i * kBP + j];
  }
}

// Trailing update V[ib][jb] -= L[ib][kb] L[jb][kb]^T for kb < jb <= ib.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ V, int N, int kb, int T) {
  __shared__ double P[kNB][kBP];  // P[k][i] = L[ib*64+i][kb*64+k]
  __shared__ double Q[kNB][kBP];
  // lower-triangle tiles (ib >= jb) among the T trailing block rows
  const int t = blockIdx.x;
  int ib = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((ib + 1) * (ib + 2) / 2 <= t) ++ib;
  while (ib * (ib + 1) / 2 > t) --ib;
  int jb = t - ib * (ib + 1) / 2;
  ib += kb + 1;
  jb += kb + 1;
  const int i0 = ib * kNB, j0 = jb * kNB, k0 = kb * kNB;
  const int ni = N - i0 < kNB ? N - i0 : kNB;
  const int nj = N - j0 < kNB ? N - j0 : kNB;
  const int nk = N - k0 < kNB ? N - k0 : kNB;
  for (int e = threadIdx.x; e < kNB * kNB; e += blockDim.x) {
    const int i = e / kNB, k = e - i * kNB;
    P[k][i] = (i < ni && k < nk) ? V[(int64_t)(i0 + i) * N + k0 + k] : 0.0;
    Q[k][i] = (i < nj && k < nk) ? V[(int64_t)(j0 + i) * N + k0 + k] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int wi = wid >> 1, wj = wid & 1;
  dbl4 acc[2][2];
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
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // FP64 MFMA: accumulator v holds row lane/16 + 4*v, column lane%16
        const int r = wi * 32 + p * 16 + (lane / 16) + 4 * v;
        const int c = wj * 32 + q * 16 + (lane & 15);
        if (r < ni && c < nj && (ib != jb || c <= r)) V[(int64_t)(i0 + r) * N + j0 + c] -= acc[p][q][v];
      }
}

// Both triangular solves of L L^T x = alpha*rhs, one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_chol_trsv(const double* __restrict__ L, int N,
                                                    const double* __restrict__ rhs, double alpha,
                                                    double* __restrict__ x) {
  extern __shared__ double sm[];
  double* c = sm;                 // N
  double* d = sm + N;             // diagonal block, 64 x 65
  double* rinv = d + kNB * kBP;   // 64
  for (int i = threadIdx.x; i < N; i += blockDim.x) c[i] = alpha * rhs[i];
  const int nb = (N + kNB - 1) / kNB;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  // forward: L z = c
  for (int kb = 0; kb < nb; ++kb) {
    const int r0 = kb * kNB;
    const int nk = N - r0 < kNB ? N - r0 : kNB;
    __syncthreads();
    for (int e = threadIdx.x; e < nk * nk; e += blockDim.x) {
      const int i = e / nk, j = e - i * nk;
      d[i * kBP + j] = j <= i ? L[(int64_t)(r0 + i) * N + r0 + j] : 0.0;
    }
    for (int j = threadIdx.x; j < nk; j += blockDim.x) rinv[j] = 1.0 / L[(int64_t)(r0 + j) * N + r0 + j];
    __syncthreads();
    if (wid == 0) {
      double v = lane < nk ? c[r0 + lane] : 0.0;
      for (int k = 0; k < nk; ++k) {
        const double zk = __shfl(v, k, kWave) * rinv[k];
        if (lane == k) v = zk;
        else if (lane > k && lane < nk) v -= d[lane * kBP + k] * zk;
      }
      if (lane < nk) c[r0 + lane] = v;
    }
    __syncthreads();
    // rows below: c_i -= sum_{k in block} L_ik z_k  (one wave per row)
    for (int i = r0 + nk + wid; i < N; i += nw) {
      double s = lane < nk ? L[(int64_t)i * N + r0 + lane] * c[r0 + lane] : 0.0;
      s = wave_sum(s);
      if (lane == 0) c[i] -= s;
    }
  }
  // backward: L^T x = z
  for (int kb = nb - 1; kb >= 0; --kb) {
    const int r0 = kb * kNB;
    const int nk = N - r0 < kNB ? N - r0 : kNB;
    __syncthreads();
    for (int e = threadIdx.x; e < nk * nk; e += blockDim.x) {
      const int i = e / nk, j = e - i * nk;
      d[i * kBP + j] = j <= i ? L[(int64_t)(r0 + i) * N + r0 + j] : 0.0;
    }
    for (int j = threadIdx.x; j < nk; j += blockDim.x) rinv[j] = 1.0 / L[(int64_t)(r0 + j) * N + r0 + j];
    __syncthreads();
    if (wid == 0) {
      double v = lane < nk ? c[r0 + lane] : 0.0;
      for (int k = nk - 1; k >= 0; --k) {
        const double xk = __shfl(v, k, kWave) * rinv[k];
        if (lane == k) v = xk;
        else if (lane < k) v -= d[k * kBP + lane] * xk;
      }
      if (lane < nk) c[r0 + lane] = v;
    }
    __syncthreads();
    // rows above: c_i -= sum_{k in block} L_ki x_k  (thread per row, coalesced over i)
    for (int i = threadIdx.x; i < r0; i += blockDim.x) {
      double s = 0.0;
      for (int k = 0; k < nk; ++k) s += L[(int64_t)(r0 + k) * N + i] * c[r0 + k];
      c[i] -= s;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) x[i] = c[i];
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
hipError_t chol_init() {
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_small,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_chol_trsv, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024 - 1024);
}

hipError_t chol_factor_solve_small(double* V, int N, const double* rhs, double alpha, double* x,
                                   int* info_dev, hipStream_t st) {
  if (N > kSmallN) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * ((size_t)N * (N + 1) + 2 * N);
  hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(256), lds, st, V, N, rhs, alpha, x, info_dev,
                     rhs ? 0 : 1);
  return hipGetLastError();
}

hipError_t cholesky(double* V, int N, int* info_dev, hipStream_t st) {
  if (N <= kSmallN) {
    const size_t lds = sizeof(double) * ((size_t)N * (N + 1) + 2 * N);
    hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(256), lds, st, V, N, (const double*)nullptr, 1.0,
                       (double*)nullptr, info_dev, 1);
    return hipGetLastError();
  }
  const int nb = (N + kNB - 1) / kNB;
  for (int kb = 0; kb < nb; ++kb) {
    hipLaunchKernelGGL(k_chol_panel, dim3(nb - kb), dim3(256), 0, st, V, N, kb, info_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int T = nb - kb - 1;
    if (T > 0) {
      hipLaunchKernelGGL(k_chol_update, dim3(T * (T + 1) / 2), dim3(256), 0, st, V, N, kb, T);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t chol_solve(const double* L, int N, const double* rhs, double alpha, double* x,
                      hipStream_t st) {
  const size_t lds = sizeof(double) * ((size_t)N + kNB * kBP + kNB);
  hipLaunchKernelGGL(k_chol_trsv, dim3(1), dim3(1024), lds, st, L, N, rhs, alpha, x);
  return hipGetLastError();
}

hipError_t zero_upper(double* V, int N, hipStream_t st) {
  int64_t nb = ((int64_t)N * N + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)nb), dim3(256), 0, st, V, N);
  return hipGetLastError();
}

}  // namespace ssnal
