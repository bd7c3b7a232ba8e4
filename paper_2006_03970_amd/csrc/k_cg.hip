// Conjugate gradients on the Newton system V d = -g, V = I + kappa A_J A_J^T
// (eq. AJ_system): the approximate direction of Sec. 3.2 for systems too
// large to factor.  V is never formed: s = A_J^T p runs on the A^T v kernel
// over the columns J, A_J s on the gathered kernel, and the finisher here
// forms q = p + kappa A_J s.  The iterate, residual, search direction and
// every scalar stay on the device; each kernel returns at once after the
// done flag is set, so the host queues several iterations between
// read-backs.  Each reduction adds per-block partials in a fixed order (every
// block that needs a total sums the same partials in the same order), so a
// run is bitwise repeatable.
#include "common.hpp"
#include "kernels.hpp"
#include "scal.hpp"

namespace ssnal {

constexpr int kCgNT = 256;
constexpr int kCgEPT = 4;  // m-vector entries per thread
constexpr int kCgRows = kCgNT * kCgEPT;

int cg_blocks(int m) { return (m + kCgRows - 1) / kCgRows; }

__device__ __forceinline__ bool cg_done(const double* scal) { return scal[SC_CG_DONE] != 0.0; }

// Sum of nb block partials, the same value in every thread of every block.
__device__ __forceinline__ double ordered_sum(const double* __restrict__ part, int nb, double* red) {
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += kCgNT) t += part[b];
  return block_sum<kCgNT>(t, red);
}

// d = 0, res = p = -g; block partials of |g|^2.
__global__ __launch_bounds__(kCgNT) void k_cg_init(const double* __restrict__ g, double* __restrict__ d,
                                                   double* __restrict__ res, double* __restrict__ p,
                                                   int m, double* __restrict__ blk) {
  __shared__ double red[kCgNT / kWave];
  const int base = blockIdx.x * kCgRows + threadIdx.x;
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kCgEPT; ++k) {
    const int i = base + k * kCgNT;
    if (i < m) {
      const double v = -g[i];
      d[i] = 0.0;
      res[i] = v;
      p[i] = v;
      t += v * v;
    }
  }
  t = block_sum<kCgNT>(t, red);
  if (threadIdx.x == 0) blk[blockIdx.x] = t;
}

__global__ __launch_bounds__(kCgNT) void k_cg_start(const double* __restrict__ blk, int nb, double eps2,
                                                    double* __restrict__ scal) {
  __shared__ double red[kCgNT / kWave];
  const double rr = ordered_sum(blk, nb, red);
  if (threadIdx.x == 0) {
    const double stop = eps2 * rr;
    scal[SC_CG_RR] = rr;
    scal[SC_CG_RR + 1] = 0.0;
    scal[SC_CG_STOP] = stop;
    scal[SC_CG_DONE] = rr <= stop ? 1.0 : 0.0;
    scal[SC_CG_IT] = 0.0;
  }
}

// q = p + kappa sum_c part[c*m + i] (the nc chunk sums of A_J s, in chunk
// order), one row per thread; block partials of p^T q.
__global__ __launch_bounds__(kCgNT) void k_cg_q(const double* __restrict__ part, int nc, int m,
                                                double kappa, const double* __restrict__ p,
                                                double* __restrict__ q, double* __restrict__ blk,
                                                const double* __restrict__ scal) {
  if (cg_done(scal)) return;
  __shared__ double red[kCgNT / kWave];
  const int i = blockIdx.x * kCgNT + threadIdx.x;
  const int ic = i < m ? i : m - 1;
  double S = 0.0;
  int c = 0;
  for (; c + 8 <= nc; c += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(c + u) * m + ic];
#pragma unroll
    for (int u = 0; u < 8; ++u) S += v[u];
  }
  for (; c < nc; ++c) S += part[(int64_t)c * m + ic];
  double t = 0.0;
  if (i < m) {
    const double pi = p[i];
    const double qi = pi + kappa * S;
    q[i] = qi;
    t = pi * qi;
  }
  t = block_sum<kCgNT>(t, red);
  if (threadIdx.x == 0) blk[blockIdx.x] = t;
}

// alpha = rr / p^T q; d += alpha p; res -= alpha q; block partials of |res|^2.
__global__ __launch_bounds__(kCgNT) void k_cg_update(const double* __restrict__ blk, int nb, int m,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ d, double* __restrict__ res,
                                                     double* __restrict__ blk2,
                                                     const double* __restrict__ scal, int par) {
  if (cg_done(scal)) return;
  __shared__ double red[kCgNT / kWave];
  const double pq = ordered_sum(blk, nb, red);
  const double alpha = scal[SC_CG_RR + par] / pq;
  const int base = blockIdx.x * kCgRows + threadIdx.x;
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kCgEPT; ++k) {
    const int i = base + k * kCgNT;
    if (i < m) {
      d[i] += alpha * p[i];
      const double ri = res[i] - alpha * q[i];
      res[i] = ri;
      t += ri * ri;
    }
  }
  t = block_sum<kCgNT>(t, red);
  if (threadIdx.x == 0) blk2[blockIdx.x] = t;
}

// beta = rr_new / rr; p = res + beta p.  Block 0 stores rr_new in the other
// parity slot, counts the iteration and raises the done flag once
// rr_new <= stop (blocks that start after that skip the now unneeded update
// of p).
__global__ __launch_bounds__(kCgNT) void k_cg_dir(const double* __restrict__ blk2, int nb, int m,
                                                  const double* __restrict__ res,
                                                  double* __restrict__ p, double* scal, int par) {
  if (cg_done(scal)) return;
  __shared__ double red[kCgNT / kWave];
  const double rr_new = ordered_sum(blk2, nb, red);
  const double beta = rr_new / scal[SC_CG_RR + par];
  const int base = blockIdx.x * kCgRows + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kCgEPT; ++k) {
    const int i = base + k * kCgNT;
    if (i < m) p[i] = res[i] + beta * p[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[SC_CG_RR + (par ^ 1)] = rr_new;
    scal[SC_CG_IT] += 1.0;
    if (rr_new <= scal[SC_CG_STOP]) scal[SC_CG_DONE] = 1.0;
  }
}

hipError_t cg_init(const double* g, double* d, double* res, double* p, int m, double eps2,
                   double* blk, double* scal, hipStream_t st) {
  const int nb = cg_blocks(m);
  hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(kCgNT), 0, st, g, d, res, p, m, blk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kCgNT), 0, st, blk, nb, eps2, scal);
  return hipGetLastError();
}

hipError_t cg_iteration(const void* A, int dtype, int64_t lda, int m, const int32_t* J, int64_t r,
                        double kappa, bool acc64, double* d, double* res, double* p, double* q,
                        double* s, double* gpart, double* blk, int par, double* scal,
                        hipStream_t st) {
  const double* done = scal + SC_CG_DONE;
  hipError_t e = gemv_t(A, dtype, lda, m, r, J, p, s, acc64, st, nullptr, nullptr, done);
  if (e != hipSuccess) return e;
  e = gather_gemv_partial(A, dtype, lda, m, J, s, nullptr, r, gpart, st, done);
  if (e != hipSuccess) return e;
  const int nb = cg_blocks(m);
  const int nbq = (m + kCgNT - 1) / kCgNT;
  const int nc = gather_nchunks(r, m);
  hipLaunchKernelGGL(k_cg_q, dim3(nbq), dim3(kCgNT), 0, st, gpart, nc, m, kappa, p, q, blk, scal);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kCgNT), 0, st, blk, nbq, m, p, q, d, res, blk + nbq,
                     scal, par);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(kCgNT), 0, st, blk + nbq, nb, m, res, p, scal, par);
  return hipGetLastError();
}

}  // namespace ssnal
