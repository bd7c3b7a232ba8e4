// Passes over the n-vectors (x, A^T y, A^T d) and the gathers over the
// active set J.  These read a few bytes per feature, next to the m bytes per
// feature of the A^T v pass, so their time is latency: 256 threads and 2
// elements per thread, one block per 512 features (many short blocks spread
// over the CUs; measured faster than 8 elements per thread at n = 1e5), and
// sums across blocks finished by a one-block kernel (no device-wide fences).
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "scal.hpp"

namespace ssnal {

constexpr int kNT = 256;
constexpr int kEPT = 2;
constexpr int kChunk = kNT * kEPT;

int prox_blocks(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }

__device__ __forceinline__ bool active(double t, double thr) { return (t > thr) | (t < -thr); }

// Element loads below read at a clamped, always valid index and mask the
// value afterwards.  A load guarded by `if (i < n)`, or selected by a
// short-circuit condition, is compiled into a branch that waits for the load
// before the join, which serialises the loads of a thread.
__device__ __forceinline__ int64_t clampi(int64_t i, int64_t n) { return i < n ? i : n - 1; }

// ------------------------------------------------------------------ finishers
// Reductions that span blocks finish in a second, single-block kernel: the
// kernel boundary makes every block's partials visible, with no device-wide
// cache write-back inside the producing kernel.
// The end of a kernel that publishes the scalar slots to the host (one
// workgroup): once the workgroup's slot writes are in place, copy the slots
// to coherent pinned memory, a system-scope fence, then the flag with
// release semantics, so a host that observes the flag reads the new slots.
__device__ __forceinline__ void publish_block(const double* scal, const Pub& pub) {
  __syncthreads();
  for (int i = threadIdx.x; i < SC_SIZE; i += blockDim.x) pub.dst[i] = scal[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(pub.flag, pub.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// out and yy_out point into the slots that a publish request copies (scal).
template <int K>
__global__ __launch_bounds__(kNT) void k_final(const double* __restrict__ part, int nb, double* out,
                                               const double* __restrict__ y, int m, double* yy_out,
                                               const double* scal, Pub pub) {
  __shared__ double red[K * kNT / kWave];
  final_sums<kNT, K>(part, nb, out, red);
  if (y) {
    double t = 0.0;
    for (int i = threadIdx.x; i < m; i += kNT) t += y[i] * y[i];
    t = block_sum<kNT>(t, red);
    if (threadIdx.x == 0) *yy_out = t;
  }
  if (pub.flag) publish_block(scal, pub);
}

// ------------------------------------------------------------------ compaction
// Active set J = {i : |t_i| > sigma*lambda1} (eq. Q_def), t = x - sigma*w.
template <bool UPDATE, bool SUPPORT>
__global__ __launch_bounds__(kNT) void k_count(const double* __restrict__ x, double* __restrict__ w,
                                                const double* __restrict__ wd,
                                                const double* __restrict__ s_dev, int64_t n,
                                                double sigma, double thr, int* __restrict__ counts) {
  const double s = UPDATE ? *s_dev : 0.0;
  int cnt = 0;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double xv[kEPT], wv[kEPT], dv[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int64_t ic = clampi(base + k * kNT + threadIdx.x, n);
    xv[k] = x[ic];
    if (!SUPPORT) wv[k] = w[ic];
    if (UPDATE) dv[k] = wd[ic];
  }
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int64_t i = base + k * kNT + threadIdx.x;
    const bool in = i < n;
    if (SUPPORT) {
      cnt += in & (xv[k] != 0.0);
    } else {
      double wi = wv[k];
      if (UPDATE) {
        wi = fma(s, dv[k], wi);  // w_y += s * w_d
        if (in) w[i] = wi;
      }
      cnt += in & active(fma(-sigma, wi, xv[k]), thr);
    }
  }
  __shared__ int red[kNT / kWave];
  const int tot = block_sum<kNT>(cnt, red);
  if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

template <bool SUPPORT>
__global__ __launch_bounds__(kNT) void k_write(const double* __restrict__ x,
                                                const double* __restrict__ w, int64_t n,
                                                double sigma, double thr, double den,
                                                const int* __restrict__ counts, int nblocks,
                                                int32_t* __restrict__ J, double* __restrict__ uJ,
                                                double* __restrict__ r_out) {
  __shared__ int red[kNT / kWave];
  __shared__ int wtot[kNT / kWave];
  int part = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kNT) part += counts[b];
  int off = block_sum<kNT>(part, red);
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double tv[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int64_t ic = clampi(base + k * kNT + threadIdx.x, n);
    tv[k] = SUPPORT ? x[ic] : fma(-sigma, w[ic], x[ic]);
  }
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int64_t i = base + k * kNT + threadIdx.x;
    const double t = tv[k];
    const bool act = (i < n) & (SUPPORT ? (t != 0.0) : active(t, thr));
    const unsigned long long mask = __ballot(act);
    const int pre = __popcll(mask & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) wtot[wid] = __popcll(mask);
    __syncthreads();
    int wo = 0, bt = 0;
#pragma unroll
    for (int q = 0; q < kNT / kWave; ++q) {
      if (q < wid) wo += wtot[q];
      bt += wtot[q];
    }
    if (act) {
      const int pos = off + wo + pre;
      J[pos] = (int32_t)i;
      uJ[pos] = SUPPORT ? t : prox_en(t, thr, den);
    }
    off += bt;
  }
  if ((int)blockIdx.x == nblocks - 1 && threadIdx.x == 0) *r_out = (double)off;
}

hipError_t prox_count(const double* x, double* w, const double* wd, const double* s_dev, int64_t n,
                      ProxArgs pa, int* counts, hipStream_t st) {
  const int nb = prox_blocks(n);
  if (s_dev)
    hipLaunchKernelGGL((k_count<true, false>), dim3(nb), dim3(kNT), 0, st, x, w, wd, s_dev, n,
                       pa.sigma, pa.thr, counts);
  else
    hipLaunchKernelGGL((k_count<false, false>), dim3(nb), dim3(kNT), 0, st, x, w, wd, s_dev, n,
                       pa.sigma, pa.thr, counts);
  return hipGetLastError();
}

hipError_t prox_write(const double* x, const double* w, int64_t n, ProxArgs pa, const int* counts,
                      int32_t* J, double* uJ, double* r_out, hipStream_t st) {
  const int nb = prox_blocks(n);
  hipLaunchKernelGGL((k_write<false>), dim3(nb), dim3(kNT), 0, st, x, w, n, pa.sigma, pa.thr, pa.den,
                     counts, nb, J, uJ, r_out);
  return hipGetLastError();
}

hipError_t support_count(const double* x, int64_t n, int* counts, hipStream_t st) {
  const int nb = prox_blocks(n);
  hipLaunchKernelGGL((k_count<false, true>), dim3(nb), dim3(kNT), 0, st, x, (double*)nullptr,
                     (const double*)nullptr, (const double*)nullptr, n, 0.0, 0.0, counts);
  return hipGetLastError();
}

hipError_t support_write(const double* x, int64_t n, const int* counts, int32_t* J, double* uJ,
                         double* r_out, hipStream_t st) {
  const int nb = prox_blocks(n);
  hipLaunchKernelGGL((k_write<true>), dim3(nb), dim3(kNT), 0, st, x, (const double*)nullptr, n, 0.0,
                     0.0, 1.0, counts, nb, J, uJ, r_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ A_J c
// Chunk k of J is reduced by one block into a partial m-vector; the finisher
// adds the partials in chunk order, so the sum is reproducible.  r may live
// on the device (it comes from the compaction pass): the grid is sized for
// the largest possible r and blocks past the last chunk return at once.
// Most chunks an r-column gather over m rows takes: 1024; columns longer than
// 4096 rows already multiply the blocks by their row panels and take fewer
// (>= 64), which keeps the partial sums (nc m-vectors) small next to A_J.
__host__ __device__ __forceinline__ int64_t chunk_cap(int m) {
  if (m <= 4096) return 1024;
  const int64_t c = (int64_t)1024 * 4096 / m;
  return c < 64 ? 64 : c;
}

__host__ __device__ __forceinline__ void chunk_plan(int64_t r, int m, int& nc, int64_t& ck) {
  if (r <= 0) {
    nc = 0;
    ck = 0;
    return;
  }
  int64_t c = (r + chunk_cap(m) - 1) / chunk_cap(m);
  c = (c + 15) / 16 * 16;  // whole groups of 16 columns
  nc = (int)((r + c - 1) / c);
  ck = c;
}

// Upper bound of the chunk count for any r <= r_bound over m rows: nc(r, m)
// <= ceil(r/16) and <= chunk_cap(m) (nc itself is not monotone in r).
int gather_chunks(int64_t r_bound, int m) {
  if (r_bound <= 0) return 0;
  const int64_t c = (r_bound + 15) / 16;
  const int64_t cap = chunk_cap(m);
  return (int)(c < cap ? c : cap);
}

// Block (b, p) sums columns [b*ck, (b+1)*ck) of A_J weighted by c, for the
// rows [p*NQ*kNT, (p+1)*NQ*kNT); a thread keeps the loads of 16 columns in
// flight.  skip (nullable): the block returns at once while *skip != 0.
template <typename T, int NQ>
__global__ __launch_bounds__(kNT) void k_gather_partial(const T* __restrict__ A, int64_t lda, int m,
                                                         const int32_t* __restrict__ J,
                                                         const double* __restrict__ c,
                                                         const double* __restrict__ r_dev,
                                                         int64_t r_host, double* __restrict__ part,
                                                         const double* __restrict__ skip) {
  if (skip && *skip != 0.0) return;
  const int64_t r = r_dev ? (int64_t)(*r_dev) : r_host;
  const int rbase = (int)blockIdx.y * (NQ * kNT);
  int nc;
  int64_t ck;
  chunk_plan(r, m, nc, ck);
  if ((int)blockIdx.x >= nc) return;
  const int64_t k0 = (int64_t)blockIdx.x * ck;
  const int64_t k1 = k0 + ck < r ? k0 + ck : r;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int64_t kb = k0; kb < k1; kb += 16) {
    int64_t col[16];
    double cv[16];
    bool ok[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t k = kb + u;
      ok[u] = k < k1;
      const int64_t kc = ok[u] ? k : k1 - 1;  // past the chunk: a valid column, weight 0
      col[u] = (int64_t)J[kc] * lda;
      cv[u] = c[kc];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int row = rbase + threadIdx.x + q * kNT;
      if (row < m) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = load1<double>(A + col[u] + row);
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[q] += ok[u] ? v[u] * cv[u] : 0.0;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int row = rbase + threadIdx.x + q * kNT;
    if (row < m) part[(int64_t)blockIdx.x * m + row] = acc[q];
  }
}

// The same sums with 16-byte loads (VN consecutive rows per load) for FP32
// and FP64 designs whose columns start 16-byte aligned; each row adds the chunk's
// columns in the same order as above, so the sums are the same.  Loads of
// FP32/BF16 values go to FP32 registers (exact) and widen to FP64 at use.
template <typename T, int NQ>
__global__ __launch_bounds__(kNT) void k_gather_partial_v(const T* __restrict__ A, int64_t lda, int m,
                                                           const int32_t* __restrict__ J,
                                                           const double* __restrict__ c,
                                                           const double* __restrict__ r_dev,
                                                           int64_t r_host, double* __restrict__ part,
                                                           const double* __restrict__ skip) {
  using LT = typename std::conditional<std::is_same<T, double>::value, double, float>::type;
  constexpr int VN = 16 / (int)sizeof(T);
  if (skip && *skip != 0.0) return;
  const int64_t r = r_dev ? (int64_t)(*r_dev) : r_host;
  int nc;
  int64_t ck;
  chunk_plan(r, m, nc, ck);
  if ((int)blockIdx.x >= nc) return;
  const int64_t k0 = (int64_t)blockIdx.x * ck;
  const int64_t k1 = k0 + ck < r ? k0 + ck : r;
  double acc[NQ][VN];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int e = 0; e < VN; ++e) acc[q][e] = 0.0;
  for (int64_t kb = k0; kb < k1; kb += 16) {
    int64_t col[16];
    double cv[16];
    bool ok[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t k = kb + u;
      ok[u] = k < k1;
      const int64_t kc = ok[u] ? k : k1 - 1;  // past the chunk: a valid column, weight 0
      col[u] = (int64_t)J[kc] * lda;
      cv[u] = c[kc];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      // rows row0 .. row0 + VN - 1 < lda: lda is a multiple of VN
      const int row0 = (q * kNT + (int)threadIdx.x) * VN;
      if (row0 < m) {
        LT v[16][VN];
#pragma unroll
        for (int u = 0; u < 16; ++u) loadv<16>(A + col[u] + row0, v[u]);
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
          for (int e = 0; e < VN; ++e) acc[q][e] += ok[u] ? (double)v[u][e] * cv[u] : 0.0;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int row0 = (q * kNT + (int)threadIdx.x) * VN;
#pragma unroll
    for (int e = 0; e < VN; ++e)
      if (row0 + e < m) part[(int64_t)blockIdx.x * m + row0 + e] = acc[q][e];
  }
}

// Rows past 16 * kNT go to further row panels (grid.y).
template <typename T>
static hipError_t launch_gather(const T* A, int64_t lda, int m, const int32_t* J, const double* c,
                                const double* r_dev, int64_t r_bound, double* part, hipStream_t st,
                                const double* skip) {
  const int nb = gather_chunks(r_bound, m);
  if (nb == 0) return hipSuccess;
  constexpr int VN = 16 / (int)sizeof(T);
  const int nv = (m + kNT * VN - 1) / (kNT * VN);  // row groups of kNT * VN
  // FP32/FP64 columns of one row panel (16 BF16 columns of 8 rows would not
  // fit the registers; over several row panels the element loads measured
  // faster)
  if (sizeof(T) >= 4 && nv <= 4 && ((uintptr_t)A) % 16 == 0 && lda % VN == 0) {
    if (nv <= 1)
      hipLaunchKernelGGL((k_gather_partial_v<T, 1>), dim3(nb), dim3(kNT), 0, st, A, lda, m, J, c, r_dev,
                         r_bound, part, skip);
    else if (nv <= 2)
      hipLaunchKernelGGL((k_gather_partial_v<T, 2>), dim3(nb), dim3(kNT), 0, st, A, lda, m, J, c, r_dev,
                         r_bound, part, skip);
    else
      hipLaunchKernelGGL((k_gather_partial_v<T, 4>), dim3(nb), dim3(kNT), 0, st, A, lda, m, J, c, r_dev,
                         r_bound, part, skip);
    return hipGetLastError();
  }
  const int nq = (m + kNT - 1) / kNT;
#define SSNAL_GATHER_CASE(Q)                                                                   \
  if (nq <= Q) {                                                                               \
    hipLaunchKernelGGL((k_gather_partial<T, Q>), dim3(nb), dim3(kNT), 0, st, A, lda, m, J, c,     \
                       r_dev, r_bound, part, skip);                                            \
    return hipGetLastError();                                                                  \
  }
  SSNAL_GATHER_CASE(1)
  SSNAL_GATHER_CASE(2)
  SSNAL_GATHER_CASE(4)
  SSNAL_GATHER_CASE(8)
#undef SSNAL_GATHER_CASE
  const unsigned np = (unsigned)((m + 16 * kNT - 1) / (16 * kNT));
  hipLaunchKernelGGL((k_gather_partial<T, 16>), dim3(nb, np), dim3(kNT), 0, st, A, lda, m, J, c,
                     r_dev, r_bound, part, skip);
  return hipGetLastError();
}

hipError_t gather_gemv_partial(const void* A, int dtype, int64_t lda, int m, const int32_t* J,
                               const double* c, const double* r_dev, int64_t r_bound, double* part,
                               hipStream_t st, const double* skip) {
  switch (dtype) {
    case kF64:
      return launch_gather<double>((const double*)A, lda, m, J, c, r_dev, r_bound, part, st, skip);
    case kF32:
      return launch_gather<float>((const float*)A, lda, m, J, c, r_dev, r_bound, part, st, skip);
    case kBF16:
      return launch_gather<uint16_t>((const uint16_t*)A, lda, m, J, c, r_dev, r_bound, part, st, skip);
  }
  return hipErrorInvalidValue;
}

int gather_nchunks(int64_t r, int m) {
  int nc;
  int64_t ck;
  chunk_plan(r, m, nc, ck);
  return nc;
}

// sum_{c < nchunks} part[c m + row], added in chunk order, eight loads in
// flight.
__device__ __forceinline__ double chunk_sum(const double* __restrict__ part, int nchunks, int m, int row) {
  double S = 0.0;
  int c = 0;
  for (; c + 8 <= nchunks; c += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(c + u) * m + row];
#pragma unroll
    for (int u = 0; u < 8; ++u) S += v[u];
  }
  for (; c < nchunks; ++c) S += part[(int64_t)c * m + row];
  return S;
}

__global__ __launch_bounds__(kNT) void k_gather_finish(const double* __restrict__ part,
                                                        const double* __restrict__ r_dev,
                                                        int64_t r_host, int m, int mode,
                                                        const double* __restrict__ y,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ g,
                                                        double* __restrict__ out2,
                                                        double* __restrict__ blk) {
  const int64_t r = r_dev ? (int64_t)(*r_dev) : r_host;
  int nchunks;
  int64_t ck;
  chunk_plan(r, m, nchunks, ck);
  const int row = blockIdx.x * kNT + threadIdx.x;
  const double S = row < m ? chunk_sum(part, nchunks, m, row) : 0.0;
  double v1 = 0.0, v2 = 0.0, v3 = 0.0;
  if (row < m) {
    if (mode == 0) {  // gradient of psi (eq. grad_phy) and the primal residual A u - b
      const double gi = y[row] + b[row] - S;
      const double rho = S - b[row];
      g[row] = gi;
      out2[row] = rho;
      v1 = gi * gi;
      v2 = rho * rho;
      v3 = b[row] * rho;
    } else if (mode == 1) {  // Woodbury direction d = -g + A_J w
      out2[row] = -g[row] + S;
    } else {  // y = A x - b
      out2[row] = S - b[row];
    }
  }
  if (mode != 0) return;
  __shared__ double red[3 * kNT / kWave];
  double sv[3] = {v1, v2, v3};
  block_sums<kNT, 3>(sv, red);
  if (threadIdx.x == 0) {
    blk[3 * blockIdx.x + 0] = sv[0];
    blk[3 * blockIdx.x + 1] = sv[1];
    blk[3 * blockIdx.x + 2] = sv[2];
  }
}

// Mode 0 by one workgroup of 512 threads (m <= kFin1Max): the chunk sums,
// g, rho and the three sums of k_gather_finish + k_final<3> in one launch,
// optionally publishing the slots to the host at the end.
constexpr int kFin1NT = 512;
constexpr int kFin1Max = 2048;
__global__ __launch_bounds__(kFin1NT) void k_gather_finish1(const double* __restrict__ part,
                                                            const double* __restrict__ r_dev, int m,
                                                            const double* __restrict__ y,
                                                            const double* __restrict__ b,
                                                            double* __restrict__ g,
                                                            double* __restrict__ rho,
                                                            double* __restrict__ scal, Pub pub) {
  int nchunks;
  int64_t ck;
  chunk_plan((int64_t)(*r_dev), m, nchunks, ck);
  double v1 = 0.0, v2 = 0.0, v3 = 0.0;
  for (int row = threadIdx.x; row < m; row += kFin1NT) {
    const double S = chunk_sum(part, nchunks, m, row);
    // gradient of psi (eq. grad_phy) and the primal residual A u - b
    const double gi = y[row] + b[row] - S;
    const double rh = S - b[row];
    g[row] = gi;
    rho[row] = rh;
    v1 += gi * gi;
    v2 += rh * rh;
    v3 += b[row] * rh;
  }
  __shared__ double red[3 * kFin1NT / kWave];
  double sv[3] = {v1, v2, v3};
  block_sums<kFin1NT, 3>(sv, red);
  if (threadIdx.x == 0) {
    scal[SC_GG + 0] = sv[0];
    scal[SC_GG + 1] = sv[1];
    scal[SC_GG + 2] = sv[2];
  }
  if (pub.flag) publish_block(scal, pub);
}

hipError_t gather_finish(const double* part, const double* r_dev, int64_t r_host, int m, int mode,
                         const double* y, const double* b, double* g, double* out2, double* scal,
                         hipStream_t st, Pub pub, double* blk) {
  if (mode == 0 && r_dev && m <= kFin1Max) {
    hipLaunchKernelGGL(k_gather_finish1, dim3(1), dim3(kFin1NT), 0, st, part, r_dev, m, y, b, g, out2,
                       scal, pub);
    return hipGetLastError();
  }
  const int nb = (m + kNT - 1) / kNT;
  // the block partials of mode 0 fit the scalar block up to kScalBlocks blocks
  if (mode == 0 && !blk) {
    if (nb > kScalBlocks) return hipErrorInvalidValue;
    blk = scal + SC_BLK;
  }
  hipLaunchKernelGGL(k_gather_finish, dim3(nb), dim3(kNT), 0, st, part, r_dev, r_host, m, mode, y, b,
                     g, out2, blk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || mode != 0) return e;
  hipLaunchKernelGGL((k_final<3>), dim3(1), dim3(kNT), 0, st, blk, nb, scal + SC_GG,
                     (const double*)nullptr, 0, (double*)nullptr, (const double*)scal, pub);
  return hipGetLastError();
}

// ------------------------------------------------------------------ line search
// Delta(s) = psi(y + s d) - psi(y) = s g^T d + s^2/2 |d|^2 + sum_i e_i(s), with
// e_i(s) = den/(2 sigma) (prox(t_i - s sigma wd_i)^2 - prox(t_i)^2) + s wd_i prox(t_i),
// which is s^2 kappa wd_i^2 / 2 while t_i stays on one active side
// (Prop. 2 (1) expanded along the line; eq. line_search).  A feature that is
// inactive for every trial step contributes nothing and is skipped; one that
// stays active on its side for every step contributes s^2 times a common sum.
constexpr int kLsSlots = kMaxTrials + 1;  // 32 trial sums + the common second-order sum
// One feature per thread, grid-stride past kLsMaxBlocks blocks: only features
// near the threshold run the trial loop, so spreading them over many waves
// keeps that loop off a few SIMDs, while the cap bounds the 33-slot partial
// rows the selection kernel sums (256 measured faster than 1024 at n = 1e5).
constexpr int kLsMaxBlocks = 256;
int ls_blocks(int64_t n) {
  const int64_t nb = (n + kNT - 1) / kNT;
  return (int)(nb < kLsMaxBlocks ? nb : kLsMaxBlocks);
}
size_t ls_part_doubles(int64_t n) { return (size_t)ls_blocks(n) * kLsSlots; }

__global__ __launch_bounds__(kNT) void k_linesearch(const double* __restrict__ x,
                                                     const double* __restrict__ w,
                                                     const double* __restrict__ wd, int64_t n,
                                                     LsArgs la,
                                                     double* __restrict__ part) {
  const double sigma = la.sigma, thr = la.thr, den = la.den, kappa = la.kappa;
  const int K = la.K;
  double e[kMaxTrials];
#pragma unroll
  for (int k = 0; k < kMaxTrials; ++k) e[k] = 0.0;
  double e2 = 0.0;
  const double smax = la.s[0];
  const double rden = 1.0 / den, h = den / (2.0 * sigma);
  for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
    const double t0 = fma(-sigma, w[i], x[i]);
    const double wi = wd[i];
    const double a0 = fabs(t0);
    const double reach = smax * sigma * fabs(wi) * (1.0 + 1e-12);
    if (a0 + reach < thr) continue;  // inactive for every trial step
    if (((t0 > thr) & (t0 - reach > thr)) | ((t0 < -thr) & (t0 + reach < -thr))) {
      e2 += 0.5 * kappa * wi * wi;  // same active side for every trial step
      continue;
    }
    const double u0 = prox_en(t0, thr, den);
    const double hk = 0.5 * kappa * wi * wi;
#pragma unroll
    for (int k = 0; k < kMaxTrials; ++k) {
      const double s = la.s[k];
      const double t1 = fma(-(s * sigma), wi, t0);
      const bool same = ((t0 > thr) & (t1 > thr)) | ((t0 < -thr) & (t1 < -thr));
      const double num = t1 > thr ? t1 - thr : (t1 < -thr ? t1 + thr : 0.0);
      const double u1 = num * rden;
      const double other = h * (u1 * u1 - u0 * u0) + s * wi * u0;
      e[k] += (k < K) ? (same ? s * s * hk : other) : 0.0;
    }
  }
  // block reduction of the 33 sums
  __shared__ double wsum[kNT / kWave][kLsSlots];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kMaxTrials; ++k) {
    const double v = wave_sum(e[k]);
    if (lane == 0) wsum[wid][k] = v;
  }
  {
    const double v = wave_sum(e2);
    if (lane == 0) wsum[wid][kMaxTrials] = v;
  }
  __syncthreads();
  if (threadIdx.x < kLsSlots) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kNT / kWave; ++q) t += wsum[q][threadIdx.x];
    part[(int64_t)blockIdx.x * kLsSlots + threadIdx.x] = t;
  }
}

// Trial selection (one block of 576 threads): the 33 sums over the partial
// rows (16 lanes per sum, rows b = j mod 16, loads issued 16 at a time, then
// a 16-lane DPP sum, all in a fixed order), Delta_k, the first k with
// Delta_k <= mu s_k g^T d, y += s d.  With select == 0 only the increments
// are produced (for the caller's g^T d and |d|^2).
constexpr int kSelNT = kLsSlots * 16 + (kWave - (kLsSlots * 16) % kWave) % kWave;  // 576

__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<kQuadXor1>(v);
  v += dpp_d<kQuadXor2>(v);
  v += dpp_d<kRowHalfMirror>(v);
  v += dpp_d<kRowMirror>(v);
  return v;
}

__global__ __launch_bounds__(kSelNT) void k_ls_select(const double* __restrict__ part, int nb,
                                                      LsArgs la, const double* __restrict__ g,
                                                      const double* __restrict__ d,
                                                      double* __restrict__ y, int m,
                                                      double* __restrict__ scal, int select,
                                                      double gd_in, double dd_in) {
  __shared__ double tot[kLsSlots];
  __shared__ double red[2][kSelNT / kWave];
  __shared__ double sh_s;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wid = tid / kWave;
  {
    // sum k = tid/16 over rows b = j, j+16, ... (j = tid%16); threads past
    // the 33 sums run the same code on component 0 and discard it
    const int k = tid / 16 < kLsSlots ? tid / 16 : 0;
    const int j = tid & 15;
    double acc = 0.0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int b = b0 + j + 16 * u;
        v[u] = part[(int64_t)(b < nb ? b : 0) * kLsSlots + k];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += (b0 + j + 16 * u < nb) ? v[u] : 0.0;
    }
    acc = row16_sum(acc);
    if (j == 0 && tid / 16 < kLsSlots) tot[tid / 16] = acc;
  }
  double gd = gd_in, dd = dd_in;
  if (select) {
    double pgd = 0.0, pdd = 0.0;
    for (int i = tid; i < m; i += kSelNT) {
      const double gi = g[i], di = d[i];
      pgd = fma(gi, di, pgd);
      pdd = fma(di, di, pdd);
    }
    pgd = wave_sum(pgd);
    pdd = wave_sum(pdd);
    if (lane == 0) {
      red[0][wid] = pgd;
      red[1][wid] = pdd;
    }
  }
  __syncthreads();
  if (select) {
    gd = 0.0;
    dd = 0.0;
#pragma unroll
    for (int q = 0; q < kSelNT / kWave; ++q) {
      gd += red[0][q];
      dd += red[1][q];
    }
  }
  if (wid == 0) {
    // lane k evaluates trial k; the first passing trial wins
    const double s = lane < la.K ? la.s[lane < kMaxTrials ? lane : 0] : 0.0;
    const double second = tot[kMaxTrials];
    const double delta = s * gd + 0.5 * s * s * dd + s * s * second + tot[lane < kMaxTrials ? lane : 0];
    if (lane < la.K) scal[SC_DELTA + lane] = delta;
    const bool pass = (lane < la.K) & (delta <= la.mu * s * gd);
    const unsigned long long mask = __ballot(pass);
    const int acc_k = mask ? __ffsll((long long)mask) - 1 : -1;
    if (lane == 0) {
      const double acc_s = acc_k >= 0 ? la.s[acc_k] : 0.0;
      scal[SC_GD] = gd;
      scal[SC_DD] = dd;
      if (select) {
        scal[SC_S] = acc_s;
        scal[SC_LSK] = (double)acc_k;
      }
      sh_s = acc_s;
    }
  }
  __syncthreads();
  if (select) {
    const double s = sh_s;
    if (s > 0.0)
      for (int i = tid; i < m; i += kSelNT) y[i] = fma(s, d[i], y[i]);
  }
}

hipError_t linesearch(const double* x, const double* w, const double* wd, int64_t n, LsArgs la,
                      const double* g, const double* d, double* y, int m, double* part,
                      double* scal, hipStream_t st) {
  const int nb = ls_blocks(n);
  hipLaunchKernelGGL(k_linesearch, dim3(nb), dim3(kNT), 0, st, x, w, wd, n, la, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ls_select, dim3(1), dim3(kSelNT), 0, st, part, nb, la, g, d, y, m, scal, 1,
                     0.0, 0.0);
  return hipGetLastError();
}

hipError_t ls_delta(const double* x, const double* w, const double* wd, int64_t n, LsArgs la,
                    double gd, double dd, double* part, double* scal, hipStream_t st) {
  const int nb = ls_blocks(n);
  hipLaunchKernelGGL(k_linesearch, dim3(nb), dim3(kNT), 0, st, x, w, wd, n, la, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ls_select, dim3(1), dim3(kSelNT), 0, st, part, nb, la, (const double*)nullptr,
                     (const double*)nullptr, (double*)nullptr, 0, scal, 0, gd, dd);
  return hipGetLastError();
}

// ------------------------------------------------------------------ multiplier update
// x <- x - sigma (A^T y + z) = prox_{sigma p}(x - sigma A^T y) by the Moreau
// decomposition; z = prox_{p^*/sigma}(x/sigma - A^T y) (Prop. 2 (2)) only
// enters the kkt3 denominator.
__global__ __launch_bounds__(kNT) void k_outer(double* __restrict__ x, const double* __restrict__ w,
                                                int64_t n, double sigma, double thr, double den,
                                                double l1, double l2,
                                                double* __restrict__ part) {
  double xu = 0.0, zz = 0.0;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double xv[kEPT], wv[kEPT];
#pragma unroll
  for (int q = 0; q < kEPT; ++q) {
    const int64_t ic = clampi(base + q * kNT + threadIdx.x, n);
    xv[q] = x[ic];
    wv[q] = w[ic];
  }
#pragma unroll
  for (int q = 0; q < kEPT; ++q) {
    const int64_t i = base + q * kNT + threadIdx.x;
    const double xi = xv[q];
    const double t = fma(-sigma, wv[q], xi);
    const double u = prox_en(t, thr, den);
    const double z = t >= thr ? (t * l2 + l1) / den : (t <= -thr ? (t * l2 - l1) / den : t / sigma);
    const double e = xi - u;
    const bool in = i < n;
    xu += in ? e * e : 0.0;
    zz += in ? z * z : 0.0;
    if (in) x[i] = u;
  }
  __shared__ double red[kNT / kWave];
  const double s1 = block_sum<kNT>(xu, red);
  const double s2 = block_sum<kNT>(zz, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

hipError_t outer_update(double* x, const double* w, int64_t n, ProxArgs pa, double l1, double l2,
                        const double* y, int m, double* part, double* scal, hipStream_t st,
                        Pub pub) {
  const int nb = prox_blocks(n);
  hipLaunchKernelGGL(k_outer, dim3(nb), dim3(kNT), 0, st, x, w, n, pa.sigma, pa.thr, pa.den, l1, l2,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_final<2>), dim3(1), dim3(kNT), 0, st, part, nb, scal + SC_XU, y, m,
                     scal + SC_YY, (const double*)scal, pub);
  return hipGetLastError();
}

// ------------------------------------------------------------------ eta pass
// q = A^T rho with rho = A x - b.  Sums for the relative KKT residual
// eta = |x - prox_p(x - q)| / (1 + |x| + |rho|), prox_p(v) = soft(v,l1)/(1+l2),
// and for the objectives F(x) and D(rho) (p^* of Prop. 1 at -q).
__global__ __launch_bounds__(kNT) void k_eta(const double* __restrict__ x,
                                              const double* __restrict__ q, int64_t n, double l1,
                                              double den1, double* __restrict__ part) {
  double se = 0.0, sxx = 0.0, sx1 = 0.0, sps = 0.0;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double xv[kEPT], qv[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const int64_t ic = clampi(base + k * kNT + threadIdx.x, n);
    xv[k] = x[ic];
    qv[k] = q[ic];
  }
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const bool in = base + k * kNT + threadIdx.x < n;
    const double xi = in ? xv[k] : 0.0, qi = in ? qv[k] : 0.0;
    const double p = prox_en(xi - qi, l1, den1);
    const double e = xi - p;
    se += e * e;
    sxx += xi * xi;
    sx1 += fabs(xi);
    const double a = fabs(qi) - l1;
    sps += a > 0.0 ? a * a : 0.0;
  }
  __shared__ double red[kNT / kWave];
  const double r0 = block_sum<kNT>(se, red);
  const double r1 = block_sum<kNT>(sxx, red);
  const double r2 = block_sum<kNT>(sx1, red);
  const double r3 = block_sum<kNT>(sps, red);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = r0;
    part[4 * blockIdx.x + 1] = r1;
    part[4 * blockIdx.x + 2] = r2;
    part[4 * blockIdx.x + 3] = r3;
  }
}

// Copy n scalars to coherent pinned host memory, then raise the host-visible
// sequence flag: the stores, a system-scope fence, then the flag with release
// semantics, so a host that observes the flag reads the new scalars.
__global__ __launch_bounds__(256) void k_publish(const double* __restrict__ s, int n,
                                                 double* __restrict__ dst,
                                                 unsigned long long* __restrict__ flag,
                                                 unsigned long long seq) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = s[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t publish_scalars(const double* scal, int n, double* host_dst, unsigned long long* host_flag,
                           unsigned long long seq, hipStream_t st) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, st, scal, n, host_dst, host_flag, seq);
  return hipGetLastError();
}

hipError_t sum_parts(const double* part, int nb, double* out, const double* y, int m,
                     double* yy_out, hipStream_t st) {
  hipLaunchKernelGGL((k_final<1>), dim3(1), dim3(kNT), 0, st, part, nb, out, y, m, yy_out,
                     (const double*)nullptr, Pub{});
  return hipGetLastError();
}

hipError_t eta_pass(const double* x, const double* q, int64_t n, double l1, double l2, double* part,
                    double* scal, hipStream_t st) {
  const int nb = prox_blocks(n);
  const double den1 = 1.0 + l2;
  hipLaunchKernelGGL(k_eta, dim3(nb), dim3(kNT), 0, st, x, q, n, l1, den1, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_final<4>), dim3(1), dim3(kNT), 0, st, part, nb, scal + SC_ETA_E,
                     (const double*)nullptr, 0, (double*)nullptr, (const double*)nullptr, Pub{});
  return hipGetLastError();
}

// ------------------------------------------------------------------ max |v_i|
// (lambda_max of a path: ||A^T b||_inf).  Per-block maxima, then one block.
// NaN entries are ignored by fmax; callers check finiteness separately.
constexpr int kMaxBlocks = 1024;

__global__ __launch_bounds__(kNT) void k_absmax(const double* __restrict__ v, int64_t n,
                                                 double* __restrict__ part) {
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT)
    mx = fmax(mx, fabs(v[i]));
  __shared__ double red[kNT / kWave];
  mx = wave_max(mx);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
#pragma unroll
    for (int q = 1; q < kNT / kWave; ++q) t = fmax(t, red[q]);
    part[blockIdx.x] = t;
  }
}
__global__ __launch_bounds__(kNT) void k_absmax_final(const double* __restrict__ part, int nb,
                                                       double* __restrict__ out) {
  double mx = 0.0;
  for (int b = threadIdx.x; b < nb; b += kNT) mx = fmax(mx, part[b]);
  __shared__ double red[kNT / kWave];
  mx = wave_max(mx);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
#pragma unroll
    for (int q = 1; q < kNT / kWave; ++q) t = fmax(t, red[q]);
    *out = t;
  }
}

hipError_t absmax(const double* v, int64_t n, double* part, double* out, hipStream_t st) {
  int64_t nb = (n + kNT - 1) / kNT;
  if (nb > kMaxBlocks) nb = kMaxBlocks;
  hipLaunchKernelGGL(k_absmax, dim3((unsigned)nb), dim3(kNT), 0, st, v, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(kNT), 0, st, part, (int)nb, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ helpers
__global__ void k_scale_copy(const double* __restrict__ src, double alpha, double* __restrict__ dst,
                             int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = alpha * src[i];
}
__global__ void k_fill(double* __restrict__ dst, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

static unsigned grid_for(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  return (unsigned)nb;
}

hipError_t vec_scale_copy(const double* src, double alpha, double* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, st, src, alpha, dst, n);
  return hipGetLastError();
}
__global__ __launch_bounds__(kNT) void k_scatter(const int32_t* __restrict__ J,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ r_dev,
                                                  double* __restrict__ out) {
  const int64_t r = (int64_t)*r_dev;
  for (int64_t k = (int64_t)blockIdx.x * kNT + threadIdx.x; k < r; k += (int64_t)gridDim.x * kNT)
    out[J[k]] = v[k];
}

hipError_t scatter(const int32_t* J, const double* v, const double* r_dev, int64_t r_bound,
                   double* out, hipStream_t st) {
  int64_t nb = (r_bound + kNT - 1) / kNT;
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)nb), dim3(kNT), 0, st, J, v, r_dev, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ k-fold
// Fold row lists by one workgroup of 1024 threads: thread t owns the
// contiguous rows [t*c, t*c + c), c = ceil(m / 1024), so a block scan of the
// per-thread counts orders the compacted rows (any m).
constexpr int kFoldNT = 1024;
__global__ __launch_bounds__(kFoldNT) void k_fold_rows(const int32_t* __restrict__ fold, int m, int k,
                                                       int f, int32_t* __restrict__ rows,
                                                       double* __restrict__ scal) {
  __shared__ int cnt[kFoldNT];
  __shared__ double red[kFoldNT / kWave];
  const int t = threadIdx.x;
  const int c = (m + kFoldNT - 1) / kFoldNT;
  const int r0 = t * c, r1 = min(r0 + c, m);
  int mine = 0, bad = 0, val = 0;
  for (int i = r0; i < r1; ++i) {
    const int fi = fold[i];
    bad += (fi < 0) | (fi >= k);
    val += fi == f;
    mine += fi != f;
  }
  cnt[t] = mine;
  __syncthreads();
  // exclusive scan of cnt (Hillis-Steele over 1024 entries)
  for (int d = 1; d < kFoldNT; d *= 2) {
    const int v = t >= d ? cnt[t - d] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  int pos = cnt[t] - mine;
  for (int i = r0; i < r1; ++i)
    if (fold[i] != f) rows[pos++] = i;
  const double nbad = block_sum<kFoldNT>((double)bad, red);
  const double nval = block_sum<kFoldNT>((double)val, red);
  if (t == 0) {
    scal[SC_CV_MT] = (double)cnt[kFoldNT - 1];
    scal[SC_CV_MV] = nval;
    scal[SC_CV_BAD] = nbad;
  }
}

hipError_t fold_rows(const int32_t* fold, int m, int k, int f, int32_t* rows, double* scal,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_fold_rows, dim3(1), dim3(kFoldNT), 0, st, fold, m, k, f, rows, scal);
  return hipGetLastError();
}

// A_t[:, j] = A[rows, j] (mt rows, leading dimension mt) and b_t = b[rows].
template <typename T>
__global__ __launch_bounds__(kNT) void k_gather_rows(const T* __restrict__ A, int64_t lda,
                                                     int64_t n, const int32_t* __restrict__ rows,
                                                     int mt, const double* __restrict__ b,
                                                     T* __restrict__ At, double* __restrict__ bt) {
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    const T* a = A + j * lda;
    T* o = At + j * mt;
    for (int i = threadIdx.x; i < mt; i += kNT) o[i] = a[rows[i]];
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < mt; i += kNT) bt[i] = b[rows[i]];
}

hipError_t gather_rows(const void* A, int dtype, int64_t lda, int64_t n, const int32_t* rows, int mt,
                       const double* b, void* At, double* bt, hipStream_t st) {
  const unsigned nb = (unsigned)std::min<int64_t>(n, 8192);
  if (dtype == kF64)
    hipLaunchKernelGGL(k_gather_rows<double>, dim3(nb), dim3(kNT), 0, st, (const double*)A, lda, n,
                       rows, mt, b, (double*)At, bt);
  else if (dtype == kF32)
    hipLaunchKernelGGL(k_gather_rows<float>, dim3(nb), dim3(kNT), 0, st, (const float*)A, lda, n,
                       rows, mt, b, (float*)At, bt);
  else
    hipLaunchKernelGGL(k_gather_rows<uint16_t>, dim3(nb), dim3(kNT), 0, st, (const uint16_t*)A, lda,
                       n, rows, mt, b, (uint16_t*)At, bt);
  return hipGetLastError();
}

// *out = sum over the rows of fold f of res_i^2 (one workgroup, fixed order).
__global__ __launch_bounds__(kFoldNT) void k_fold_sq(const double* __restrict__ res,
                                                     const int32_t* __restrict__ fold, int m, int f,
                                                     double* __restrict__ out) {
  __shared__ double red[kFoldNT / kWave];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += kFoldNT) s += fold[i] == f ? res[i] * res[i] : 0.0;
  s = block_sum<kFoldNT>(s, red);
  if (threadIdx.x == 0) *out = s;
}

hipError_t fold_sq(const double* res, const int32_t* fold, int m, int f, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_fold_sq, dim3(1), dim3(kFoldNT), 0, st, res, fold, m, f, out);
  return hipGetLastError();
}

hipError_t vec_fill(double* dst, double v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, st, dst, v, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(kNT) void k_nonfinite(const double* __restrict__ v, int64_t n,
                                                    double* __restrict__ part) {
  int c = 0;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double vv[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) vv[k] = v[clampi(base + k * kNT + threadIdx.x, n)];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) c += (base + k * kNT + threadIdx.x < n) ? (int)!isfinite(vv[k]) : 0;
  __shared__ int red[kNT / kWave];
  const int t = block_sum<kNT>(c, red);
  if (threadIdx.x == 0) part[blockIdx.x] = (double)t;
}

hipError_t nonfinite_count(const double* v, int64_t n, double* scal_slot, double* part,
                           hipStream_t st) {
  const int nb = prox_blocks(n);
  hipLaunchKernelGGL(k_nonfinite, dim3(nb), dim3(kNT), 0, st, v, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_final<1>), dim3(1), dim3(kNT), 0, st, part, nb, scal_slot,
                     (const double*)nullptr, 0, (double*)nullptr, (const double*)nullptr, Pub{});
  return hipGetLastError();
}

}  // namespace ssnal
