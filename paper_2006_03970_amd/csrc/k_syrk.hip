// Newton matrix of the semi-smooth Newton step (eq. AJ_system / eq. smw_formula):
//   form 0:  V = shift*I_m + scale * A_J A_J^T   (m x m, contraction over the r active columns)
//   form 1:  W = shift*I_r + scale * A_J^T A_J   (r x r, contraction over the m rows)
// Both are C = Z Z^T for a gathered operand Z (N x K), computed on the matrix
// cores: 64 x 64 output tiles of the upper triangle, four waves per tile each
// owning a 32 x 32 quarter as 2 x 2 blocks of 16 x 16 MFMA accumulators, the K
// range split across workgroups (split-K) so that even a handful of tiles
// fills the chip.  Partial tiles are stored in FP64 and summed in split order
// by a second kernel, which also applies scale/shift and mirrors the result,
// so V is exactly symmetric and reproducible.
//
// FP64 storage runs v_mfma_f64_16x16x4 (FP64 accumulation), FP32 storage
// v_mfma_f32_16x16x4 and BF16 storage v_mfma_f32_16x16x32_bf16, both with FP32
// accumulation inside a split (BF16 values and their products are exact in
// FP32).
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace ssnal {

constexpr int kTile = 64;
constexpr int kKS = 32;          // K elements staged per step
constexpr int kPitch = kTile + 1;  // LDS row pitch (odd, to spread banks)

template <typename T> struct MfmaOf { using C = float; };
template <> struct MfmaOf<double> { using C = double; };

__device__ __forceinline__ dbl4 mfma_step(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma_step(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename C> constexpr bool kIs64 = false;
template <> constexpr bool kIs64<double> = true;

template <typename C> struct Acc4;
template <> struct Acc4<double> { using type = dbl4; };
template <> struct Acc4<float> { using type = flt4; };

__device__ __forceinline__ void tile_of(int t, int& ti, int& tj) {
  // upper-triangle tiles enumerated column by column: t = tj(tj+1)/2 + ti, ti <= tj
  int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  while (j * (j + 1) / 2 > t) --j;
  tj = j;
  ti = t - j * (j + 1) / 2;
}

// Z element loaders.  form 0: Z[a][k] = A[a, J[k]] (a < m, k < r).
//                     form 1: Z[a][k] = A[k, J[a]] (a < r, k < m).
// A stage is 64 rows x kKS k-values = 2048 elements, 8 per thread, fetched
// into registers (the next stage's loads are in flight while the matrix
// cores work on the current one) and then stored to LDS.
template <typename T, typename C, int FORM>
__device__ __forceinline__ void fetch(const T* __restrict__ A, int64_t lda, int N, int64_t K,
                                      const int32_t* __restrict__ J, int row0, int64_t k0,
                                      C (&v)[8]) {
  const int t = threadIdx.x;
  if (FORM == 0) {
    const int kk = t / 8;           // 32 columns
    const int a0 = (t % 8) * 8;     // 8 consecutive rows
    const int64_t k = k0 + kk;
    const bool kok = k < K;
    const T* col = A + (int64_t)J[kok ? k : K - 1] * lda;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int a = row0 + a0 + q;
      const C x = load1<C>(col + (a < N ? a : N - 1));
      v[q] = (kok & (a < N)) ? x : (C)0;
    }
  } else {
    const int aa = t / 4;           // 64 gathered columns
    const int kq = (t % 4) * 8;     // 8 consecutive rows of that column
    const int a = row0 + aa;
    const bool aok = a < N;
    const T* col = A + (int64_t)J[aok ? a : N - 1] * lda;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t k = k0 + kq + q;
      const C x = load1<C>(col + (k < K ? k : K - 1));
      v[q] = (aok & (k < K)) ? x : (C)0;
    }
  }
}

template <typename C, int FORM>
__device__ __forceinline__ void store_stage(const C (&v)[8], C (*dst)[kPitch]) {
  const int t = threadIdx.x;
  if (FORM == 0) {
    const int kk = t / 8, a0 = (t % 8) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[kk][a0 + q] = v[q];
  } else {
    const int aa = t / 4, kq = (t % 4) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[kq + q][aa] = v[q];
  }
}

template <typename T, int FORM>
__global__ __launch_bounds__(256) void k_syrk_partial(const T* __restrict__ A, int64_t lda, int N,
                                                      int64_t K, const int32_t* __restrict__ J,
                                                      int ntiles, int64_t kchunk,
                                                      double* __restrict__ part) {
  using C = typename MfmaOf<T>::C;
  using V4 = typename Acc4<C>::type;
  __shared__ C zi[kKS][kPitch];
  __shared__ C zj[kKS][kPitch];
  const int tile = blockIdx.x % ntiles;
  const int split = blockIdx.x / ntiles;
  int ti, tj;
  tile_of(tile, ti, tj);
  const bool diag = (ti == tj);
  const int64_t kb = (int64_t)split * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;

  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int wi = wid >> 1, wj = wid & 1;
  V4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = V4{0, 0, 0, 0};

  C ri[8], rj[8];
  fetch<T, C, FORM>(A, lda, N, ke, J, ti * kTile, kb, ri);
  if (!diag) fetch<T, C, FORM>(A, lda, N, ke, J, tj * kTile, kb, rj);
  for (int64_t k0 = kb; k0 < ke; k0 += kKS) {
    __syncthreads();
    store_stage<C, FORM>(ri, zi);
    if (!diag) store_stage<C, FORM>(rj, zj);
    __syncthreads();
    if (k0 + kKS < ke) {
      fetch<T, C, FORM>(A, lda, N, ke, J, ti * kTile, k0 + kKS, ri);
      if (!diag) fetch<T, C, FORM>(A, lda, N, ke, J, tj * kTile, k0 + kKS, rj);
    }
    C (*zb)[kPitch] = diag ? zi : zj;
#pragma unroll
    for (int ks = 0; ks < kKS; ks += 4) {
      const int kr = ks + lane / 16;
      C a[2], b[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) a[p] = zi[kr][wi * 32 + p * 16 + (lane & 15)];
#pragma unroll
      for (int q = 0; q < 2; ++q) b[q] = zb[kr][wj * 32 + q * 16 + (lane & 15)];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = mfma_step(a[p], b[q], acc[p][q]);
    }
  }
  // accumulator v of a 16 x 16 block holds row 4*(lane/16)+v (FP32 MFMA) or
  // row lane/16 + 4*v (FP64 MFMA), column lane%16
  double* out = part + ((int64_t)split * ntiles + tile) * (kTile * kTile);
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = kIs64<C> ? (lane / 16) + 4 * v : 4 * (lane / 16) + v;
        const int r = wi * 32 + p * 16 + rr;
        const int c = wj * 32 + q * 16 + (lane & 15);
        out[r * kTile + c] = (double)acc[p][q][v];
      }
}

// BF16 storage on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation): the products of two BF16 values are exact in FP32, as in the
// FP32 path, but one instruction covers 32 k-values.  A stage holds 64 rows x
// kKS k-values of each operand in LDS as BF16 with the k-values of a row
// contiguous (zs[row][k]); a lane's MFMA operand is 8 consecutive k-values of
// one row, one 16-byte LDS read.  Thread t fetches row t/4, k-values
// 8 (t % 4) .. + 7: form 1 reads them from one column of A (16 bytes when
// the column starts allow it), form 0 from eight gathered columns (row a of
// each, adjacent lanes reading adjacent rows).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kBPitch = kKS + 8;  // BF16 elements per LDS row (80 bytes: 16-byte aligned, banks spread)

template <int FORM>
__device__ __forceinline__ void fetch_bf16(const uint16_t* __restrict__ A, int64_t lda, int N, int64_t K,
                                           const int32_t* __restrict__ J, int row0, int64_t k0, bool v16,
                                           uint4& out) {
  const int t = threadIdx.x;
  const int a = row0 + t / 4;
  const int64_t kb = k0 + (t % 4) * 8;
  const bool aok = a < N;
  uint16_t v[8];
  if (FORM == 1) {
    const uint16_t* col = A + (int64_t)J[aok ? a : N - 1] * lda;
    if (v16 && kb + 8 <= K) {
      const uint4 x = *reinterpret_cast<const uint4*>(col + kb);
      out = aok ? x : uint4{0, 0, 0, 0};
      return;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t k = kb + q;
      const uint16_t x = col[k < K ? k : K - 1];
      v[q] = (aok & (k < K)) ? x : (uint16_t)0;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t k = kb + q;
      const bool kok = k < K;
      const uint16_t x = A[(int64_t)J[kok ? k : K - 1] * lda + (aok ? a : N - 1)];
      v[q] = (aok & kok) ? x : (uint16_t)0;
    }
  }
  out.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
  out.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
  out.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
  out.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
}

template <int FORM>
__global__ __launch_bounds__(256) void k_syrk_partial_bf16(const uint16_t* __restrict__ A, int64_t lda,
                                                           int N, int64_t K, const int32_t* __restrict__ J,
                                                           int ntiles, int64_t kchunk, bool v16,
                                                           double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint16_t zi[kTile][kBPitch];
  __shared__ __attribute__((aligned(16))) uint16_t zj[kTile][kBPitch];
  const int tile = blockIdx.x % ntiles;
  const int split = blockIdx.x / ntiles;
  int ti, tj;
  tile_of(tile, ti, tj);
  const bool diag = (ti == tj);
  const int64_t kb = (int64_t)split * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;

  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int wi = wid >> 1, wj = wid & 1;
  flt4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = flt4{0, 0, 0, 0};

  const int t = threadIdx.x;
  uint4 ri, rj;
  fetch_bf16<FORM>(A, lda, N, ke, J, ti * kTile, kb, v16, ri);
  if (!diag) fetch_bf16<FORM>(A, lda, N, ke, J, tj * kTile, kb, v16, rj);
  for (int64_t k0 = kb; k0 < ke; k0 += kKS) {
    __syncthreads();
    *reinterpret_cast<uint4*>(&zi[t / 4][(t % 4) * 8]) = ri;
    if (!diag) *reinterpret_cast<uint4*>(&zj[t / 4][(t % 4) * 8]) = rj;
    __syncthreads();
    if (k0 + kKS < ke) {
      fetch_bf16<FORM>(A, lda, N, ke, J, ti * kTile, k0 + kKS, v16, ri);
      if (!diag) fetch_bf16<FORM>(A, lda, N, ke, J, tj * kTile, k0 + kKS, v16, rj);
    }
    uint16_t(*zb)[kBPitch] = diag ? zi : zj;
    const int kq = 8 * (lane / 16);
    bf16x8 a[2], b[2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
      a[p] = *reinterpret_cast<const bf16x8*>(&zi[wi * 32 + p * 16 + (lane & 15)][kq]);
#pragma unroll
    for (int q = 0; q < 2; ++q)
      b[q] = *reinterpret_cast<const bf16x8*>(&zb[wj * 32 + q * 16 + (lane & 15)][kq]);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[p], b[q], acc[p][q], 0, 0, 0);
  }
  // accumulator v of a 16 x 16 block holds row 4*(lane/16)+v, column lane%16
  double* out = part + ((int64_t)split * ntiles + tile) * (kTile * kTile);
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wi * 32 + p * 16 + 4 * (lane / 16) + v;
        const int c = wj * 32 + q * 16 + (lane & 15);
        out[r * kTile + c] = (double)acc[p][q][v];
      }
}

// One thread per tile element (16 workgroups per tile); the split partials
// are summed in split order, eight loads in flight.
__global__ __launch_bounds__(256) void k_syrk_finish(const double* __restrict__ part, int N,
                                                     int ntiles, int nsplit, double shift,
                                                     double scale, double* __restrict__ out) {
  const int tile = blockIdx.x / 16;
  const int e = (blockIdx.x % 16) * 256 + threadIdx.x;
  int ti, tj;
  tile_of(tile, ti, tj);
  const int li = e / kTile, lj = e % kTile;
  const int i = ti * kTile + li, j = tj * kTile + lj;
  if (i >= N || j >= N) return;
  if (ti == tj && li > lj) return;  // diagonal tile: upper half, mirrored below
  const double* src = part + (int64_t)tile * (kTile * kTile) + e;
  const int64_t stride = (int64_t)ntiles * (kTile * kTile);
  double s = 0.0;
  int sp = 0;
  for (; sp + 8 <= nsplit; sp += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[(sp + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; sp < nsplit; ++sp) s += src[sp * stride];
  double v = scale * s;
  if (i == j) v += shift;
  out[(int64_t)i * N + j] = v;
  out[(int64_t)j * N + i] = v;
}

namespace {
struct SyrkPlan {
  int N, T, ntiles, nsplit;
  int64_t K, kchunk;
};
SyrkPlan plan(int form, int m, int64_t r) {
  SyrkPlan p;
  p.N = form == 0 ? m : (int)r;
  p.K = form == 0 ? r : m;
  p.T = (p.N + kTile - 1) / kTile;
  p.ntiles = p.T * (p.T + 1) / 2;
  int64_t want = (1024 + p.ntiles - 1) / p.ntiles;
  int64_t maxs = (p.K + 63) / 64;
  if (maxs < 1) maxs = 1;
  int64_t s = want < maxs ? want : maxs;
  if (s < 1) s = 1;
  int64_t kc = (p.K + s - 1) / s;
  kc = (kc + kKS - 1) / kKS * kKS;
  if (kc < kKS) kc = kKS;
  p.kchunk = kc;
  p.nsplit = (int)((p.K + kc - 1) / kc);
  if (p.nsplit < 1) p.nsplit = 1;
  return p;
}
}  // namespace

size_t syrk_workspace_bytes(int form, int m, int64_t r) {
  SyrkPlan p = plan(form, m, r);
  return (size_t)p.nsplit * p.ntiles * kTile * kTile * sizeof(double);
}

template <typename T>
static hipError_t launch_syrk(const T* A, int64_t lda, int m, const int32_t* J, int64_t r, int form,
                              double shift, double scale, double* out, double* work, hipStream_t st) {
  SyrkPlan p = plan(form, m, r);
  if (p.N <= 0) return hipSuccess;
  const unsigned nb = (unsigned)(p.ntiles * p.nsplit);
  if (std::is_same<T, uint16_t>::value) {
    // 16-byte fetches of a column need 16-byte aligned column starts
    const bool v16 = ((uintptr_t)A % 16 == 0) && (lda % 8 == 0);
    const uint16_t* Ab = reinterpret_cast<const uint16_t*>(A);
    if (form == 0)
      hipLaunchKernelGGL((k_syrk_partial_bf16<0>), dim3(nb), dim3(256), 0, st, Ab, lda, p.N, p.K, J,
                         p.ntiles, p.kchunk, v16, work);
    else
      hipLaunchKernelGGL((k_syrk_partial_bf16<1>), dim3(nb), dim3(256), 0, st, Ab, lda, p.N, p.K, J,
                         p.ntiles, p.kchunk, v16, work);
  } else if (form == 0)
    hipLaunchKernelGGL((k_syrk_partial<T, 0>), dim3(nb), dim3(256), 0, st, A, lda, p.N, p.K, J,
                       p.ntiles, p.kchunk, work);
  else
    hipLaunchKernelGGL((k_syrk_partial<T, 1>), dim3(nb), dim3(256), 0, st, A, lda, p.N, p.K, J,
                       p.ntiles, p.kchunk, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_syrk_finish, dim3(p.ntiles * 16), dim3(256), 0, st, work, p.N, p.ntiles,
                     p.nsplit, shift, scale, out);
  return hipGetLastError();
}

hipError_t syrk(const void* A, int dtype, int64_t lda, int m, const int32_t* J, int64_t r, int form,
                double shift, double scale, double* out, void* work, hipStream_t st) {
  switch (dtype) {
    case kF64:
      return launch_syrk<double>((const double*)A, lda, m, J, r, form, shift, scale, out, (double*)work, st);
    case kF32:
      return launch_syrk<float>((const float*)A, lda, m, J, r, form, shift, scale, out, (double*)work, st);
    case kBF16:
      return launch_syrk<uint16_t>((const uint16_t*)A, lda, m, J, r, form, shift, scale, out, (double*)work,
                                   st);
  }
  return hipErrorInvalidValue;
}

}  // namespace ssnal
