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

// ---- 128 x 128 output tiles for the large systems (K of thousands of
// columns and more: the early Newton steps of an m = 1000, n = 10^6 solve
// contract over r = 5 * 10^5 active columns).  Four waves, each a 64 x 64
// quarter as 4 x 4 blocks of 16 x 16 accumulators, so every operand read
// from LDS feeds four MFMAs; a stage is 128 bytes of k per row (16 FP64, 32
// FP32 or 64 BF16 values) for both operand panels, double-buffered in LDS
// (one barrier a stage) with the next stage's 16-byte global loads in flight
// during the current stage's MFMAs (BF16: the next two stages'); registers
// are held to 256 a lane so that two workgroups share a CU (64 KB of LDS
// each).  LDS holds each operand row's k-values
// contiguously in 16-byte chunks, chunk c of row a at a * 128 + 16 (c ^
// ((a >> 1) & 7)) bytes, so the 16 rows of one MFMA operand read hit
// distinct banks.  Lane group g = lane / 16 reads chunk 4q + g of its row:
// for FP32 and FP64 the elements of that chunk feed consecutive MFMA steps
// (step e of read q contracts k = 4q*EPB + g*EPB + e over the four groups),
// for BF16 the chunk is one 16x16x32 operand; both operands use the same
// assignment, so every k of the stage is contracted exactly once.
//   form 1 (k contiguous in A): thread t loads chunks t + 256 q of a panel,
//     row (t + 256 q) / 8, chunk t % 8, straight into LDS;
//   form 0 (rows contiguous in A): a thread loads EPB-row chunks of
//     several gathered columns and transposes them in registers into
//     row chunks (adjacent lanes read adjacent rows of one column).
constexpr int kBT = 128;                 // output tile
constexpr int kRowB = 128;               // bytes of k per operand row and stage
constexpr int kPanelB = kBT * kRowB;     // 16 KB

template <typename T> struct BigT;
template <> struct BigT<double> { using V4 = dbl4; static constexpr int EPB = 2; };
template <> struct BigT<float> { using V4 = flt4; static constexpr int EPB = 4; };
template <> struct BigT<uint16_t> { using V4 = flt4; static constexpr int EPB = 8; };

__device__ __forceinline__ int swz(int row, int chunk) { return row * kRowB + ((chunk ^ ((row >> 1) & 7)) << 4); }

// zero the elements of a 16-byte chunk from element nv on (nv in 0..EPB)
template <typename T>
__device__ __forceinline__ uint4 keep_first(uint4 v, int nv) {
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
  constexpr int EPB = 16 / (int)sizeof(T);
#pragma unroll
  for (int e = 0; e < EPB; ++e) {
    const bool z = e >= nv;
    if (sizeof(T) == 8) {
      w[2 * e] = z ? 0u : w[2 * e];
      w[2 * e + 1] = z ? 0u : w[2 * e + 1];
    } else if (sizeof(T) == 4) {
      w[e] = z ? 0u : w[e];
    } else {
      const uint32_t m = (e & 1) ? 0xffff0000u : 0x0000ffffu;
      w[e >> 1] = z ? (w[e >> 1] & ~m) : w[e >> 1];
    }
  }
  return uint4{w[0], w[1], w[2], w[3]};
}

// The gathered indices a thread's loads of one stage need (4 per panel):
// form 0 the columns J[k] of its k-values, form 1 the columns J[a] of its
// rows (the same in every stage), clamped into the index range.  They are
// loaded one stage ahead of the operand loads that use them: the vector
// memory counter retires in order, so an index load issued after a stage's
// operand loads would make the next stage wait for those as well.
template <typename T, int FORM>
__device__ __forceinline__ void big_jload(const int32_t* __restrict__ J, int N, int64_t K, int row0,
                                          int64_t k0, int (&jv)[4]) {
  constexpr int EPB = BigT<T>::EPB;
  const int t = threadIdx.x;
  if (FORM == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = row0 + (t >> 3) + 32 * q;
      jv[q] = J[a < N ? a : N - 1];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // FP32: column 4 (t / 32) + q; FP64: 2 ((t + 256 h) / 64) + j, q = 2h + j; BF16: 4 (t / 16) + q
      const int64_t k = k0 + (EPB == 4   ? 4 * (t >> 5) + q
                              : EPB == 2 ? 2 * ((t + 256 * (q >> 1)) >> 6) + (q & 1)
                                         : 4 * (t >> 4) + q);
      jv[q] = J[k < K ? k : K - 1];
    }
  }
}

// Global loads of one operand panel's stage (4 x 16 bytes per thread), at
// addresses clamped into the matrix and issued unconditionally (a load under
// a branch makes the compiler wait for it where the branches join, which
// would serialise the prefetch).  Values outside the matrix are zeroed by
// big_mask, only in stages at an edge: the masks cost more vector
// instructions than a BF16 stage has MFMAs.
template <typename T, int FORM>
__device__ __forceinline__ void big_fetch(const T* __restrict__ A, int64_t lda, int N, int64_t K,
                                          const int (&jv)[4], int row0, int64_t k0, uint4 (&v)[4]) {
  constexpr int EPB = BigT<T>::EPB;
  const int t = threadIdx.x;
  if (FORM == 1) {
    // chunk c = t + 256 q: row c / 8, elements k0 + EPB (c % 8) ..
    const int64_t kc = k0 + (int64_t)EPB * (t & 7);
    const int64_t klast = (K - 1) / EPB * EPB;  // last chunk start inside the column
    const int64_t kl = kc < klast ? kc : klast;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const uint4*>(A + (int64_t)jv[q] * lda + kl);
  } else {
    // rows EPB-aligned: FP32 4 (t % 32), FP64 2 ((t + 256 h) % 64), BF16 8 (t % 16)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = row0 + (EPB == 4 ? 4 * (t & 31) : EPB == 2 ? 2 * ((t + 256 * (q >> 1)) & 63) : 8 * (t & 15));
      v[q] = *reinterpret_cast<const uint4*>(A + (int64_t)jv[q] * lda + (a < N ? a : 0));
    }
  }
}

// Zero what big_fetch loaded from outside the matrix (rows >= N, k >= K).
template <typename T, int FORM>
__device__ __forceinline__ void big_mask(int N, int64_t K, int row0, int64_t k0, uint4 (&v)[4]) {
  constexpr int EPB = BigT<T>::EPB;
  const int t = threadIdx.x;
  auto nvalid = [](int64_t left) { return (int)(left < EPB ? (left > 0 ? left : 0) : EPB); };
  if (FORM == 1) {
    const int nv = nvalid(K - (k0 + (int64_t)EPB * (t & 7)));
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = keep_first<T>(v[q], row0 + (t >> 3) + 32 * q < N ? nv : 0);
  } else if (EPB == 4) {
    const int nv = nvalid(N - (row0 + 4 * (t & 31)));
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = keep_first<T>(v[q], k0 + 4 * (t >> 5) + q < K ? nv : 0);
  } else if (EPB == 2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = t + 256 * h;
      const int nv = nvalid(N - (row0 + 2 * (b & 63)));
#pragma unroll
      for (int j = 0; j < 2; ++j) v[2 * h + j] = keep_first<T>(v[2 * h + j], k0 + 2 * (b >> 6) + j < K ? nv : 0);
    }
  } else {
    const int nv = nvalid(N - (row0 + 8 * (t & 15)));
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = keep_first<T>(v[q], k0 + 4 * (t >> 4) + q < K ? nv : 0);
  }
}

// The staged chunks into an LDS panel (layout above).
template <typename T, int FORM>
__device__ __forceinline__ void big_store(const uint4 (&v)[4], unsigned char* __restrict__ P) {
  constexpr int EPB = BigT<T>::EPB;
  const int t = threadIdx.x;
  if (FORM == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<uint4*>(P + swz((t >> 3) + 32 * q, t & 7)) = v[q];
  } else if (EPB == 4) {
    // v[q] = rows a..a+3 of column q; row i gets {v[0].i, v[1].i, v[2].i, v[3].i}
    const int r = 4 * (t & 31), c = t >> 5;
    const uint32_t w[4][4] = {{v[0].x, v[0].y, v[0].z, v[0].w}, {v[1].x, v[1].y, v[1].z, v[1].w},
                              {v[2].x, v[2].y, v[2].z, v[2].w}, {v[3].x, v[3].y, v[3].z, v[3].w}};
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *reinterpret_cast<uint4*>(P + swz(r + i, c)) = uint4{w[0][i], w[1][i], w[2][i], w[3][i]};
  } else if (EPB == 2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = t + 256 * h;
      const int r = 2 * (b & 63), c = b >> 6;
      const uint4 x0 = v[2 * h], x1 = v[2 * h + 1];  // columns 2c, 2c+1; rows r, r+1 in .xy / .zw
      *reinterpret_cast<uint4*>(P + swz(r, c)) = uint4{x0.x, x0.y, x1.x, x1.y};
      *reinterpret_cast<uint4*>(P + swz(r + 1, c)) = uint4{x0.z, x0.w, x1.z, x1.w};
    }
  } else {
    // BF16: v[q] = rows r..r+7 of column 4 (t / 16) + q; row i gets 4 values, 8 bytes,
    // half (t / 16) % 2 of chunk (t / 16) / 2
    const int r = 8 * (t & 15), kq = t >> 4;
    const uint32_t w[4][4] = {{v[0].x, v[0].y, v[0].z, v[0].w}, {v[1].x, v[1].y, v[1].z, v[1].w},
                              {v[2].x, v[2].y, v[2].z, v[2].w}, {v[3].x, v[3].y, v[3].z, v[3].w}};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      // byte permute: the low (even i) or high (odd i) halves of two words
      const uint32_t sel = (i & 1) ? 0x07060302u : 0x05040100u;
      const uint32_t lo = __builtin_amdgcn_perm(w[1][i >> 1], w[0][i >> 1], sel);
      const uint32_t hi = __builtin_amdgcn_perm(w[3][i >> 1], w[2][i >> 1], sel);
      *reinterpret_cast<uint2*>(P + swz(r + i, kq >> 1) + 8 * (kq & 1)) = uint2{lo, hi};
    }
  }
}

template <typename T>
__device__ __forceinline__ void big_mfma(const uint4* a, const uint4* b, typename BigT<T>::V4 (&acc)[4][4]);

template <>
__device__ __forceinline__ void big_mfma<float>(const uint4* a, const uint4* b, flt4 (&acc)[4][4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float x[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t ua[4] = {a[i].x, a[i].y, a[i].z, a[i].w};
      const uint32_t ub[4] = {b[i].x, b[i].y, b[i].z, b[i].w};
      x[i] = __uint_as_float(ua[e]);
      y[i] = __uint_as_float(ub[e]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[i], y[j], acc[i][j], 0, 0, 0);
  }
}
template <>
__device__ __forceinline__ void big_mfma<double>(const uint4* a, const uint4* b, dbl4 (&acc)[4][4]) {
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    double x[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t la = e ? a[i].z : a[i].x, ha = e ? a[i].w : a[i].y;
      const uint32_t lb = e ? b[i].z : b[i].x, hb = e ? b[i].w : b[i].y;
      x[i] = __hiloint2double((int)ha, (int)la);
      y[i] = __hiloint2double((int)hb, (int)lb);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i], y[j], acc[i][j], 0, 0, 0);
  }
}
template <>
__device__ __forceinline__ void big_mfma<uint16_t>(const uint4* a, const uint4* b, flt4 (&acc)[4][4]) {
  bf16x8 x[4], y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    x[i] = __builtin_bit_cast(bf16x8, a[i]);
    y[i] = __builtin_bit_cast(bf16x8, b[i]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[i], y[j], acc[i][j], 0, 0, 0);
}

// Work items (split, tile) are numbered split-major, o = split * ntiles +
// tile, and spread so that each XCD (workgroup b runs on XCD b % 8) takes a
// contiguous range of them: the tiles of one split, which read the same
// operand panels over the same k range, share that XCD's L2 instead of
// each fetching the panels from HBM (nwork items; the grid is a multiple of
// 8 and the items past nwork return at once).
template <typename T, int FORM>
__global__ __launch_bounds__(256, 2) void k_syrk_big(const T* __restrict__ A, int64_t lda, int N, int64_t K,
                                                  const int32_t* __restrict__ J, int ntiles, int nwork,
                                                  int64_t kchunk, double* __restrict__ part) {
  using V4 = typename BigT<T>::V4;
  constexpr int KS = kRowB / (int)sizeof(T);  // k-values per stage
  __shared__ __attribute__((aligned(16))) unsigned char lds[4 * kPanelB];  // [buffer][operand]
  const int o = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
  if (o >= nwork) return;
  const int tile = o % ntiles;
  const int split = o / ntiles;
  int ti, tj;
  tile_of(tile, ti, tj);
  const bool diag = (ti == tj);
  const int64_t kb = (int64_t)split * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int wi = wid >> 1, wj = wid & 1;
  // a diagonal tile's lower-left quarter is never read: its wave only stages
  const bool work = !(diag && wi > wj);
  V4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = V4{0, 0, 0, 0};

  auto compute = [&](int buf) {
    const unsigned char* Pi = lds + (2 * buf) * kPanelB;
    const unsigned char* Pj = diag ? Pi : Pi + kPanelB;
    if (!work) return;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int ch = 4 * q + (lane >> 4);
      uint4 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *reinterpret_cast<const uint4*>(Pi + swz(wi * 64 + 16 * i + (lane & 15), ch));
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = *reinterpret_cast<const uint4*>(Pj + swz(wj * 64 + 16 * j + (lane & 15), ch));
      big_mfma<T>(a, b, acc);
    }
  };
  const int64_t nst = (ke - kb + KS - 1) / KS;  // stages of this split
  // k of stage st, clamped to the last stage: loads past the end repeat it
  // (unconditional loads, see big_fetch) and are never stored
  auto kst = [&](int64_t st) { return kb + (st < nst ? st : nst - 1) * KS; };
  auto jload2 = [&](int64_t st, int (&ji)[4], int (&jj)[4]) {
    big_jload<T, FORM>(J, N, ke, ti * kBT, kst(st), ji);
    if (!diag) big_jload<T, FORM>(J, N, ke, tj * kBT, kst(st), jj);
  };
  auto fetch2 = [&](int64_t st, const int (&ji)[4], const int (&jj)[4], uint4 (&ri)[4], uint4 (&rj)[4]) {
    big_fetch<T, FORM>(A, lda, N, ke, ji, ti * kBT, kst(st), ri);
    if (!diag) big_fetch<T, FORM>(A, lda, N, ke, jj, tj * kBT, kst(st), rj);
  };
  // stage st into LDS buffer buf, masked where it meets an edge (a uniform branch)
  auto store2 = [&](uint4 (&ri)[4], uint4 (&rj)[4], int buf, int64_t st) {
    const int64_t k0 = kst(st);
    if (k0 + KS > ke || (tj + 1) * kBT > N) {
      big_mask<T, FORM>(N, ke, ti * kBT, k0, ri);
      if (!diag) big_mask<T, FORM>(N, ke, tj * kBT, k0, rj);
    }
    unsigned char* Q = lds + (2 * buf) * kPanelB;
    big_store<T, FORM>(ri, Q);
    if (!diag) big_store<T, FORM>(rj, Q + kPanelB);
  };
  if (sizeof(T) >= 4) {
    // FP64 and FP32: one stage of operand loads in flight, which a stage of
    // 64 FP64 or 128 FP32 MFMAs covers (a second register set measured
    // slower for FP32, 6.2 against 5.8 ms at m = 1000, r = 520000, and would
    // pass 256 registers for FP64); the indices of stage st + 2 are loaded
    // after the operand loads of stage st + 1, which the store of stage
    // st + 1 waits for anyway
    int ji[4], jj[4];
    uint4 ri[4], rj[4];
    jload2(0, ji, jj);
    fetch2(0, ji, jj, ri, rj);
    jload2(1, ji, jj);
    store2(ri, rj, 0, 0);
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
      fetch2(st + 1, ji, jj, ri, rj);
      jload2(st + 2, ji, jj);
      compute((int)(st & 1));
      if (st + 1 < nst) store2(ri, rj, (int)((st + 1) & 1), st + 1);
      __syncthreads();
    }
  } else {
    // BF16: the operand loads of stage s + 2 are issued while stage s is
    // computed and stage s + 1 waits in the other register set, so a stage's
    // loads have two stages' MFMAs to arrive (a BF16 stage is only 32
    // MFMAs).  Index set st % 2 serves stage st; it is loaded before the
    // operand loads of stage st - 1, so those may stay in flight.
    int j0i[4], j0j[4], j1i[4], j1j[4];
    uint4 r0i[4], r0j[4], r1i[4], r1j[4];
    jload2(0, j0i, j0j);
    jload2(1, j1i, j1j);
    fetch2(0, j0i, j0j, r0i, r0j);
    jload2(2, j0i, j0j);
    fetch2(1, j1i, j1j, r1i, r1j);
    jload2(3, j1i, j1j);
    store2(r0i, r0j, 0, 0);
    __syncthreads();
    for (int64_t st = 0; st < nst; st += 2) {
      // stage st (buffer 0); stage st + 1 in set 1; set 0 takes stage st + 2
      fetch2(st + 2, j0i, j0j, r0i, r0j);
      jload2(st + 4, j0i, j0j);
      compute(0);
      if (st + 1 < nst) store2(r1i, r1j, 1, st + 1);
      __syncthreads();
      if (st + 1 >= nst) break;
      // stage st + 1 (buffer 1); stage st + 2 in set 0; set 1 takes stage st + 3
      fetch2(st + 3, j1i, j1j, r1i, r1j);
      jload2(st + 5, j1i, j1j);
      compute(1);
      if (st + 2 < nst) store2(r0i, r0j, 0, st + 2);
      __syncthreads();
    }
  }
  // accumulator v of a 16 x 16 block: row 4*(lane/16)+v (FP32 acc) or lane/16 + 4v (FP64), column lane%16
  double* out = part + ((int64_t)split * ntiles + tile) * (kBT * kBT);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = std::is_same<T, double>::value ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
        const int r = wi * 64 + 16 * i + rr;
        const int c = wj * 64 + 16 * j + (lane & 15);
        out[r * kBT + c] = work ? (double)acc[i][j][v] : 0.0;
      }
}

// One thread per tile element (TL*TL/256 workgroups per tile); the split partials
// are summed in split order, eight loads in flight.
template <int TL>
__global__ __launch_bounds__(256) void k_syrk_finish(const double* __restrict__ part, int N,
                                                     int ntiles, int nsplit, double shift,
                                                     double scale, double* __restrict__ out) {
  constexpr int kPer = TL * TL / 256;  // workgroups per tile
  const int tile = blockIdx.x / kPer;
  const int e = (blockIdx.x % kPer) * 256 + threadIdx.x;
  int ti, tj;
  tile_of(tile, ti, tj);
  const int li = e / TL, lj = e % TL;
  const int i = ti * TL + li, j = tj * TL + lj;
  if (i >= N || j >= N) return;
  if (ti == tj && li > lj) return;  // diagonal tile: upper half, mirrored below
  const double* src = part + (int64_t)tile * (TL * TL) + e;
  const int64_t stride = (int64_t)ntiles * (TL * TL);
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

// The 128-tile kernel: one round of at most 512 workgroups (two per CU; a
// second, part-filled round would double the time) from the split of K, at
// least 256 k-values a split, and no more partial tiles than fit the workspace:
// (1024 + T64 (T64 + 1) / 2) tiles of 64 x 64 up to N = 512 (the bound of
// the no-allocation entry point, whose m is at most 512), twice the 1024
// beyond; nsplit = 0 when not even one split fits.
SyrkPlan plan_big(int form, int m, int64_t r) {
  SyrkPlan p;
  p.N = form == 0 ? m : (int)r;
  p.K = form == 0 ? r : m;
  p.T = (p.N + kBT - 1) / kBT;
  p.ntiles = p.T * (p.T + 1) / 2;
  const int64_t t64 = (p.N + kTile - 1) / kTile;
  const int64_t cap = ((p.N > 512 ? 2048 : 1024) + t64 * (t64 + 1) / 2) / 4 / p.ntiles;
  int64_t s = p.ntiles <= 512 ? 512 / p.ntiles : 1;
  const int64_t maxs = (p.K + 255) / 256;
  if (s > maxs) s = maxs;
  if (s > cap) s = cap;
  if (s < 1) {
    p.nsplit = 0;
    p.kchunk = 0;
    return p;
  }
  int64_t kc = (p.K + s - 1) / s;
  kc = (kc + 63) / 64 * 64;
  p.kchunk = kc;
  p.nsplit = (int)((p.K + kc - 1) / kc);
  return p;
}

// The large systems (N >= 256 outputs over K >= 4096 terms) go to the
// 128-tile kernel when its 16-byte loads are aligned (A on 16 bytes, a
// column pitch of whole 16-byte chunks) and, for FP64, when its tiles fit
// one round: past 512 tiles (N > 4000) the 64-tile kernel keeps more FP64
// MFMAs busy (3.7 against 4.0 ms at N = 4096, K = 8192).
bool use_big(int form, int m, int64_t r, const void* A, int64_t lda, int esize) {
  const int64_t N = form == 0 ? m : r, K = form == 0 ? r : m;
  if (N < 256 || K < 4096) return false;
  if ((uintptr_t)A % 16 != 0 || (lda * esize) % 16 != 0) return false;
  const SyrkPlan q = plan_big(form, m, r);
  if (esize == 8 && q.ntiles > 512) return false;
  return q.nsplit >= 1;
}
}  // namespace

size_t syrk_workspace_bytes(int form, int m, int64_t r) {
  SyrkPlan p = plan(form, m, r);
  size_t b = (size_t)p.nsplit * p.ntiles * kTile * kTile * sizeof(double);
  SyrkPlan q = plan_big(form, m, r);
  const size_t c = (size_t)q.nsplit * q.ntiles * kBT * kBT * sizeof(double);
  return c > b ? c : b;
}

template <typename T>
static hipError_t launch_syrk(const T* A, int64_t lda, int m, const int32_t* J, int64_t r, int form,
                              double shift, double scale, double* out, double* work, hipStream_t st) {
  if (use_big(form, m, r, A, lda, (int)sizeof(T))) {
    SyrkPlan q = plan_big(form, m, r);
    const int nwork = q.ntiles * q.nsplit;
    const unsigned nb = (unsigned)((nwork + 7) / 8 * 8);
    if (form == 0)
      hipLaunchKernelGGL((k_syrk_big<T, 0>), dim3(nb), dim3(256), 0, st, A, lda, q.N, q.K, J, q.ntiles,
                         nwork, q.kchunk, work);
    else
      hipLaunchKernelGGL((k_syrk_big<T, 1>), dim3(nb), dim3(256), 0, st, A, lda, q.N, q.K, J, q.ntiles,
                         nwork, q.kchunk, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_syrk_finish<kBT>, dim3(q.ntiles * (kBT * kBT / 256)), dim3(256), 0, st, work, q.N,
                       q.ntiles, q.nsplit, shift, scale, out);
    return hipGetLastError();
  }
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
  hipLaunchKernelGGL(k_syrk_finish<kTile>, dim3(p.ntiles * 16), dim3(256), 0, st, work, p.N, p.ntiles,
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
