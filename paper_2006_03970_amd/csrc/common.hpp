// Shared device helpers for the SsNAL-EN HIP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssnal {

constexpr int kWave = 64;

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- reductions
// Wave sums on DPP lane permutations (no LDS traffic): xor-1 and xor-2
// inside quads, then the half-row and row mirrors, which leaves every lane of
// a 16-lane row holding the row sum; the four row sums are then combined
// across rows with permlane swaps in a fixed order.  At each step a lane adds
// the same two values as
// its partner (a + b == b + a), so every lane ends with the same bits and
// the result is reproducible run to run.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v));
  const int hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int kQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

// Cross-row steps of the wave sums (gfx950 permlane swaps, plain vector
// operations): with a value per 16-lane row r0..r3 in every lane of its row,
// pair_rows gives every lane r(2p) + r(2p + 1) of its row pair and then
// pair_halves (lower 32 lanes + upper 32 lanes) gives (r0 + r1) + (r2 + r3)
// in every lane: the operands and order of a sum of the four rows' first
// lanes, without a broadcast through a scalar register (about 70 cycles
// before its first use).
__device__ __forceinline__ double pair_rows(double v) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double pair_halves(double v) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ float pair_rows(float v) {
  const auto x = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
  return __int_as_float((int)x[0]) + __int_as_float((int)x[1]);
}
__device__ __forceinline__ float pair_halves(float v) {
  const auto x = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
  return __int_as_float((int)x[0]) + __int_as_float((int)x[1]);
}
__device__ __forceinline__ int pair_rows(int v) {
  const auto x = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return (int)x[0] + (int)x[1];
}
__device__ __forceinline__ int pair_halves(int v) {
  const auto x = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return (int)x[0] + (int)x[1];
}

// Sum over the wave; every lane receives the same bits.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kQuadXor1>(v);
  v += dpp_d<kQuadXor2>(v);
  v += dpp_d<kRowHalfMirror>(v);
  v += dpp_d<kRowMirror>(v);
  return pair_halves(pair_rows(v));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<kQuadXor1>(v);
  v += dpp_f<kQuadXor2>(v);
  v += dpp_f<kRowHalfMirror>(v);
  v += dpp_f<kRowMirror>(v);
  return pair_halves(pair_rows(v));
}
__device__ __forceinline__ int wave_sum(int v) {
  v += dpp_i<kQuadXor1>(v);
  v += dpp_i<kQuadXor2>(v);
  v += dpp_i<kRowHalfMirror>(v);
  v += dpp_i<kRowMirror>(v);
  return pair_halves(pair_rows(v));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<kQuadXor1>(v));
  v = fmax(v, dpp_d<kQuadXor2>(v));
  v = fmax(v, dpp_d<kRowHalfMirror>(v));
  v = fmax(v, dpp_d<kRowMirror>(v));
  auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  v = fmax(__hiloint2double((int)hi[0], (int)lo[0]), __hiloint2double((int)hi[1], (int)lo[1]));
  lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  return fmax(__hiloint2double((int)hi[0], (int)lo[0]), __hiloint2double((int)hi[1], (int)lo[1]));
}
// Sum over aligned groups of 8 lanes (every lane of a group gets the sum);
// only the lanes of each group need to be active.
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_d<kQuadXor1>(v);
  v += dpp_d<kQuadXor2>(v);
  v += dpp_d<kRowHalfMirror>(v);
  return v;
}

// Block sum for NT threads; `lds` holds NT/64 slots.  The result is valid in
// every thread.  Waves are combined in index order.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
  __syncthreads();
  T t = lds[0];
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i) t += lds[i];
  return t;
}

// K block sums at once (lds: K * NT / kWave entries): the bits of K calls
// of block_sum, with one pair of barriers instead of K.
template <int NT, int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* lds) {
  constexpr int NW = NT / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * NW + w] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = lds[k * NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) t += lds[k * NW + i];
    v[k] = t;
  }
}

// Sums of K components over nb partial rows part[b*K + k], by one block of
// NT threads: thread t adds rows t, t+NT, ... (each row's K loads issued
// together), then one tree per component (lds: K * NT / kWave entries).
// out[k] is written by thread 0.
// Fixed partition and order: reproducible.
template <int NT, int K>
__device__ __forceinline__ void final_sums(const double* part, int nb, double* out, double* lds) {
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) {
    double row[K];
#pragma unroll
    for (int k = 0; k < K; ++k) row[k] = part[(int64_t)b * K + k];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += row[k];
  }
  block_sums<NT, K>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = v[k];
  }
}

// ---------------------------------------------------------------- storage types
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t bits16) {
  return __uint_as_float(bits16 << 16);
}

// 16-byte vector load of VN consecutive stored elements, converted to ACC.
template <typename T> struct Vec16;
template <> struct Vec16<double> { static constexpr int N = 2; };
template <> struct Vec16<float> { static constexpr int N = 4; };
template <> struct Vec16<uint16_t> { static constexpr int N = 8; };

template <typename ACC>
__device__ __forceinline__ void load16(const double* p, ACC* e) {
  double2 q = *reinterpret_cast<const double2*>(p);
  e[0] = (ACC)q.x;
  e[1] = (ACC)q.y;
}
template <typename ACC>
__device__ __forceinline__ void load16(const float* p, ACC* e) {
  float4 q = *reinterpret_cast<const float4*>(p);
  e[0] = (ACC)q.x;
  e[1] = (ACC)q.y;
  e[2] = (ACC)q.z;
  e[3] = (ACC)q.w;
}
template <typename ACC>
__device__ __forceinline__ void load16(const uint16_t* p, ACC* e) {
  uint4 q = *reinterpret_cast<const uint4*>(p);
  uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    e[2 * i] = (ACC)bf16_bits_to_f32(w[i] & 0xFFFFu);
    e[2 * i + 1] = (ACC)bf16_bits_to_f32(w[i] >> 16);
  }
}

// 8-byte vector loads (A 8-byte aligned, lda*sizeof(elem) a multiple of 8).
template <typename ACC>
__device__ __forceinline__ void load8(const double* p, ACC* e) {
  e[0] = (ACC)*p;
}
template <typename ACC>
__device__ __forceinline__ void load8(const float* p, ACC* e) {
  float2 q = *reinterpret_cast<const float2*>(p);
  e[0] = (ACC)q.x;
  e[1] = (ACC)q.y;
}
template <typename ACC>
__device__ __forceinline__ void load8(const uint16_t* p, ACC* e) {
  uint2 q = *reinterpret_cast<const uint2*>(p);
  e[0] = (ACC)bf16_bits_to_f32(q.x & 0xFFFFu);
  e[1] = (ACC)bf16_bits_to_f32(q.x >> 16);
  e[2] = (ACC)bf16_bits_to_f32(q.y & 0xFFFFu);
  e[3] = (ACC)bf16_bits_to_f32(q.y >> 16);
}
// VB-byte vector load (VB = 16 or 8) of VB / sizeof(T) elements.
template <int VB, typename T, typename ACC>
__device__ __forceinline__ void loadv(const T* p, ACC* e) {
  if constexpr (VB == 16) load16<ACC>(p, e);
  else load8<ACC>(p, e);
}

template <typename ACC>
__device__ __forceinline__ ACC load1(const double* p) { return (ACC)*p; }
template <typename ACC>
__device__ __forceinline__ ACC load1(const float* p) { return (ACC)*p; }
template <typename ACC>
__device__ __forceinline__ ACC load1(const uint16_t* p) { return (ACC)bf16_bits_to_f32(*p); }

// ---------------------------------------------------------------- prox
// prox_{sigma p}(t) = soft(t, thr)/den with thr = sigma*lambda1 and
// den = 1 + sigma*lambda2 precomputed by the host (eq. prox_elastic).
__device__ __forceinline__ double prox_en(double t, double thr, double den) {
  if (t > thr) return (t - thr) / den;
  if (t < -thr) return (t + thr) / den;
  return 0.0;
}

}  // namespace ssnal
