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
// Butterfly sums: every lane ends with the same value (a + b == b + a), and
// the order is fixed, so results are bitwise reproducible run to run.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
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

// "Last block finishes" protocol: each block publishes its partials, then
// counts itself in; the block that arrives last sees every partial (agent-
// scope release/acquire fences make the writes of other XCDs visible) and
// resets the counter for the next launch.  Returns true in the last block.
__device__ __forceinline__ bool arrive_last(unsigned int* counter, unsigned int nblocks) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int prev = atomicAdd(counter, 1u);
    last = (prev == nblocks - 1);
    if (last) atomicExch(counter, 0u);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
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
