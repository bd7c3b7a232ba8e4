// A^T v over a column-major design: the HBM-bound pass of every Newton
// iteration (w_d = A^T d), of the initial A^T y and of the KKT residual.
//
// Layout: each wave streams whole columns.  Lane l owns rows
// [(it*64 + l)*VN, +VN) for it < ITERS, where VN elements make one VB-byte
// load (16 bytes, or 8 when the column stride allows no more), so a wave
// reads 1 KiB (512 B) per instruction and the matching slice of v stays in
// registers for the whole kernel.  A wave keeps COLS columns in
// flight (COLS*ITERS loads outstanding per lane), then reduces each column
// across the wave.  A block owns a contiguous range of columns, so the four
// waves of a block read neighbouring columns.
#include <hip/hip_ext.h>

#include "common.hpp"
#include "kernels.hpp"

namespace ssnal {

// Columns in flight per wave for ITERS loads per lane and element size ES
// (ES = 0: the long-column kernel).  FP32 columns of two loads per lane keep
// 4 in flight (fewer registers, more waves: measured faster than 8), BF16
// ones 8; FP64 columns of four loads with non-temporal loads 2 (measured at
// m = 500: 60.2 against 66.0 us for 4 cached).
constexpr int cols_for(int iters, int es, bool nt = false) {
  return iters <= 1 ? 8
                    : (iters <= 2 ? (es == 4 ? 4 : 8)
                                  : (iters <= 4 ? (nt && es == 8 ? 2 : 4) : (iters <= 8 ? 2 : 1)));
}
template <int ITERS, int ES = 0, bool NT = false>
struct ColsFor {
  static constexpr int value = cols_for(ITERS, ES, NT);
};

// Designs larger than this stream past the Infinity Cache (256 MB): their
// FP64 passes take non-temporal loads, which do not allocate in the caches
// (measured: m = 500, n = 1e5, 400 MB: 60.2 against 66.0 us; m = 1000,
// n = 1e6, 8 GB: 1138 against 1214 us; FP32 and BF16 gain nothing or lose,
// their smaller designs partly hitting the cache from pass to pass).
constexpr double kNtBytes = 256.0 * 1024 * 1024;

// VB-byte vector load of VB / 8 doubles that does not allocate in the caches.
template <int VB>
__device__ __forceinline__ void loadv_nt(const double* p, double* e) {
  if constexpr (VB == 16) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 q = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
    e[0] = q[0];
    e[1] = q[1];
  } else {
    e[0] = __builtin_nontemporal_load(p);
  }
}

// NT: non-temporal loads (FP64 only).
template <typename T, typename ACC, int ITERS, bool COLSQ, int VB, bool NT = false>
__global__ __launch_bounds__(256) void k_gemv_t(const T* __restrict__ A, int64_t lda, int m,
                                                int64_t ncols, const double* __restrict__ v,
                                                double* __restrict__ w, int64_t cpb,
                                                double* __restrict__ colsq_part) {
  constexpr int VN = VB / (int)sizeof(T);
  constexpr int COLS = ColsFor<ITERS, (int)sizeof(T), NT>::value;
  static_assert(!NT || (sizeof(T) == 8 && sizeof(ACC) == 8), "non-temporal loads for FP64 designs");
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;

  ACC vr[ITERS][VN];
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int r0 = (it * kWave + lane) * VN;
#pragma unroll
    for (int q = 0; q < VN; ++q) {
      const ACC x = (ACC)v[r0 + q < m ? r0 + q : m - 1];
      vr[it][q] = (r0 + q < m) ? x : (ACC)0;
    }
  }

  const int64_t c0 = (int64_t)blockIdx.x * cpb;
  const int64_t c1 = c0 + cpb < ncols ? c0 + cpb : ncols;
  double sq = 0.0;

  for (int64_t cb = c0 + (int64_t)wid * COLS; cb < c1; cb += 4 * COLS) {
    ACC e[COLS][ITERS][VN];
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      // loads are unconditional (clamped column and row start) and masked
      // below: a guarded load would be compiled into a branch that waits for
      // it, serialising the COLS x ITERS loads of the lane
      const int64_t j = cb + c;
      const T* a = A + (j < c1 ? j : c0) * lda;
#pragma unroll
      for (int it = 0; it < ITERS; ++it) {
        const int r0 = (it * kWave + lane) * VN;
        if constexpr (NT)
          loadv_nt<VB>(reinterpret_cast<const double*>(a + (r0 < m ? r0 : 0)), reinterpret_cast<double*>(e[c][it]));
        else
          loadv<VB>(a + (r0 < m ? r0 : 0), e[c][it]);
      }
    }
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      // rows past m inside the padded leading dimension may hold anything
#pragma unroll
      for (int it = 0; it < ITERS; ++it) {
        const int r0 = (it * kWave + lane) * VN;
        if (r0 + VN > m) {
#pragma unroll
          for (int q = 0; q < VN; ++q)
            if (r0 + q >= m) e[c][it][q] = (ACC)0;
        }
      }
      ACC acc = (ACC)0;
#pragma unroll
      for (int it = 0; it < ITERS; ++it)
#pragma unroll
        for (int q = 0; q < VN; ++q) acc += e[c][it][q] * vr[it][q];
      if (COLSQ) {
        const bool ok = cb + c < c1;
#pragma unroll
        for (int it = 0; it < ITERS; ++it)
#pragma unroll
          for (int q = 0; q < VN; ++q) sq += ok ? (double)e[c][it][q] * (double)e[c][it][q] : 0.0;
      }
      const double s = (double)wave_sum(acc);
      if (lane == 0 && cb + c < c1) w[cb + c] = s;
    }
  }
  if (COLSQ) {
    __shared__ double red[4];
    const double t = block_sum<256>(sq, red);
    if (threadIdx.x == 0) colsq_part[blockIdx.x] = t;
  }
}

// Long or gathered columns: the rows go in panels of PR = ITERS*64*VN, each
// with its slice of v in registers (as above); a block owns at most
// kLongCols consecutive columns (or entries of J) and carries their partial
// sums from panel to panel in LDS, each column in the same wave and lane in
// every panel, so the panels add up in a fixed order.
constexpr int kLongCols = 256;
template <typename T, typename ACC, int ITERS, int VB, bool GATHER>
__global__ __launch_bounds__(256) void k_gemv_t_long(const T* __restrict__ A, int64_t lda, int m,
                                                     int64_t ncols, const int32_t* __restrict__ J,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ w, int64_t cpb,
                                                     const double* __restrict__ skip) {
  if (skip && *skip != 0.0) return;
  constexpr int VN = VB / (int)sizeof(T);
  constexpr int COLS = ColsFor<ITERS>::value;
  constexpr int PR = ITERS * kWave * VN;
  __shared__ double lw[kLongCols];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int64_t c0 = (int64_t)blockIdx.x * cpb;
  const int64_t c1 = c0 + cpb < ncols ? c0 + cpb : ncols;
  for (int p0 = 0; p0 < m; p0 += PR) {
    const int mp = m - p0 < PR ? m - p0 : PR;
    const bool first = p0 == 0, last = p0 + PR >= m;
    ACC vr[ITERS][VN];
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const int r0 = (it * kWave + lane) * VN;
#pragma unroll
      for (int q = 0; q < VN; ++q) {
        const ACC x = (ACC)v[p0 + (r0 + q < mp ? r0 + q : mp - 1)];
        vr[it][q] = (r0 + q < mp) ? x : (ACC)0;
      }
    }
    for (int64_t cb = c0 + (int64_t)wid * COLS; cb < c1; cb += 4 * COLS) {
      ACC e[COLS][ITERS][VN];
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        const int64_t j = cb + c < c1 ? cb + c : c0;
        const int64_t col = GATHER ? (int64_t)J[j] : j;
        // r0 + VN <= lda - p0 whenever r0 < mp: lda is a multiple of VN
        const T* a = A + col * lda + p0;
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
          const int r0 = (it * kWave + lane) * VN;
          loadv<VB>(a + (r0 < mp ? r0 : 0), e[c][it]);
        }
      }
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
          const int r0 = (it * kWave + lane) * VN;
          if (r0 + VN > mp) {
#pragma unroll
            for (int q = 0; q < VN; ++q)
              if (r0 + q >= mp) e[c][it][q] = (ACC)0;
          }
        }
        ACC acc = (ACC)0;
#pragma unroll
        for (int it = 0; it < ITERS; ++it)
#pragma unroll
          for (int q = 0; q < VN; ++q) acc += e[c][it][q] * vr[it][q];
        const double sp = (double)wave_sum(acc);
        if (lane == 0 && cb + c < c1) {
          const int k = (int)(cb + c - c0);
          const double t = first ? sp : lw[k] + sp;
          if (last)
            w[cb + c] = t;
          else
            lw[k] = t;
        }
      }
    }
  }
}

// Any alignment, any m, optional column index list: one element per lane.
template <typename T, typename ACC, bool GATHER>
__global__ __launch_bounds__(256) void k_gemv_t_gen(const T* __restrict__ A, int64_t lda, int m,
                                                    int64_t ncols, const int32_t* __restrict__ J,
                                                    const double* __restrict__ v,
                                                    double* __restrict__ w,
                                                    const double* __restrict__ skip) {
  if (skip && *skip != 0.0) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t j = gw; j < ncols; j += nw) {
    const int64_t col = GATHER ? (int64_t)J[j] : j;
    const T* a = A + col * lda;
    ACC acc = (ACC)0;
    for (int i = lane; i < m; i += kWave) acc += load1<ACC>(a + i) * (ACC)v[i];
    const double s = (double)wave_sum(acc);
    if (lane == 0) w[j] = s;
  }
}

// sum_j ||a_j||^2 for any alignment (one partial per block).
template <typename T>
__global__ __launch_bounds__(256) void k_colsq_gen(const T* __restrict__ A, int64_t lda, int m,
                                                   int64_t n, double* __restrict__ part) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
  double sq = 0.0;
  for (int64_t j = gw; j < n; j += nw) {
    const T* a = A + j * lda;
    for (int i = lane; i < m; i += kWave) {
      const double e = load1<double>(a + i);
      sq += e * e;
    }
  }
  __shared__ double red[4];
  const double t = block_sum<256>(sq, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

namespace {

// Loads per lane and panel: the slice of v held in registers stays within 64
// VGPRs (beyond that the kernels spill).
template <typename T, typename ACC, int VB>
constexpr int max_iters() {
  constexpr int v = 256 / ((VB / (int)sizeof(T)) * (int)sizeof(ACC));
  return v < 16 ? v : 16;
}
template <typename T, typename ACC>
bool fits_fast(int vb, int m) {
  const int cap = vb == 16 ? max_iters<T, ACC, 16>() : max_iters<T, ACC, 8>();
  return m <= cap * kWave * (vb / (int)sizeof(T));
}

// ev0/ev1 (nullable): events stamped by the dispatch itself around the kernel.
template <typename T, typename ACC, bool COLSQ, int VB, bool NT = false>
hipError_t launch_fast(const T* A, int64_t lda, int m, int64_t n, const double* v, double* w,
                       double* colsq_part, int* nparts, hipStream_t st, hipEvent_t ev0,
                       hipEvent_t ev1) {
  constexpr int VN = VB / (int)sizeof(T);
  const int need = (m + kWave * VN - 1) / (kWave * VN);
  int iters = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
  const int cols = cols_for(iters, (int)sizeof(T), NT);
  const int64_t step = 4 * (int64_t)cols;
  const int64_t nsteps = (n + step - 1) / step;
  // one column step (4 waves x cols columns) per block: the many short blocks
  // balance across the CUs better than fewer long ones (measured: -4% on the
  // pass at n = 1e5, -3% at n = 1e6); the pass with column sums keeps one
  // partial per block, at most 2048
  const int64_t maxb = COLSQ ? 2048 : nsteps;
  int64_t spb = (nsteps + maxb - 1) / maxb;
  if (spb < 1) spb = 1;
  const int64_t cpb = spb * step;
  const int64_t nb = (n + cpb - 1) / cpb;
  if (nparts) *nparts = (int)nb;
  dim3 g((unsigned)nb), b(256);
#define SSNAL_GEMV_CASE(IT)                                                                  \
  case IT:                                                                                   \
    if constexpr (IT <= max_iters<T, ACC, VB>()) {                                           \
      if (ev0)                                                                               \
        hipExtLaunchKernelGGL((k_gemv_t<T, ACC, IT, COLSQ, VB, NT>), g, b, 0, st, ev0, ev1, 0, \
                              A, lda, m, n, v, w, cpb, colsq_part);                          \
      else                                                                                   \
        hipLaunchKernelGGL((k_gemv_t<T, ACC, IT, COLSQ, VB, NT>), g, b, 0, st, A, lda, m, n, v, \
                           w, cpb, colsq_part);                                              \
    } else {                                                                                 \
      return hipErrorInvalidValue;                                                           \
    }                                                                                        \
    break;
  switch (iters) {
    SSNAL_GEMV_CASE(1)
    SSNAL_GEMV_CASE(2)
    SSNAL_GEMV_CASE(4)
    SSNAL_GEMV_CASE(8)
    SSNAL_GEMV_CASE(16)
  }
#undef SSNAL_GEMV_CASE
  return hipGetLastError();
}

template <typename T, typename ACC>
hipError_t launch_gen(const T* A, int64_t lda, int m, int64_t n, const int32_t* J, const double* v,
                      double* w, hipStream_t st, const double* skip) {
  int64_t nb = (n + 3) / 4;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  if (J)
    hipLaunchKernelGGL((k_gemv_t_gen<T, ACC, true>), dim3((unsigned)nb), dim3(256), 0, st, A, lda, m,
                       n, J, v, w, skip);
  else
    hipLaunchKernelGGL((k_gemv_t_gen<T, ACC, false>), dim3((unsigned)nb), dim3(256), 0, st, A, lda,
                       m, n, J, v, w, skip);
  return hipGetLastError();
}

// Panels of up to 16 loads per lane; a block owns cpb <= kLongCols columns:
// up to 8 column groups per wave, fewer while that leaves under 1024 blocks.
template <typename T, typename ACC, int VB, bool GATHER>
hipError_t launch_long(const T* A, int64_t lda, int m, int64_t n, const int32_t* J, const double* v,
                       double* w, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                       const double* skip) {
  constexpr int VN = VB / (int)sizeof(T);
  const int need = (m + kWave * VN - 1) / (kWave * VN);
  int iters = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
  if (iters > max_iters<T, ACC, VB>()) iters = max_iters<T, ACC, VB>();
  const int cols = cols_for(iters, 0);
  const int64_t step = 4 * (int64_t)cols;
  const int64_t nsteps = (n + step - 1) / step;
  int64_t spb = (nsteps + 1023) / 1024;
  if (spb > 8) spb = 8;
  if (spb * step > kLongCols) spb = kLongCols / step;
  if (spb < 1) spb = 1;
  const int64_t cpb = spb * step;
  const int64_t nb = (n + cpb - 1) / cpb;
  dim3 g((unsigned)nb), b(256);
#define SSNAL_LONG_CASE(IT)                                                                      \
  case IT:                                                                                       \
    if constexpr (IT <= max_iters<T, ACC, VB>()) {                                               \
      if (ev0)                                                                                   \
        hipExtLaunchKernelGGL((k_gemv_t_long<T, ACC, IT, VB, GATHER>), g, b, 0, st, ev0, ev1, 0,   \
                              A, lda, m, n, J, v, w, cpb, skip);                                 \
      else                                                                                       \
        hipLaunchKernelGGL((k_gemv_t_long<T, ACC, IT, VB, GATHER>), g, b, 0, st, A, lda, m, n, J,  \
                           v, w, cpb, skip);                                                     \
    }                                                                                            \
    break;
  switch (iters) {
    SSNAL_LONG_CASE(1)
    SSNAL_LONG_CASE(2)
    SSNAL_LONG_CASE(4)
    SSNAL_LONG_CASE(8)
    SSNAL_LONG_CASE(16)
  }
#undef SSNAL_LONG_CASE
  return hipGetLastError();
}

// Widest vector load (16 or 8 bytes) that every column start allows, with
// the column held in at most 16 loads per lane; 0 = no such width.
int fast_vb(const void* A, int dtype, int64_t lda, int m) {
  const int es = dtype_size(dtype);
  for (int vb = 16; vb >= 8; vb /= 2) {
    if (((uintptr_t)A) % vb != 0 || (lda * es) % vb != 0) continue;
    if (m <= 16 * kWave * (vb / es)) return vb;
  }
  return 0;
}
// Widest vector load that every column start allows, for any m (panels).
int align_vb(const void* A, int dtype, int64_t lda) {
  const int es = dtype_size(dtype);
  for (int vb = 16; vb >= 8; vb /= 2)
    if (((uintptr_t)A) % vb == 0 && (lda * es) % vb == 0) return vb;
  return 0;
}

template <typename T, typename ACC, bool COLSQ>
hipError_t launch_vb(int vb, const T* A, int64_t lda, int m, int64_t n, const double* v, double* w,
                     double* colsq_part, int* nparts, hipStream_t st, hipEvent_t ev0,
                     hipEvent_t ev1) {
  if constexpr (sizeof(T) == 8 && sizeof(ACC) == 8 && !COLSQ) {
    if ((double)lda * (double)n * 8.0 > kNtBytes) {
      if (vb == 16)
        return launch_fast<T, ACC, COLSQ, 16, true>(A, lda, m, n, v, w, colsq_part, nparts, st, ev0, ev1);
      return launch_fast<T, ACC, COLSQ, 8, true>(A, lda, m, n, v, w, colsq_part, nparts, st, ev0, ev1);
    }
  }
  if (vb == 16)
    return launch_fast<T, ACC, COLSQ, 16>(A, lda, m, n, v, w, colsq_part, nparts, st, ev0, ev1);
  return launch_fast<T, ACC, COLSQ, 8>(A, lda, m, n, v, w, colsq_part, nparts, st, ev0, ev1);
}

template <typename T, typename ACC>
hipError_t dispatch_long(int lvb, const T* A, int64_t lda, int m, int64_t n, const int32_t* J,
                         const double* v, double* w, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                         const double* skip) {
  if (lvb == 16)
    return J ? launch_long<T, ACC, 16, true>(A, lda, m, n, J, v, w, st, ev0, ev1, skip)
             : launch_long<T, ACC, 16, false>(A, lda, m, n, J, v, w, st, ev0, ev1, skip);
  return J ? launch_long<T, ACC, 8, true>(A, lda, m, n, J, v, w, st, ev0, ev1, skip)
           : launch_long<T, ACC, 8, false>(A, lda, m, n, J, v, w, st, ev0, ev1, skip);
}

template <typename T>
hipError_t dispatch(const T* A, int64_t lda, int m, int64_t n, const int32_t* J, const double* v,
                    double* w, bool acc64, int vb, int lvb, hipStream_t st, hipEvent_t ev0,
                    hipEvent_t ev1, const double* skip) {
  if (n <= 0) return hipSuccess;
  if (vb && !J && !skip) {
    if (acc64 && fits_fast<T, double>(vb, m))
      return launch_vb<T, double, false>(vb, A, lda, m, n, v, w, nullptr, nullptr, st, ev0, ev1);
    if (!acc64 && fits_fast<T, float>(vb, m))
      return launch_vb<T, float, false>(vb, A, lda, m, n, v, w, nullptr, nullptr, st, ev0, ev1);
  }
  if (lvb) {
    if (acc64) return dispatch_long<T, double>(lvb, A, lda, m, n, J, v, w, st, ev0, ev1, skip);
    return dispatch_long<T, float>(lvb, A, lda, m, n, J, v, w, st, ev0, ev1, skip);
  }
  if (ev0) {
    hipError_t e = hipEventRecord(ev0, st);
    if (e != hipSuccess) return e;
  }
  hipError_t e = acc64 ? launch_gen<T, double>(A, lda, m, n, J, v, w, st, skip)
                       : launch_gen<T, float>(A, lda, m, n, J, v, w, st, skip);
  if (e == hipSuccess && ev1) e = hipEventRecord(ev1, st);
  return e;
}

}  // namespace

hipError_t gemv_t(const void* A, int dtype, int64_t lda, int m, int64_t ncols, const int32_t* J,
                  const double* v, double* w, bool acc64, hipStream_t st, hipEvent_t ev0,
                  hipEvent_t ev1, const double* skip) {
  const int vb = fast_vb(A, dtype, lda, m);
  const int lvb = align_vb(A, dtype, lda);
  switch (dtype) {
    case kF64:
      return dispatch<double>((const double*)A, lda, m, ncols, J, v, w, true, vb, lvb, st, ev0, ev1,
                              skip);
    case kF32:
      return dispatch<float>((const float*)A, lda, m, ncols, J, v, w, acc64, vb, lvb, st, ev0, ev1,
                             skip);
    case kBF16:
      return dispatch<uint16_t>((const uint16_t*)A, lda, m, ncols, J, v, w, acc64, vb, lvb, st, ev0,
                                ev1, skip);
  }
  return hipErrorInvalidValue;
}

hipError_t gemv_t_colsq(const void* A, int dtype, int64_t lda, int m, int64_t n, const double* v,
                        double* w, double* colsq_part, int* nparts, hipStream_t st, hipEvent_t ev0,
                        hipEvent_t ev1) {
  int vb = fast_vb(A, dtype, lda, m);
  // the pass with column sums accumulates in FP64
  if (vb && !(dtype == kF64   ? fits_fast<double, double>(vb, m)
              : dtype == kF32 ? fits_fast<float, double>(vb, m)
                              : fits_fast<uint16_t, double>(vb, m)))
    vb = 0;
  if (!vb) {
    hipError_t e = gemv_t(A, dtype, lda, m, n, nullptr, v, w, true, st, ev0, ev1);
    if (e != hipSuccess) return e;
    const int nb = 1024;
    *nparts = nb;
    switch (dtype) {
      case kF64:
        hipLaunchKernelGGL(k_colsq_gen<double>, dim3(nb), dim3(256), 0, st, (const double*)A, lda, m, n, colsq_part);
        break;
      case kF32:
        hipLaunchKernelGGL(k_colsq_gen<float>, dim3(nb), dim3(256), 0, st, (const float*)A, lda, m, n, colsq_part);
        break;
      case kBF16:
        hipLaunchKernelGGL(k_colsq_gen<uint16_t>, dim3(nb), dim3(256), 0, st, (const uint16_t*)A, lda, m, n,
                           colsq_part);
        break;
    }
    return hipGetLastError();
  }
  switch (dtype) {
    case kF64:
      return launch_vb<double, double, true>(vb, (const double*)A, lda, m, n, v, w, colsq_part,
                                             nparts, st, ev0, ev1);
    case kF32:
      return launch_vb<float, double, true>(vb, (const float*)A, lda, m, n, v, w, colsq_part, nparts,
                                            st, ev0, ev1);
    case kBF16:
      return launch_vb<uint16_t, double, true>(vb, (const uint16_t*)A, lda, m, n, v, w, colsq_part,
                                               nparts, st, ev0, ev1);
  }
  return hipErrorInvalidValue;
}

}  // namespace ssnal
