// Internal helpers of libspca: error reporting, launch checks and
// deterministic block reductions for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace spca {

constexpr int kWave = 64;

// Thread-local last-error message (exported through spca_last_error).
void set_error(const std::string& msg);
const char* last_error();

struct Status {
  int code;
};

#define SPCA_HIP_TRY(expr)                                                   \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess) {                                                  \
      ::spca::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));  \
      return SPCA_EHIP;                                                      \
    }                                                                        \
  } while (0)

#define SPCA_LAUNCH_CHECK(what)                                              \
  do {                                                                       \
    hipError_t _e = hipGetLastError();                                       \
    if (_e != hipSuccess) {                                                  \
      ::spca::set_error(std::string("launch of ") + (what) + ": " +          \
                        hipGetErrorString(_e));                              \
      return SPCA_EHIP;                                                      \
    }                                                                        \
  } while (0)

#define SPCA_REQUIRE(cond, msg)                                              \
  do {                                                                       \
    if (!(cond)) {                                                           \
      ::spca::set_error(msg);                                                \
      return SPCA_EINVAL;                                                    \
    }                                                                        \
  } while (0)

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
__host__ __device__ inline int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }

// ---------------------------------------------------------------------------
// Deterministic reductions.  A wave reduces with a fixed xor butterfly and
// lane 0's value is taken; waves are then summed in wave order by one thread.
// The result does not depend on timing, only on the block size.
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Sums NV values per thread over the block; every thread receives the
// totals.  scratch must hold NV * (blockDim/64 + 1) elements of T.
template <typename T, int NV>
__device__ __forceinline__ void block_sum_n(T (&v)[NV], T* scratch) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = wave_sum(v[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) scratch[wave * NV + c] = v[c];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    T acc = 0;
    for (int w = 0; w < nwaves; ++w) acc += scratch[w * NV + threadIdx.x];
    scratch[nwaves * NV + threadIdx.x] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = scratch[nwaves * NV + c];
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
  T a[1] = {v};
  block_sum_n<T, 1>(a, scratch);
  return a[0];
}

// Block max; scratch holds blockDim/64 + 1 elements.
template <typename T>
__device__ __forceinline__ T block_max(T v, T* scratch) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  v = wave_max(v);
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T m = scratch[0];
    for (int w = 1; w < nwaves; ++w) m = scratch[w] > m ? scratch[w] : m;
    scratch[nwaves] = m;
  }
  __syncthreads();
  v = scratch[nwaves];
  __syncthreads();
  return v;
}

// Exclusive prefix sum of one value per thread in thread order; returns the
// thread's offset and writes the block total to *total.  scratch holds
// blockDim/64 + 1 values.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* scratch, T* total) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  T incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T o = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += o;
  }
  if (lane == kWave - 1) scratch[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int w = 0; w < nwaves; ++w) {
      T t = scratch[w];
      scratch[w] = run;
      run += t;
    }
    scratch[nwaves] = run;
  }
  __syncthreads();
  T res = scratch[wave] + incl - v;
  *total = scratch[nwaves];
  __syncthreads();
  return res;
}

// FP32 -> BF16 bit pattern, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

// Per-start state machine shared by the iteration kernels.
constexpr int32_t kRunning = -1;

}  // namespace spca
