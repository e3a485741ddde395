// Counter-based synthetic spiked matrices generated in device memory, for
// workloads too large to build on the host and for requests that carry only
// a seed.  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): entry (i, j)
// uses counter (i, j, 0, 0) and key (seed low, seed high); its four outputs
// give four uniform 24-bit integers whose scaled sum
//   g = (sum * 2^-24 - 2) * sqrt(3)        (FP64, one rounding to FP32)
// has mean 0 and variance 1.  The spikes add sum_k (theta_k u_k[i]) v_k[j]
// in FP64, left to right, with explicitly rounded operations so that no
// multiply-add is contracted; the FP32 result is therefore reproducible
// bit for bit by any IEEE implementation of the same definition.
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr double kSqrt3 = 1.7320508075688772;
constexpr int kMaxSpikes = 16;

struct SpikeArgs {
  int32_t k;
  double theta[kMaxSpikes];
};

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0,
                                              uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ __launch_bounds__(256) void gen_spiked_kernel(
    uint32_t key0, uint32_t key1, int64_t n, int64_t p, float* __restrict__ A,
    int64_t lda, SpikeArgs sa, const double* __restrict__ U, int64_t ldu,
    const double* __restrict__ V, int64_t ldv) {
  for (int64_t j = blockIdx.y; j < p; j += gridDim.y) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
      uint32_t c[4] = {(uint32_t)i, (uint32_t)j, 0u, 0u};
      philox4x32_10(c, key0, key1);
      const double sum = (double)(c[0] >> 8) + (double)(c[1] >> 8) +
                         (double)(c[2] >> 8) + (double)(c[3] >> 8);
      double acc = __dmul_rn(__dadd_rn(__dmul_rn(sum, 0x1p-24), -2.0), kSqrt3);
      for (int t = 0; t < sa.k; ++t)
        acc = __dadd_rn(acc, __dmul_rn(__dmul_rn(sa.theta[t], U[i + t * ldu]),
                                       V[j + t * ldv]));
      A[i + j * lda] = (float)acc;
    }
  }
}

}  // namespace
}  // namespace spca

using namespace spca;

extern "C" int spca_generate_spiked(void* stream, uint64_t seed, int64_t n,
                                    int64_t p, float* A, int64_t lda, int32_t k,
                                    const double* thetas, const double* U,
                                    int64_t ldu, const double* V, int64_t ldv) {
  SPCA_REQUIRE(A != nullptr, "A must not be NULL");
  SPCA_REQUIRE(n >= 1 && p >= 1 && lda >= n, "need n, p >= 1 and lda >= n");
  SPCA_REQUIRE(n <= UINT32_MAX && p <= UINT32_MAX, "n and p must fit in 32 bits");
  SPCA_REQUIRE(k >= 0 && k <= kMaxSpikes, "k must be in 0..16");
  SPCA_REQUIRE(k == 0 || (thetas && U && V && ldu >= n && ldv >= p),
               "spikes need thetas, U (ldu >= n) and V (ldv >= p)");
  SpikeArgs sa{};
  sa.k = k;
  for (int t = 0; t < k; ++t) sa.theta[t] = thetas[t];
  const unsigned gx = (unsigned)ceil_div(n, 256) < 64 ? (unsigned)ceil_div(n, 256) : 64;
  const unsigned gy = (unsigned)(p < 65535 ? p : 65535);
  hipLaunchKernelGGL(gen_spiked_kernel, dim3(gx, gy), dim3(256), 0,
                     (hipStream_t)stream, (uint32_t)(seed & 0xFFFFFFFFu),
                     (uint32_t)(seed >> 32), n, p, A, lda, sa, U, ldu, V, ldv);
  SPCA_LAUNCH_CHECK("gen_spiked");
  return SPCA_OK;
}
