// The x-update operator (Table 3, rows S3-S6) for callers that cannot
// allocate device memory: the same computation as spca_x_update, with the
// scratch of the chunked kernels (rows longer than 12288) in a fixed
// per-device array instead of an allocation.
//
// The array below is a device symbol: in host code its name is not a
// device address.  Its address on each device is looked up once, with that
// device current, at the first call there, and only that address is ever
// handed to kernels.
#include <stdint.h>

#include <mutex>
#include <string>

#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr size_t kScratchBytes = (size_t)SPCA_X_UPDATE_NOALLOC_SCRATCH;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// The scratch address on the current device (looked up on first use).
int scratch_on_current_device(void** out) {
  int dev = -1;
  SPCA_HIP_TRY(hipGetDevice(&dev));
  SPCA_REQUIRE(dev >= 0 && dev < kMaxDevices, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    SPCA_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SPCA_REQUIRE(p != nullptr && (uintptr_t)p % 256 == 0,
                 "scratch symbol has no 256-byte aligned device address");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SPCA_OK;
}

// Zero fill (a kernel rather than a memset node, so the call can be
// captured into a graph).
__global__ __launch_bounds__(256) void clear_words_kernel(uint32_t* __restrict__ w,
                                                          int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    w[i] = 0u;
}

}  // namespace
}  // namespace spca

using namespace spca;

extern "C" int spca_x_update_noalloc(void* stream, int formulation, const float* V,
                                     int64_t ldv, int64_t r, int64_t p,
                                     double s_or_gamma, float* X, int64_t ldx,
                                     double* phi, int32_t* nnz) {
  SPCA_REQUIRE(V && X && phi && nnz, "V, X, phi and nnz must not be NULL");
  int rc = check_problem(1, p, 1, formulation, s_or_gamma, r, 0.0, 1);
  if (rc != SPCA_OK) return rc;
  SPCA_REQUIRE(ldv >= p && ldx >= p, "leading dimensions too small");
  const size_t wb = x_update_wide_bytes(formulation, r, p);
  if (wb > kScratchBytes) {
    set_error("x-update scratch of " + std::to_string(wb) + " bytes for r = " +
              std::to_string(r) + ", p = " + std::to_string(p) +
              " exceeds the fixed " + std::to_string(kScratchBytes) +
              " bytes (SPCA_X_UPDATE_NOALLOC_SCRATCH); split the rows into batches");
    return SPCA_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  void* wide = nullptr;
  if (wb) {
    rc = scratch_on_current_device(&wide);
    if (rc != SPCA_OK) return rc;
    // the digit histograms must start at zero (the kernels leave them
    // zero, but an earlier call's state is not relied on)
    const int64_t words = x_update_wide_clear_words(r);
    const int64_t blocks = ceil_div(words, (int64_t)256);
    hipLaunchKernelGGL(clear_words_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)),
                       dim3(256), 0, st, (uint32_t*)wide, words);
  }
  StartState s{phi, nullptr, nnz, nullptr, nullptr};
  x_update(st, formulation, s_or_gamma, V, ldv, r, p, X, ldx, nullptr, nullptr, 0, 0, s,
           -1.0, 1, nullptr, nullptr, wide);
  hipError_t le = hipGetLastError();
  if (le != hipSuccess) {
    set_error(std::string("x_update_noalloc: ") + hipGetErrorString(le));
    return SPCA_EHIP;
  }
  return SPCA_OK;
}
