// The per-device solver context (workspace, pinned poll word, event pools,
// the polish sub-context, the capture stream) and helpers shared by the
// host drivers of the solves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

namespace spca {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
      (void)hipSetDevice(prev);
  }
};

}  // namespace spca

// Pool of HIP events recorded in begin/end pairs around selected launches.
struct EventPairs {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipError_t mark(hipStream_t st) {
    if (used == ev.size()) {
      hipEvent_t e;
      hipError_t rc = hipEventCreate(&e);
      if (rc != hipSuccess) return rc;
      ev.push_back(e);
    }
    return hipEventRecord(ev[used++], st);
  }
  // sum of (end - begin) over the recorded pairs, in ms
  hipError_t total_ms(double* ms) {
    double t = 0.0;
    for (size_t i = 0; i + 1 < used; i += 2) {
      float x = 0.f;
      hipError_t rc = hipEventElapsedTime(&x, ev[i], ev[i + 1]);
      if (rc != hipSuccess) return rc;
      t += x;
    }
    *ms = t;
    return hipSuccess;
  }
  void reset() { used = 0; }
  void destroy() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    used = 0;
  }
};

struct spca_ctx {
  int device = 0;
  size_t budget = 0;
  void* ws = nullptr;
  size_t ws_cap = 0;
  bool ws_external = false;  // ws belongs to the caller
  int32_t* host_poll = nullptr;  // pinned
  EventPairs t_aty, t_xup, t_ax;
  spca_ctx* polish = nullptr;  // context of the FP32 polish sub-solves
  hipStream_t capture = nullptr;  // stream that graphs are captured on
  std::mutex mu;
};

// Grows the context's workspace to at least `bytes` (SPCA_ENOMEM beyond
// the context budget or a caller-provided workspace).
int ensure_workspace(spca_ctx* ctx, hipStream_t st, size_t bytes);

// The solve-wide warning (spca_result.warning) from the final statuses of
// the l starts of a solve with stop tolerance tol.
int32_t solve_warning(const std::vector<int32_t>& st, int64_t l, double tol);
