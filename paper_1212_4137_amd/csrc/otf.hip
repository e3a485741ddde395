// On-the-fly replacement of finished starts (the OTF scheme of Section
// 4.3): total_starts starting points flow through r slots.  After every
// x-update the slots whose start just stopped (any status other than
// running) are evaluated in FP64 (objective of Table 1 and explained
// variance, the same kernels as the final evaluation), their results are
// stored under their start's index, the best start so far is kept (largest
// f, ties to the lowest start index, as in the final selection), and the
// next unissued starts are loaded into the freed slots in slot order.  All
// of it runs on the device inside the iteration, so the host only polls the
// number of running slots, and the iteration can be captured in a graph.
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

__global__ void otf_init_kernel(Otf o, int64_t r) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < r) {
    o.slot_start[s] = s < o.total ? (int32_t)s : -1;
    o.retiring[s] = 0;
    o.refill[s] = -1;
  }
  if (s == 0) {
    o.ctl[0] = (int32_t)(r < o.total ? r : o.total);
    o.ctl[1] = INT32_MAX;
    o.ctl[2] = -1;
    *o.best_f = -INFINITY;
  }
}

// finished slots of this x-update; with force, every occupied slot (a start
// still running is closed as MAXIT)
__global__ void otf_mark_kernel(Otf o, StartState s, int64_t r, int force) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  int ret = 0;
  if (o.slot_start[j] >= 0) {
    if (s.status[j] != kRunning)
      ret = 1;
    else if (force) {
      s.status[j] = SPCA_MAXIT;
      ret = 1;
    }
  }
  o.retiring[j] = ret;
}

// one thread, slots in order: results, best so far, next starts
__global__ void otf_commit_kernel(Otf o, StartState s, int64_t r,
                                  const double* __restrict__ f,
                                  const double* __restrict__ ev) {
  if (threadIdx.x != 0) return;
  o.ctl[2] = -1;
  for (int64_t j = 0; j < r; ++j) {
    o.refill[j] = -1;
    if (!o.retiring[j]) continue;
    const int32_t id = o.slot_start[j];
    const int32_t stj = s.status[j];
    const bool live = stj != SPCA_DEGENERATE && stj != SPCA_ZERO;
    o.f[id] = f[j];
    o.ev[id] = ev[j];
    o.phi[id] = s.phi[j];
    o.iters[id] = s.iters[j];
    o.status[id] = stj;
    o.nnz[id] = live ? s.nnz[j] : 0;
    o.retiring[j] = id + 1;  // the copy kernel files the iterate under id
    if (f[j] > *o.best_f || (f[j] == *o.best_f && id < o.ctl[1])) {
      *o.best_f = f[j];
      o.ctl[1] = id;
      o.ctl[2] = (int32_t)j;
    }
    const int32_t next = o.ctl[0];
    if (next < o.total) {
      o.refill[j] = next;
      o.slot_start[j] = next;
      o.ctl[0] = next + 1;
    } else {
      o.slot_start[j] = -1;
    }
  }
}

// per slot: keep the best start's iterate (and, when asked, every finished
// start's), then load the slot's next start
__global__ __launch_bounds__(256) void otf_copy_kernel(
    Otf o, StartState s, float* __restrict__ X, int64_t ldx,
    const float* __restrict__ X0, int64_t p) {
  const int64_t j = blockIdx.x;
  float* x = X + j * ldx;
  if (o.ctl[2] == j)
    for (int64_t i = threadIdx.x; i < p; i += 256) o.best_x[i] = x[i];
  const int32_t done_id = o.retiring[j] - 1;
  if (o.x_all != nullptr && done_id >= 0) {
    float* dst = o.x_all + (int64_t)done_id * p;
    for (int64_t i = threadIdx.x; i < p; i += 256) dst[i] = x[i];
  }
  __syncthreads();
  const int32_t id = o.refill[j];
  if (id < 0) return;
  const float* x0 = X0 + (int64_t)id * p;
  for (int64_t i = threadIdx.x; i < p; i += 256) x[i] = x0[i];
  if (threadIdx.x == 0) {
    s.phi[j] = 0.0;
    s.phi_prev[j] = 0.0;
    s.iters[j] = 0;
    s.nnz[j] = (int32_t)p;
    s.status[j] = kRunning;
    if (s.thr != nullptr) s.thr[j] = 0.f;
  }
}

// x = best_x / ||best_x||_2 in FP64 and its support in index order
__global__ __launch_bounds__(1024) void otf_output_kernel(
    Otf o, int64_t p, int32_t* best, double* x_out, int32_t* support_out) {
  __shared__ double red[17];
  __shared__ int scan[17];
  const int64_t chunk = ceil_div(p, (int64_t)1024);
  const int64_t b = threadIdx.x * chunk;
  const int64_t e = b + chunk < p ? b + chunk : p;
  double sq = 0.0;
  int cnt = 0;
  for (int64_t i = b; i < e; ++i) {
    const double v = o.best_x[i];
    sq += v * v;
    cnt += v != 0.0;
  }
  sq = block_sum(sq, red);
  int total;
  int off = block_exclusive_scan(cnt, scan, &total);
  const double nrm = sqrt(sq);
  const bool live = o.ctl[1] != INT32_MAX && nrm > 0.0 &&
                    o.status[o.ctl[1]] != SPCA_DEGENERATE &&
                    o.status[o.ctl[1]] != SPCA_ZERO;
  for (int64_t i = b; i < e; ++i) {
    const float v = o.best_x[i];
    x_out[i] = live ? (double)v / nrm : 0.0;
    if (live && v != 0.f) support_out[off++] = (int32_t)i;
  }
  if (threadIdx.x == 0) {
    best[0] = o.ctl[1] == INT32_MAX ? 0 : o.ctl[1];
    best[1] = live ? total : 0;
  }
}

}  // namespace

void otf_init(hipStream_t st, Otf o, int64_t r) {
  hipLaunchKernelGGL(otf_init_kernel, dim3((unsigned)ceil_div(r, 256)), dim3(256), 0,
                     st, o, r);
}

void otf_step(hipStream_t st, int fid, double s_or_gamma, const float* A,
              int64_t lda, int64_t n, int64_t p, float* X, int64_t ldx,
              const float* X0, int32_t* list_idx, float* list_val, int64_t ldl,
              StartState s, int64_t r, double* partial, double* f, double* ev,
              double* xnorm, Otf o, int force) {
  const dim3 g((unsigned)ceil_div(r, 256));
  hipLaunchKernelGGL(otf_mark_kernel, g, dim3(256), 0, st, o, s, r, force);
  compact_rows(st, X, ldx, r, p, list_idx, list_val, ldl, s.nnz, nullptr, nullptr,
               nullptr, o.retiring);
  evaluate_rows(st, fid, s_or_gamma, A, lda, n, list_idx, list_val, ldl, s, r,
                partial, f, ev, xnorm, o.retiring);
  hipLaunchKernelGGL(otf_commit_kernel, dim3(1), dim3(64), 0, st, o, s, r, f, ev);
  hipLaunchKernelGGL(otf_copy_kernel, dim3((unsigned)r), dim3(256), 0, st, o, s, X,
                     ldx, X0, p);
}

void otf_output(hipStream_t st, Otf o, int64_t p, int32_t* best, double* x_out,
                int32_t* support_out) {
  hipLaunchKernelGGL(otf_output_kernel, dim3(1), dim3(1024), 0, st, o, p, best,
                     x_out, support_out);
}

}  // namespace spca
