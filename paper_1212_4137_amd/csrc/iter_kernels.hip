// Staging, planning and y-update kernels of the AM iteration (Algorithm 2):
// the layout copies of A, the start x0 = e_{i*}, the per-start state, the
// choice between the dense and the list-based product A x, and the y-update
// y = sgn(u) or u / ||u||_2 (Table 3, rows S1 and S2).
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

// ---------------------------------------------------------------------------
// Layout copies
// ---------------------------------------------------------------------------

constexpr int kTT = 64;  // transpose tile

__global__ __launch_bounds__(256) void transpose_kernel(
    const float* __restrict__ A, int64_t lda, float* __restrict__ At,
    int64_t ldat, int64_t n, int64_t p) {
  __shared__ float tile[kTT][kTT + 1];
  const int64_t i0 = (int64_t)blockIdx.x * kTT;  // rows of A (n)
  const int64_t k0 = (int64_t)blockIdx.y * kTT;  // columns of A (p)
  const int tx = threadIdx.x % kTT;
  const int ty = threadIdx.x / kTT;  // 0..3
  for (int kk = ty; kk < kTT; kk += 4) {
    int64_t i = i0 + tx, k = k0 + kk;
    tile[kk][tx] = (i < n && k < p) ? A[i + k * lda] : 0.f;
  }
  __syncthreads();
  for (int ii = ty; ii < kTT; ii += 4) {
    int64_t i = i0 + ii, k = k0 + tx;
    if (i < n && k < p) At[i * ldat + k] = tile[tx][ii];
  }
}

// one block per column (grid-stride over columns)
__global__ __launch_bounds__(256) void copy_columns_kernel(
    const float* __restrict__ A, int64_t lda, float* __restrict__ B,
    int64_t ldb, int64_t n, int64_t p) {
  for (int64_t k = blockIdx.x; k < p; k += gridDim.x)
    for (int64_t i = threadIdx.x; i < ldb; i += 256)
      B[i + k * ldb] = i < n ? A[i + k * lda] : 0.f;
}

__global__ __launch_bounds__(256) void count_nonfinite_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n, int64_t p,
    int32_t* count) {
  int bad = 0;
  for (int64_t k = blockIdx.x; k < p; k += gridDim.x)
    for (int64_t i = threadIdx.x; i < n; i += 256) bad += !isfinite(A[i + k * lda]);
  if (bad) atomicAdd(count, bad);
}

// ---------------------------------------------------------------------------
// x0 = e_{i*}
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void column_sq_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n, int64_t p,
    double* colsq) {
  __shared__ double red[8];
  const int64_t k = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double a = A[i + k * lda];
    acc += a * a;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) colsq[k] = acc;
}

__global__ __launch_bounds__(1024) void argmax_start_kernel(
    const double* __restrict__ colsq, int64_t p, float* X) {
  __shared__ double bv[16];
  __shared__ int64_t bi[16];
  double best = -1.0;
  int64_t arg = 0;
  for (int64_t k = threadIdx.x; k < p; k += 1024) {
    if (colsq[k] > best) {
      best = colsq[k];
      arg = k;
    }
  }
  // reduce (value desc, index asc)
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(best, off, kWave);
    int64_t oi = __shfl_xor(arg, off, kWave);
    if (ov > best || (ov == best && oi < arg)) {
      best = ov;
      arg = oi;
    }
  }
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (lane == 0) {
    bv[wave] = best;
    bi[wave] = arg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w)
      if (bv[w] > best || (bv[w] == best && bi[w] < arg)) {
        best = bv[w];
        arg = bi[w];
      }
    bi[0] = arg;
  }
  __syncthreads();
  arg = bi[0];
  for (int64_t k = threadIdx.x; k < p; k += 1024) X[k] = (k == arg) ? 1.f : 0.f;
}

// ---------------------------------------------------------------------------
// Lists of nonzeros of the rows of X, in index order
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void compact_rows_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t p, int32_t* list_idx,
    float* list_val, int64_t ldl, int32_t* nnz, const int32_t* status) {
  __shared__ int scan[20];
  const int64_t j = blockIdx.x;
  if (status != nullptr && status[j] != kRunning) return;
  const float* x = X + j * ldx;
  const int64_t chunk = ceil_div(p, blockDim.x);
  const int64_t b = threadIdx.x * chunk;
  const int64_t e = b + chunk < p ? b + chunk : p;
  int cnt = 0;
  for (int64_t i = b; i < e; ++i) cnt += x[i] != 0.f;
  int total;
  int off = block_exclusive_scan(cnt, scan, &total);
  for (int64_t i = b; i < e; ++i) {
    float v = x[i];
    if (v != 0.f) {
      list_idx[j * ldl + off] = (int32_t)i;
      list_val[j * ldl + off] = v;
      ++off;
    }
  }
  if (threadIdx.x == 0) nnz[j] = total;
}

__global__ void init_state_kernel(StartState s, int64_t r) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  s.phi[j] = 0.0;
  s.phi_prev[j] = 0.0;
  s.iters[j] = 0;
  s.status[j] = kRunning;
}

// One block: count running starts and their nonzeros, pick the product.
__global__ __launch_bounds__(1024) void plan_kernel(StartState s, int64_t r,
                                                    int64_t p, double frac,
                                                    int dense_only, Plan* plan) {
  __shared__ int64_t red[2 * 17];
  int64_t v[2] = {0, 0};
  for (int64_t j = threadIdx.x; j < r; j += blockDim.x) {
    if (s.status[j] == kRunning) {
      v[0] += 1;
      v[1] += s.nnz[j];
    }
  }
  block_sum_n<int64_t, 2>(v, red);
  if (threadIdx.x == 0) {
    plan->active = (int32_t)v[0];
    plan->total_nnz = v[1];
    const double dense_work = (double)p * (double)v[0];
    plan->sparse = (!dense_only && (double)v[1] <= frac * dense_work) ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// y-update (Algorithm 2; Table 3, S1 for L2 variance, S2 for L1 variance)
// ---------------------------------------------------------------------------

template <bool L1VAR>
__global__ __launch_bounds__(256) void y_update_kernel(
    const float* __restrict__ U, int splits, int64_t split_stride,
    float* __restrict__ Y, int64_t ldu, int64_t n, StartState s,
    const Plan* plan) {
  __shared__ double red[8];
  if (plan->sparse) return;
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  const float* u = U + j * ldu;
  float* y = Y + j * ldu;
  // u_i = sum of the split partials in split order; each thread keeps the
  // values it owns in y until the norm is known
  double sq = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    float t = u[i];
    for (int sp = 1; sp < splits; ++sp) t += u[i + sp * split_stride];
    y[i] = t;
    double td = t;
    sq += td * td;
  }
  sq = block_sum(sq, red);
  if (sq == 0.0) {
    if (threadIdx.x == 0) s.status[j] = SPCA_DEGENERATE;
    return;
  }
  const double inv = 1.0 / sqrt(sq);
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    float t = y[i];
    y[i] = L1VAR ? (float)((t > 0.f) - (t < 0.f)) : (float)((double)t * inv);
  }
}

// Sparse A x (x given by its list) fused with the y-update; one block per
// start, rows of A strided over the threads so that every term reads a
// contiguous run of a column.  FP64 accumulation.
constexpr int kSpThreads = 256;
constexpr int kSpRows = 8;      // rows per thread per sweep of the list
constexpr int kSpStage = 256;   // list entries staged in LDS at a time

template <bool L1VAR>
__global__ __launch_bounds__(kSpThreads) void sparse_ax_y_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n,
    const int32_t* __restrict__ list_idx, const float* __restrict__ list_val,
    int64_t ldl, float* __restrict__ Y, int64_t ldu, StartState s,
    const Plan* plan) {
  __shared__ int32_t sidx[kSpStage];
  __shared__ float sval[kSpStage];
  __shared__ double red[8];
  if (!plan->sparse) return;
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  const int32_t cnt = s.nnz[j];
  const int32_t* li = list_idx + j * ldl;
  const float* lv = list_val + j * ldl;
  float* y = Y + j * ldu;

  double sq = 0.0;
  for (int64_t base = 0; base < n; base += (int64_t)kSpThreads * kSpRows) {
    double acc[kSpRows];
#pragma unroll
    for (int q = 0; q < kSpRows; ++q) acc[q] = 0.0;
    for (int32_t t0 = 0; t0 < cnt; t0 += kSpStage) {
      const int32_t m = cnt - t0 < kSpStage ? cnt - t0 : kSpStage;
      __syncthreads();
      if (threadIdx.x < m) {
        sidx[threadIdx.x] = li[t0 + threadIdx.x];
        sval[threadIdx.x] = lv[t0 + threadIdx.x];
      }
      __syncthreads();
      for (int32_t t = 0; t < m; ++t) {
        const float* col = A + (int64_t)sidx[t] * lda;
        const double xv = sval[t];
#pragma unroll
        for (int q = 0; q < kSpRows; ++q) {
          int64_t i = base + q * kSpThreads + threadIdx.x;
          if (i < n) acc[q] += (double)col[i] * xv;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kSpRows; ++q) {
      int64_t i = base + q * kSpThreads + threadIdx.x;
      if (i < n) {
        float u = (float)acc[q];
        y[i] = u;  // u for now; scaled below once ||u|| is known
        double uu = u;
        sq += uu * uu;
      }
    }
  }
  sq = block_sum(sq, red);
  if (sq == 0.0) {
    if (threadIdx.x == 0) s.status[j] = SPCA_DEGENERATE;
    return;
  }
  const double inv = 1.0 / sqrt(sq);
  // each thread rescales exactly the entries it wrote
  for (int64_t base = 0; base < n; base += (int64_t)kSpThreads * kSpRows) {
#pragma unroll
    for (int q = 0; q < kSpRows; ++q) {
      int64_t i = base + q * kSpThreads + threadIdx.x;
      if (i < n) {
        float t = y[i];
        y[i] = L1VAR ? (float)((t > 0.f) - (t < 0.f)) : (float)((double)t * inv);
      }
    }
  }
}

}  // namespace

void transpose_f32(hipStream_t st, const float* A, int64_t lda, float* At,
                   int64_t ldat, int64_t n, int64_t p) {
  dim3 grid((unsigned)ceil_div(n, kTT), (unsigned)ceil_div(p, kTT));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, A, lda, At, ldat,
                     n, p);
}

void copy_columns_f32(hipStream_t st, const float* A, int64_t lda, float* B,
                      int64_t ldb, int64_t n, int64_t p) {
  dim3 grid((unsigned)(p < 65536 ? p : 65536));
  hipLaunchKernelGGL(copy_columns_kernel, grid, dim3(256), 0, st, A, lda, B, ldb,
                     n, p);
}

void count_nonfinite(hipStream_t st, const float* A, int64_t lda, int64_t n,
                     int64_t p, int32_t* count) {
  dim3 grid((unsigned)(p < 65536 ? p : 65536));
  hipLaunchKernelGGL(count_nonfinite_kernel, grid, dim3(256), 0, st, A, lda, n,
                     p, count);
}

void max_norm_column_start(hipStream_t st, const float* A, int64_t lda,
                           int64_t n, int64_t p, double* colsq, float* X,
                           int64_t ldx) {
  (void)ldx;
  hipLaunchKernelGGL(column_sq_kernel, dim3((unsigned)p), dim3(256), 0, st, A,
                     lda, n, p, colsq);
  hipLaunchKernelGGL(argmax_start_kernel, dim3(1), dim3(1024), 0, st, colsq, p,
                     X);
}

void compact_rows(hipStream_t st, const float* X, int64_t ldx, int64_t r,
                  int64_t p, int32_t* list_idx, float* list_val, int64_t ldl,
                  int32_t* nnz, const int32_t* status) {
  hipLaunchKernelGGL(compact_rows_kernel, dim3((unsigned)r), dim3(1024), 0, st,
                     X, ldx, p, list_idx, list_val, ldl, nnz, status);
}

void init_state(hipStream_t st, StartState s, int64_t r) {
  hipLaunchKernelGGL(init_state_kernel, dim3((unsigned)ceil_div(r, 256)),
                     dim3(256), 0, st, s, r);
}

void plan_next(hipStream_t st, StartState s, int64_t r, int64_t p,
               double sparse_fraction, int dense_only, Plan* plan) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, st, s, r, p,
                     sparse_fraction, dense_only, plan);
}

void y_update(hipStream_t st, int fid, const float* U, int splits,
              int64_t split_stride, float* Y, int64_t ldu, int64_t r,
              int64_t n, StartState s, const Plan* plan) {
  if (l1_variance(fid))
    hipLaunchKernelGGL(y_update_kernel<true>, dim3((unsigned)r), dim3(256), 0,
                       st, U, splits, split_stride, Y, ldu, n, s, plan);
  else
    hipLaunchKernelGGL(y_update_kernel<false>, dim3((unsigned)r), dim3(256), 0,
                       st, U, splits, split_stride, Y, ldu, n, s, plan);
}

void sparse_ax_y_update(hipStream_t st, int fid, const float* A, int64_t lda,
                        int64_t n, const int32_t* list_idx,
                        const float* list_val, int64_t ldl, float* Y,
                        int64_t ldu, int64_t r, StartState s, const Plan* plan) {
  if (l1_variance(fid))
    hipLaunchKernelGGL(sparse_ax_y_kernel<true>, dim3((unsigned)r),
                       dim3(kSpThreads), 0, st, A, lda, n, list_idx, list_val,
                       ldl, Y, ldu, s, plan);
  else
    hipLaunchKernelGGL(sparse_ax_y_kernel<false>, dim3((unsigned)r),
                       dim3(kSpThreads), 0, st, A, lda, n, list_idx, list_val,
                       ldl, Y, ldu, s, plan);
}

}  // namespace spca
