// The two products of the AM iteration for a sparse A (the paper's text
// corpora are word-count matrices), stored twice: compressed sparse columns
// for A^T Y and for A x from a sparse x, compressed sparse rows for A x from a
// dense x.  The iterates keep the start-major layout of the dense path, so the
// y-update, x-update, planner and stop test are shared; the products read
// the transposed operand (all starts of a row of Y, or of a column of X, are
// contiguous) so that every stored entry of A is used against 64 starts with
// one 256-byte read, and tiles of the result go back to start-major order
// through LDS.  Every sum runs in a fixed order.
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr int kST = 64;  // rows or columns per tile, and starts per group

// U tile (64 rows x 64 starts) from the rows of A against X^T
__global__ __launch_bounds__(256) void sp_csr_ax_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const float* __restrict__ val, int64_t n, const float* __restrict__ XT, int64_t ldxt,
    int64_t r, float* __restrict__ U, int64_t ldu, const Plan* plan) {
  __shared__ float tile[kST][kST + 1];
  if (plan->mode != kAxDense) return;
  const int64_t i0 = (int64_t)blockIdx.x * kST;
  const int64_t j0 = (int64_t)blockIdx.y * kST;
  const int lane = threadIdx.x % kST, wave = threadIdx.x / kST;
  const int64_t j = j0 + lane;
  for (int rr = wave; rr < kST; rr += 4) {
    const int64_t i = i0 + rr;
    float acc = 0.f;
    if (i < n && j < r)
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
        acc += val[k] * XT[(int64_t)col_idx[k] * ldxt + j];
    tile[rr][lane] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kST * kST; e += 256) {
    const int jj = e / kST, rr = e % kST;
    if (i0 + rr < n && j0 + jj < r) U[(j0 + jj) * ldu + i0 + rr] = tile[rr][jj];
  }
}

// one workgroup per running start: u = sum over its support columns, column
// by column (the rows of one column are distinct, so no two threads add to
// the same entry at once)
__global__ __launch_bounds__(256) void sp_csc_ax_list_kernel(
    const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
    const float* __restrict__ val, int64_t n, const int32_t* __restrict__ list_idx,
    const float* __restrict__ list_val, int64_t ldl, float* __restrict__ U, int64_t ldu,
    StartState s, const Plan* plan) {
  if (plan->mode != kAxListRows) return;
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  float* u = U + j * ldu;
  for (int64_t i = threadIdx.x; i < n; i += 256) u[i] = 0.f;
  __syncthreads();
  const int32_t cnt = s.nnz[j];
  for (int32_t t = 0; t < cnt; ++t) {
    const int32_t c = list_idx[j * ldl + t];
    const float x = list_val[j * ldl + t];
    for (int64_t k = col_ptr[c] + threadIdx.x; k < col_ptr[c + 1]; k += 256)
      u[row_idx[k]] += val[k] * x;
    __syncthreads();
  }
}

// V tile (64 columns x 64 starts) from the columns of A against Y^T
__global__ __launch_bounds__(256) void sp_csc_aty_kernel(
    const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
    const float* __restrict__ val, int64_t p, const float* __restrict__ YT, int64_t ldyt,
    int64_t r, float* __restrict__ V, int64_t ldv) {
  __shared__ float tile[kST][kST + 1];
  const int64_t c0 = (int64_t)blockIdx.x * kST;
  const int64_t j0 = (int64_t)blockIdx.y * kST;
  const int lane = threadIdx.x % kST, wave = threadIdx.x / kST;
  const int64_t j = j0 + lane;
  for (int cc = wave; cc < kST; cc += 4) {
    const int64_t c = c0 + cc;
    float acc = 0.f;
    if (c < p && j < r)
      for (int64_t k = col_ptr[c]; k < col_ptr[c + 1]; ++k)
        acc += val[k] * YT[(int64_t)row_idx[k] * ldyt + j];
    tile[cc][lane] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kST * kST; e += 256) {
    const int jj = e / kST, cc = e % kST;
    if (c0 + cc < p && j0 + jj < r) V[(j0 + jj) * ldv + c0 + cc] = tile[cc][jj];
  }
}

// final evaluation: u = A x / ||x|| in FP64 from the support columns, then
// sum u_i^2 and sum |u_i| (one partial per start)
__global__ __launch_bounds__(256) void sp_final_kernel(
    const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
    const float* __restrict__ val, int64_t n, const int32_t* __restrict__ list_idx,
    const float* __restrict__ list_val, int64_t ldl, StartState s,
    const double* __restrict__ xnorm, double* __restrict__ u64, double* partial) {
  __shared__ double red[2 * 5];
  const int64_t j = blockIdx.x;
  double* u = u64 + j * n;
  for (int64_t i = threadIdx.x; i < n; i += 256) u[i] = 0.0;
  __syncthreads();
  const double nrm = xnorm[j];
  const bool live = s.status[j] != SPCA_DEGENERATE && s.status[j] != SPCA_ZERO && nrm > 0.0;
  const int32_t cnt = live ? s.nnz[j] : 0;
  for (int32_t t = 0; t < cnt; ++t) {
    const int32_t c = list_idx[j * ldl + t];
    const double x = (double)list_val[j * ldl + t] / nrm;
    for (int64_t k = col_ptr[c] + threadIdx.x; k < col_ptr[c + 1]; k += 256)
      u[row_idx[k]] += (double)val[k] * x;
    __syncthreads();
  }
  double acc[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    acc[0] += u[i] * u[i];
    acc[1] += fabs(u[i]);
  }
  block_sum_n<double, 2>(acc, red);
  if (threadIdx.x == 0) {
    partial[2 * j] = acc[0];
    partial[2 * j + 1] = acc[1];
  }
}

}  // namespace

void sparse_ax_dense(hipStream_t st, SparseA a, const float* XT, int64_t ldxt, int64_t r,
                     float* U, int64_t ldu, const Plan* plan) {
  const dim3 g((unsigned)ceil_div(a.n, (int64_t)kST), (unsigned)ceil_div(r, (int64_t)kST));
  hipLaunchKernelGGL(sp_csr_ax_kernel, g, dim3(256), 0, st, a.row_ptr, a.col_idx, a.row_val,
                     a.n, XT, ldxt, r, U, ldu, plan);
}

void sparse_ax_list(hipStream_t st, SparseA a, const int32_t* list_idx,
                    const float* list_val, int64_t ldl, float* U, int64_t ldu, int64_t r,
                    StartState s, const Plan* plan) {
  hipLaunchKernelGGL(sp_csc_ax_list_kernel, dim3((unsigned)r), dim3(256), 0, st, a.col_ptr,
                     a.row_idx, a.col_val, a.n, list_idx, list_val, ldl, U, ldu, s, plan);
}

void sparse_aty(hipStream_t st, SparseA a, const float* YT, int64_t ldyt, int64_t r,
                float* V, int64_t ldv) {
  const dim3 g((unsigned)ceil_div(a.p, (int64_t)kST), (unsigned)ceil_div(r, (int64_t)kST));
  hipLaunchKernelGGL(sp_csc_aty_kernel, g, dim3(256), 0, st, a.col_ptr, a.row_idx, a.col_val,
                     a.p, YT, ldyt, r, V, ldv);
}

void sparse_final(hipStream_t st, SparseA a, const int32_t* list_idx,
                  const float* list_val, int64_t ldl, StartState s, int64_t r,
                  const double* xnorm, double* u64, double* partial) {
  hipLaunchKernelGGL(sp_final_kernel, dim3((unsigned)r), dim3(256), 0, st, a.col_ptr,
                     a.row_idx, a.col_val, a.n, list_idx, list_val, ldl, s, xnorm, u64,
                     partial);
}

}  // namespace spca
