// FP64 finalisation of a multi-start solve.  Per start j the FP32 iterate is
// renormalised in FP64 on its support, x64 = x / ||x||_2; then u = A x64 is
// formed in FP64 and f(x64) of Table 1 and the explained variance
// (||Ax||_2^2 for L2 variance, ||Ax||_1 for L1 variance) follow.  The best
// start is the largest f, ties to the lowest index (Section 4: keep the
// solution with the largest objective value).  Starts that ended DEGENERATE
// or ZERO report x = 0 and f = 0.
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr int kFT = 256;       // rows of A per block of the matvec
constexpr int kFStage = 256;   // list entries staged in LDS at a time

__global__ __launch_bounds__(256) void x_norms_kernel(
    const float* __restrict__ list_val, int64_t ldl, StartState s, int64_t r,
    double* xnorm, const int32_t* only) {
  __shared__ double red[2 * 5];
  const int64_t j = blockIdx.x;
  if (only != nullptr && only[j] == 0) return;
  const bool live = s.status[j] != SPCA_DEGENERATE && s.status[j] != SPCA_ZERO;
  const int32_t cnt = live ? s.nnz[j] : 0;
  double acc[2] = {0.0, 0.0};
  for (int32_t t = threadIdx.x; t < cnt; t += 256) {
    double v = list_val[j * ldl + t];
    acc[0] += v * v;
    acc[1] += fabs(v);
  }
  block_sum_n<double, 2>(acc, red);
  if (threadIdx.x == 0) {
    double nrm = sqrt(acc[0]);
    xnorm[j] = nrm;               // ||x||_2 of the FP32 iterate
    xnorm[r + j] = nrm > 0.0 ? acc[1] / nrm : 0.0;  // ||x64||_1
  }
}

__global__ __launch_bounds__(kFT) void final_matvec_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n,
    const int32_t* __restrict__ list_idx, const float* __restrict__ list_val,
    int64_t ldl, StartState s, const double* __restrict__ xnorm,
    double* partial, int nchunks, const int32_t* only, Defl defl) {
  __shared__ int32_t sidx[kFStage];
  __shared__ double sval[kFStage];
  __shared__ double red[2 * 5];
  const int64_t j = blockIdx.x;
  const int c = blockIdx.y;
  if (only != nullptr && only[j] == 0) return;
  const double nrm = xnorm[j];
  double* out = partial + ((int64_t)j * nchunks + c) * 2;
  if (!(nrm > 0.0)) {
    if (threadIdx.x == 0) {
      out[0] = 0.0;
      out[1] = 0.0;
    }
    return;
  }
  const bool live = s.status[j] != SPCA_DEGENERATE && s.status[j] != SPCA_ZERO;
  const int32_t cnt = live ? s.nnz[j] : 0;
  const double inv = 1.0 / nrm;
  const int64_t i = (int64_t)c * kFT + threadIdx.x;
  double u = 0.0;
  for (int32_t t0 = 0; t0 < cnt; t0 += kFStage) {
    const int32_t m = cnt - t0 < kFStage ? cnt - t0 : kFStage;
    __syncthreads();
    if (threadIdx.x < m) {
      sidx[threadIdx.x] = list_idx[j * ldl + t0 + threadIdx.x];
      sval[threadIdx.x] = (double)list_val[j * ldl + t0 + threadIdx.x] * inv;
    }
    __syncthreads();
    if (i < n) {
      for (int32_t t = 0; t < m; ++t)
        u += (double)A[i + (int64_t)sidx[t] * lda] * sval[t];
    }
  }
  // deflated problem: A_k x = A x - sum_l alpha_l A x_l
  if (defl.k > 0 && i < n)
    for (int l = 0; l < defl.k; ++l)
      u -= defl.alpha[j * kMaxDefl + l] * defl.scores[i * kMaxDefl + l];
  double acc[2] = {u * u, fabs(u)};
  block_sum_n<double, 2>(acc, red);
  if (threadIdx.x == 0) {
    out[0] = acc[0];
    out[1] = acc[1];
  }
}

__global__ void objective_kernel(int fid, double gamma, StartState s,
                                 int64_t r, const double* __restrict__ partial,
                                 int nchunks, const double* __restrict__ xnorm,
                                 double* f, double* ev, const int32_t* only,
                                 const double* __restrict__ gam) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  if (only != nullptr && only[j] == 0) return;
  const bool live = s.status[j] != SPCA_DEGENERATE && s.status[j] != SPCA_ZERO &&
                    xnorm[j] > 0.0;
  if (!live) {
    f[j] = 0.0;
    ev[j] = 0.0;
    return;
  }
  double sq = 0.0, l1 = 0.0;
  for (int c = 0; c < nchunks; ++c) {
    sq += partial[(j * nchunks + c) * 2];
    l1 += partial[(j * nchunks + c) * 2 + 1];
  }
  const bool l1var = fid % 2 == 0;
  const double var = l1var ? l1 : sqrt(sq);
  if (gam != nullptr) gamma = gam[j];
  ev[j] = l1var ? l1 : sq;
  double fv;
  if (fid <= 4)
    fv = var;                                   // ||Ax||
  else if (fid <= 6)
    fv = var * var - gamma * (double)s.nnz[j];  // ||Ax||^2 - g ||x||_0
  else
    fv = var - gamma * xnorm[r + j];            // ||Ax|| - g ||x||_1
  f[j] = fv;
}

__global__ __launch_bounds__(1024) void best_kernel(
    const double* __restrict__ f, StartState s, int64_t r, int64_t p,
    const int32_t* __restrict__ list_idx, const float* __restrict__ list_val,
    int64_t ldl, const double* __restrict__ xnorm, int32_t* best_out,
    double* x_out, int32_t* support_out) {
  __shared__ double bv[16];
  __shared__ int64_t bi[16];
  double best = -INFINITY;
  int64_t arg = r;
  for (int64_t j = threadIdx.x; j < r; j += 1024) {
    if (f[j] > best || (f[j] == best && j < arg)) {
      best = f[j];
      arg = j;
    }
  }
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
    if (arg >= r) arg = 0;
    bi[0] = arg;
    best_out[0] = (int32_t)arg;
  }
  __syncthreads();
  const int64_t jb = bi[0];
  for (int64_t k = threadIdx.x; k < p; k += 1024) x_out[k] = 0.0;
  __syncthreads();
  const double nrm = xnorm[jb];
  const bool live = s.status[jb] != SPCA_DEGENERATE && s.status[jb] != SPCA_ZERO &&
                    nrm > 0.0;
  const int32_t cnt = live ? s.nnz[jb] : 0;
  for (int32_t t = threadIdx.x; t < cnt; t += 1024) {
    int32_t idx = list_idx[jb * ldl + t];
    x_out[idx] = (double)list_val[jb * ldl + t] / nrm;
    support_out[t] = idx;
  }
  if (threadIdx.x == 0) best_out[1] = cnt;
}

}  // namespace

void evaluate_rows(hipStream_t st, int fid, double s_or_gamma, const float* A,
                   int64_t lda, int64_t n, const int32_t* list_idx,
                   const float* list_val, int64_t ldl, StartState s, int64_t r,
                   double* partial, double* f, double* ev, double* xnorm,
                   const int32_t* only, const double* gam, Defl defl) {
  const int nchunks = (int)ceil_div(n, kFT);
  hipLaunchKernelGGL(x_norms_kernel, dim3((unsigned)r), dim3(256), 0, st,
                     list_val, ldl, s, r, xnorm, only);
  hipLaunchKernelGGL(final_matvec_kernel, dim3((unsigned)r, (unsigned)nchunks),
                     dim3(kFT), 0, st, A, lda, n, list_idx, list_val, ldl, s,
                     xnorm, partial, nchunks, only, defl);
  hipLaunchKernelGGL(objective_kernel, dim3((unsigned)ceil_div(r, 256)),
                     dim3(256), 0, st, fid, s_or_gamma, s, r, partial, nchunks,
                     xnorm, f, ev, only, gam);
}

void x_norms(hipStream_t st, const float* list_val, int64_t ldl, StartState s, int64_t r,
             double* xnorm) {
  hipLaunchKernelGGL(x_norms_kernel, dim3((unsigned)r), dim3(256), 0, st, list_val, ldl, s,
                     r, xnorm, nullptr);
}

void objective_and_best(hipStream_t st, int fid, double s_or_gamma, StartState s,
                        int64_t r, int64_t p, const double* partial, int nchunks,
                        const int32_t* list_idx, const float* list_val, int64_t ldl,
                        const double* xnorm, double* f, double* ev, int32_t* best,
                        double* x_out, int32_t* support_out, const double* gam,
                        bool by_ev) {
  hipLaunchKernelGGL(objective_kernel, dim3((unsigned)ceil_div(r, 256)), dim3(256), 0, st,
                     fid, s_or_gamma, s, r, partial, nchunks, xnorm, f, ev, nullptr, gam);
  hipLaunchKernelGGL(best_kernel, dim3(1), dim3(1024), 0, st, by_ev ? ev : f, s, r, p,
                     list_idx, list_val, ldl, xnorm, best, x_out, support_out);
}

void finalize(hipStream_t st, int fid, double s_or_gamma, const float* A,
              int64_t lda, int64_t n, int64_t p, const int32_t* list_idx,
              const float* list_val, int64_t ldl, StartState s, int64_t r,
              double* partial, double* f, double* ev, double* xnorm,
              int32_t* best, double* x_out, int32_t* support_out,
              const double* gam, bool by_ev, Defl defl) {
  evaluate_rows(st, fid, s_or_gamma, A, lda, n, list_idx, list_val, ldl, s, r,
                partial, f, ev, xnorm, nullptr, gam, defl);
  hipLaunchKernelGGL(best_kernel, dim3(1), dim3(1024), 0, st, by_ev ? ev : f, s, r, p,
                     list_idx, list_val, ldl, xnorm, best, x_out, support_out);
}

}  // namespace spca
