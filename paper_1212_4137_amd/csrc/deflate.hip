// Deflation for further components: the solve works on
//   A_k = A (I - x_1 x_1^T)(I - x_2 x_2^T) ... (I - x_k x_k^T)
// (projection deflation of the data matrix by the loadings found before)
// without forming it.  With P_i = I - x_i x_i^T:
//   A_k x   = A z,  z = P_1 ... P_k x = x - sum_i alpha_i x_i,
//             alpha_i = x_i^T x - sum_{l > i} G_il alpha_l   (i = k .. 1)
//   A_k^T y = P_k ... P_1 (A^T y) = v - sum_i beta_i x_i,
//             beta_i  = x_i^T v - sum_{l < i} G_il beta_l    (i = 1 .. k)
// with G the Gram matrix of the loadings.  So u = A x is corrected by
// - sum alpha_i (A x_i) before the y-update and v = A^T y by
// - sum beta_i x_i (on the supports of the x_i) before the x-update; the
// scores A x_i are formed once per solve in FP64.  The loadings are sparse,
// so the per-iteration work is O(r k (n + |S|)).  All sums run in a fixed
// order.
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr int kDT = 256;

// loading i as an (index, value) list of its nonzeros, in index order
__global__ __launch_bounds__(1024) void defl_compact_kernel(const double* __restrict__ Xd,
                                                            int64_t p, Defl d) {
  __shared__ int scan[17];
  const int64_t i = blockIdx.x;
  const double* x = Xd + i * p;
  const int64_t chunk = ceil_div(p, (int64_t)1024);
  const int64_t b = threadIdx.x * chunk < p ? threadIdx.x * chunk : p;
  const int64_t e = b + chunk < p ? b + chunk : p;
  int cnt = 0;
  for (int64_t t = b; t < e; ++t) cnt += x[t] != 0.0;
  int total;
  int off = block_exclusive_scan(cnt, scan, &total);
  for (int64_t t = b; t < e; ++t) {
    if (x[t] != 0.0) {
      d.idx[i * p + off] = (int32_t)t;
      d.val[i * p + off] = x[t];
      ++off;
    }
  }
  if (threadIdx.x == 0) d.cnt[i] = total;
}

// G_il = x_i^T x_l (block i, all l)
__global__ __launch_bounds__(kDT) void defl_gram_kernel(const double* __restrict__ Xd,
                                                        int64_t p, Defl d) {
  __shared__ double red[2 * kMaxDefl * (kDT / kWave + 1)];
  const int i = blockIdx.x;
  double acc[kMaxDefl];
#pragma unroll
  for (int l = 0; l < kMaxDefl; ++l) acc[l] = 0.0;
  for (int t = threadIdx.x; t < d.cnt[i]; t += kDT) {
    const int32_t c = d.idx[i * p + t];
    const double v = d.val[i * p + t];
#pragma unroll
    for (int l = 0; l < kMaxDefl; ++l)
      if (l < d.k) acc[l] += v * Xd[l * p + c];
  }
  block_sum_n<double, kMaxDefl>(acc, red);
  if (threadIdx.x == 0)
    for (int l = 0; l < d.k; ++l) d.gram[i * kMaxDefl + l] = acc[l];
}

// scores B[:, i] = A x_i in FP64 (rows in chunks of kDT)
__global__ __launch_bounds__(kDT) void defl_scores_kernel(const float* __restrict__ A,
                                                          int64_t lda, int64_t n,
                                                          int64_t p, Defl d) {
  const int i = blockIdx.x;
  const int64_t row = (int64_t)blockIdx.y * kDT + threadIdx.x;
  if (row >= n) return;
  double u = 0.0;
  for (int t = 0; t < d.cnt[i]; ++t)
    u += (double)A[row + (int64_t)d.idx[i * p + t] * lda] * d.val[i * p + t];
  d.scores[row * kMaxDefl + i] = u;
}

// dot products of a row (an iterate, or v) with the loadings, over their
// supports; every thread receives them
__device__ __forceinline__ void loading_dots(const Defl& d, const float* __restrict__ x,
                                             int64_t p, double (&dot)[kMaxDefl],
                                             double* red) {
#pragma unroll
  for (int l = 0; l < kMaxDefl; ++l) dot[l] = 0.0;
  for (int l = 0; l < d.k; ++l)
    for (int t = threadIdx.x; t < d.cnt[l]; t += kDT)
      dot[l] += d.val[l * p + t] * (double)x[d.idx[l * p + t]];
  block_sum_n<double, kMaxDefl>(dot, red);
}

// alpha from the dots (i = k .. 1)
__device__ __forceinline__ void alphas(const Defl& d, double (&a)[kMaxDefl]) {
  for (int i = d.k - 1; i >= 0; --i) {
    double t = a[i];
    for (int l = i + 1; l < d.k; ++l) t -= d.gram[i * kMaxDefl + l] * a[l];
    a[i] = t;
  }
}

// u_j (first partial of U) -= sum_i alpha_i B[:, i], for the running starts,
// in the modes whose U goes through the separate y-update.  Workgroup
// (b, j) corrects rows [b kDR, (b + 1) kDR) of start j (alpha is formed
// again by every block of the start: k dot products over the loadings'
// supports).
constexpr int64_t kDR = 4096;

__global__ __launch_bounds__(kDT) void defl_u_kernel(const float* __restrict__ X,
                                                     int64_t ldx, int64_t p,
                                                     float* __restrict__ U, int64_t ldu,
                                                     int64_t n, StartState s,
                                                     const Plan* plan, Defl d) {
  __shared__ double red[kMaxDefl * (kDT / kWave + 1)];
  if (plan->mode == kAxList) return;
  const int64_t j = blockIdx.y;
  if (s.status[j] != kRunning) return;
  double a[kMaxDefl];
  loading_dots(d, X + j * ldx, p, a, red);
  alphas(d, a);
  float* u = U + j * ldu;
  const int64_t b0 = (int64_t)blockIdx.x * kDR;
  const int64_t b1 = b0 + kDR < n ? b0 + kDR : n;
  for (int64_t row = b0 + threadIdx.x; row < b1; row += kDT) {
    double c = 0.0;
    for (int l = 0; l < d.k; ++l) c += a[l] * d.scores[row * kMaxDefl + l];
    u[row] = (float)((double)u[row] - c);
  }
}

// v_j -= sum_i beta_i x_i on the supports of the loadings
__global__ __launch_bounds__(kDT) void defl_v_kernel(float* __restrict__ V, int64_t ldv,
                                                     int64_t p, StartState s, Defl d) {
  __shared__ double red[kMaxDefl * (kDT / kWave + 1)];
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  float* v = V + j * ldv;
  double b[kMaxDefl];
  loading_dots(d, v, p, b, red);
  for (int i = 0; i < d.k; ++i) {
    double t = b[i];
    for (int l = 0; l < i; ++l) t -= d.gram[i * kMaxDefl + l] * b[l];
    b[i] = t;
  }
  for (int i = 0; i < d.k; ++i) {
    for (int t = threadIdx.x; t < d.cnt[i]; t += kDT) {
      const int32_t c = d.idx[i * p + t];
      v[c] = (float)((double)v[c] - b[i] * d.val[i * p + t]);
    }
    __syncthreads();  // overlapping supports: loadings in order
  }
}

// alpha of every start for the final FP64 evaluation, for the unit FP64
// iterate x / ||x||_2
__global__ __launch_bounds__(kDT) void defl_final_alpha_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t p, Defl d) {
  __shared__ double red[kMaxDefl * (kDT / kWave + 1)];
  const int64_t j = blockIdx.x;
  const float* x = X + j * ldx;
  double sq = 0.0;
  for (int64_t t = threadIdx.x; t < p; t += kDT) sq += (double)x[t] * (double)x[t];
  sq = block_sum(sq, red);
  double a[kMaxDefl];
  loading_dots(d, x, p, a, red);
  const double inv = sq > 0.0 ? 1.0 / sqrt(sq) : 0.0;
#pragma unroll
  for (int l = 0; l < kMaxDefl; ++l) a[l] *= inv;
  alphas(d, a);
  if (threadIdx.x == 0)
    for (int l = 0; l < d.k; ++l) d.alpha[j * kMaxDefl + l] = a[l];
}

}  // namespace

size_t deflate_bytes(int64_t n, int64_t p, int64_t r, int k) {
  if (k <= 0) return 0;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  return up(sizeof(int32_t) * k * p) + up(sizeof(double) * k * p) + up(sizeof(int32_t) * k) +
         up(sizeof(double) * kMaxDefl * kMaxDefl) + up(sizeof(double) * kMaxDefl * n) +
         up(sizeof(double) * kMaxDefl * r);
}

Defl carve_deflate(void* base, int64_t n, int64_t p, int64_t r, int k) {
  Defl d;
  d.k = k;
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = c + off;
    off += (bytes + 255) / 256 * 256;
    return q;
  };
  d.idx = (int32_t*)take(sizeof(int32_t) * k * p);
  d.val = (double*)take(sizeof(double) * k * p);
  d.cnt = (int32_t*)take(sizeof(int32_t) * k);
  d.gram = (double*)take(sizeof(double) * kMaxDefl * kMaxDefl);
  d.scores = (double*)take(sizeof(double) * kMaxDefl * n);
  d.alpha = (double*)take(sizeof(double) * kMaxDefl * r);
  return d;
}

void deflate_loadings(hipStream_t st, const double* Xd, int64_t p, Defl d) {
  hipLaunchKernelGGL(defl_compact_kernel, dim3((unsigned)d.k), dim3(1024), 0, st, Xd, p, d);
  hipLaunchKernelGGL(defl_gram_kernel, dim3((unsigned)d.k), dim3(kDT), 0, st, Xd, p, d);
}

void deflate_setup(hipStream_t st, const double* Xd, const float* A, int64_t lda,
                   int64_t n, int64_t p, Defl d) {
  deflate_loadings(st, Xd, p, d);
  hipLaunchKernelGGL(defl_scores_kernel, dim3((unsigned)d.k, (unsigned)ceil_div(n, kDT)),
                     dim3(kDT), 0, st, A, lda, n, p, d);
}

void deflate_u(hipStream_t st, const float* X, int64_t ldx, int64_t p, float* U,
               int64_t ldu, int64_t n, int64_t r, StartState s, const Plan* plan, Defl d) {
  hipLaunchKernelGGL(defl_u_kernel, dim3((unsigned)ceil_div(n, kDR), (unsigned)r), dim3(kDT),
                     0, st, X, ldx, p, U, ldu, n, s, plan, d);
}

void deflate_v(hipStream_t st, float* V, int64_t ldv, int64_t p, int64_t r, StartState s,
               Defl d) {
  hipLaunchKernelGGL(defl_v_kernel, dim3((unsigned)r), dim3(kDT), 0, st, V, ldv, p, s, d);
}

void deflate_final_alpha(hipStream_t st, const float* X, int64_t ldx, int64_t p,
                         int64_t r, Defl d) {
  hipLaunchKernelGGL(defl_final_alpha_kernel, dim3((unsigned)r), dim3(kDT), 0, st, X, ldx,
                     p, d);
}

}  // namespace spca
