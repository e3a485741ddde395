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

// The same partial sums for mostly dense iterates, as one FP64 product on the
// matrix cores: U = A Xs with Xs[c][j] = x_j[c] / ||x_j|| (x_j the FP32
// iterate, A exact in FP64).  Workgroup (t, g) owns rows [64 t, 64 t + 64)
// and starts [64 g, 64 g + 64); its 2 x 2 waves own 32 x 32, four 16 x 16
// blocks of v_mfma_f64_16x16x4f64 (operand lane l: A[l % 16][l / 16] and
// B[l / 16][l % 16]; result element e of lane l: D[4 e + l / 16][l % 16]).
// The columns advance 16 at a time through LDS, the next 16 already in
// registers.  Partial pairs per (start, 64-row tile), summed in a fixed order.
// With a column split (blockIdx.z of gridDim.z splits, pc columns each) the
// workgroups write their part of u to upart[(z r + j) n + i] instead, and
// final_pairs_kernel sums the splits in order before forming the pairs:
// more workgroups than the (row, start) tiles alone give.
typedef double double4_t __attribute__((ext_vector_type(4)));
constexpr int kGT = 64;  // rows and starts per workgroup tile
constexpr int kGK = 16;  // columns per stage

__global__ __launch_bounds__(256) void final_gemm64_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n, int64_t p,
    const float* __restrict__ X, int64_t ldx, StartState s, int64_t r,
    const double* __restrict__ xnorm, double* partial, int ntiles, Defl defl, int64_t pc,
    double* __restrict__ upart) {
  __shared__ double sA[kGK][kGT];  // A[row][col] by column
  __shared__ double sB[kGK][kGT];  // Xs[col][start] by column
  __shared__ double scale[kGT];
  __shared__ double red[2][4][kGT][2];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int wm = wave % 2, wn = wave / 2;
  const int64_t i0 = (int64_t)blockIdx.x * kGT, j0 = (int64_t)blockIdx.y * kGT;
  if (tid < kGT) {
    const int64_t j = j0 + tid;
    double sc = 0.0;
    if (j < r) {
      const double nrm = xnorm[j];
      const bool live = s.status[j] != SPCA_DEGENERATE && s.status[j] != SPCA_ZERO;
      if (live && nrm > 0.0) sc = 1.0 / nrm;
    }
    scale[tid] = sc;
  }
  // staging: A as (row tid % 64, columns 4 (tid / 64) .. + 3); X as
  // (start tid / 4, columns 4 (tid % 4) .. + 3)
  const int ar = tid % kGT, ac = 4 * (tid / kGT);
  const int xj = tid / 4, xc = 4 * (tid % 4);
  float pa[4], px[4];
  const int64_t cbeg = (int64_t)blockIdx.z * pc;
  const int64_t cend = cbeg + pc < p ? cbeg + pc : p;
  auto fetch = [&](int64_t c0) {
    const int64_t i = i0 + ar, j = j0 + xj;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t ca = c0 + ac + e, cx = c0 + xc + e;
      pa[e] = (i < n && ca < cend) ? A[i + ca * lda] : 0.f;
      px[e] = (j < r && cx < cend) ? X[j * ldx + cx] : 0.f;
    }
  };
  double4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = {0.0, 0.0, 0.0, 0.0};
  fetch(cbeg);
  __syncthreads();  // scale
  for (int64_t c0 = cbeg; c0 < cend; c0 += kGK) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      sA[ac + e][ar] = (double)pa[e];
      sB[xc + e][xj] = (double)px[e] * scale[xj];
    }
    __syncthreads();
    if (c0 + kGK < cend) fetch(c0 + kGK);
#pragma unroll
    for (int k0 = 0; k0 < kGK; k0 += 4) {
      const int k = k0 + lane / 16, q = lane % 16;
      double fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) fa[a] = sA[k][wm * 32 + a * 16 + q];
#pragma unroll
      for (int b = 0; b < 2; ++b) fb[b] = sB[k][wn * 32 + b * 16 + q];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: lane holds rows wm 32 + a 16 + 4 e + lane / 16 of start
  // wn 32 + b 16 + lane % 16
  if (gridDim.z > 1) {  // this split's part of u
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t j = j0 + wn * 32 + b * 16 + lane % 16;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t i = i0 + wm * 32 + a * 16 + 4 * e + lane / 16;
          if (i < n && j < r) upart[((int64_t)blockIdx.z * r + j) * n + i] = acc[a][b][e];
        }
    }
    return;
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int jl = wn * 32 + b * 16 + lane % 16;
    const int64_t j = j0 + jl;
    double sq = 0.0, ab = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = i0 + wm * 32 + a * 16 + 4 * e + lane / 16;
        if (i < n && j < r) {
          double u = acc[a][b][e];
          if (defl.k > 0)
            for (int l = 0; l < defl.k; ++l)
              u -= defl.alpha[j * kMaxDefl + l] * defl.scores[i * kMaxDefl + l];
          sq += u * u;
          ab += fabs(u);
        }
      }
    red[wm][lane / 16][jl][0] = sq;
    red[wm][lane / 16][jl][1] = ab;
  }
  __syncthreads();
  if (tid < kGT && j0 + tid < r) {
    double sq = 0.0, ab = 0.0;
    for (int m = 0; m < 2; ++m)
      for (int g = 0; g < 4; ++g) {
        sq += red[m][g][tid][0];
        ab += red[m][g][tid][1];
      }
    partial[((j0 + tid) * ntiles + blockIdx.x) * 2] = sq;
    partial[((j0 + tid) * ntiles + blockIdx.x) * 2 + 1] = ab;
  }
}

// The split parts of u summed in split order, the deflation correction,
// then the partial pairs (sum u_i^2, sum |u_i|) of each (start, 64-row
// tile): thread t sums rows 16 (t / 64) .. + 15 of start t % 64, and the
// four row groups are added in order.
__global__ __launch_bounds__(256) void final_pairs_kernel(const double* __restrict__ upart,
                                                          int splits, int64_t n, int64_t r,
                                                          double* partial, int ntiles,
                                                          Defl defl) {
  __shared__ double red[4][kGT][2];
  const int tid = threadIdx.x, jl = tid % kGT, g = tid / kGT;
  const int64_t i0 = (int64_t)blockIdx.x * kGT, j = (int64_t)blockIdx.y * kGT + jl;
  double sq = 0.0, ab = 0.0;
  if (j < r) {
    for (int q = 0; q < kGT / 4; ++q) {
      const int64_t i = i0 + 16 * g + q;
      if (i >= n) break;
      double u = 0.0;
      for (int z = 0; z < splits; ++z) u += upart[((int64_t)z * r + j) * n + i];
      if (defl.k > 0)
        for (int l = 0; l < defl.k; ++l)
          u -= defl.alpha[j * kMaxDefl + l] * defl.scores[i * kMaxDefl + l];
      sq += u * u;
      ab += fabs(u);
    }
  }
  red[g][jl][0] = sq;
  red[g][jl][1] = ab;
  __syncthreads();
  if (g == 0 && j < r) {
    for (int h = 1; h < 4; ++h) {
      sq += red[h][jl][0];
      ab += red[h][jl][1];
    }
    partial[(j * ntiles + blockIdx.x) * 2] = sq;
    partial[(j * ntiles + blockIdx.x) * 2 + 1] = ab;
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

int final_gemm64_splits(int64_t n, int64_t p, int64_t r) {
  const int64_t base = ceil_div(n, (int64_t)kGT) * ceil_div(r, (int64_t)kGT);
  int sp = 1;
  // at least 512 workgroups where the columns allow, each split at least
  // 256 columns, and the parts of u (splits r n doubles) within r p floats
  while (sp < 8 && base * sp < 512 && p / (2 * sp) >= 256 && 2 * sp * 2 * n <= p) sp *= 2;
  return sp;
}

void finalize(hipStream_t st, int fid, double s_or_gamma, const float* A,
              int64_t lda, int64_t n, int64_t p, const int32_t* list_idx,
              const float* list_val, int64_t ldl, StartState s, int64_t r,
              double* partial, double* f, double* ev, double* xnorm,
              int32_t* best, double* x_out, int32_t* support_out,
              const double* gam, bool by_ev, Defl defl, const float* X_dense,
              int64_t ldx, double* upart) {
  if (X_dense == nullptr) {
    evaluate_rows(st, fid, s_or_gamma, A, lda, n, list_idx, list_val, ldl, s, r,
                  partial, f, ev, xnorm, nullptr, gam, defl);
  } else {
    const int ntiles = (int)ceil_div(n, (int64_t)kGT);
    const int rtiles = (int)ceil_div(r, (int64_t)kGT);
    const int splits = upart != nullptr ? final_gemm64_splits(n, p, r) : 1;
    const int64_t pc = round_up(ceil_div(p, (int64_t)splits), (int64_t)kGK);
    hipLaunchKernelGGL(x_norms_kernel, dim3((unsigned)r), dim3(256), 0, st, list_val, ldl, s,
                       r, xnorm, nullptr);
    hipLaunchKernelGGL(final_gemm64_kernel, dim3((unsigned)ntiles, (unsigned)rtiles,
                       (unsigned)splits), dim3(256), 0, st, A, lda, n, p, X_dense, ldx, s, r,
                       xnorm, partial, ntiles, defl, pc, upart);
    if (splits > 1)
      hipLaunchKernelGGL(final_pairs_kernel, dim3((unsigned)ntiles, (unsigned)rtiles),
                         dim3(256), 0, st, upart, splits, n, r, partial, ntiles, defl);
    hipLaunchKernelGGL(objective_kernel, dim3((unsigned)ceil_div(r, 256)), dim3(256), 0, st,
                       fid, s_or_gamma, s, r, partial, ntiles, xnorm, f, ev, nullptr, gam);
  }
  hipLaunchKernelGGL(best_kernel, dim3(1), dim3(1024), 0, st, by_ev ? ev : f, s, r, p,
                     list_idx, list_val, ldl, xnorm, best, x_out, support_out);
}

}  // namespace spca
