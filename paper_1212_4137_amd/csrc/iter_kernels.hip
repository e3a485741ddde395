// Staging, planning and y-update kernels of the AM iteration (Algorithm 2):
// the layout copies of A, the start x0 = e_{i*}, the per-start state, the
// choice between the dense and the list-based product A x, and the y-update
// y = sgn(u) or u / ||u||_2 (Table 3, rows S1 and S2).
#include <algorithm>

#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

// ---------------------------------------------------------------------------
// Layout copies
// ---------------------------------------------------------------------------

// K-split partials summed in split order, four entries per thread and step
// (stride and count multiples of 4 take the 16-byte path)
__global__ __launch_bounds__(256) void sum_splits_kernel(float* __restrict__ V, int64_t stride,
                                                         int splits, int64_t count) {
  const bool vec = stride % 4 == 0 && count % 4 == 0 && ((uintptr_t)V & 15) == 0;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; 4 * q < count;
       q += (int64_t)gridDim.x * 256) {
    const int64_t i = 4 * q;
    if (vec) {
      float4 a = *reinterpret_cast<const float4*>(V + i);
      for (int sp = 1; sp < splits; ++sp) {
        const float4 b = *reinterpret_cast<const float4*>(V + sp * stride + i);
        a.x += b.x;
        a.y += b.y;
        a.z += b.z;
        a.w += b.w;
      }
      *reinterpret_cast<float4*>(V + i) = a;
    } else {
      for (int e = 0; e < 4 && i + e < count; ++e) {
        float a = V[i + e];
        for (int sp = 1; sp < splits; ++sp) a += V[sp * stride + i + e];
        V[i + e] = a;
      }
    }
  }
}

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

// BF16 conversions of A.  Column-major: one block per column (grid-stride).
__global__ __launch_bounds__(256) void to_bf16_col_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n, int64_t p,
    uint16_t* __restrict__ Ab, int64_t ldab) {
  for (int64_t k = blockIdx.x; k < p; k += gridDim.x)
    for (int64_t i = threadIdx.x; i < ldab; i += 256)
      Ab[i + k * ldab] = i < n ? f32_to_bf16(A[i + k * lda]) : (uint16_t)0;
}

// Row-major: 64 x 64 tiles transposed through LDS.
__global__ __launch_bounds__(256) void to_bf16_row_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n, int64_t p,
    uint16_t* __restrict__ Atb, int64_t ldatb) {
  __shared__ float tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64;  // rows of A
  const int64_t k0 = (int64_t)blockIdx.y * 64;  // columns of A
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  for (int kk = ty; kk < 64; kk += 4) {
    const int64_t i = i0 + tx, k = k0 + kk;
    tile[kk][tx] = (i < n && k < p) ? A[i + k * lda] : 0.f;
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t i = i0 + ii, k = k0 + tx;
    if (i < n && k < ldatb) Atb[i * ldatb + k] = k < p ? f32_to_bf16(tile[tx][ii]) : (uint16_t)0;
  }
}

__global__ __launch_bounds__(256) void rows_to_bf16_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t p,
    uint16_t* __restrict__ Xb, int64_t ldxb, const Plan* plan) {
  if (plan != nullptr && plan->mode != kAxDense) return;
  const int64_t j = blockIdx.x;
  for (int64_t i = threadIdx.x; i < ldxb; i += 256)
    Xb[j * ldxb + i] = i < p ? f32_to_bf16(X[j * ldx + i]) : (uint16_t)0;
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

// 16 consecutive entries of a row from position i0 (zeros past len); one
// 16-byte load per four entries when the whole run is inside and aligned
template <typename T>
__device__ __forceinline__ void load16(const T* __restrict__ a, int64_t i0, int64_t len,
                                       T (&v)[16]) {
  static_assert(sizeof(T) == 4, "4-byte entries");
  if (i0 + 16 <= len && ((uintptr_t)(a + i0) & 15) == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int4 w = *reinterpret_cast<const int4*>(a + i0 + 4 * q);
      v[4 * q] = __builtin_bit_cast(T, w.x);
      v[4 * q + 1] = __builtin_bit_cast(T, w.y);
      v[4 * q + 2] = __builtin_bit_cast(T, w.z);
      v[4 * q + 3] = __builtin_bit_cast(T, w.w);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = i0 + k < len ? a[i0 + k] : T(0);
  }
}

// One block per start: the (index, value) list of the row's nonzeros in
// index order.  The row is read in passes of 16 consecutive entries per
// thread (coalesced), one block scan per pass.
__global__ __launch_bounds__(1024) void compact_rows_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t p, int32_t* list_idx,
    float* list_val, int64_t ldl, int32_t* nnz, const int32_t* status,
    int32_t* colmark, const Plan* plan, const int32_t* only) {
  __shared__ int scan[20];
  const int64_t j = blockIdx.x;
  if (status != nullptr && status[j] != kRunning) return;
  if (only != nullptr && only[j] == 0) return;
  const int32_t epoch = colmark != nullptr ? plan->epoch : 0;
  const float* x = X + j * ldx;
  int run = 0;
  for (int64_t base = 0; base < p; base += 16 * (int64_t)blockDim.x) {
    const int64_t i0 = base + 16 * (int64_t)threadIdx.x;
    float v[16];
    load16(x, i0, p, v);
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) cnt += v[k] != 0.f;
    int total;
    int off = run + block_exclusive_scan(cnt, scan, &total);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (v[k] != 0.f) {
        list_idx[j * ldl + off] = (int32_t)(i0 + k);
        list_val[j * ldl + off] = v[k];
        ++off;
        if (colmark != nullptr) colmark[i0 + k] = epoch;
      }
    }
    run += total;
  }
  if (threadIdx.x == 0) nnz[j] = run;
}

__global__ void init_state_kernel(StartState s, int64_t r) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  s.phi[j] = 0.0;
  s.phi_prev[j] = 0.0;
  s.iters[j] = 0;
  s.status[j] = kRunning;
  if (s.thr != nullptr) s.thr[j] = 0.f;
}

// One block: count running starts and their nonzeros, gather the union of
// their supports, pick the product for the next A x.
//
// Cost model of the ways to form U = X A^T (r x n), in microseconds on
// MI355X: the dense MFMA product runs at about 100 TFLOP/s over all p
// columns (but reads all of A however few the starts); the union product at about 80 TFLOP/s over the u union columns
// plus its gathers (about 2 TB/s) and a fixed 6 us; the list product reads
// a column of A per list entry, at about 12 TB/s while the distinct columns
// it touches (the last measured union, else all list entries) stay within
// the 256 MB Infinity Cache (192 MB taken as usable) and at about 3 TB/s
// beyond that.
// The union is only gathered when the last x-update marked columns: while
// the union product wins, every iteration, otherwise on the first two
// planner calls and every 16th (a probe).
__global__ __launch_bounds__(1024) void plan_kernel(
    StartState s, int64_t r, int64_t n, int64_t p, int list_cap,
    int dense_only, int dense_splits, int64_t ucap,
    const int32_t* __restrict__ colmark, int32_t* __restrict__ ulist,
    Plan* plan, int no_fused, int allow_union) {
  __shared__ int64_t red[2 * 17];
  __shared__ int32_t mred[17];
  __shared__ int scan[20];
  int64_t v[2] = {0, 0};
  int32_t mx = 0;
  for (int64_t j = threadIdx.x; j < r; j += blockDim.x) {
    if (s.status[j] == kRunning) {
      v[0] += 1;
      v[1] += s.nnz[j];
      mx = s.nnz[j] > mx ? s.nnz[j] : mx;
    }
  }
  block_sum_n<int64_t, 2>(v, red);
  mx = block_max(mx, mred);
  // union of the marked columns, in index order
  const int32_t epoch = plan->epoch;
  const bool marked = colmark != nullptr && plan->mark != 0;
  int u = -1;
  if (marked) {
    // passes of 16 consecutive columns per thread (coalesced)
    u = 0;
    for (int64_t base = 0; base < p; base += 16 * (int64_t)blockDim.x) {
      const int64_t i0 = base + 16 * (int64_t)threadIdx.x;
      int32_t m[16];
      load16(colmark, i0, p, m);
      int cnt = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) cnt += i0 + k < p && m[k] == epoch;
      int total;
      int off = u + block_exclusive_scan(cnt, scan, &total);
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (i0 + k < p && m[k] == epoch) ulist[off++] = (int32_t)(i0 + k);
      u += total;
    }
  }
  if (threadIdx.x == 0) {
    plan->active = (int32_t)v[0];
    plan->total_nnz = v[1];
    plan->max_nnz = mx;
    plan->union_size = u < 0 ? 0 : u;
    if (u >= 0) plan->last_union = u;
    const double rd = (double)r, nd = (double)n;
    // the dense product: MFMA time (starts padded to a 32-row tile) or one
    // read of A at about 4 TB/s, whichever is longer, plus launch costs
    const double mfma_us = 2.0 * (rd > 32.0 ? rd : 32.0) * nd * (double)p / 1.0e8;
    const double read_us = nd * (double)p * 4.0 / 4.0e6;
    const double dense_us = (mfma_us > read_us ? mfma_us : read_us) + 5.0;
    const double union_us = u >= 1 && u <= ucap
                                ? 2.0 * rd * nd * u / 0.8e8 + 6.0 +
                                      (rd + nd) * u * 8.0 / 2.0e6
                                : 1e300;
    const double cols = plan->last_union > 0 ? (double)plan->last_union
                                             : (double)(v[1] < p ? v[1] : p);
    const double list_bw = cols * nd * 4.0 <= 192.0e6 ? 12.0e6 : 3.0e6;
    // the one-workgroup-per-start kernel needs about 512 workgroups to reach
    // that rate; the row-block kernel has r * ceil(n / 1024) of them and
    // pays the separate y-update
    const double wg1 = (double)v[0], wgr = (double)v[0] * ceil(nd / 1024.0);
    const double list_us =
        mx <= list_cap && !no_fused
            ? (double)v[1] * nd * 4.0 / (list_bw * (wg1 < 512.0 ? wg1 / 512.0 : 1.0)) + 3.0
            : 1e300;
    const double rows_us =
        mx <= list_cap && rows_product_possible(n, no_fused)
            ? (double)v[1] * nd * 4.0 / (list_bw * (wgr < 512.0 ? wgr / 512.0 : 1.0)) + 8.0
            : 1e300;
    int mode = kAxDense;
    double best = dense_us;
    if (!dense_only) {
      // the best product without the union one: dense, list or row-block
      double other = dense_us;
      other = list_us < other ? list_us : other;
      other = rows_us < other ? rows_us : other;
      if (allow_union && union_us < best) {
        best = union_us;
        mode = kAxUnion;
      }
      if (list_us < best) {
        best = list_us;
        mode = kAxList;
      }
      if (rows_us < best) {
        best = rows_us;
        mode = kAxListRows;
      }
      // evidence for the host's decision to keep launching the union
      // product (it reads this at its polls)
      if (mode == kAxUnion)
        plan->union_close = 1;
      else if (u >= 0)
        plan->union_close = union_us < 1.25 * other ? 1 : 0;
    }
    plan->mode = mode;
    plan->ax_splits = mode == kAxDense ? dense_splits : 1;
    plan->mode_count[mode] += v[0] > 0 ? 1 : 0;
    plan->active_sum += (double)v[0];
    plan->nnz_sum += (double)v[1];
    plan->epoch = epoch + 1;
    const int32_t it = plan->iter + 1;
    plan->iter = it;
    plan->mark = (colmark != nullptr && !dense_only &&
                  (mode == kAxUnion || it % 16 == 0 || it <= 2)) ? 1 : 0;
  }
}

__global__ void init_plan_kernel(Plan* plan, int dense_splits) {
  plan->mode = kAxDense;
  plan->active = 0;
  plan->union_close = 0;
  plan->total_nnz = 0;
  plan->max_nnz = 0;
  plan->union_size = 0;
  plan->last_union = 0;
  plan->epoch = 1;
  plan->ax_splits = dense_splits;
  plan->mark = 1;
  plan->iter = 0;
  plan->mode_count[0] = plan->mode_count[1] = plan->mode_count[2] = 0;
  plan->mode_count[3] = 0;
  plan->active_sum = 0.0;
  plan->nnz_sum = 0.0;
}

// Union gathers: the blocks copy the union columns of the rows of X, then
// transpose 64 x 64 tiles of A's union columns into the row-major Qc.
constexpr int kGT = 64;
__global__ __launch_bounds__(256) void union_gather_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t r,
    const float* __restrict__ A, int64_t lda, int64_t n,
    const int32_t* __restrict__ ulist, const Plan* plan, float* __restrict__ Xc,
    int64_t ldxc, float* __restrict__ Qc, int64_t ldqc) {
  __shared__ float tile[kGT][kGT + 1];
  if (plan->mode != kAxUnion) return;
  const int u = plan->union_size;
  for (int64_t j = blockIdx.x; j < r; j += gridDim.x)
    for (int c = threadIdx.x; c < u; c += 256) Xc[j * ldxc + c] = X[j * ldx + ulist[c]];
  const int64_t tiles_i = ceil_div(n, kGT);
  const int64_t tiles = tiles_i * ceil_div(u, kGT);
  const int tx = threadIdx.x % kGT, ty = threadIdx.x / kGT;  // ty in 0..3
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t i0 = (t % tiles_i) * kGT;
    const int64_t c0 = (t / tiles_i) * kGT;
    __syncthreads();
    for (int cc = ty; cc < kGT; cc += 4) {
      const int64_t c = c0 + cc, i = i0 + tx;
      tile[cc][tx] = (c < u && i < n) ? A[i + (int64_t)ulist[c] * lda] : 0.f;
    }
    __syncthreads();
    for (int ii = ty; ii < kGT; ii += 4) {
      const int64_t i = i0 + ii, c = c0 + tx;
      if (i < n && c < u) Qc[i * ldqc + c] = tile[tx][ii];
    }
  }
}

// ---------------------------------------------------------------------------
// y-update (Algorithm 2; Table 3, S1 for L2 variance, S2 for L1 variance)
// ---------------------------------------------------------------------------

typedef float yvec4 __attribute__((ext_vector_type(4)));

// u = the split partials summed in split order, for the four consecutive
// entries i .. i + 3 of a row (entries at n and beyond read as 0).  The
// loads of all partials are issued before the first add, so a thread waits
// for memory once per group instead of once per partial.  Rows and split
// strides are multiples of 4 floats and 16-byte aligned.
__device__ __forceinline__ yvec4 sum_partials4(const float* __restrict__ u, int64_t i,
                                               int64_t n, int splits, int64_t stride) {
  yvec4 part[kSplitsMax];
#pragma unroll
  for (int sp = 0; sp < kSplitsMax; ++sp)
    if (sp < splits) part[sp] = *reinterpret_cast<const yvec4*>(u + i + sp * stride);
  yvec4 t = part[0];
#pragma unroll
  for (int sp = 1; sp < kSplitsMax; ++sp)
    if (sp < splits) t += part[sp];
  if (i + 3 >= n) {
    if (i + 1 >= n) t.y = 0.f;
    if (i + 2 >= n) t.z = 0.f;
    if (i + 3 >= n) t.w = 0.f;
  }
  return t;
}

__device__ __forceinline__ void store4(float* __restrict__ y, int64_t i, int64_t n, yvec4 t) {
  if (i + 3 < n) {
    *reinterpret_cast<yvec4*>(y + i) = t;
  } else {
    y[i] = t.x;
    if (i + 1 < n) y[i + 1] = t.y;
    if (i + 2 < n) y[i + 2] = t.z;
  }
}

// One block per start.  Thread t owns the groups of four entries starting
// at 4 (t + 256 k), in increasing order whatever the row length; it keeps
// its sums in y until the FP64 norm (entries squared in index order per
// thread, then the block sum) is known.
template <bool L1VAR>
__device__ __forceinline__ void y_update_row(const float* __restrict__ u, int64_t stride,
                                             int splits, float* __restrict__ y, int64_t n,
                                             int32_t* status, uint16_t* __restrict__ yb,
                                             double* red) {
  double sq = 0.0;
  for (int64_t i = 4 * (int64_t)threadIdx.x; i < n; i += 4 * 256) {
    const yvec4 t = sum_partials4(u, i, n, splits, stride);
    store4(y, i, n, t);
    const double t0 = t.x, t1 = t.y, t2 = t.z, t3 = t.w;
    sq += t0 * t0;
    sq += t1 * t1;
    sq += t2 * t2;
    sq += t3 * t3;
  }
  sq = block_sum(sq, red);
  if (sq == 0.0) {
    if (threadIdx.x == 0) *status = SPCA_DEGENERATE;
    return;
  }
  const double inv = 1.0 / sqrt(sq);
  for (int64_t i = 4 * (int64_t)threadIdx.x; i < n; i += 4 * 256) {
    const yvec4 t = *reinterpret_cast<const yvec4*>(y + i);
    yvec4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      o[e] = L1VAR ? (float)((t[e] > 0.f) - (t[e] < 0.f)) : (float)((double)t[e] * inv);
    store4(y, i, n, o);
    if (yb != nullptr)
      for (int e = 0; e < 4 && i + e < n; ++e) yb[i + e] = f32_to_bf16(o[e]);
  }
}

template <bool L1VAR>
__global__ __launch_bounds__(256) void y_update_kernel(
    const float* __restrict__ U, int64_t split_stride, float* __restrict__ Y,
    int64_t ldu, int64_t n, StartState s, const Plan* plan,
    uint16_t* __restrict__ Yb, int64_t ldyb) {
  __shared__ double red[8];
  if (plan->mode == kAxList) return;
  const int splits = plan->ax_splits;
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  y_update_row<L1VAR>(U + j * ldu, split_stride, splits, Y + j * ldu, n, s.status + j,
                      Yb != nullptr ? Yb + j * ldyb : nullptr, red);
}

// Grouped solves: y_update_kernel with the variance type and the partial
// count taken per start from its request.
__global__ __launch_bounds__(256) void group_y_update_kernel(
    const float* __restrict__ U, int64_t split_stride, float* __restrict__ Y,
    int64_t ldu, int64_t n, StartState s) {
  __shared__ double red[8];
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  const int splits = s.cfg[j].splits;
  if (s.cfg[j].l1 != 0)
    y_update_row<true>(U + j * ldu, split_stride, splits, Y + j * ldu, n, s.status + j,
                       nullptr, red);
  else
    y_update_row<false>(U + j * ldu, split_stride, splits, Y + j * ldu, n, s.status + j,
                        nullptr, red);
}

// Grouped solves: one block per start sums its A^T y partials in order.
__global__ __launch_bounds__(256) void group_sum_splits_kernel(float* __restrict__ V,
                                                               int64_t stride, int64_t ldv,
                                                               int64_t p, StartState s) {
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  const int splits = s.cfg[j].aty_splits;
  if (splits <= 1) return;
  float* v = V + j * ldv;
  for (int64_t i = 4 * (int64_t)threadIdx.x; i < p; i += 4 * 256)
    store4(v, i, p, sum_partials4(v, i, p, splits, stride));
}

// Running starts per request and in total; one block of 16 waves, a wave
// per request at a time.
__global__ __launch_bounds__(1024) void group_count_kernel(const int32_t* __restrict__ status,
                                                           const int64_t* __restrict__ first,
                                                           int count,
                                                           int32_t* __restrict__ running) {
  __shared__ int32_t tot[16];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  int32_t mine = 0;
  for (int q = wave; q < count; q += 16) {
    int32_t c = 0;
    for (int64_t j = first[q] + lane; j < first[q + 1]; j += kWave) c += status[j] == kRunning;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) running[q] = c;
    mine += c;
  }
  if (lane == 0) tot[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int w = 0; w < 16; ++w) t += tot[w];
    running[count] = t;
  }
}

// Sparse A x (x given by its list) fused with the y-update; one block per
// start.  Thread t owns groups of 4 consecutive rows (one 16-byte load per
// list entry and group), so a column of A is read with 16-byte loads; list
// entries are taken four at a time so that 4 R independent loads are in
// flight.  FP64 accumulation.  Needs lda % 4 == 0 and a 16-byte aligned A.
constexpr int kSpThreads = 256;
constexpr int kSpStage = 256;   // list entries staged in LDS at a time
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// four consecutive entries of a column as floats (FP32 or BF16 storage)
__device__ __forceinline__ floatx4_t load4(const float* c, int64_t row) {
  return *reinterpret_cast<const floatx4_t*>(c + row);
}
__device__ __forceinline__ floatx4_t load4(const uint16_t* c, int64_t row) {
  const uint2 w = *reinterpret_cast<const uint2*>(c + row);
  floatx4_t f = {__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u),
                 __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xffff0000u)};
  return f;
}
__device__ __forceinline__ float load1(const float* c, int64_t row) { return c[row]; }
__device__ __forceinline__ float load1(const uint16_t* c, int64_t row) {
  return bf16_to_f32(c[row]);
}

template <bool L1VAR, int R, typename TA>
__global__ __launch_bounds__(kSpThreads) void sparse_ax_y_kernel(
    const TA* __restrict__ A, int64_t lda, int64_t n,
    const int32_t* __restrict__ list_idx, const float* __restrict__ list_val,
    int64_t ldl, float* __restrict__ Y, int64_t ldu, StartState s,
    const Plan* plan, uint16_t* __restrict__ Yb, int64_t ldyb) {
  __shared__ int32_t sidx[kSpStage];
  __shared__ double sval[kSpStage];
  __shared__ double red[8];
  if (plan->mode != kAxList) return;
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  const int32_t cnt = s.nnz[j];
  const int32_t* li = list_idx + j * ldl;
  const float* lv = list_val + j * ldl;
  float* y = Y + j * ldu;
  const int64_t groups = ceil_div(n, 4);

  double sq = 0.0;
  for (int64_t gbase = 0; gbase < groups; gbase += (int64_t)kSpThreads * R) {
    double acc[R][4];
    int64_t g[R];
    bool ok[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      g[q] = gbase + q * kSpThreads + threadIdx.x;
      ok[q] = g[q] < groups;
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[q][e] = 0.0;
    }
    for (int32_t t0 = 0; t0 < cnt; t0 += kSpStage) {
      const int32_t m = cnt - t0 < kSpStage ? cnt - t0 : kSpStage;
      __syncthreads();
      if (threadIdx.x < m) {
        sidx[threadIdx.x] = li[t0 + threadIdx.x];
        sval[threadIdx.x] = (double)lv[t0 + threadIdx.x];
      }
      __syncthreads();
      int32_t t = 0;
      for (; t + 4 <= m; t += 4) {
        const TA* c[4];
        double xv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          c[e] = A + (int64_t)sidx[t + e] * lda;
          xv[e] = sval[t + e];
        }
        floatx4_t a[4][R];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int q = 0; q < R; ++q) {
            if (ok[q]) {
              const int64_t row = 4 * g[q];
              if (row + 3 < n) {
                a[e][q] = load4(c[e], row);
              } else {
                floatx4_t z = {0.f, 0.f, 0.f, 0.f};
                if (row < n) z.x = load1(c[e], row);
                if (row + 1 < n) z.y = load1(c[e], row + 1);
                if (row + 2 < n) z.z = load1(c[e], row + 2);
                a[e][q] = z;
              }
            } else {
              a[e][q] = floatx4_t{0.f, 0.f, 0.f, 0.f};
            }
          }
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            acc[q][0] += (double)a[e][q].x * xv[e];
            acc[q][1] += (double)a[e][q].y * xv[e];
            acc[q][2] += (double)a[e][q].z * xv[e];
            acc[q][3] += (double)a[e][q].w * xv[e];
          }
      }
      for (; t < m; ++t) {
        const TA* c0 = A + (int64_t)sidx[t] * lda;
        const double x0 = sval[t];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          if (!ok[q]) continue;
          const int64_t row = 4 * g[q];
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (row + e < n) acc[q][e] += (double)load1(c0, row + e) * x0;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (!ok[q]) continue;
      const int64_t row = 4 * g[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (row + e < n) {
          float u = (float)acc[q][e];
          y[row + e] = u;  // u for now; scaled below once ||u|| is known
          double uu = u;
          sq += uu * uu;
        }
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
  for (int64_t gbase = 0; gbase < groups; gbase += (int64_t)kSpThreads * R) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t gq = gbase + q * kSpThreads + threadIdx.x;
      if (gq >= groups) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = 4 * gq + e;
        if (i < n) {
          float t = y[i];
          const float o = L1VAR ? (float)((t > 0.f) - (t < 0.f)) : (float)((double)t * inv);
          y[i] = o;
          if (Yb != nullptr) Yb[j * ldyb + i] = f32_to_bf16(o);
        }
      }
    }
  }
}

template <bool L1VAR, typename TA>
void launch_sparse(hipStream_t st, const TA* A, int64_t lda, int64_t n,
                   const int32_t* li, const float* lv, int64_t ldl, float* Y,
                   int64_t ldu, int64_t r, StartState s, const Plan* plan,
                   uint16_t* Yb, int64_t ldyb) {
  const int64_t per = ceil_div(ceil_div(n, 4), kSpThreads);
  dim3 g((unsigned)r), b(kSpThreads);
  if (per <= 1)
    hipLaunchKernelGGL((sparse_ax_y_kernel<L1VAR, 1, TA>), g, b, 0, st, A, lda, n, li, lv, ldl, Y, ldu, s, plan, Yb, ldyb);
  else
    hipLaunchKernelGGL((sparse_ax_y_kernel<L1VAR, 2, TA>), g, b, 0, st, A, lda, n, li, lv, ldl, Y, ldu, s, plan, Yb, ldyb);
}

// Row-block list product: workgroup (c, j) forms rows [1024 c, 1024 c + 1024)
// of u_j = sum_t A[:, idx_t] val_t, each thread four consecutive rows with
// 16-byte loads, in list order, in FP64.
constexpr int kRowsBlock = 4 * kSpThreads;
static_assert(kRowsBlock == kRowsBlockN, "row-block height");

template <typename TA>
__global__ __launch_bounds__(kSpThreads) void sparse_ax_rows_kernel(
    const TA* __restrict__ A, int64_t lda, int64_t n,
    const int32_t* __restrict__ list_idx, const float* __restrict__ list_val,
    int64_t ldl, float* __restrict__ U, int64_t ldu, StartState s,
    const Plan* plan) {
  __shared__ int32_t sidx[kSpStage];
  __shared__ float sval[kSpStage];
  if (plan->mode != kAxListRows) return;
  const int64_t j = blockIdx.y;
  if (s.status[j] != kRunning) return;
  const int32_t cnt = s.nnz[j];
  const int64_t row = (int64_t)blockIdx.x * kRowsBlock + 4 * threadIdx.x;
  const bool full = row + 3 < n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t t0 = 0; t0 < cnt; t0 += kSpStage) {
    const int32_t m = cnt - t0 < kSpStage ? cnt - t0 : kSpStage;
    __syncthreads();
    if ((int)threadIdx.x < m) {
      sidx[threadIdx.x] = list_idx[j * ldl + t0 + threadIdx.x];
      sval[threadIdx.x] = list_val[j * ldl + t0 + threadIdx.x];
    }
    __syncthreads();
    if (row < n) {
      for (int32_t t = 0; t < m; ++t) {
        const TA* c = A + (int64_t)sidx[t] * lda;
        const double w = (double)sval[t];
        if (full) {
          const floatx4_t a = load4(c, row);
          acc[0] += (double)a.x * w;
          acc[1] += (double)a.y * w;
          acc[2] += (double)a.z * w;
          acc[3] += (double)a.w * w;
        } else {
          for (int e = 0; e < 4; ++e)
            if (row + e < n) acc[e] += (double)load1(c, row + e) * w;
        }
      }
    }
  }
  float* u = U + j * ldu;
  if (full) {
    const floatx4_t o = {(float)acc[0], (float)acc[1], (float)acc[2], (float)acc[3]};
    *reinterpret_cast<floatx4_t*>(u + row) = o;
  } else {
    for (int e = 0; e < 4; ++e)
      if (row + e < n) u[row + e] = (float)acc[e];
  }
}

template <typename TA>
void launch_rows(hipStream_t st, const TA* A, int64_t lda, int64_t n,
                 const int32_t* li, const float* lv, int64_t ldl, float* U,
                 int64_t ldu, int64_t r, StartState s, const Plan* plan) {
  const dim3 g((unsigned)ceil_div(n, (int64_t)kRowsBlock), (unsigned)r);
  hipLaunchKernelGGL(sparse_ax_rows_kernel<TA>, g, dim3(kSpThreads), 0, st, A, lda, n,
                     li, lv, ldl, U, ldu, s, plan);
}

}  // namespace

void sparse_ax_rows(hipStream_t st, const float* A, int64_t lda, int64_t n,
                    const int32_t* list_idx, const float* list_val, int64_t ldl,
                    float* U, int64_t ldu, int64_t r, StartState s, const Plan* plan) {
  launch_rows<float>(st, A, lda, n, list_idx, list_val, ldl, U, ldu, r, s, plan);
}

void sparse_ax_rows_bf16(hipStream_t st, const uint16_t* Ab, int64_t ldab, int64_t n,
                         const int32_t* list_idx, const float* list_val, int64_t ldl,
                         float* U, int64_t ldu, int64_t r, StartState s,
                         const Plan* plan) {
  launch_rows<uint16_t>(st, Ab, ldab, n, list_idx, list_val, ldl, U, ldu, r, s, plan);
}

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
                  int32_t* nnz, const int32_t* status, int32_t* colmark,
                  const Plan* plan, const int32_t* only) {
  hipLaunchKernelGGL(compact_rows_kernel, dim3((unsigned)r), dim3(1024), 0, st,
                     X, ldx, p, list_idx, list_val, ldl, nnz, status, colmark,
                     plan, only);
}

void init_state(hipStream_t st, StartState s, int64_t r) {
  hipLaunchKernelGGL(init_state_kernel, dim3((unsigned)ceil_div(r, 256)),
                     dim3(256), 0, st, s, r);
}

void plan_next(hipStream_t st, StartState s, int64_t r, int64_t n, int64_t p,
               int list_cap, int dense_only, int dense_splits, int64_t ucap,
               const int32_t* colmark, int32_t* ulist, Plan* plan, int no_fused,
               int allow_union) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, st, s, r, n, p,
                     list_cap, dense_only, dense_splits, ucap, colmark, ulist,
                     plan, no_fused, allow_union);
}

void init_plan(hipStream_t st, Plan* plan, int dense_splits) {
  hipLaunchKernelGGL(init_plan_kernel, dim3(1), dim3(1), 0, st, plan, dense_splits);
}

void union_gather(hipStream_t st, const float* X, int64_t ldx, int64_t r,
                  const float* A, int64_t lda, int64_t n,
                  const int32_t* ulist, const Plan* plan, float* Xc,
                  int64_t ldxc, float* Qc, int64_t ldqc) {
  const unsigned blocks = 512;
  hipLaunchKernelGGL(union_gather_kernel, dim3(blocks),
                     dim3(256), 0, st, X, ldx, r, A, lda, n, ulist, plan, Xc,
                     ldxc, Qc, ldqc);
}

void sum_splits(hipStream_t st, float* V, int64_t stride, int splits, int64_t count) {
  if (splits <= 1 || count <= 0) return;
  const int64_t n4 = ceil_div(count, (int64_t)4);
  const unsigned g = (unsigned)std::min<int64_t>(ceil_div(n4, (int64_t)256), 8192);
  hipLaunchKernelGGL(sum_splits_kernel, dim3(g), dim3(256), 0, st, V, stride, splits, count);
}

void y_update(hipStream_t st, int fid, const float* U, int64_t split_stride,
              float* Y, int64_t ldu, int64_t r, int64_t n, StartState s,
              const Plan* plan, uint16_t* Yb, int64_t ldyb) {
  if (l1_variance(fid))
    hipLaunchKernelGGL(y_update_kernel<true>, dim3((unsigned)r), dim3(256), 0,
                       st, U, split_stride, Y, ldu, n, s, plan, Yb, ldyb);
  else
    hipLaunchKernelGGL(y_update_kernel<false>, dim3((unsigned)r), dim3(256), 0,
                       st, U, split_stride, Y, ldu, n, s, plan, Yb, ldyb);
}

void group_y_update(hipStream_t st, const float* U, int64_t split_stride, float* Y,
                    int64_t ldu, int64_t r, int64_t n, StartState s) {
  hipLaunchKernelGGL(group_y_update_kernel, dim3((unsigned)r), dim3(256), 0, st, U,
                     split_stride, Y, ldu, n, s);
}

void group_sum_splits(hipStream_t st, float* V, int64_t split_stride, int64_t ldv,
                      int64_t r, int64_t p, StartState s) {
  hipLaunchKernelGGL(group_sum_splits_kernel, dim3((unsigned)r), dim3(256), 0, st, V,
                     split_stride, ldv, p, s);
}

void group_count(hipStream_t st, const int32_t* status, const int64_t* first, int count,
                 int32_t* running) {
  hipLaunchKernelGGL(group_count_kernel, dim3(1), dim3(1024), 0, st, status, first, count,
                     running);
}

void to_bf16_colmajor(hipStream_t st, const float* A, int64_t lda, int64_t n,
                      int64_t p, uint16_t* Ab, int64_t ldab) {
  hipLaunchKernelGGL(to_bf16_col_kernel, dim3((unsigned)(p < 65536 ? p : 65536)),
                     dim3(256), 0, st, A, lda, n, p, Ab, ldab);
}

void to_bf16_rowmajor(hipStream_t st, const float* A, int64_t lda, int64_t n,
                      int64_t p, uint16_t* Atb, int64_t ldatb) {
  dim3 grid((unsigned)ceil_div(n, 64), (unsigned)ceil_div(ldatb, 64));
  hipLaunchKernelGGL(to_bf16_row_kernel, grid, dim3(256), 0, st, A, lda, n, p,
                     Atb, ldatb);
}

void rows_to_bf16(hipStream_t st, const float* X, int64_t ldx, int64_t r,
                  int64_t p, uint16_t* Xb, int64_t ldxb, const Plan* plan) {
  hipLaunchKernelGGL(rows_to_bf16_kernel, dim3((unsigned)r), dim3(256), 0, st,
                     X, ldx, p, Xb, ldxb, plan);
}

__global__ __launch_bounds__(256) void gather_columns_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n,
    const int32_t* __restrict__ idx, int64_t m, float* __restrict__ As,
    int64_t ldas) {
  for (int64_t t = blockIdx.x; t < m; t += gridDim.x) {
    const float* col = A + (int64_t)idx[t] * lda;
    for (int64_t i = threadIdx.x; i < ldas; i += 256)
      As[t * ldas + i] = i < n ? col[i] : 0.f;
  }
}

void gather_columns(hipStream_t st, const float* A, int64_t lda, int64_t n,
                    const int32_t* idx, int64_t m, float* As, int64_t ldas) {
  if (m <= 0) return;
  hipLaunchKernelGGL(gather_columns_kernel, dim3((unsigned)(m < 65536 ? m : 65536)),
                     dim3(256), 0, st, A, lda, n, idx, m, As, ldas);
}

void sparse_ax_y_update(hipStream_t st, int fid, const float* A, int64_t lda,
                        int64_t n, const int32_t* list_idx,
                        const float* list_val, int64_t ldl, float* Y,
                        int64_t ldu, int64_t r, StartState s, const Plan* plan) {
  if (l1_variance(fid))
    launch_sparse<true, float>(st, A, lda, n, list_idx, list_val, ldl, Y, ldu, r, s, plan, nullptr, 0);
  else
    launch_sparse<false, float>(st, A, lda, n, list_idx, list_val, ldl, Y, ldu, r, s, plan, nullptr, 0);
}

void sparse_ax_y_update_bf16(hipStream_t st, int fid, const uint16_t* Ab,
                             int64_t ldab, int64_t n, const int32_t* list_idx,
                             const float* list_val, int64_t ldl, float* Y,
                             int64_t ldu, uint16_t* Yb, int64_t ldyb, int64_t r,
                             StartState s, const Plan* plan) {
  if (l1_variance(fid))
    launch_sparse<true, uint16_t>(st, Ab, ldab, n, list_idx, list_val, ldl, Y, ldu, r, s, plan, Yb, ldyb);
  else
    launch_sparse<false, uint16_t>(st, Ab, ldab, n, list_idx, list_val, ldl, Y, ldu, r, s, plan, Yb, ldyb);
}

}  // namespace spca
