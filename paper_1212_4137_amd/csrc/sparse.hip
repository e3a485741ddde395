// The two products of the AM iteration for a sparse A (the paper's text
// corpora are word-count matrices), stored twice: compressed sparse columns
// for A^T Y and for A x from a sparse x, compressed sparse rows for A x from a
// dense x.  The iterates keep the start-major layout of the dense path, so the
// y-update, x-update, planner and stop test are shared.
//
// Products with a dense operand (A^T Y from the columns, A X from the rows)
// are balanced over the nonzeros, not over the columns or rows: word counts
// follow Zipf's law, so a few columns hold a large share of all nonzeros and
// a column-per-wave split leaves one wave with most of the work.  Each wave
// takes a fixed chunk of kW consecutive nonzeros of the compressed layout;
// every lane group of the wave takes one nonzero at a time and the lanes of a
// group are the starts, so every stored entry of A meets one contiguous row
// of the transposed operand.  A column (or row) that lies inside one chunk is
// written directly; one that crosses chunk boundaries leaves a partial per
// chunk, summed afterwards in chunk order.  Results go to a transposed
// buffer (major index x starts), then to start-major order through LDS.
//
// A x from a sparse x (the support lists) and the FP64 final evaluation are
// split by blocks of rows: a workgroup owns one start and one block of rows,
// accumulates the block of u in LDS column by column (the rows of a column
// are distinct, so no two threads add to the same entry at once), and finds
// its range in each column by a 64-way search of the sorted row indices.
//
// Every sum runs in a fixed order.
#include <algorithm>

#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr int64_t kW = 2048;  // nonzeros per wave chunk
constexpr int kWPB = 4;       // waves per workgroup
constexpr int kTT = 64;       // tile of the transposed-to-start-major copy
constexpr int kRB = 8192;     // rows per block, FP32 list product (32 KB LDS)
constexpr int kRB64 = 4096;   // rows per block, FP64 evaluation (32 KB LDS)
// gathers of rows spread over more than about 16 MB run several times slower
// than within it (address translation reach, measured on MI355X); a panel's
// slice of YT stays well inside that window
#ifndef SPCA_PANEL_BYTES
#define SPCA_PANEL_BYTES (8 << 20)
#endif
constexpr int64_t kPanelBytes = SPCA_PANEL_BYTES;
constexpr int kScanB = 4096;  // elements per block of the panel offset scan

// --------------------------------------------------------------------------
// validation and chunk tables
// --------------------------------------------------------------------------

// ptr non-decreasing (bit 1)
__global__ __launch_bounds__(256) void sp_check_ptr_kernel(const int64_t* __restrict__ ptr,
                                                           int64_t m, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m && ptr[i] > ptr[i + 1]) atomicOr(bad, 1);
}

// every index in [0, lim) (bit 2)
__global__ __launch_bounds__(256) void sp_check_idx_kernel(const int32_t* __restrict__ idx,
                                                           int64_t nnz, int64_t lim,
                                                           int32_t* bad) {
  bool ok = true;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * 256)
    ok = ok && idx[k] >= 0 && idx[k] < lim;
  if (!ok) atomicOr(bad, 2);
}

// first[w] = the nonempty major (column or row) holding nonzero w * kW
__global__ __launch_bounds__(256) void sp_first_kernel(const int64_t* __restrict__ ptr,
                                                       int64_t m, int64_t nchunks,
                                                       int32_t* __restrict__ first) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  const int64_t cb = ptr[c], ce = ptr[c + 1];
  for (int64_t w = ceil_div(cb < 0 ? 0 : cb, kW); w * kW < ce && w < nchunks; ++w)
    first[w] = (int32_t)c;
}

// strictly increasing indices within each major (bit 4), walking the chunks
// as the products do; bounded for any ptr, so it runs before ptr is known
// to be valid
__global__ __launch_bounds__(256) void sp_check_sorted_kernel(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t m,
    int64_t nnz, const int32_t* __restrict__ first, int32_t* bad) {
  const int lane = threadIdx.x % kWave;
  const int64_t w =
      (int64_t)blockIdx.x * kWPB + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t lo = w * kW;
  if (lo >= nnz) return;
  const int64_t hi = lo + kW < nnz ? lo + kW : nnz;
  int64_t c = first[w];
  if (c < 0 || c >= m) c = 0;
  bool ok = true;
  for (int64_t k = lo; k < hi && c < m; ++c) {
    const int64_t ce = ptr[c + 1] < nnz ? ptr[c + 1] : nnz;
    const int64_t e = ce < hi ? ce : hi;
    for (int64_t t = k + lane; t < e; t += kWave)
      ok = ok && (t + 1 >= ce || idx[t] < idx[t + 1]);
    k = e > k ? e : k;
  }
  if (!ok) atomicOr(bad, 4);
}

// --------------------------------------------------------------------------
// row panels of the columns (for A^T Y): the chunks run in panel order, so
// at any time the gathers fall into one or two panels' slices of YT
// --------------------------------------------------------------------------

// first position in [lo, hi) whose index is >= target (hi if none)
__device__ __forceinline__ int64_t lower_bound_idx(const int32_t* __restrict__ a, int64_t lo,
                                                   int64_t hi, int64_t target) {
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// src[M], cnt[M] for M = P p + c: where column c's rows of panel P begin in
// the columns, and how many there are
__global__ __launch_bounds__(256) void sp_pan_bounds_kernel(
    const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx, int64_t p,
    int32_t npan, int64_t prow, int64_t* __restrict__ src, int64_t* __restrict__ cnt) {
  const int64_t M = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (M >= npan * p) return;
  const int64_t P = M / p, c = M % p;
  const int64_t cb = col_ptr[c], ce = col_ptr[c + 1];
  const int64_t b = P == 0 ? cb : lower_bound_idx(row_idx, cb, ce, P * prow);
  const int64_t e = P + 1 == npan ? ce : lower_bound_idx(row_idx, b, ce, (P + 1) * prow);
  src[M] = b;
  cnt[M] = e - b;
}

// block totals of cnt (kScanB elements per block of 1024 threads)
__global__ __launch_bounds__(1024) void sp_scan_sums_kernel(const int64_t* __restrict__ cnt,
                                                            int64_t len, int64_t* bsum) {
  __shared__ int64_t scan[17];
  const int64_t base = (int64_t)blockIdx.x * kScanB + 4 * threadIdx.x;
  int64_t v = 0;
  for (int e = 0; e < 4; ++e)
    if (base + e < len) v += cnt[base + e];
  int64_t total;
  block_exclusive_scan<int64_t>(v, scan, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// bsum -> exclusive offsets, bsum[nb] = the grand total (one thread)
__global__ void sp_scan_top_kernel(int64_t* bsum, int64_t nb) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t run = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t t = bsum[b];
    bsum[b] = run;
    run += t;
  }
  bsum[nb] = run;
}

// pptr = exclusive scan of cnt, pptr[len] = total
__global__ __launch_bounds__(1024) void sp_scan_out_kernel(const int64_t* __restrict__ cnt,
                                                           int64_t len,
                                                           const int64_t* __restrict__ bsum,
                                                           int64_t nb, int64_t* pptr) {
  __shared__ int64_t scan[17];
  const int64_t base = (int64_t)blockIdx.x * kScanB + 4 * threadIdx.x;
  int64_t c4[4], v = 0;
  for (int e = 0; e < 4; ++e) {
    c4[e] = base + e < len ? cnt[base + e] : 0;
    v += c4[e];
  }
  int64_t total;
  int64_t off = block_exclusive_scan<int64_t>(v, scan, &total) + bsum[blockIdx.x];
  for (int e = 0; e < 4; ++e) {
    if (base + e < len) pptr[base + e] = off;
    off += c4[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) pptr[len] = bsum[nb];
}

// copies the columns into the panel layout, one wave per chunk of kW
// destination positions (walking the panel majors of the chunk from its
// first one)
__global__ __launch_bounds__(256) void sp_pan_copy_kernel(
    const int64_t* __restrict__ src, const int64_t* __restrict__ pptr, int64_t len,
    int64_t nnz, const int32_t* __restrict__ pfirst, const int32_t* __restrict__ row_idx,
    const float* __restrict__ col_val, int32_t* __restrict__ pidx,
    float* __restrict__ pval) {
  const int lane = threadIdx.x % kWave;
  const int64_t w =
      (int64_t)blockIdx.x * kWPB + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t lo = w * kW;
  if (lo >= nnz) return;
  const int64_t hi = lo + kW < nnz ? lo + kW : nnz;
  int64_t M = pfirst[w];
  for (int64_t k = lo; k < hi && M < len; ++M) {
    const int64_t e = pptr[M + 1] < hi ? pptr[M + 1] : hi;
    const int64_t off = src[M] - pptr[M];  // source position - destination position
    for (int64_t t = k + lane; t < e; t += kWave) {
      pidx[t] = row_idx[t + off];
      pval[t] = col_val[t + off];
    }
    k = e > k ? e : k;
  }
}

// --------------------------------------------------------------------------
// balanced products with a dense operand
// --------------------------------------------------------------------------

// which launches run (bits): those of an iteration planned dense, those
// with a running start
enum SegGate { kGateNone = 0, kGateDense = 1, kGateActive = 2 };

// OT[c][j] = sum over the nonzeros (c, i) of val * BT[i][j] for the majors
// inside this wave's chunk, for the starts j0 .. j0 + 4 L - 1 of this block;
// partials of majors crossing a chunk boundary go to carry[w][slot] (slot 0:
// the major holding the chunk's first nonzero, slot 1: the major holding its
// last one).
//
// A row of BT (4 L floats, a power of two, aligned) is read by L lanes with
// one 16-byte load each, so one load instruction covers 64 / L nonzeros and
// touches one cache line per row; every lane keeps the running sums of its
// four starts for the current major.  The indices and values reach the wave
// kSS at a time through LDS: the next stage is loaded with coalesced 16-byte
// loads while the current one is worked off in steps of kU 64 / L nonzeros
// (each of the 64 / L lane slots takes kU consecutive ones), independent of
// where majors begin and end; where a major ends, the sums of the slots are
// combined by a fixed xor butterfly and written.
// OFF32: every byte offset into BT fits in 32 bits.
constexpr int kU = 8;      // row loads per lane and step
constexpr int kSS = 512;   // nonzeros per stage

template <int L, bool OFF32>
__global__ __launch_bounds__(256) void sp_seg_kernel(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
    const float* __restrict__ val, int64_t m, int64_t nnz,
    const int32_t* __restrict__ first, const float* __restrict__ BT, int64_t ldb, int64_t r,
    float* __restrict__ OT, int64_t ldo, float* __restrict__ carry, const Plan* plan,
    int gate) {
  constexpr int NPI = kWave / L;      // nonzeros per load instruction
  constexpr int NS = kU * NPI;        // nonzeros per step
  static_assert(kSS % NS == 0 && kU % 4 == 0, "a stage holds whole steps");
  __shared__ int32_t sidx[kWPB][2][kSS];
  __shared__ float sval[kWPB][2][kSS];
  if ((gate & kGateDense) && plan->mode != kAxDense) return;
  if ((gate & kGateActive) && plan->active == 0) return;
  // the wave index is the same on every lane; saying so keeps the chunk, the
  // majors and all loop control in scalar registers
  const int lane = threadIdx.x % kWave;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int slot = lane / L, quad = lane % L;
  const int64_t j0 = (int64_t)blockIdx.y * 4 * L + 4 * quad;  // this lane's first start
  const int64_t w = (int64_t)blockIdx.x * kWPB + wv;
  const int64_t lo = w * kW;
  if (lo >= nnz) return;
  const int64_t hi = lo + kW < nnz ? lo + kW : nnz;

  // stage at sb: lane l holds positions sb + 8 l .. sb + 8 l + 7 (index 0 and
  // value 0 past hi)
  int4 gi0, gi1;
  float4 gv0, gv1;
  auto load_stage = [&](int64_t sb) {
    const int64_t t = sb + 8 * lane;
    if (sb + kSS <= hi) {
      gi0 = *reinterpret_cast<const int4*>(idx + t);
      gi1 = *reinterpret_cast<const int4*>(idx + t + 4);
      gv0 = *reinterpret_cast<const float4*>(val + t);
      gv1 = *reinterpret_cast<const float4*>(val + t + 4);
    } else {
      int32_t e[8];
      float f[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        e[k] = t + k < hi ? idx[t + k] : 0;
        f[k] = t + k < hi ? val[t + k] : 0.f;
      }
      gi0 = {e[0], e[1], e[2], e[3]};
      gi1 = {e[4], e[5], e[6], e[7]};
      gv0 = {f[0], f[1], f[2], f[3]};
      gv1 = {f[4], f[5], f[6], f[7]};
    }
  };
  auto store_stage = [&](int buf) {
    *reinterpret_cast<int4*>(&sidx[wv][buf][8 * lane]) = gi0;
    *reinterpret_cast<int4*>(&sidx[wv][buf][8 * lane + 4]) = gi1;
    *reinterpret_cast<float4*>(&sval[wv][buf][8 * lane]) = gv0;
    *reinterpret_cast<float4*>(&sval[wv][buf][8 * lane + 4]) = gv1;
  };
  auto flush = [&](float4 a, int64_t c, int64_t cb, int64_t ce) {
#pragma unroll
    for (int off = L; off < kWave; off <<= 1) {
      a.x += __shfl_xor(a.x, off, kWave);
      a.y += __shfl_xor(a.y, off, kWave);
      a.z += __shfl_xor(a.z, off, kWave);
      a.w += __shfl_xor(a.w, off, kWave);
    }
    if (slot == 0 && j0 < r) {
      const bool whole = cb >= lo && ce <= hi;
      float* o = whole ? OT + c * ldo + j0 : carry + (w * 2 + (cb <= lo ? 0 : 1)) * ldo + j0;
      if (j0 + 4 <= r) {
        *reinterpret_cast<float4*>(o) = a;
      } else {
        o[0] = a.x;
        if (j0 + 1 < r) o[1] = a.y;
        if (j0 + 2 < r) o[2] = a.z;
      }
    }
  };

  float4 acc = {0.f, 0.f, 0.f, 0.f};
  int64_t c = first[w];
  int64_t cb = ptr[c], ce = ptr[c + 1];
  int64_t cn = c + 2 <= m ? ptr[c + 2] : ce;  // end of the next major
  bool open = true;  // major c still collects nonzeros of this chunk
  load_stage(lo);
  store_stage(0);
  if (lo + kSS < hi) load_stage(lo + kSS);
  int buf = 0;
  for (int64_t sb = lo; sb < hi && open; sb += kSS, buf ^= 1) {
    const int64_t send = sb + kSS < hi ? sb + kSS : hi;
    for (int64_t tb = sb; tb < send && open; tb += NS) {
      // slot s takes positions tb + s kU .. tb + s kU + kU - 1 (wide LDS reads)
      const int base = (int)(tb - sb) + slot * kU;
      float v[kU];
      float4 b[kU];
      int32_t ii[kU];
#pragma unroll
      for (int u = 0; u < kU; u += 4) {
        const int4 q4 = *reinterpret_cast<const int4*>(&sidx[wv][buf][base + u]);
        const float4 f4 = *reinterpret_cast<const float4*>(&sval[wv][buf][base + u]);
        ii[u] = q4.x;
        ii[u + 1] = q4.y;
        ii[u + 2] = q4.z;
        ii[u + 3] = q4.w;
        v[u] = f4.x;
        v[u + 1] = f4.y;
        v[u + 2] = f4.z;
        v[u + 3] = f4.w;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int32_t i = ii[u];
        if (OFF32)
          b[u] = *reinterpret_cast<const float4*>(
              reinterpret_cast<const char*>(BT) +
              ((uint32_t)i * (uint32_t)ldb + (uint32_t)j0) * (uint32_t)sizeof(float));
        else
          b[u] = *reinterpret_cast<const float4*>(BT + (int64_t)i * ldb + j0);
      }
      const int64_t bend = tb + NS < send ? tb + NS : send;
      for (;;) {
        // the step's positions tb + u NPI + slot inside [cb, min(ce, bend))
        const int rlo = cb > tb ? (int)(cb - tb) : 0;
        const int rhi = (int)((ce < bend ? ce : bend) - tb);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int rel = slot * kU + u;
          if (rel >= rlo && rel < rhi) {
            acc.x = fmaf(v[u], b[u].x, acc.x);
            acc.y = fmaf(v[u], b[u].y, acc.y);
            acc.z = fmaf(v[u], b[u].z, acc.z);
            acc.w = fmaf(v[u], b[u].w, acc.w);
          }
        }
        if (ce > bend) break;  // major c goes on past this step
        flush(acc, c, cb, ce);
        acc = {0.f, 0.f, 0.f, 0.f};
        ++c;
        if (c >= m) {
          open = false;
          break;
        }
        cb = ce;
        ce = cn;
        cn = c + 2 <= m ? ptr[c + 2] : ce;
        if (cb >= hi) {
          open = false;
          break;
        }
      }
    }
    if (sb + kSS < hi) {
      store_stage(buf ^ 1);
      if (sb + 2 * kSS < hi) load_stage(sb + 2 * kSS);
    }
  }
  if (open) flush(acc, c, cb, ce);  // crosses into the next chunk
}

// majors crossing chunk boundaries (listed once per solve): sum of their
// chunk partials in chunk order.  One wave per listed major.
__global__ __launch_bounds__(256) void sp_fix_kernel(const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ split,
                                                     int64_t nsplit,
                                                     const float* __restrict__ carry,
                                                     int64_t r, float* __restrict__ OT,
                                                     int64_t ldo, const Plan* plan, int gate) {
  if ((gate & kGateDense) && plan->mode != kAxDense) return;
  if ((gate & kGateActive) && plan->active == 0) return;
  const int64_t k =
      (int64_t)blockIdx.x * kWPB + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (k >= nsplit) return;
  const int lane = threadIdx.x % kWave;
  const int64_t c = split[k];
  const int64_t cb = ptr[c], ce = ptr[c + 1];
  const int64_t w0 = cb / kW, w1 = (ce - 1) / kW;
  const int64_t s0 = cb == w0 * kW ? 0 : 1;
  for (int64_t j = lane; j < r; j += kWave) {
    float acc = carry[(w0 * 2 + s0) * ldo + j];
#pragma unroll 8
    for (int64_t w = w0 + 1; w <= w1; ++w) acc += carry[w * 2 * ldo + j];
    OT[c * ldo + j] = acc;
  }
}

// the nonempty majors crossing a chunk boundary, in any order
__global__ __launch_bounds__(256) void sp_split_list_kernel(const int64_t* __restrict__ ptr,
                                                            int64_t m, int32_t* split,
                                                            int32_t* count) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  const int64_t cb = ptr[c], ce = ptr[c + 1];
  if (cb < ce && cb / kW != (ce - 1) / kW) split[atomicAdd(count, 1)] = (int32_t)c;
}

// O[j][c] = sum over the npan panels of OT[P m + c][j] (in panel order),
// through 64 x 64 LDS tiles
__global__ __launch_bounds__(256) void sp_to_starts_kernel(const float* __restrict__ OT,
                                                           int64_t ldo, int64_t m, int64_t r,
                                                           int32_t npan, float* __restrict__ O,
                                                           int64_t ld, const Plan* plan,
                                                           int gate) {
  __shared__ float tile[kTT][kTT + 1];
  if ((gate & kGateDense) && plan->mode != kAxDense) return;
  if ((gate & kGateActive) && plan->active == 0) return;
  const int64_t c0 = (int64_t)blockIdx.x * kTT, j0 = (int64_t)blockIdx.y * kTT;
  const int tx = threadIdx.x % kTT, ty = threadIdx.x / kTT;
  for (int cc = ty; cc < kTT; cc += 4) {
    const int64_t c = c0 + cc, j = j0 + tx;
    float v = 0.f;
    if (c < m && j < r) {
      v = OT[c * ldo + j];
      for (int32_t P = 1; P < npan; ++P) v += OT[(P * m + c) * ldo + j];
    }
    tile[cc][tx] = v;
  }
  __syncthreads();
  for (int jj = ty; jj < kTT; jj += 4) {
    const int64_t c = c0 + tx, j = j0 + jj;
    if (c < m && j < r) O[j * ld + c] = tile[tx][jj];
  }
}

// --------------------------------------------------------------------------
// y-update into the transposed layout (Table 3: y = u / ||u||_2 for the L2
// variance, y = sgn(u) for the L1 variance), parallel over starts and rows
// --------------------------------------------------------------------------

constexpr int kYB = 4096;  // rows per norm partial

// partial[j * nb + b] = sum of u_ji^2 over rows [b kYB, (b + 1) kYB)
__global__ __launch_bounds__(256) void sp_ynorm_kernel(const float* __restrict__ U,
                                                       int64_t ldu, int64_t n, StartState s,
                                                       double* __restrict__ partial) {
  __shared__ double red[8];
  const int64_t j = blockIdx.y;
  if (s.status[j] != kRunning) return;
  const float* u = U + j * ldu;
  const int64_t b0 = (int64_t)blockIdx.x * kYB;
  const int64_t b1 = b0 + kYB < n ? b0 + kYB : n;
  double sq = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
    const double t = u[i];
    sq += t * t;
  }
  sq = block_sum(sq, red);
  if (threadIdx.x == 0) partial[j * gridDim.x + blockIdx.x] = sq;
}

// YT[i][j] = y_ji for a tile of 64 rows x 64 starts (running starts with
// u != 0); a start with u = 0 becomes degenerate (set by the tiles of the
// first row block)
template <bool L1VAR>
__global__ __launch_bounds__(256) void sp_yapply_kernel(const float* __restrict__ U,
                                                        int64_t ldu, int64_t n, int64_t r,
                                                        StartState s,
                                                        const double* __restrict__ partial,
                                                        int64_t nb, float* __restrict__ YT,
                                                        int64_t ldt) {
  __shared__ float tile[kTT][kTT + 1];
  __shared__ double scale[kTT];
  __shared__ int live[kTT];
  const int64_t i0 = (int64_t)blockIdx.x * kTT, j0 = (int64_t)blockIdx.y * kTT;
  const int tx = threadIdx.x % kTT, ty = threadIdx.x / kTT;
  if (threadIdx.x < kTT) {
    const int64_t j = j0 + threadIdx.x;
    int ok = 0;
    double sc = 0.0;
    if (j < r && s.status[j] == kRunning) {
      double sq = 0.0;
      for (int64_t b = 0; b < nb; ++b) sq += partial[j * nb + b];
      if (L1VAR) {
        // ||u||_1 > 0 iff some u_i != 0 iff ||u||_2 > 0
        ok = sq > 0.0;
      } else if (sq > 0.0) {
        ok = 1;
        sc = 1.0 / sqrt(sq);
      }
      if (!ok && blockIdx.x == 0) s.status[j] = SPCA_DEGENERATE;
    }
    live[threadIdx.x] = ok;
    scale[threadIdx.x] = sc;
  }
  __syncthreads();
  for (int jj = ty; jj < kTT; jj += 4) {
    const int64_t i = i0 + tx, j = j0 + jj;
    float y = 0.f;
    if (i < n && live[jj]) {
      const float t = U[j * ldu + i];
      y = L1VAR ? (float)((t > 0.f) - (t < 0.f)) : (float)((double)t * scale[jj]);
    }
    tile[jj][tx] = y;
  }
  __syncthreads();
  for (int ii = ty; ii < kTT; ii += 4) {
    const int64_t i = i0 + ii, j = j0 + tx;
    if (i < n && j < r && live[tx]) YT[i * ldt + j] = tile[tx][ii];
  }
}

// --------------------------------------------------------------------------
// row-block products from the support lists
// --------------------------------------------------------------------------

// first position in [lo, hi) whose index is >= target (hi if none), for
// indices sorted ascending; one wave, 64 probes per round.  Stays inside
// [lo, hi] for any contents.
__device__ __forceinline__ int64_t wave_lower_bound(const int32_t* __restrict__ a, int64_t lo,
                                                    int64_t hi, int64_t target) {
  const int lane = threadIdx.x % kWave;
  while (hi - lo > kWave) {
    const int64_t len = hi - lo;
    const int64_t pos = lo + (int64_t)(lane + 1) * len / (kWave + 1);
    const int cnt = __popcll(__ballot(a[pos] < target));
    const int64_t plo = lo + (int64_t)cnt * len / (kWave + 1);  // probe cnt - 1
    const int64_t phi = lo + (int64_t)(cnt + 1) * len / (kWave + 1);
    if (cnt > 0) lo = plo + 1;
    if (cnt < kWave) hi = phi;
  }
  const int64_t pos = lo + lane;
  const int cnt = __popcll(__ballot(pos < hi && a[pos] < target));
  return lo + cnt;
}

// rows [b0, b1) of the running start j's u = sum over its support columns
__global__ __launch_bounds__(256) void sp_list_rows_kernel(
    const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
    const float* __restrict__ val, int64_t n, const int32_t* __restrict__ list_idx,
    const float* __restrict__ list_val, int64_t ldl, float* __restrict__ U, int64_t ldu,
    StartState s, const Plan* plan) {
  __shared__ float ub[kRB];
  __shared__ int64_t bnd[2];
  if (plan->mode != kAxListRows) return;
  const int64_t j = blockIdx.y;
  if (s.status[j] != kRunning) return;
  const int64_t b0 = (int64_t)blockIdx.x * kRB;
  const int64_t b1 = b0 + kRB < n ? b0 + kRB : n;
  const int wave = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kRB; i += 256) ub[i] = 0.f;
  const int32_t cnt = s.nnz[j];
  for (int32_t t = 0; t < cnt; ++t) {
    const int32_t c = list_idx[j * ldl + t];
    const float x = list_val[j * ldl + t];
    const int64_t cb = col_ptr[c], ce = col_ptr[c + 1];
    if (wave < 2) {
      const int64_t pos = wave_lower_bound(row_idx, cb, ce, wave == 0 ? b0 : b1);
      if (threadIdx.x % kWave == 0) bnd[wave] = pos;
    }
    __syncthreads();
    const int64_t kb = bnd[0], ke = bnd[1];
    for (int64_t k = kb + threadIdx.x; k < ke; k += 256) {
      const int64_t i = row_idx[k];
      if (i >= b0 && i < b1) ub[i - b0] += val[k] * x;
    }
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; b0 + i < b1; i += 256) U[j * ldu + b0 + i] = ub[i];
}

// FP64 evaluation: rows [b0, b1) of u = A x / ||x||_2, then the block's
// sum of u_i^2 and of |u_i| (one partial pair per start and block)
__global__ __launch_bounds__(256) void sp_final_kernel(
    const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
    const float* __restrict__ val, int64_t n, const int32_t* __restrict__ list_idx,
    const float* __restrict__ list_val, int64_t ldl, StartState s,
    const double* __restrict__ xnorm, double* __restrict__ partial, Defl defl) {
  __shared__ double ub[kRB64];
  __shared__ int64_t bnd[2];
  __shared__ double red[2 * 5];
  const int64_t j = blockIdx.y;
  const int64_t nb = gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * kRB64;
  const int64_t b1 = b0 + kRB64 < n ? b0 + kRB64 : n;
  const int wave = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kRB64; i += 256) ub[i] = 0.0;
  const double nrm = xnorm[j];
  const bool live = s.status[j] != SPCA_DEGENERATE && s.status[j] != SPCA_ZERO && nrm > 0.0;
  const int32_t cnt = live ? s.nnz[j] : 0;
  for (int32_t t = 0; t < cnt; ++t) {
    const int32_t c = list_idx[j * ldl + t];
    const double x = (double)list_val[j * ldl + t] / nrm;
    const int64_t cb = col_ptr[c], ce = col_ptr[c + 1];
    if (wave < 2) {
      const int64_t pos = wave_lower_bound(row_idx, cb, ce, wave == 0 ? b0 : b1);
      if (threadIdx.x % kWave == 0) bnd[wave] = pos;
    }
    __syncthreads();
    const int64_t kb = bnd[0], ke = bnd[1];
    for (int64_t k = kb + threadIdx.x; k < ke; k += 256) {
      const int64_t i = row_idx[k];
      if (i >= b0 && i < b1) ub[i - b0] += (double)val[k] * x;
    }
    __syncthreads();
  }
  // deflated problem: A_k x = A x - sum_l alpha_l A x_l
  if (live && defl.k > 0)
    for (int64_t i = threadIdx.x; b0 + i < b1; i += 256)
      for (int l = 0; l < defl.k; ++l)
        ub[i] -= defl.alpha[j * kMaxDefl + l] * defl.scores[(b0 + i) * kMaxDefl + l];
  double acc[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; b0 + i < b1; i += 256) {
    acc[0] += ub[i] * ub[i];
    acc[1] += fabs(ub[i]);
  }
  block_sum_n<double, 2>(acc, red);
  if (threadIdx.x == 0) {
    partial[(j * nb + blockIdx.x) * 2] = acc[0];
    partial[(j * nb + blockIdx.x) * 2 + 1] = acc[1];
  }
}

// rows of BT: 4 L floats, L a power of two (2 .. 16); 64 starts per block
// above 64 starts
int seg_lanes(int64_t r) { return r <= 8 ? 2 : r <= 16 ? 4 : r <= 32 ? 8 : 16; }
int64_t seg_blocks(int64_t r) { return ceil_div(r, (int64_t)4 * seg_lanes(r)); }

// FP64 scores of the deflation loadings: rows [b0, b1) of B[:, i] = A x_i
// from the loading's (index, value) list, in LDS, column by column
__global__ __launch_bounds__(256) void sp_scores_kernel(
    const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
    const float* __restrict__ val, int64_t n, int64_t p, Defl d) {
  __shared__ double ub[kRB64];
  __shared__ int64_t bnd[2];
  const int i = blockIdx.y;
  const int64_t b0 = (int64_t)blockIdx.x * kRB64;
  const int64_t b1 = b0 + kRB64 < n ? b0 + kRB64 : n;
  const int wave = threadIdx.x / kWave;
  for (int e = threadIdx.x; e < kRB64; e += 256) ub[e] = 0.0;
  const int32_t cnt = d.cnt[i];
  for (int32_t t = 0; t < cnt; ++t) {
    const int32_t c = d.idx[i * p + t];
    const double x = d.val[i * p + t];
    const int64_t cb = col_ptr[c], ce = col_ptr[c + 1];
    if (wave < 2) {
      const int64_t pos = wave_lower_bound(row_idx, cb, ce, wave == 0 ? b0 : b1);
      if (threadIdx.x % kWave == 0) bnd[wave] = pos;
    }
    __syncthreads();
    const int64_t kb = bnd[0], ke = bnd[1];
    for (int64_t k = kb + threadIdx.x; k < ke; k += 256) {
      const int64_t row = row_idx[k];
      if (row >= b0 && row < b1) ub[row - b0] += (double)val[k] * x;
    }
    __syncthreads();
  }
  for (int64_t e = threadIdx.x; b0 + e < b1; e += 256) d.scores[(b0 + e) * kMaxDefl + i] = ub[e];
}

template <int L>
void launch_seg(hipStream_t st, const int64_t* ptr, const int32_t* idx, const float* val,
                int64_t m, int64_t nnz, const int32_t* first, const float* BT, int64_t ldb,
                int64_t minor, int64_t r, float* OT, int64_t ldo, float* carry,
                const Plan* plan, int gate) {
  const int64_t nchunks = ceil_div(nnz, kW);
  if (nchunks == 0) return;
  const dim3 g((unsigned)ceil_div(nchunks, (int64_t)kWPB), (unsigned)seg_blocks(r));
  // BT (minor rows of ldb floats) within 4 GiB: 32-bit address arithmetic
  if (minor * ldb * (int64_t)sizeof(float) <= (int64_t)UINT32_MAX)
    hipLaunchKernelGGL((sp_seg_kernel<L, true>), g, dim3(256), 0, st, ptr, idx, val, m, nnz,
                       first, BT, ldb, r, OT, ldo, carry, plan, gate);
  else
    hipLaunchKernelGGL((sp_seg_kernel<L, false>), g, dim3(256), 0, st, ptr, idx, val, m, nnz,
                       first, BT, ldb, r, OT, ldo, carry, plan, gate);
}

// O (r x mo, start-major, ld) = the product of A's compressed layout (ptr,
// idx, val; m = npan mo majors) with BT, through OT (m x ldo; the rows of
// empty majors hold zeros) and carry; split: the majors crossing chunks
void seg_product(hipStream_t st, const int64_t* ptr, const int32_t* idx, const float* val,
                 int64_t m, int64_t nnz, const int32_t* first, const int32_t* split,
                 int64_t nsplit, const float* BT, int64_t ldb, int64_t minor, int64_t r,
                 float* OT, int64_t ldo, float* carry, float* O, int64_t ld, const Plan* plan,
                 int gate, int32_t npan) {
  const int64_t mo = npan > 0 ? m / npan : m;
  switch (seg_lanes(r)) {
    case 2:
      launch_seg<2>(st, ptr, idx, val, m, nnz, first, BT, ldb, minor, r, OT, ldo, carry, plan,
                    gate);
      break;
    case 4:
      launch_seg<4>(st, ptr, idx, val, m, nnz, first, BT, ldb, minor, r, OT, ldo, carry, plan,
                    gate);
      break;
    case 8:
      launch_seg<8>(st, ptr, idx, val, m, nnz, first, BT, ldb, minor, r, OT, ldo, carry, plan,
                    gate);
      break;
    default:
      launch_seg<16>(st, ptr, idx, val, m, nnz, first, BT, ldb, minor, r, OT, ldo, carry, plan,
                     gate);
  }
  if (nsplit > 0)
    hipLaunchKernelGGL(sp_fix_kernel, dim3((unsigned)ceil_div(nsplit, (int64_t)kWPB)),
                       dim3(256), 0, st, ptr, split, nsplit, carry, r, OT, ldo, plan, gate);
  const dim3 g((unsigned)ceil_div(mo, (int64_t)kTT), (unsigned)ceil_div(r, (int64_t)kTT));
  hipLaunchKernelGGL(sp_to_starts_kernel, g, dim3(256), 0, st, OT, ldo, mo, r,
                     npan > 0 ? npan : 1, O, ld, plan, gate);
}

}  // namespace

int64_t sparse_chunks(int64_t nnz) { return ceil_div(nnz, kW); }
// rows of the transposed operands: a power of two of at least 8 floats up to
// 64 starts (one 128-byte line for 17 .. 32), then whole blocks of 64
int64_t sparse_ld(int64_t r) { return seg_blocks(r) * 4 * seg_lanes(r); }

int32_t sparse_panels(int64_t n, int64_t p, int64_t nnz, int64_t ldt, int force) {
  (void)p;
  const int64_t bytes = n * ldt * (int64_t)sizeof(float);
  if (force < 0 || n < 2 || nnz == 0) return 0;
  if (force == 0 && (bytes <= 2 * kPanelBytes || nnz < (1 << 20))) return 0;
  const int64_t np = std::max<int64_t>(2, ceil_div(bytes, kPanelBytes));
  return (int32_t)std::min<int64_t>(np, std::min<int64_t>(n, 64));
}

int64_t sparse_panel_tmp(int32_t npan, int64_t p) {
  const int64_t len = npan * p;
  return 2 * len + ceil_div(len, (int64_t)kScanB) + 1;
}

void sparse_split_lists(hipStream_t st, const SparseA& a, int32_t* counts) {
  if (a.nnz == 0) return;
  hipLaunchKernelGGL(sp_split_list_kernel, dim3((unsigned)ceil_div(a.n, (int64_t)256)),
                     dim3(256), 0, st, a.row_ptr, a.n, a.row_split, counts);
  const int64_t mc = a.npan > 0 ? a.npan * a.p : a.p;
  hipLaunchKernelGGL(sp_split_list_kernel, dim3((unsigned)ceil_div(mc, (int64_t)256)),
                     dim3(256), 0, st, a.npan > 0 ? a.pptr : a.col_ptr, mc, a.col_split,
                     counts + 1);
}

void sparse_build_panels(hipStream_t st, SparseA& a) {
  const int64_t len = a.npan * a.p, nb = ceil_div(len, (int64_t)kScanB);
  int64_t* src = a.ptmp;
  int64_t* cnt = a.ptmp + len;
  int64_t* bsum = a.ptmp + 2 * len;
  hipLaunchKernelGGL(sp_pan_bounds_kernel, dim3((unsigned)ceil_div(len, (int64_t)256)),
                     dim3(256), 0, st, a.col_ptr, a.row_idx, a.p, a.npan, a.prow, src, cnt);
  hipLaunchKernelGGL(sp_scan_sums_kernel, dim3((unsigned)nb), dim3(1024), 0, st, cnt, len,
                     bsum);
  hipLaunchKernelGGL(sp_scan_top_kernel, dim3(1), dim3(64), 0, st, bsum, nb);
  hipLaunchKernelGGL(sp_scan_out_kernel, dim3((unsigned)nb), dim3(1024), 0, st, cnt, len,
                     bsum, nb, a.pptr);
  const int64_t nch = sparse_chunks(a.nnz);
  (void)hipMemsetAsync(a.pfirst, 0, sizeof(int32_t) * nch, st);
  hipLaunchKernelGGL(sp_first_kernel, dim3((unsigned)ceil_div(len, (int64_t)256)), dim3(256),
                     0, st, a.pptr, len, nch, a.pfirst);
  hipLaunchKernelGGL(sp_pan_copy_kernel, dim3((unsigned)ceil_div(nch, (int64_t)kWPB)),
                     dim3(256), 0, st, src, a.pptr, len, a.nnz, a.pfirst, a.row_idx,
                     a.col_val, a.pidx, a.pval);
}

int64_t sparse_final_parts(int64_t n) { return ceil_div(n, (int64_t)kRB64); }

void sparse_prepare(hipStream_t st, const SparseA& a, int32_t* bad) {
  const int64_t nch = sparse_chunks(a.nnz);
  const unsigned gi = (unsigned)std::min<int64_t>(ceil_div(a.nnz, (int64_t)256), 16384);
  if (a.p > 0)
    hipLaunchKernelGGL(sp_check_ptr_kernel, dim3((unsigned)ceil_div(a.p, (int64_t)256)),
                       dim3(256), 0, st, a.col_ptr, a.p, bad);
  if (a.n > 0)
    hipLaunchKernelGGL(sp_check_ptr_kernel, dim3((unsigned)ceil_div(a.n, (int64_t)256)),
                       dim3(256), 0, st, a.row_ptr, a.n, bad);
  if (a.nnz == 0) return;
  hipLaunchKernelGGL(sp_check_idx_kernel, dim3(gi), dim3(256), 0, st, a.row_idx, a.nnz, a.n,
                     bad);
  hipLaunchKernelGGL(sp_check_idx_kernel, dim3(gi), dim3(256), 0, st, a.col_idx, a.nnz, a.p,
                     bad);
  (void)hipMemsetAsync(a.col_first, 0, sizeof(int32_t) * nch, st);
  (void)hipMemsetAsync(a.row_first, 0, sizeof(int32_t) * nch, st);
  hipLaunchKernelGGL(sp_first_kernel, dim3((unsigned)ceil_div(a.p, (int64_t)256)), dim3(256),
                     0, st, a.col_ptr, a.p, nch, a.col_first);
  hipLaunchKernelGGL(sp_first_kernel, dim3((unsigned)ceil_div(a.n, (int64_t)256)), dim3(256),
                     0, st, a.row_ptr, a.n, nch, a.row_first);
  hipLaunchKernelGGL(sp_check_sorted_kernel, dim3((unsigned)ceil_div(nch, (int64_t)kWPB)),
                     dim3(256), 0, st, a.col_ptr, a.row_idx, a.p, a.nnz, a.col_first, bad);
}

void sparse_ax_dense(hipStream_t st, const SparseA& a, const float* XT, int64_t ldxt,
                     int64_t r, float* UT, float* carry, float* U, int64_t ldu,
                     StartState s, const Plan* plan) {
  seg_product(st, a.row_ptr, a.col_idx, a.row_val, a.n, a.nnz, a.row_first, a.row_split,
              a.nrow_split, XT, ldxt, a.p, r, UT, ldxt, carry, U, ldu, plan,
              kGateDense | kGateActive, 0);
}

void sparse_aty(hipStream_t st, const SparseA& a, const float* YT, int64_t ldyt, int64_t r,
                float* VT, float* carry, float* V, int64_t ldv, StartState s,
                const Plan* plan) {
  if (a.npan > 0)
    seg_product(st, a.pptr, a.pidx, a.pval, a.npan * a.p, a.nnz, a.pfirst, a.col_split,
                a.ncol_split, YT, ldyt, a.n, r, VT, ldyt, carry, V, ldv, plan, kGateActive,
                a.npan);
  else
    seg_product(st, a.col_ptr, a.row_idx, a.col_val, a.p, a.nnz, a.col_first, a.col_split,
                a.ncol_split, YT, ldyt, a.n, r, VT, ldyt, carry, V, ldv, plan, kGateActive, 0);
}

int64_t sparse_y_parts(int64_t n) { return ceil_div(n, (int64_t)kYB); }

void sparse_y_update(hipStream_t st, int fid, const float* U, int64_t ldu, int64_t n,
                     int64_t r, StartState s, double* partial, float* YT, int64_t ldt) {
  const int64_t nb = sparse_y_parts(n);
  hipLaunchKernelGGL(sp_ynorm_kernel, dim3((unsigned)nb, (unsigned)r), dim3(256), 0, st, U,
                     ldu, n, s, partial);
  const dim3 g((unsigned)ceil_div(n, (int64_t)kTT), (unsigned)ceil_div(r, (int64_t)kTT));
  if (l1_variance(fid))
    hipLaunchKernelGGL(sp_yapply_kernel<true>, g, dim3(256), 0, st, U, ldu, n, r, s, partial,
                       nb, YT, ldt);
  else
    hipLaunchKernelGGL(sp_yapply_kernel<false>, g, dim3(256), 0, st, U, ldu, n, r, s, partial,
                       nb, YT, ldt);
}

void sparse_ax_list(hipStream_t st, const SparseA& a, const int32_t* list_idx,
                    const float* list_val, int64_t ldl, float* U, int64_t ldu, int64_t r,
                    StartState s, const Plan* plan) {
  if (a.n == 0) return;
  const dim3 g((unsigned)ceil_div(a.n, (int64_t)kRB), (unsigned)r);
  hipLaunchKernelGGL(sp_list_rows_kernel, g, dim3(256), 0, st, a.col_ptr, a.row_idx,
                     a.col_val, a.n, list_idx, list_val, ldl, U, ldu, s, plan);
}

void sparse_final(hipStream_t st, const SparseA& a, const int32_t* list_idx,
                  const float* list_val, int64_t ldl, StartState s, int64_t r,
                  const double* xnorm, double* partial, Defl defl) {
  const dim3 g((unsigned)sparse_final_parts(a.n), (unsigned)r);
  hipLaunchKernelGGL(sp_final_kernel, g, dim3(256), 0, st, a.col_ptr, a.row_idx, a.col_val,
                     a.n, list_idx, list_val, ldl, s, xnorm, partial, defl);
}

void sparse_deflate_scores(hipStream_t st, const SparseA& a, Defl d) {
  if (d.k <= 0 || a.n == 0) return;
  const dim3 g((unsigned)sparse_final_parts(a.n), (unsigned)d.k);
  hipLaunchKernelGGL(sp_scores_kernel, g, dim3(256), 0, st, a.col_ptr, a.row_idx, a.col_val,
                     a.n, a.p, d);
}

}  // namespace spca
