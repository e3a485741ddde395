// FP32 "NT" GEMM on CDNA4 matrix cores: C = P * Q^T with P (M x K) and
// Q (N x K) both K-contiguous.  Both products of an AM iteration have this
// shape once A is held column-major (for A^T Y) and row-major (for A X):
//   V^T (r x p) = Y^T (r x n) * [A columns] (p x n)^T     K = n
//   U^T (r x n) = X^T (r x p) * [A rows]    (n x p)^T     K = p
//
// Tiling: a workgroup of WM x WN waves owns a BM x BN tile of C; each wave
// owns (BM/WM) x (BN/WN) built from 32 x 32 v_mfma_f32_32x32x2_f32 blocks.
// K advances 32 at a time through two LDS stages: while the waves multiply
// out of one stage, the next K slab is already in registers and is written
// to the other stage, so one barrier per slab suffices.
// Within an 8-wide K chunk, lane l feeds row (l % 32) at k offset
// 4 * (l / 32) .. +3 as one 16-byte LDS read; the i-th of the four MFMAs of
// the chunk takes element i.  The order in which k terms enter the sum does
// not change the product, so every LDS read is 16 bytes wide.
// LDS rows are 128 bytes with no padding; the 16-byte chunk c of row r is
// stored at chunk c ^ ((r ^ (r >> 3)) & 7), so that any 8 consecutive rows
// (and any 16 rows of alternating parity pairs) read at one chunk index
// fall in distinct banks for 32- and 64-bank LDS alike.
// Split-K: when splits > 1, slab range s of every tile writes its partial
// product to C + s * split_stride; the consumer sums the partials in order.
// BF16 operands: the same 128-byte LDS rows hold 64 bf16 of K; each 16-byte
// chunk (8 bf16 of one row) feeds one v_mfma_f32_32x32x16_bf16 instead of
// four FP32 MFMAs, and the products accumulate in FP32.
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBK = 32;              // floats per LDS row (128 bytes)
constexpr int kChunks = kBK / 4;     // 16-byte chunks per LDS row

// Element traits: how many K elements a 16-byte chunk holds.
template <typename T>
struct Elem;
template <>
struct Elem<float> {
  static constexpr int kPerChunk = 4;
};
template <>
struct Elem<uint16_t> {  // bf16 bit patterns
  static constexpr int kPerChunk = 8;
};

template <int BM, int BN, int WM, int WN>
struct GemmCfg {
  static constexpr int kThreads = WM * WN * kWave;
  static constexpr int kTM = BM / WM;  // rows per wave
  static constexpr int kTN = BN / WN;  // cols per wave
  static constexpr int kFM = kTM / 32;
  static constexpr int kFN = kTN / 32;
  static constexpr int kPVec = BM * kChunks / kThreads;  // float4 per thread
  static constexpr int kQVec = BN * kChunks / kThreads;
  static constexpr int kStage = (BM + BN) * kBK;  // floats per LDS stage
  static_assert(kTM % 32 == 0 && kTN % 32 == 0, "wave tile must be 32-aligned");
  static_assert((BM * kChunks) % kThreads == 0, "P slab load must divide");
  static_assert((BN * kChunks) % kThreads == 0, "Q slab load must divide");
};

__device__ __forceinline__ int swz(int row, int chunk) {
  return row * kBK + ((chunk ^ ((row ^ (row >> 3)) & 7)) << 2);
}

// 16 bytes of row `row` starting at element k (zero past kend or nrows).
template <typename T>
__device__ __forceinline__ floatx4 load_chunk(const T* __restrict__ base,
                                              int64_t ld, int row, int nrows,
                                              int k, int kend) {
  constexpr int E = Elem<T>::kPerChunk;
  floatx4 v = {0.f, 0.f, 0.f, 0.f};
  if (row < nrows) {
    const T* p = base + (int64_t)row * ld + k;
    if (k + E - 1 < kend) {
      v = *reinterpret_cast<const floatx4*>(p);
    } else {
      T tmp[E];
#pragma unroll
      for (int e = 0; e < E; ++e) tmp[e] = k + e < kend ? p[e] : T(0);
      v = *reinterpret_cast<const floatx4*>(tmp);
    }
  }
  return v;
}

// One BM x BN tile of C = P * Q^T over K range [kbeg, kend): rows m0.. of P
// and C, rows n0.. of Q (columns of C); lds holds 2 * kStage floats.
// DEPTH = slabs in flight between global memory and LDS: 1 (one register
// set), or 2 (two register sets, the slab loop taken two at a time).
template <typename T, int BM, int BN, int WM, int WN, int DEPTH = 1>
__device__ __forceinline__ void gemm_tile(const T* __restrict__ P, int64_t ldp,
                                          const T* __restrict__ Q, int64_t ldq,
                                          float* __restrict__ Cs, int64_t ldc, int M,
                                          int N, int m0, int n0, int kbeg, int kend,
                                          float* lds) {
  using Cfg = GemmCfg<BM, BN, WM, WN>;
  constexpr int E = Elem<T>::kPerChunk;
  constexpr int SK = kChunks * E;  // K elements per slab
  const int nslabs = kend > kbeg ? (kend - kbeg + SK - 1) / SK : 0;

  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wave = tid / kWave;
  const int wm = wave % WM;
  const int wn = wave / WM;
  const int lrow = lane % 32;
  const int lhalf = lane / 32;

  const T* Pblk = P + (int64_t)m0 * ldp;
  const T* Qblk = Q + (int64_t)n0 * ldq;
  const int mrows = M - m0;
  const int nrows = N - n0;

  floatx16 acc[Cfg::kFM][Cfg::kFN];
#pragma unroll
  for (int i = 0; i < Cfg::kFM; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::kFN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  static_assert(DEPTH == 1 || DEPTH == 2, "one or two slabs in flight");
  floatx4 pre_p[DEPTH][Cfg::kPVec];
  floatx4 pre_q[DEPTH][Cfg::kQVec];

  // Small wave tiles (at most two MFMA blocks) load interior slabs of full
  // tiles without per-row or per-K guards, and read the operands of the
  // next 8-wide K chunk from LDS while the current chunk's MFMAs run (two
  // register sets).  Larger wave tiles issue enough MFMAs per LDS read to
  // cover its latency, and measured slower with either change.
  constexpr bool kPrefetch = Cfg::kFM * Cfg::kFN <= 2;
  const bool full_rows = mrows >= BM && nrows >= BN;
  auto fetch = [&](auto set_tag, int k0) {
    constexpr int R = decltype(set_tag)::value;
    if (kPrefetch && full_rows && k0 + SK <= kend) {
#pragma unroll
      for (int v = 0; v < Cfg::kPVec; ++v) {
        const int f = tid + v * Cfg::kThreads;
        pre_p[R][v] = *reinterpret_cast<const floatx4*>(
            Pblk + (int64_t)(f / kChunks) * ldp + k0 + (f % kChunks) * E);
      }
#pragma unroll
      for (int v = 0; v < Cfg::kQVec; ++v) {
        const int f = tid + v * Cfg::kThreads;
        pre_q[R][v] = *reinterpret_cast<const floatx4*>(
            Qblk + (int64_t)(f / kChunks) * ldq + k0 + (f % kChunks) * E);
      }
      return;
    }
#pragma unroll
    for (int v = 0; v < Cfg::kPVec; ++v) {
      int f = tid + v * Cfg::kThreads;
      pre_p[R][v] = load_chunk<T>(Pblk, ldp, f / kChunks, mrows, k0 + (f % kChunks) * E, kend);
    }
#pragma unroll
    for (int v = 0; v < Cfg::kQVec; ++v) {
      int f = tid + v * Cfg::kThreads;
      pre_q[R][v] = load_chunk<T>(Qblk, ldq, f / kChunks, nrows, k0 + (f % kChunks) * E, kend);
    }
  };
  auto stash = [&](auto set_tag, float* st) {
    constexpr int R = decltype(set_tag)::value;
#pragma unroll
    for (int v = 0; v < Cfg::kPVec; ++v) {
      int f = tid + v * Cfg::kThreads;
      *reinterpret_cast<floatx4*>(&st[swz(f / kChunks, f % kChunks)]) = pre_p[R][v];
    }
    float* sq = st + BM * kBK;
#pragma unroll
    for (int v = 0; v < Cfg::kQVec; ++v) {
      int f = tid + v * Cfg::kThreads;
      *reinterpret_cast<floatx4*>(&sq[swz(f / kChunks, f % kChunks)]) = pre_q[R][v];
    }
  };

  // the MFMAs of slab ks, from LDS stage ks & 1
  auto compute = [&](int ks) {
    const float* sp = lds + (ks & 1) * Cfg::kStage;
    const float* sq = sp + BM * kBK;
    floatx4 a[2][Cfg::kFM];
    floatx4 bq[2][Cfg::kFN];
    auto read_ops = [&](int buf, int c8) {
      const int chunk = c8 + lhalf;  // k offset 4 * chunk within the slab
#pragma unroll
      for (int i = 0; i < Cfg::kFM; ++i)
        a[buf][i] = *reinterpret_cast<const floatx4*>(
            &sp[swz(wm * Cfg::kTM + i * 32 + lrow, chunk)]);
#pragma unroll
      for (int j = 0; j < Cfg::kFN; ++j)
        bq[buf][j] = *reinterpret_cast<const floatx4*>(
            &sq[swz(wn * Cfg::kTN + j * 32 + lrow, chunk)]);
    };
    if (kPrefetch) read_ops(0, 0);
#pragma unroll
    for (int c8 = 0; c8 < kChunks; c8 += 2) {
      const int cur = kPrefetch ? (c8 / 2) & 1 : 0;
      if (!kPrefetch) {
        read_ops(0, c8);
      } else if (c8 + 2 < kChunks) {
        read_ops(cur ^ 1, c8 + 2);
        // keep the scheduler from sinking those reads below the MFMAs
        __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (E == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int i = 0; i < Cfg::kFM; ++i)
#pragma unroll
            for (int j = 0; j < Cfg::kFN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cur][i][e], bq[cur][j][e],
                                                               acc[i][j], 0, 0, 0);
      } else {
#pragma unroll
        for (int i = 0; i < Cfg::kFM; ++i)
#pragma unroll
          for (int j = 0; j < Cfg::kFN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, a[cur][i]), __builtin_bit_cast(bf16x8, bq[cur][j]),
                acc[i][j], 0, 0, 0);
      }
    }
  };
  using S0 = std::integral_constant<int, 0>;
  if constexpr (DEPTH == 1) {
    if (nslabs > 0) {
      fetch(S0{}, kbeg);
      stash(S0{}, lds);
    }
    __syncthreads();
    for (int ks = 0; ks < nslabs; ++ks) {
      if (ks + 1 < nslabs) fetch(S0{}, kbeg + (ks + 1) * SK);
      compute(ks);
      if (ks + 1 < nslabs) stash(S0{}, lds + ((ks + 1) & 1) * Cfg::kStage);
      __syncthreads();
    }
  } else {
    // slab ks + 2 loads into the register set that slab ks left while
    // slab ks is multiplied and slab ks + 1 waits in the other set
    using S1 = std::integral_constant<int, 1>;
    if (nslabs > 0) {
      fetch(S0{}, kbeg);
      stash(S0{}, lds);
    }
    if (nslabs > 1) fetch(S1{}, kbeg + SK);
    __syncthreads();
    int ks = 0;
    for (; ks + 1 < nslabs; ks += 2) {
      if (ks + 2 < nslabs) fetch(S0{}, kbeg + (ks + 2) * SK);
      compute(ks);
      stash(S1{}, lds + Cfg::kStage);
      __syncthreads();
      if (ks + 3 < nslabs) fetch(S1{}, kbeg + (ks + 3) * SK);
      compute(ks + 1);
      if (ks + 2 < nslabs) stash(S0{}, lds);
      __syncthreads();
    }
    if (ks < nslabs) compute(ks);
  }

  // Accumulator layout of the 32x32 block: register e of lane l holds
  // row 8 * (e / 4) + 4 * (l / 32) + e % 4, column l % 32.
#pragma unroll
  for (int i = 0; i < Cfg::kFM; ++i) {
#pragma unroll
    for (int j = 0; j < Cfg::kFN; ++j) {
      const int col = n0 + wn * Cfg::kTN + j * 32 + lrow;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = m0 + wm * Cfg::kTM + i * 32 + 8 * (e / 4) + 4 * lhalf + (e % 4);
        if (row < M && col < N) Cs[(int64_t)row * ldc + col] = acc[i][j][e];
      }
    }
  }
}

// DEPTH 2 holds two register sets of slabs; its one compiled shape
// (64 x 128) is held to 168 registers so that a CU keeps three workgroups.
template <typename T, int BM, int BN, int WM, int WN, int DEPTH = 1>
__global__ __launch_bounds__(WM* WN* kWave, DEPTH == 2 ? 3 : 1) void gemm_nt_kernel(
    const T* __restrict__ P, int64_t ldp, const T* __restrict__ Q,
    int64_t ldq, float* __restrict__ C, int64_t ldc, int M, int N, int K,
    int tiles_m, int tiles_mn, int splits, int kslabs_per_split,
    int64_t split_stride, const int32_t* __restrict__ gate, int32_t gate_run,
    const int32_t* __restrict__ kdev) {
  using Cfg = GemmCfg<BM, BN, WM, WN>;
  constexpr int SK = kChunks * Elem<T>::kPerChunk;  // K elements per slab
  if (gate != nullptr && *gate != gate_run) return;
  if (kdev != nullptr) {
    K = *kdev;
    kslabs_per_split = (K + SK - 1) / SK;
  }

  __shared__ __attribute__((aligned(16))) float lds[2 * Cfg::kStage];

  // Blocks are dealt to the 8 XCDs round-robin (block b to XCD b mod 8).
  // Unsplit, renumber so that runs of consecutive tiles (the M tiles sharing
  // one Q tile) stay on one XCD and reuse its L2.  Split, keep the split
  // index fastest: with a power-of-two split count the blocks of one K range
  // share XCDs, so each XCD reads only its K ranges of P and Q (the whole P
  // on every XCD cost 12% at 256 x 5000 x 50000 with 8 splits).
  int b = blockIdx.x;
  if (splits == 1) {
    const int per_xcd = tiles_mn / 8;
    if (b < per_xcd * 8) b = (b % 8) * per_xcd + b / 8;
  }
  const int split = b % splits;
  const int t = b / splits;
  const int tm = t % tiles_m;
  const int tn = t / tiles_m;
  const int kbeg = split * kslabs_per_split * SK;
  int kend = kbeg + kslabs_per_split * SK;
  kend = kend < K ? kend : K;
  gemm_tile<T, BM, BN, WM, WN, DEPTH>(P, ldp, Q, ldq, C + (int64_t)split * split_stride, ldc,
                               M, N, tm * BM, tn * BN, kbeg, kend, lds);
}

// Grouped products: one launch over the tiles of several independent
// products (GemmGroupDesc), each tile owned by the product whose tile range
// holds its block index.  The products of a request none of whose starts
// still runs (running[req] == 0) are skipped.
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(WM* WN* kWave) void gemm_group_kernel(
    const GemmGroupDesc* __restrict__ d, int count, const int32_t* __restrict__ running) {
  using Cfg = GemmCfg<BM, BN, WM, WN>;
  constexpr int SK = kChunks * Elem<float>::kPerChunk;
  __shared__ __attribute__((aligned(16))) float lds[2 * Cfg::kStage];
  const int b = blockIdx.x;
  // the last product whose first tile is at or below b (tile0 ascending)
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (d[mid].tile0 <= b) lo = mid; else hi = mid - 1;
  }
  const GemmGroupDesc g = d[lo];
  if (running != nullptr && running[g.req] == 0) return;
  const int local = b - g.tile0;
  const int split = local % g.splits;
  const int t = local / g.splits;
  const int tm = t % g.tiles_m;
  const int tn = t / g.tiles_m;
  const int kbeg = split * g.kslabs_per_split * SK;
  int kend = kbeg + g.kslabs_per_split * SK;
  kend = kend < g.K ? kend : g.K;
  gemm_tile<float, BM, BN, WM, WN>(g.P, g.ldp, g.Q, g.ldq, g.C + (int64_t)split * g.split_stride,
                                   g.ldc, g.M, g.N, tm * BM, tn * BN, kbeg, kend, lds);
}

// Compiled tile shapes.  occ = workgroups a CU holds at once (LDS and
// registers); eff = relative MFMA efficiency of the shape measured on
// MI355X (larger per-wave tiles reuse each LDS read for more MFMAs); eff16
// the same for BF16 operands, where a tile's operand bytes per MFMA (global
// and LDS) limit it long before the matrix cores do, so the largest tiles
// win (measured on 256 x 50000 x 5000 and 256 x 5000 x 50000); with one
// workgroup per CU, 8 waves (two per SIMD) hide more of its load latency
// than 4.  A shape with eff (eff16) 0 is never planned for FP32 (BF16) by
// the model, only by the autotuner.
struct Shape {
  int bm, bn, occ;
  double eff, eff16;
};
constexpr Shape kShapes[] = {
    {128, 128, 2, 1.00, 0.73},  // 2x2 waves of 64x64
    {128, 160, 2, 1.00, 0.80},  // 4x1 waves of 32x160
    {128, 96, 2, 0.92, 0.73},   // 4x1 waves of 32x96
    {128, 64, 3, 0.85, 0.64},   // 2x2 waves of 64x32
    {64, 128, 3, 0.85, 0.65},   // 2x2 waves of 32x64
    {32, 128, 3, 0.70, 0.48},   // 1x4 waves of 32x32
    {64, 256, 2, 0.85, 0.57},   // 1x4 waves of 64x64
    {256, 128, 1, 0.90, 0.85},  // 2x2 waves of 128x64
    {256, 256, 1, 0.90, 1.25},  // 2x2 waves of 128x128
    {256, 256, 1, 0.0, 1.36},   // 2x4 waves of 128x64: BF16 only (2 waves per SIMD)
    {256, 256, 1, 0.0, 0.0},    // 4x2 waves of 64x128: tuning candidate only
    {64, 128, 3, 0.0, 0.0},     // 2x2 waves of 32x64, two slabs in flight: tuning candidate only
};
constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));

template <typename T, int BM, int BN, int WM, int WN, int DEPTH = 1>
void launch(hipStream_t st, const T* P, int64_t ldp, const T* Q,
            int64_t ldq, float* C, int64_t ldc, int64_t M, int64_t N,
            int64_t K, int splits, int64_t split_stride, const int32_t* gate,
            int32_t gate_run, const int32_t* kdev) {
  const int tiles_m = (int)ceil_div(M, BM);
  const int tiles_n = (int)ceil_div(N, BN);
  const int kslabs = (int)ceil_div(K, kChunks * Elem<T>::kPerChunk);
  const int per_split = (int)ceil_div(kslabs, splits);
  const int total = tiles_m * tiles_n * splits;
  hipLaunchKernelGGL((gemm_nt_kernel<T, BM, BN, WM, WN, DEPTH>), dim3(total),
                     dim3(WM * WN * kWave), 0, st, P, ldp, Q, ldq, C, ldc,
                     (int)M, (int)N, (int)K, tiles_m, tiles_m * tiles_n, splits,
                     per_split, split_stride, gate, gate_run, kdev);
}

template <typename T>
void dispatch(int shape, hipStream_t st, const T* P, int64_t ldp,
              const T* Q, int64_t ldq, float* C, int64_t ldc, int64_t M,
              int64_t N, int64_t K, int splits, int64_t split_stride,
              const int32_t* gate, int32_t gate_run, const int32_t* kdev) {
  switch (shape) {
    case 0:
      launch<T, 128, 128, 2, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 1:
      launch<T, 128, 160, 4, 1>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 2:
      launch<T, 128, 96, 4, 1>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 3:
      launch<T, 128, 64, 2, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 4:
      launch<T, 64, 128, 2, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 5:
      launch<T, 32, 128, 1, 4>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 6:
      launch<T, 64, 256, 1, 4>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 7:
      launch<T, 256, 128, 2, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 8:
      launch<T, 256, 256, 2, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 9:
      launch<T, 256, 256, 2, 4>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    case 10:
      launch<T, 256, 256, 4, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
    default:
      launch<T, 64, 128, 2, 2, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, splits, split_stride, gate, gate_run, kdev);
      break;
  }
}

}  // namespace

// Choice of tile shape and K split: a measured winner from the tuning table
// when there is one, else the deterministic model below.
// Model of one launch, in cycles of one CU:
//   a workgroup's MFMA work  w = BM * BN * (K slabs per split * 32)
//                               / (128 MACs per cycle * eff);
//   the workgroups fill rounds of 256 CUs x occ slots; a CU running k
//   workgroups at once takes w * max(k, 1.5) (one workgroup alone cannot
//   keep the matrix cores busy), so the partial last round costs
//   w * max(ceil(rest / 256), 1.5);
//   split partials cost their HBM traffic, 8 bytes per element per split at
//   about 1.7 KB per cycle for the whole chip.
// ---------------------------------------------------------------------------
// Tuning table: measured winners keyed by element width, max splits and the
// half-octave buckets of M, N and K (round(2 log2 x)).  Filled by the
// autotuner of the solve (or imported as text); consulted before the model.
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
  int eb, ms, bm, bn, bk;
  bool operator<(const TuneKey& o) const {
    if (eb != o.eb) return eb < o.eb;
    if (ms != o.ms) return ms < o.ms;
    if (bm != o.bm) return bm < o.bm;
    if (bn != o.bn) return bn < o.bn;
    return bk < o.bk;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, GemmPlan> g_tune;

int bucket(int64_t x) { return (int)std::lround(2.0 * std::log2((double)(x > 0 ? x : 1))); }
TuneKey key_of(int64_t M, int64_t N, int64_t K, int ms, int eb) {
  return TuneKey{eb, ms, bucket(M), bucket(N), bucket(K)};
}
}  // namespace

bool tuned_plan(int64_t M, int64_t N, int64_t K, int max_splits, int elem_bytes,
                GemmPlan* out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(key_of(M, N, K, max_splits, elem_bytes));
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

void record_tuned_plan(int64_t M, int64_t N, int64_t K, int max_splits,
                       int elem_bytes, GemmPlan plan) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key_of(M, N, K, max_splits, elem_bytes)] = plan;
}

std::string tune_table_text() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::ostringstream os;
  for (const auto& kv : g_tune)
    os << kv.first.eb << ' ' << kv.first.ms << ' ' << kv.first.bm << ' ' << kv.first.bn
       << ' ' << kv.first.bk << ' ' << kv.second.shape << ' ' << kv.second.splits << '\n';
  return os.str();
}

bool tune_table_load(const char* text, std::string* err) {
  std::map<TuneKey, GemmPlan> t;
  std::istringstream is(text);
  std::string line;
  int ln = 0;
  while (std::getline(is, line)) {
    ++ln;
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    std::istringstream ls(line);
    TuneKey k;
    GemmPlan g;
    if (!(ls >> k.eb >> k.ms >> k.bm >> k.bn >> k.bk >> g.shape >> g.splits) ||
        (k.eb != 2 && k.eb != 4) || g.shape < 0 || g.shape >= gemm_num_shapes() ||
        g.splits < 1 || g.splits > k.ms) {
      *err = "bad tuning entry on line " + std::to_string(ln);
      return false;
    }
    t[k] = g;
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const auto& kv : t) g_tune[kv.first] = kv.second;
  return true;
}

void tune_table_clear() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
}

int max_feasible_splits(int64_t K, int max_splits, int elem_bytes) {
  const int64_t kslabs = ceil_div(K, 128 / elem_bytes);
  int s = 1;
  while (s * 2 <= max_splits && ceil_div(kslabs, (int64_t)s * 2) >= 8) s *= 2;
  return s;
}

GemmPlan plan_gemm_nt(int64_t M, int64_t N, int64_t K, int max_splits,
                      int elem_bytes) {
  {
    // a tuning-table entry covers a size bucket: its split count is capped
    // at what this K allows, which is what callers size split buffers for
    GemmPlan t;
    if (tuned_plan(M, N, K, max_splits, elem_bytes, &t)) {
      const int cap = max_feasible_splits(K, max_splits, elem_bytes);
      if (t.splits > cap) t.splits = cap;
      if (t.splits < 1) t.splits = 1;
      return t;
    }
  }
  return model_plan_gemm_nt(M, N, K, max_splits, elem_bytes);
}

GemmPlan model_plan_gemm_nt(int64_t M, int64_t N, int64_t K, int max_splits,
                            int elem_bytes) {
  GemmPlan best{0, 1};
  double best_cost = 1e300;
  const int64_t slab_k = 128 / elem_bytes;
  const int64_t kslabs = ceil_div(K, slab_k);
  // MACs per cycle per CU: FP32 MFMA 128; BF16 operands are limited by
  // operand traffic well below their MFMA rate, taken as 4x FP32 times the
  // shape's BF16 efficiency
  const double macs = elem_bytes == 4 ? 128.0 : 512.0;
  for (int s = 0; s < kNumShapes; ++s) {
    const Shape& sh = kShapes[s];
    if (sh.bm > 32 && M <= sh.bm / 2) continue;  // mostly padding rows
    const int64_t tiles = ceil_div(M, sh.bm) * ceil_div(N, sh.bn);
    for (int splits = 1; splits <= max_splits; splits *= 2) {
      const int64_t per = ceil_div(kslabs, splits);
      if (splits > 1 && per < 8) break;  // too little K per split
      const int64_t wgs = tiles * splits;
      const int64_t slots = 256LL * sh.occ;
      const double eff = elem_bytes == 4 ? sh.eff : sh.eff16;
      const double w = (double)sh.bm * sh.bn * (double)(per * slab_k) / (macs * eff);
      const int64_t full = wgs / slots;
      const int64_t rest = wgs % slots;
      double cost = (double)full * w * (sh.occ > 1.5 ? sh.occ : 1.5);
      if (rest > 0) {
        double k = (double)ceil_div(rest, 256);
        cost += w * (k > 1.5 ? k : 1.5);
      }
      if (splits > 1) cost += (double)splits * M * N * 8.0 / 1700.0;
      if (cost < best_cost * 0.999) {
        best_cost = cost;
        best = GemmPlan{s, splits};
      }
    }
  }
  return best;
}

int gemm_num_shapes() { return kNumShapes; }
int gemm_shape_bm(int shape) {
  return shape >= 0 && shape < kNumShapes ? kShapes[shape].bm : 0;
}

void gemm_nt_f32(hipStream_t st, const float* P, int64_t ldp, const float* Q,
                 int64_t ldq, float* C, int64_t ldc, int64_t M, int64_t N,
                 int64_t K, const int32_t* gate, int32_t gate_run,
                 GemmPlan plan, int64_t split_stride, const int32_t* kdev) {
  if (M <= 0 || N <= 0) return;
  if (kdev != nullptr) plan.splits = 1;
  dispatch<float>(plan.shape, st, P, ldp, Q, ldq, C, ldc, M, N, K, plan.splits,
                  split_stride, gate, gate_run, kdev);
}

void gemm_nt_bf16(hipStream_t st, const uint16_t* P, int64_t ldp,
                  const uint16_t* Q, int64_t ldq, float* C, int64_t ldc,
                  int64_t M, int64_t N, int64_t K, const int32_t* gate,
                  int32_t gate_run, GemmPlan plan, int64_t split_stride) {
  if (M <= 0 || N <= 0) return;
  dispatch<uint16_t>(plan.shape, st, P, ldp, Q, ldq, C, ldc, M, N, K,
                     plan.splits, split_stride, gate, gate_run, nullptr);
}

void gemm_group_tiles(GemmGroupDesc* d, int count, int* total_tiles) {
  int t = 0;
  for (int q = 0; q < count; ++q) {
    d[q].tiles_m = (int32_t)ceil_div((int64_t)d[q].M, (int64_t)kGroupBM);
    const int tiles_n = (int)ceil_div((int64_t)d[q].N, (int64_t)kGroupBN);
    const int kslabs = (int)ceil_div((int64_t)d[q].K, (int64_t)kChunks * 4);
    if (d[q].splits < 1) d[q].splits = 1;
    d[q].kslabs_per_split = (int32_t)ceil_div((int64_t)kslabs, (int64_t)d[q].splits);
    d[q].tile0 = t;
    t += d[q].tiles_m * tiles_n * d[q].splits;
  }
  *total_tiles = t;
}

void gemm_nt_f32_group(hipStream_t st, const GemmGroupDesc* d_dev, int count, int total_tiles,
                       const int32_t* running) {
  if (count <= 0 || total_tiles <= 0) return;
  static_assert(kGroupBM == 64 && kGroupBN == 128, "group tile shape");
  hipLaunchKernelGGL((gemm_group_kernel<64, 128, 2, 2>), dim3((unsigned)total_tiles),
                     dim3(4 * kWave), 0, st, d_dev, count, running);
}

}  // namespace spca
