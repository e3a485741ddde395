// FP32 "NT" GEMM on CDNA4 matrix cores: C = P * Q^T with P (M x K) and
// Q (N x K) both K-contiguous.  Both products of an AM iteration have this
// shape once A is held column-major (for A^T Y) and row-major (for A X):
//   V^T (r x p) = Y^T (r x n) * [A columns] (p x n)^T     K = n
//   U^T (r x n) = X^T (r x p) * [A rows]    (n x p)^T     K = p
//
// Tiling: a workgroup of WM x WN waves owns a BM x BN tile of C; each wave
// owns (BM/WM) x (BN/WN) built from 32 x 32 v_mfma_f32_32x32x2_f32 blocks.
// K advances BK at a time through one LDS buffer, with the next tile
// prefetched into registers while the current one is consumed.
// Within an 8-wide K chunk, lane l of a wave feeds row (l % 32) at k offset
// 4 * (l / 32) .. +3 as one 16-byte LDS read; the i-th of the four MFMAs of
// the chunk takes element i.  The order in which k terms enter the sum does
// not change the product, so this keeps every LDS read 16 bytes wide.
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kPad = 4;  // floats of padding per LDS row

template <int BM, int BN, int BK, int WM, int WN>
struct GemmCfg {
  static constexpr int kThreads = WM * WN * kWave;
  static constexpr int kTM = BM / WM;  // rows per wave
  static constexpr int kTN = BN / WN;  // cols per wave
  static constexpr int kFM = kTM / 32;
  static constexpr int kFN = kTN / 32;
  static constexpr int kLdsRow = BK + kPad;
  static constexpr int kPVec = BM * BK / 4 / kThreads;  // float4 per thread
  static constexpr int kQVec = BN * BK / 4 / kThreads;
  static_assert(kTM % 32 == 0 && kTN % 32 == 0, "wave tile must be 32-aligned");
  static_assert(BK % 8 == 0, "BK must be a multiple of 8");
  static_assert((BM * BK / 4) % kThreads == 0, "P tile load must divide");
  static_assert((BN * BK / 4) % kThreads == 0, "Q tile load must divide");
};

__device__ __forceinline__ floatx4 load_row4(const float* __restrict__ base,
                                             int64_t ld, int row, int nrows,
                                             int k, int K) {
  floatx4 v = {0.f, 0.f, 0.f, 0.f};
  if (row < nrows) {
    const float* p = base + (int64_t)row * ld + k;
    if (k + 3 < K) {
      v = *reinterpret_cast<const floatx4*>(p);
    } else {
      if (k + 0 < K) v.x = p[0];
      if (k + 1 < K) v.y = p[1];
      if (k + 2 < K) v.z = p[2];
    }
  }
  return v;
}

template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM* WN* kWave) void gemm_nt_f32_kernel(
    const float* __restrict__ P, int64_t ldp, const float* __restrict__ Q,
    int64_t ldq, float* __restrict__ C, int64_t ldc, int M, int N, int K,
    int tiles_m, int tiles_total, const int32_t* __restrict__ gate,
    int32_t gate_skip) {
  using Cfg = GemmCfg<BM, BN, BK, WM, WN>;
  if (gate != nullptr && *gate == gate_skip) return;

  __shared__ __attribute__((aligned(16))) float Ps[BM * Cfg::kLdsRow];
  __shared__ __attribute__((aligned(16))) float Qs[BN * Cfg::kLdsRow];

  // Blocks are dealt to the 8 XCDs round-robin; renumber so that runs of
  // consecutive tiles (the M tiles sharing one Q tile) stay on one XCD and
  // reuse its L2.
  int b = blockIdx.x;
  const int per_xcd = tiles_total / 8;
  if (b < per_xcd * 8) b = (b % 8) * per_xcd + b / 8;
  const int tm = b % tiles_m;
  const int tn = b / tiles_m;
  const int m0 = tm * BM;
  const int n0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wave = tid / kWave;
  const int wm = wave % WM;
  const int wn = wave / WM;
  const int lrow = lane % 32;
  const int lk = 4 * (lane / 32);

  const float* Pblk = P + (int64_t)m0 * ldp;
  const float* Qblk = Q + (int64_t)n0 * ldq;
  const int mrows = M - m0;
  const int nrows = N - n0;

  floatx16 acc[Cfg::kFM][Cfg::kFN];
#pragma unroll
  for (int i = 0; i < Cfg::kFM; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::kFN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  floatx4 pre_p[Cfg::kPVec];
  floatx4 pre_q[Cfg::kQVec];
  constexpr int kVecPerRow = BK / 4;

  auto fetch = [&](int k0) {
#pragma unroll
    for (int v = 0; v < Cfg::kPVec; ++v) {
      int f = tid + v * Cfg::kThreads;
      int row = f / kVecPerRow;
      int kc = (f % kVecPerRow) * 4;
      pre_p[v] = load_row4(Pblk, ldp, row, mrows, k0 + kc, K);
    }
#pragma unroll
    for (int v = 0; v < Cfg::kQVec; ++v) {
      int f = tid + v * Cfg::kThreads;
      int row = f / kVecPerRow;
      int kc = (f % kVecPerRow) * 4;
      pre_q[v] = load_row4(Qblk, ldq, row, nrows, k0 + kc, K);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int v = 0; v < Cfg::kPVec; ++v) {
      int f = tid + v * Cfg::kThreads;
      int row = f / kVecPerRow;
      int kc = (f % kVecPerRow) * 4;
      *reinterpret_cast<floatx4*>(&Ps[row * Cfg::kLdsRow + kc]) = pre_p[v];
    }
#pragma unroll
    for (int v = 0; v < Cfg::kQVec; ++v) {
      int f = tid + v * Cfg::kThreads;
      int row = f / kVecPerRow;
      int kc = (f % kVecPerRow) * 4;
      *reinterpret_cast<floatx4*>(&Qs[row * Cfg::kLdsRow + kc]) = pre_q[v];
    }
  };

  const int ktiles = (K + BK - 1) / BK;
  fetch(0);
  stash();
  __syncthreads();
  for (int kt = 0; kt < ktiles; ++kt) {
    if (kt + 1 < ktiles) fetch((kt + 1) * BK);
#pragma unroll
    for (int kc = 0; kc < BK; kc += 8) {
      floatx4 a[Cfg::kFM];
      floatx4 bq[Cfg::kFN];
#pragma unroll
      for (int i = 0; i < Cfg::kFM; ++i)
        a[i] = *reinterpret_cast<const floatx4*>(
            &Ps[(wm * Cfg::kTM + i * 32 + lrow) * Cfg::kLdsRow + kc + lk]);
#pragma unroll
      for (int j = 0; j < Cfg::kFN; ++j)
        bq[j] = *reinterpret_cast<const floatx4*>(
            &Qs[(wn * Cfg::kTN + j * 32 + lrow) * Cfg::kLdsRow + kc + lk]);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int i = 0; i < Cfg::kFM; ++i)
#pragma unroll
          for (int j = 0; j < Cfg::kFN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][e], bq[j][e],
                                                             acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (kt + 1 < ktiles) {
      stash();
      __syncthreads();
    }
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
        const int row = m0 + wm * Cfg::kTM + i * 32 + 8 * (e / 4) + lk + (e % 4);
        if (row < M && col < N) C[(int64_t)row * ldc + col] = acc[i][j][e];
      }
    }
  }
}

template <int BM, int BN, int BK, int WM, int WN>
void launch(hipStream_t st, const float* P, int64_t ldp, const float* Q,
            int64_t ldq, float* C, int64_t ldc, int64_t M, int64_t N,
            int64_t K, const int32_t* gate, int32_t gate_skip) {
  const int tiles_m = (int)ceil_div(M, BM);
  const int tiles_n = (int)ceil_div(N, BN);
  const int total = tiles_m * tiles_n;
  hipLaunchKernelGGL((gemm_nt_f32_kernel<BM, BN, BK, WM, WN>), dim3(total),
                     dim3(WM * WN * kWave), 0, st, P, ldp, Q, ldq, C, ldc,
                     (int)M, (int)N, (int)K, tiles_m, total, gate, gate_skip);
}

}  // namespace

void gemm_nt_f32(hipStream_t st, const float* P, int64_t ldp, const float* Q,
                 int64_t ldq, float* C, int64_t ldc, int64_t M, int64_t N,
                 int64_t K, const int32_t* gate, int32_t gate_skip) {
  if (M <= 0 || N <= 0) return;
  if (M <= 32) {
    launch<32, 128, 32, 1, 4>(st, P, ldp, Q, ldq, C, ldc, M, N, K, gate, gate_skip);
  } else if (M <= 64) {
    launch<64, 128, 32, 2, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, gate, gate_skip);
  } else {
    launch<128, 128, 32, 2, 2>(st, P, ldp, Q, ldq, C, ldc, M, N, K, gate, gate_skip);
  }
}

}  // namespace spca
