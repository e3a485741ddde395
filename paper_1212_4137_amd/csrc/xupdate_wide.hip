// x-update for long rows (p beyond what one workgroup keeps in registers):
// each row of V is cut into chunks of kWCH elements and every chunk gets its
// own workgroup, so a launch has (chunks x starts) workgroups instead of one
// per start.  Row-level decisions are taken by small per-row kernels between
// the chunk passes; every sum is reduced in a fixed order, so results do not
// depend on timing.  Operators (Table 3, rows S3-S6):
//   T_s   exact top-s by |v| with ties to the lowest index: a radix select
//         over the 31-bit keys of |v| in three digit passes (11, 10, 10
//         bits); each pass histograms the keys that share the prefix fixed
//         so far (LDS histogram per chunk, integer atomics into one global
//         histogram per row) and a per-row kernel picks the digit holding
//         the s-th largest key.  When the s-th key is shared by more
//         elements than are still needed, a counting pass gives each chunk
//         the number of such ties before it.
//   U_g   keep v_i with v_i^2 > g;  V_g  soft threshold at g.
//   V_{lambda_s}  the exact lambda of the one-workgroup kernel, found the
//         same way: the M largest |v_i| (M from the previous support size)
//         by the T_s passes, FP64 chunk sums that decide whether the
//         constraint is active and whether the root lies among them, then
//         one workgroup per row sorts the candidates and scans their
//         segments for the closed-form root (an FP64 search over float
//         intervals of the row when it does not lie there); then the soft
//         threshold at that lambda.
// Then: per-chunk FP64 partial sums (count, ||w||^2, sum (w^2 - g)), a
// per-row kernel that adds them in chunk order, applies the stop test and
// turns the counts into list offsets, and an emit pass that writes
// x = w / ||w|| (and the index list and column marks).
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr int kWT = 256;              // threads per chunk workgroup
constexpr int kWN = 16;               // elements per thread
constexpr int kWCH = kWT * kWN;       // chunk length
constexpr int kWBins = 2048;          // largest digit (11 bits)
constexpr int kNWv = kWT / kWave;
constexpr int kMaxCandW = 2048;       // lambda_s candidates sorted per row
constexpr int kNCdW = 7;              // thresholds per FP64 search step

typedef float floatx4 __attribute__((ext_vector_type(4)));

struct WRow {
  uint32_t prefix;   // key bits fixed so far (the full key after pass 3)
  int32_t need;      // elements still to take at or below the prefix
  int32_t eq_total;  // elements whose key equals the final key
  int32_t straddle;  // 1 when only part of those are taken
  int32_t live;      // row processed in this x-update
  int32_t listed;    // the index list is written
  int32_t zero;      // w = 0
  int32_t marking;   // kept columns get colmark = epoch
  int32_t epoch;
  int32_t lmode;     // lambda_s: 0 inactive, 1 candidates, 2 search
  double inv;        // 1 / ||w||
  double lam;        // lambda_s of the row
  int32_t ncand;     // lambda_s candidates (keys >= prefix)
  uint32_t mk;       // largest key of the row
};

struct Wide {
  uint32_t* ghist;  // r x kWBins
  WRow* rows;       // r
  int32_t* eqcnt;   // r x nch
  int32_t* cnt;     // r x nch: kept count, then list offset
  double* part;     // r x nch x 2
  double* lpart;    // r x nch x 4 (lambda_s sums)
  uint32_t* lmax;   // r x nch (largest key per chunk)
  float* cand;      // r x kMaxCandW
  int nch;
  int32_t warm_K;   // sparsity-targeted warm-up (0: off)
  int32_t warm_target;
  double* gam;      // r: parameter of each start under the warm-up
};

Wide carve_wide(void* base, int64_t r, int64_t p) {
  Wide w;
  w.nch = (int)ceil_div(p, kWCH);
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = c + off;
    off += (bytes + 255) / 256 * 256;
    return q;
  };
  w.ghist = (uint32_t*)take(sizeof(uint32_t) * kWBins * r);
  w.rows = (WRow*)take(sizeof(WRow) * r);
  w.eqcnt = (int32_t*)take(sizeof(int32_t) * r * w.nch);
  w.cnt = (int32_t*)take(sizeof(int32_t) * r * w.nch);
  w.part = (double*)take(sizeof(double) * 2 * r * w.nch);
  w.lpart = (double*)take(sizeof(double) * 4 * r * w.nch);
  w.lmax = (uint32_t*)take(sizeof(uint32_t) * r * w.nch);
  w.cand = (float*)take(sizeof(float) * kMaxCandW * r);
  w.warm_K = 0;
  w.warm_target = 0;
  w.gam = nullptr;
  return w;
}

__device__ __forceinline__ uint32_t wkey(float v) {
  return __float_as_uint(v) & 0x7fffffffu;
}

__device__ __forceinline__ bool row_live(const StartState& s, int64_t j) {
  return s.status == nullptr || s.status[j] == kRunning;
}

__device__ __forceinline__ void load_chunk(const float* __restrict__ vg, int p,
                                           int base, float (&v)[kWN]) {
#pragma unroll
  for (int q = 0; q < kWN; q += 4) {
    const int i = base + q;
    if (i + 3 < p) {
      const floatx4 t = *reinterpret_cast<const floatx4*>(vg + i);
      v[q] = t.x;
      v[q + 1] = t.y;
      v[q + 2] = t.z;
      v[q + 3] = t.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[q + e] = i + e < p ? vg[i + e] : 0.f;
    }
  }
}

// digit pass PASS: bits [shift, shift + bits) of the key, among keys whose
// higher bits equal the prefix
template <int PASS>
struct Digit {
  static constexpr int kShift = PASS == 0 ? 20 : PASS == 1 ? 10 : 0;
  static constexpr int kBits = PASS == 0 ? 11 : 10;
  static constexpr int kBins = 1 << kBits;
};

template <int PASS>
__global__ __launch_bounds__(kWT) void wide_hist_kernel(
    const float* __restrict__ V, int64_t ldv, int p, StartState s, Wide w) {
  using D = Digit<PASS>;
  __shared__ uint32_t lh[D::kBins];
  const int64_t j = blockIdx.y;
  if (!row_live(s, j)) return;
  const int tid = threadIdx.x;
  for (int b = tid; b < D::kBins; b += kWT) lh[b] = 0u;
  const uint32_t prefix = PASS == 0 ? 0u : w.rows[j].prefix;
  __syncthreads();
  const int base = blockIdx.x * kWCH + tid * kWN;
  float v[kWN];
  load_chunk(V + j * ldv, p, base, v);
#pragma unroll
  for (int k = 0; k < kWN; ++k) {
    const uint32_t key = wkey(v[k]);
    const bool in = base + k < p &&
                    (PASS == 0 || (key >> (D::kShift + D::kBits)) == prefix);
    if (in) atomicAdd(&lh[(key >> D::kShift) & (D::kBins - 1)], 1u);
  }
  __syncthreads();
  uint32_t* gh = w.ghist + j * kWBins;
  for (int b = tid; b < D::kBins; b += kWT)
    if (lh[b] != 0u) atomicAdd(&gh[b], lh[b]);
}

// M for lambda_s: twice the previous support plus 32 (or 4 ceil(s) + 64
// without state), at least floor(s) + 2, at most kMaxCandW and p
__device__ __forceinline__ int lambda_m(const StartState& s, int64_t j, double s_par,
                                       int p) {
  int64_t m = s.status != nullptr ? 2 * (int64_t)s.nnz[j] + 32
                                  : 4 * (int64_t)ceil(s_par) + 64;
  const int64_t smin = (int64_t)floor(s_par) + 2;
  m = m < smin ? smin : m;
  m = m > kMaxCandW ? kMaxCandW : m;
  m = m > p ? p : m;
  return (int)m;
}

// per row: the digit holding the need-th largest key (need: s for T_s, M for
// lambda_s); clears the histogram
template <int PASS>
__global__ __launch_bounds__(kWT) void wide_decide_kernel(StartState s, Wide w,
                                                          int32_t s_need, int lam_mode,
                                                          double s_par, int p) {
  using D = Digit<PASS>;
  constexpr int kPer = D::kBins / kWT;
  __shared__ int scan[kNWv + 1];
  const int64_t j = blockIdx.x;
  if (!row_live(s, j)) return;
  const int tid = threadIdx.x;
  WRow* R = w.rows + j;
  const int need = PASS == 0 ? (lam_mode ? lambda_m(s, j, s_par, p) : s_need) : R->need;
  const uint32_t prefix = PASS == 0 ? 0u : R->prefix;
  uint32_t* gh = w.ghist + j * kWBins;
  // thread 0 owns the highest bins
  const int hi = D::kBins - kPer * tid;
  int c[kPer];
  int sum = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    c[e] = (int)gh[hi - 1 - e];
    sum += c[e];
  }
  int total;
  int run = block_exclusive_scan(sum, scan, &total);
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    if (run < need && need <= run + c[e]) {
      const uint32_t key = (prefix << D::kBits) | (uint32_t)(hi - 1 - e);
      R->prefix = key;
      R->need = need - run;
      if (PASS == 2) {
        R->eq_total = c[e];
        R->straddle = key != 0u && c[e] > need - run;
      }
    }
    run += c[e];
  }
#pragma unroll
  for (int e = 0; e < kPer; ++e) gh[hi - 1 - e] = 0u;
}

__global__ __launch_bounds__(kWT) void wide_eqcount_kernel(
    const float* __restrict__ V, int64_t ldv, int p, StartState s, Wide w) {
  __shared__ int red[kNWv + 1];
  const int64_t j = blockIdx.y;
  if (!row_live(s, j) || !w.rows[j].straddle) return;
  const uint32_t t = w.rows[j].prefix;
  const int base = blockIdx.x * kWCH + threadIdx.x * kWN;
  float v[kWN];
  load_chunk(V + j * ldv, p, base, v);
  int eq = 0;
#pragma unroll
  for (int k = 0; k < kWN; ++k) eq += base + k < p && wkey(v[k]) == t;
  eq = block_sum(eq, red);
  if (threadIdx.x == 0) w.eqcnt[j * w.nch + blockIdx.x] = eq;
}

// Membership and value of each element of the thread's slice.  For T_s the
// rank of an element among the ties at the final key decides (lowest
// indices first).
template <int KIND>
struct Keep {
  uint32_t t = 0;
  int straddle = 0, need = 0, rank = 0;
  double lam = 0.0;

  __device__ void setup(const Wide& w, int64_t j, double param,
                        const float (&v)[kWN], int base, int p, int* scan,
                        int* red) {
    if (KIND == kTopS) {
      const WRow& R = w.rows[j];
      t = R.prefix;
      straddle = R.straddle;
      need = R.need;
      if (straddle) {
        int before = 0;
        for (int c = threadIdx.x; c < (int)blockIdx.x; c += kWT)
          before += w.eqcnt[j * w.nch + c];
        before = block_sum(before, red);
        int eq = 0;
#pragma unroll
        for (int k = 0; k < kWN; ++k) eq += base + k < p && wkey(v[k]) == t;
        int tot;
        rank = before + block_exclusive_scan(eq, scan, &tot);
      }
    } else if (KIND == kLambdaS || w.warm_K > 0) {
      lam = w.rows[j].lam;  // per row: lambda_s, or gamma under the warm-up
    } else {
      lam = param;
    }
  }

  // call in element order over the slice
  __device__ bool operator()(float vv, bool valid, double* wv) {
    if (!valid) return false;
    if (KIND == kTopS) {
      const uint32_t k = wkey(vv);
      *wv = (double)vv;
      if (k == 0u || k < t) return false;
      if (k > t || !straddle) return true;
      return rank++ < need;
    } else if (KIND == kHardGamma) {
      *wv = (double)vv;
      return (double)vv * (double)vv > lam;
    } else {  // soft threshold: V_gamma, and V_lambda at the row's lambda
      const double a = fabs((double)vv);
      *wv = vv > 0.f ? a - lam : lam - a;
      return a > lam;
    }
  }
};

template <int KIND>
__global__ __launch_bounds__(kWT) void wide_partial_kernel(
    const float* __restrict__ V, int64_t ldv, int p, double param, StartState s,
    Wide w) {
  __shared__ int scan[kNWv + 1];
  __shared__ int red[kNWv + 1];
  __shared__ double dred[2 * (kNWv + 1)];
  const int64_t j = blockIdx.y;
  if (!row_live(s, j)) return;
  const int base = blockIdx.x * kWCH + threadIdx.x * kWN;
  float v[kWN];
  load_chunk(V + j * ldv, p, base, v);
  Keep<KIND> keep;
  keep.setup(w, j, param, v, base, p, scan, red);
  int cnt = 0;
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kWN; ++k) {
    double wv;
    if (keep(v[k], base + k < p, &wv)) {
      ++cnt;
      acc[0] += wv * wv;
      if (KIND == kHardGamma) acc[1] += wv * wv - keep.lam;
    }
  }
  block_sum_n<double, 2>(acc, dred);
  cnt = block_sum(cnt, red);
  if (threadIdx.x == 0) {
    const int64_t c = j * w.nch + blockIdx.x;
    w.cnt[c] = cnt;
    w.part[2 * c] = acc[0];
    w.part[2 * c + 1] = acc[1];
  }
}

// one thread per row: chunk sums in chunk order, phi, the stop test (the
// same state machine as the one-workgroup kernels) and list offsets
template <int KIND>
__global__ __launch_bounds__(64) void wide_row_kernel(
    int64_t r, StartState s, double tol, int maxit, int list_cap, int have_list,
    const Plan* plan, int have_marks, Wide w, double s_par) {
  const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (j >= r) return;
  WRow* R = w.rows + j;
  const bool live = row_live(s, j);
  R->live = live;
  if (!live) return;
  double a0 = 0.0, a1 = 0.0;
  int total = 0;
  for (int c = 0; c < w.nch; ++c) {
    const int64_t q = j * w.nch + c;
    a0 += w.part[2 * q];
    a1 += w.part[2 * q + 1];
    const int k = w.cnt[q];
    w.cnt[q] = total;
    total += k;
  }
  const double nrm = sqrt(a0);
  const double phi = KIND == kHardGamma ? a1
                     : KIND == kLambdaS ? R->lam * sqrt(s_par) + nrm
                                        : nrm;
  const bool zero = !(nrm > 0.0);
  R->zero = zero;
  R->inv = zero ? 0.0 : 1.0 / nrm;
  R->listed = have_list && !zero && total <= list_cap;
  R->marking = have_marks && !zero && plan != nullptr && plan->mark != 0;
  R->epoch = R->marking ? plan->epoch : 0;
  if (s.status == nullptr) {
    s.phi[j] = phi;
    s.nnz[j] = zero ? 0 : total;
  } else {
    const int it = s.iters[j] + 1;
    if (KIND != kTopS && w.warm_K > 0 && it <= w.warm_K) w.gam[j] = R->lam;
    const double prev = s.phi[j];
    s.iters[j] = it;
    s.phi_prev[j] = prev;
    s.phi[j] = phi;
    s.nnz[j] = zero ? 0 : total;
    if (zero)
      s.status[j] = SPCA_ZERO;
    else if (it >= 2 && tol >= 0.0 && (w.warm_K == 0 || it >= w.warm_K + 1) &&
             phi <= (1.0 + tol) * prev)
      s.status[j] = SPCA_CONVERGED;
    else if (it >= maxit)
      s.status[j] = SPCA_MAXIT;
  }
}

template <int KIND>
__global__ __launch_bounds__(kWT) void wide_emit_kernel(
    const float* __restrict__ V, int64_t ldv, int p, double param,
    float* __restrict__ X, int64_t ldx, int32_t* __restrict__ list_idx,
    float* __restrict__ list_val, int64_t ldl, int32_t* __restrict__ colmark,
    Wide w) {
  __shared__ int scan[kNWv + 1];
  __shared__ int red[kNWv + 1];
  const int64_t j = blockIdx.y;
  const WRow R = w.rows[j];
  if (!R.live) return;
  const int base = blockIdx.x * kWCH + threadIdx.x * kWN;
  float v[kWN];
  load_chunk(V + j * ldv, p, base, v);
  Keep<KIND> keep;
  keep.setup(w, j, param, v, base, p, scan, red);
  float xo[kWN];
  bool kp[kWN];
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < kWN; ++k) {
    double wv = 0.0;
    kp[k] = keep(v[k], base + k < p, &wv) && !R.zero;
    xo[k] = kp[k] ? (float)(wv * R.inv) : 0.f;
    cnt += kp[k];
  }
  if (R.listed) {
    int tot;
    int off = w.cnt[j * w.nch + blockIdx.x] + block_exclusive_scan(cnt, scan, &tot);
    int32_t* li = list_idx + j * ldl;
    float* lv = list_val + j * ldl;
#pragma unroll
    for (int k = 0; k < kWN; ++k) {
      if (kp[k]) {
        li[off] = base + k;
        lv[off] = xo[k];
        ++off;
      }
    }
  }
  if (R.marking) {
#pragma unroll
    for (int k = 0; k < kWN; ++k)
      if (kp[k]) colmark[base + k] = R.epoch;
  }
  float* x = X + j * ldx;
#pragma unroll
  for (int q = 0; q < kWN; q += 4) {
    const int i = base + q;
    if (i + 3 < p) {
      floatx4 t = {xo[q], xo[q + 1], xo[q + 2], xo[q + 3]};
      *reinterpret_cast<floatx4*>(x + i) = t;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i + e < p) x[i + e] = xo[q + e];
    }
  }
}


// ---------------------------------------------------------------------------
// lambda_s
// ---------------------------------------------------------------------------

// per chunk: sum |v|, sum v^2 (all entries), sum (|v| - t0)_+ and its square,
// the number of candidates (keys >= t0) and the largest key
__global__ __launch_bounds__(kWT) void lam_stats_kernel(
    const float* __restrict__ V, int64_t ldv, int p, StartState s, Wide w) {
  __shared__ double dred[4 * (kNWv + 1)];
  __shared__ int red[kNWv + 1];
  __shared__ uint32_t ured[kNWv + 1];
  const int64_t j = blockIdx.y;
  if (!row_live(s, j)) return;
  const uint32_t t0 = w.rows[j].prefix > 1u ? w.rows[j].prefix : 1u;
  const double t0f = (double)__uint_as_float(t0);
  const int base = blockIdx.x * kWCH + threadIdx.x * kWN;
  float v[kWN];
  load_chunk(V + j * ldv, p, base, v);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int c = 0;
  uint32_t mk = 0u;
#pragma unroll
  for (int k = 0; k < kWN; ++k) {
    if (base + k >= p) continue;
    const double a = fabs((double)v[k]);
    acc[0] += a;
    acc[1] += a * a;
    double d = a - t0f;
    d = d > 0.0 ? d : 0.0;
    acc[2] += d;
    acc[3] += d * d;
    const uint32_t key = wkey(v[k]);
    c += key >= t0;
    mk = key > mk ? key : mk;
  }
  block_sum_n<double, 4>(acc, dred);
  c = block_sum(c, red);
  mk = block_max(mk, ured);
  if (threadIdx.x == 0) {
    const int64_t q = j * w.nch + blockIdx.x;
    w.lpart[4 * q] = acc[0];
    w.lpart[4 * q + 1] = acc[1];
    w.lpart[4 * q + 2] = acc[2];
    w.lpart[4 * q + 3] = acc[3];
    w.cnt[q] = c;
    w.lmax[q] = mk;
  }
}

// one thread per row: the constraint is inactive (lambda = 0) when
// ||v||_1 <= sqrt(s) ||v||_2; the root lies among the candidates when
// rho(t0) >= sqrt(s) (and they fit the buffer); offsets of the candidates
__global__ __launch_bounds__(64) void lam_row_kernel(int64_t r, StartState s, Wide w,
                                                     double s_par) {
  const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (j >= r || !row_live(s, j)) return;
  WRow* R = w.rows + j;
  if (w.warm_K > 0 && s.status != nullptr && s.iters[j] + 1 > w.warm_K) {
    R->lmode = 3;  // frozen after the warm-up
    R->lam = w.gam[j];
    return;
  }
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t nc = 0;
  uint32_t mk = 0u;
  for (int c = 0; c < w.nch; ++c) {
    const int64_t q = j * w.nch + c;
    for (int e = 0; e < 4; ++e) a[e] += w.lpart[4 * q + e];
    const int k = w.cnt[q];
    w.cnt[q] = (int)nc;
    nc += k;
    mk = w.lmax[q] > mk ? w.lmax[q] : mk;
  }
  const double rs = sqrt(s_par);
  R->mk = mk;
  R->lam = 0.0;
  R->ncand = (int32_t)(nc < INT32_MAX ? nc : INT32_MAX);
  if (!(a[0] > rs * sqrt(a[1]))) {
    R->lmode = 0;
    return;
  }
  const bool ok = nc <= kMaxCandW && a[3] > 0.0 && a[2] >= rs * sqrt(a[3]);
  R->lmode = ok ? 1 : 2;
}

__global__ __launch_bounds__(kWT) void lam_gather_kernel(
    const float* __restrict__ V, int64_t ldv, int p, StartState s, Wide w) {
  __shared__ int scan[kNWv + 1];
  const int64_t j = blockIdx.y;
  if (!row_live(s, j) || w.rows[j].lmode != 1) return;
  const uint32_t t0 = w.rows[j].prefix > 1u ? w.rows[j].prefix : 1u;
  const int base = blockIdx.x * kWCH + threadIdx.x * kWN;
  float v[kWN];
  load_chunk(V + j * ldv, p, base, v);
  int c = 0;
#pragma unroll
  for (int k = 0; k < kWN; ++k) c += base + k < p && wkey(v[k]) >= t0;
  int tot;
  int off = w.cnt[j * w.nch + blockIdx.x] + block_exclusive_scan(c, scan, &tot);
  float* cd = w.cand + j * kMaxCandW;
#pragma unroll
  for (int k = 0; k < kWN; ++k)
    if (base + k < p && wkey(v[k]) >= t0) cd[off++] = fabsf(v[k]);
}

// exclusive prefix of two doubles per thread, in thread order
__device__ __forceinline__ void excl_scan2(double (&v)[2], double* scratch) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  double inc[2] = {v[0], v[1]};
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double o = __shfl_up(inc[c], off, kWave);
      if (lane >= off) inc[c] += o;
    }
  }
  if (lane == kWave - 1) {
    scratch[2 * wave] = inc[0];
    scratch[2 * wave + 1] = inc[1];
  }
  __syncthreads();
  double b0 = 0.0, b1 = 0.0;
  for (int q = 0; q < wave; ++q) {
    b0 += scratch[2 * q];
    b1 += scratch[2 * q + 1];
  }
  v[0] = b0 + inc[0] - v[0];
  v[1] = b1 + inc[1] - v[1];
  __syncthreads();
}

// one workgroup per row: lambda from the sorted candidates, else by the
// FP64 search of the float interval that holds the root
__global__ __launch_bounds__(kWT) void lam_solve_kernel(
    const float* __restrict__ V, int64_t ldv, int p, StartState s, Wide w,
    double s_par) {
  __shared__ float cand[kMaxCandW];
  __shared__ double dscan[2 * (kNWv + 1)];
  __shared__ double dred[2 * kNCdW * (kNWv + 1)];
  __shared__ int kbest;
  __shared__ double seg[4];
  const int64_t j = blockIdx.x;
  if (!row_live(s, j)) return;
  WRow* R = w.rows + j;
  int mode = R->lmode;
  if (mode == 0 || mode == 3) return;
  const int tid = threadIdx.x;
  const double rs = sqrt(s_par);
  if (mode == 1) {
    const int nc = R->ncand;
    const uint32_t t0 = R->prefix > 1u ? R->prefix : 1u;
    const double t0f = (double)__uint_as_float(t0);
    int np2 = 2;
    while (np2 < nc) np2 <<= 1;
    for (int i = tid; i < np2; i += kWT) cand[i] = i < nc ? w.cand[j * kMaxCandW + i] : -1.f;
    // bitonic sort, descending
    for (int size = 2; size <= np2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        __syncthreads();
        for (int t = tid; t < np2 / 2; t += kWT) {
          const int pos = 2 * stride * (t / stride) + (t % stride);
          const int partner = pos + stride;
          const bool desc = (pos & size) == 0;
          const float x0 = cand[pos], x1 = cand[partner];
          if ((x0 < x1) == desc) {
            cand[pos] = x1;
            cand[partner] = x0;
          }
        }
      }
    }
    __syncthreads();
    // prefix sums of c and c^2; thread t owns sorted positions [8t, 8t + 8)
    constexpr int kCP = kMaxCandW / kWT;
    double cv[kCP];
    double pre[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kCP; ++e) {
      const int q = kCP * tid + e;
      cv[e] = q < nc ? (double)cand[q] : 0.0;
      pre[0] += cv[e];
      pre[1] += cv[e] * cv[e];
    }
    excl_scan2(pre, dscan);
    if (tid == 0) kbest = INT32_MAX;
    __syncthreads();
    double S1 = pre[0], S2 = pre[1];
    int myk = INT32_MAX;
    double sg[4] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < kCP; ++e) {
      const int q = kCP * tid + e;
      S1 += cv[e];
      S2 += cv[e] * cv[e];
      const int k = q + 1;  // top-k prefix
      if (q >= nc || (double)k <= s_par || myk != INT32_MAX) continue;
      const double lo = k < nc ? (double)cand[k] : t0f;
      const double l1 = S1 - (double)k * lo;
      const double l2 = S2 - 2.0 * lo * S1 + (double)k * lo * lo;
      if (l2 > 0.0 && l1 >= rs * sqrt(l2)) {
        myk = k;
        sg[0] = S1;
        sg[1] = S2;
        sg[2] = lo;
        sg[3] = cv[e];
      }
    }
    if (myk != INT32_MAX) atomicMin(&kbest, myk);
    __syncthreads();
    const int kb = kbest;
    if (myk == kb && kb != INT32_MAX) {
      seg[0] = sg[0];
      seg[1] = sg[1];
      seg[2] = sg[2];
      seg[3] = sg[3];
    }
    __syncthreads();
    if (kb != INT32_MAX) {
      if (tid == 0) {
        const double k = (double)kb;
        double disc = k * seg[1] - seg[0] * seg[0];
        disc = disc > 0.0 ? disc : 0.0;
        double l = (seg[0] - sqrt(s_par * disc / (k - s_par))) / k;
        l = l < seg[2] ? seg[2] : l;
        l = l > seg[3] ? seg[3] : l;
        R->lam = l;
      }
      return;
    }
    mode = 2;  // no segment among the candidates: search the row
  }
  // FP64 search over the float keys: the largest key t with
  // ||(|v| - t)_+||_1 >= sqrt(s) ||(|v| - t)_+||_2, then the closed form on
  // the interval, where the active set is fixed
  const float* vg = V + j * ldv;
  uint32_t lo = 0u, hi = R->mk;
  while (hi - lo > 1u) {
    uint32_t t[kNCdW];
    const uint32_t span = hi - lo;
#pragma unroll
    for (int c = 0; c < kNCdW; ++c) {
      const uint32_t d = span > kNCdW + 1
                             ? (uint32_t)(((uint64_t)span * (uint64_t)(c + 1)) / (kNCdW + 1))
                             : (uint32_t)(c + 1);
      t[c] = d < span ? lo + d : hi;
    }
    double acc[2 * kNCdW];
    double tf[kNCdW];
#pragma unroll
    for (int c = 0; c < kNCdW; ++c) {
      acc[2 * c] = acc[2 * c + 1] = 0.0;
      tf[c] = (double)__uint_as_float(t[c]);
    }
    for (int i = tid; i < p; i += kWT) {
      const double a = fabs((double)vg[i]);
#pragma unroll
      for (int c = 0; c < kNCdW; ++c) {
        double d = a - tf[c];
        d = d > 0.0 ? d : 0.0;
        acc[2 * c] += d;
        acc[2 * c + 1] += d * d;
      }
    }
    block_sum_n<double, 2 * kNCdW>(acc, dred);
    uint32_t nlo = lo, nhi = hi;
#pragma unroll
    for (int c = 0; c < kNCdW; ++c) {
      if (t[c] >= hi) continue;
      const bool pred = acc[2 * c + 1] > 0.0 && acc[2 * c] >= rs * sqrt(acc[2 * c + 1]);
      if (pred)
        nlo = t[c] > nlo ? t[c] : nlo;
      else
        nhi = t[c] < nhi ? t[c] : nhi;
    }
    lo = nlo;
    hi = nhi;
  }
  const double tl = (double)__uint_as_float(lo);
  const double th = (double)__uint_as_float(hi);
  double ks[3] = {0.0, 0.0, 0.0};
  for (int i = tid; i < p; i += kWT) {
    const double a = fabs((double)vg[i]);
    if (a > tl) {
      ks[0] += 1.0;
      ks[1] += a;
      ks[2] += a * a;
    }
  }
  block_sum_n<double, 3>(ks, dred);
  if (tid == 0) {
    const double k = ks[0], S1 = ks[1], S2 = ks[2];
    double l = tl;
    if (k > s_par) {
      double disc = k * S2 - S1 * S1;
      disc = disc > 0.0 ? disc : 0.0;
      l = (S1 - sqrt(s_par * disc / (k - s_par))) / k;
    }
    l = l < tl ? tl : l;
    l = l > th ? th : l;
    R->lam = l;
  }
}

// warm-up of the penalties: gamma of the row from the (target + 1)-th largest
// key found by the digit passes, or the frozen value
template <int KIND>
__global__ __launch_bounds__(64) void gam_row_kernel(int64_t r, int p, StartState s,
                                                     Wide w) {
  const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (j >= r || !row_live(s, j)) return;
  WRow* R = w.rows + j;
  const bool warming = s.status == nullptr || s.iters[j] + 1 <= w.warm_K;
  if (!warming) {
    R->lam = w.gam[j];
  } else if ((int64_t)w.warm_target >= (int64_t)p) {
    R->lam = 0.0;
  } else {
    const double t = (double)__uint_as_float(R->prefix);
    R->lam = KIND == kHardGamma ? t * t : t;
  }
}

template <int KIND>
void launch_wide_kind(hipStream_t st, double param, const float* V,
                      int64_t ldv, int64_t r, int64_t p, float* X, int64_t ldx,
                      int32_t* li, float* lv, int64_t ldl, int list_cap,
                      StartState s, double tol, int maxit, int32_t* colmark,
                      const Plan* plan, const Wide& w) {
  const dim3 g2((unsigned)w.nch, (unsigned)r);
  const int ip = (int)p;
  const bool warm_gamma = (KIND == kHardGamma || KIND == kSoftGamma) && w.warm_K > 0;
  if (KIND == kTopS || KIND == kLambdaS || warm_gamma) {
    const int lm = KIND == kLambdaS ? 1 : 0;
    const int64_t want = warm_gamma ? (int64_t)w.warm_target + 1 : (int64_t)param;
    const int32_t need = lm ? 0 : (int32_t)(want < p ? want : p);
    const dim3 g1((unsigned)r);
    hipLaunchKernelGGL(wide_hist_kernel<0>, g2, dim3(kWT), 0, st, V, ldv, ip, s, w);
    hipLaunchKernelGGL(wide_decide_kernel<0>, g1, dim3(kWT), 0, st, s, w, need, lm, param, ip);
    hipLaunchKernelGGL(wide_hist_kernel<1>, g2, dim3(kWT), 0, st, V, ldv, ip, s, w);
    hipLaunchKernelGGL(wide_decide_kernel<1>, g1, dim3(kWT), 0, st, s, w, need, lm, param, ip);
    hipLaunchKernelGGL(wide_hist_kernel<2>, g2, dim3(kWT), 0, st, V, ldv, ip, s, w);
    hipLaunchKernelGGL(wide_decide_kernel<2>, g1, dim3(kWT), 0, st, s, w, need, lm, param, ip);
  }
  if (KIND == kTopS)
    hipLaunchKernelGGL(wide_eqcount_kernel, g2, dim3(kWT), 0, st, V, ldv, ip, s, w);
  if (warm_gamma)
    hipLaunchKernelGGL(gam_row_kernel<KIND>, dim3((unsigned)ceil_div(r, 64)), dim3(64), 0,
                       st, r, ip, s, w);
  if (KIND == kLambdaS) {
    hipLaunchKernelGGL(lam_stats_kernel, g2, dim3(kWT), 0, st, V, ldv, ip, s, w);
    hipLaunchKernelGGL(lam_row_kernel, dim3((unsigned)ceil_div(r, 64)), dim3(64), 0, st,
                       r, s, w, param);
    hipLaunchKernelGGL(lam_gather_kernel, g2, dim3(kWT), 0, st, V, ldv, ip, s, w);
    hipLaunchKernelGGL(lam_solve_kernel, dim3((unsigned)r), dim3(kWT), 0, st, V, ldv, ip,
                       s, w, param);
  }
  hipLaunchKernelGGL(wide_partial_kernel<KIND>, g2, dim3(kWT), 0, st, V, ldv, ip,
                     param, s, w);
  hipLaunchKernelGGL(wide_row_kernel<KIND>, dim3((unsigned)ceil_div(r, 64)), dim3(64),
                     0, st, r, s, tol, maxit, list_cap, li != nullptr ? 1 : 0, plan,
                     colmark != nullptr ? 1 : 0, w, param);
  hipLaunchKernelGGL(wide_emit_kernel<KIND>, g2, dim3(kWT), 0, st, V, ldv, ip, param,
                     X, ldx, li, lv, ldl, colmark, w);
}

}  // namespace

size_t x_update_wide_bytes(int fid, int64_t r, int64_t p) {
  (void)fid;
  if (p <= kWideMinP || r < 1) return 0;
  const int64_t nch = ceil_div(p, kWCH);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  return up(sizeof(uint32_t) * kWBins * r) + up(sizeof(WRow) * r) +
         2 * up(sizeof(int32_t) * r * nch) + up(sizeof(double) * 2 * r * nch) +
         up(sizeof(double) * 4 * r * nch) + up(sizeof(uint32_t) * r * nch) +
         up(sizeof(float) * kMaxCandW * r);
}

hipError_t x_update_wide_reset(hipStream_t st, void* scratch, int64_t r) {
  return hipMemsetAsync(scratch, 0, sizeof(uint32_t) * kWBins * r, st);
}

int64_t x_update_wide_clear_words(int64_t r) { return (int64_t)kWBins * r; }

bool x_update_wide(hipStream_t st, int fid, double s_or_gamma, const float* V,
                   int64_t ldv, int64_t r, int64_t p, float* X, int64_t ldx,
                   int32_t* list_idx, float* list_val, int64_t ldl, int list_cap,
                   StartState s, double tol, int32_t maxit, int32_t* colmark,
                   const Plan* plan, void* scratch, Warm wm) {
  const bool aligned = ldv % 4 == 0 && ldx % 4 == 0 && (uintptr_t)V % 16 == 0 &&
                       (uintptr_t)X % 16 == 0;
  if (scratch == nullptr || !aligned || x_update_wide_bytes(fid, r, p) == 0)
    return false;
  Wide w = carve_wide(scratch, r, p);
  w.warm_K = wm.K;
  w.warm_target = wm.target;
  w.gam = wm.gam;
  switch (xkind_of(fid)) {
    case kTopS:
      launch_wide_kind<kTopS>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx, list_val,
                              ldl, list_cap, s, tol, maxit, colmark, plan, w);
      return true;
    case kHardGamma:
      launch_wide_kind<kHardGamma>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                                   list_val, ldl, list_cap, s, tol, maxit, colmark, plan, w);
      return true;
    case kSoftGamma:
      launch_wide_kind<kSoftGamma>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                                   list_val, ldl, list_cap, s, tol, maxit, colmark, plan, w);
      return true;
    case kLambdaS:
      launch_wide_kind<kLambdaS>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                                 list_val, ldl, list_cap, s, tol, maxit, colmark, plan, w);
      return true;
    default:
      return false;
  }
}

}  // namespace spca
