// x-update of Algorithm 2 (Table 3, rows S3-S6), one workgroup per start:
//   L0 constraint  x = T_s(v) / ||T_s(v)||             phi = ||T_s(v)||
//   L1 constraint  x = V_l(v) / ||V_l(v)||, l = lambda_s(v)
//                                                      phi = l sqrt(s) + ||V_l(v)||
//   L0 penalty     x = U_g(v) / ||U_g(v)||             phi = sum_kept (v_i^2 - g)
//   L1 penalty     x = V_g(v) / ||V_g(v)||             phi = ||V_g(v)||
// followed by the ratio stop test of Section 2.2.
//
// Selection without a full sort.  The bit pattern of a non-negative float
// is monotone in its value, so thresholds are searched over the 31-bit keys
// of |v_i|.  Counting searches test kNC thresholds per step with wave
// ballots (one compare and one scalar popcount per element and threshold),
// a 16-ary search that needs 8 steps for 31 bits.
//   T_s       largest key t with #{key >= t} >= s; ties at that key go to the
//             lowest indices (a block-wide prefix count finds the cut index).
//   lambda_s  the derivative of l sqrt(s) + ||V_l(v)|| is sqrt(s) - rho(l)
//             with rho = ||V_l||_1 / ||V_l||_2 non-increasing, so lambda = 0
//             when rho(0) <= sqrt(s), and otherwise the root lies in the
//             first segment [c_{k+1}, c_k] (k > s, c sorted descending) whose
//             lower end already has rho >= sqrt(s), with the closed form
//             l = (S1_k - sqrt(s (k S2_k - S1_k^2) / (k - s))) / k.
//             Fast path: the M largest |v_i| (M from the previous support
//             size) are gathered, sorted in LDS and scanned for that segment,
//             after checking rho >= sqrt(s) at their smallest key (so the
//             root cannot lie below them).  Otherwise a search over keys with
//             FP64 sums of (|v| - t)_+ and its square finds the float interval
//             holding the root, on which the active set is fixed.
// Comparisons that decide membership use FP64 on the FP32 inputs (squares
// and differences of floats are exact or correctly rounded there).
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr int kXT = 1024;  // threads per start
constexpr int kNW = kXT / kWave;
constexpr int kNC = 15;    // thresholds per counting step (ballots)
constexpr int kNCd = 7;    // thresholds per FP64 search step
constexpr int kMaxCand = 2048;        // lambda_s candidates sorted in LDS
constexpr int64_t kStageMax = 12288;  // p staged in LDS up to this size

__device__ __forceinline__ uint32_t key_of(float v) {
  return __float_as_uint(v) & 0x7fffffffu;
}

struct XSmem {
  double dred[2 * kNCd * (kNW + 1)];
  int32_t ired[kNC * (kNW + 1)];
  uint32_t ured[kNW + 1];
  int scan[kNW + 1];
  double dscan[2 * (kNW + 1)];
  float cand[kMaxCand];
  int ncand;
  int kbest;
  int64_t cut;
  double seg[4];  // S1, S2, lower end, upper end of the chosen segment
};

// Thresholds strictly inside (lo, hi), spread evenly; unused slots get hi.
template <int NC>
__device__ __forceinline__ void spread(uint32_t lo, uint32_t hi, uint32_t (&t)[NC]) {
  const uint32_t span = hi - lo;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    uint32_t d = span > NC + 1
                     ? (uint32_t)(((uint64_t)span * (uint64_t)(c + 1)) / (NC + 1))
                     : (uint32_t)(c + 1);
    t[c] = d < span ? lo + d : hi;
  }
}

// #{i : key_i >= t} for kNC thresholds, every thread gets the totals.
template <typename ValF>
__device__ __forceinline__ void count_ge(ValF val, int p, const uint32_t (&t)[kNC],
                                         int (&cnt)[kNC], int32_t* ired) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < kNC; ++c) cnt[c] = 0;
  for (int base = wave * kWave; base < p; base += kXT) {
    const int i = base + lane;
    const uint32_t k = i < p ? key_of(val(i)) : 0u;
#pragma unroll
    for (int c = 0; c < kNC; ++c) cnt[c] += __popcll(__ballot(k >= t[c]));
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < kNC; ++c) ired[wave * kNC + c] = cnt[c];
  }
  __syncthreads();
  if (threadIdx.x < kNC) {
    int a = 0;
    for (int w = 0; w < kNW; ++w) a += ired[w * kNC + threadIdx.x];
    ired[kNW * kNC + threadIdx.x] = a;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kNC; ++c) cnt[c] = ired[kNW * kNC + c];
  __syncthreads();
}

// Largest key t in [lo, hi) with #{key >= t} >= need, given that this holds
// at lo and fails at hi.
template <typename ValF>
__device__ uint32_t search_count(ValF val, int p, uint32_t lo, uint32_t hi,
                                 int64_t need, int32_t* ired) {
  while (hi - lo > 1) {
    uint32_t t[kNC];
    spread<kNC>(lo, hi, t);
    int cnt[kNC];
    count_ge(val, p, t, cnt, ired);
    uint32_t nlo = lo, nhi = hi;
#pragma unroll
    for (int c = 0; c < kNC; ++c) {
      if (t[c] >= hi) continue;
      if (cnt[c] >= need)
        nlo = t[c] > nlo ? t[c] : nlo;
      else
        nhi = t[c] < nhi ? t[c] : nhi;
    }
    lo = nlo;
    hi = nhi;
  }
  return lo;
}

__device__ __forceinline__ int count_ge1(uint32_t t, int p, const float* vs,
                                         const float* vg, bool staged,
                                         int32_t* ired) {
  uint32_t tt[kNC];
#pragma unroll
  for (int c = 0; c < kNC; ++c) tt[c] = t;
  int cnt[kNC];
  auto val = [&](int i) -> float { return staged ? vs[i] : vg[i]; };
  count_ge(val, p, tt, cnt, ired);
  return cnt[0];
}

// Exclusive prefix sums of two doubles per thread in thread order.
__device__ __forceinline__ void block_exclusive_scan2(double (&v)[2], double* scratch,
                                                     double (&total)[2]) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  double inc[2] = {v[0], v[1]};
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double o = __shfl_up(inc[c], off, kWave);
      if (lane >= off) inc[c] += o;
    }
  }
  if (lane == kWave - 1) {
    scratch[2 * wave] = inc[0];
    scratch[2 * wave + 1] = inc[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r0 = 0.0, r1 = 0.0;
    for (int w = 0; w < kNW; ++w) {
      double a = scratch[2 * w], b = scratch[2 * w + 1];
      scratch[2 * w] = r0;
      scratch[2 * w + 1] = r1;
      r0 += a;
      r1 += b;
    }
    scratch[2 * kNW] = r0;
    scratch[2 * kNW + 1] = r1;
  }
  __syncthreads();
  const double b0 = scratch[2 * wave], b1 = scratch[2 * wave + 1];
  total[0] = scratch[2 * kNW];
  total[1] = scratch[2 * kNW + 1];
  v[0] = b0 + inc[0] - v[0];
  v[1] = b1 + inc[1] - v[1];
  __syncthreads();
}

template <int KIND, bool STAGED>
__global__ __launch_bounds__(kXT) void x_update_kernel(
    const float* __restrict__ V, int64_t ldv, int p, double param,
    float* __restrict__ X, int64_t ldx, int32_t* __restrict__ list_idx,
    float* __restrict__ list_val, int64_t ldl, int list_cap, StartState s,
    double tol, int maxit, int32_t* __restrict__ colmark, const Plan* plan) {
  extern __shared__ __attribute__((aligned(16))) float vstage[];
  __shared__ XSmem sm;
  const int64_t j = blockIdx.x;
  const bool full = s.status != nullptr;
  if (full && s.status[j] != kRunning) return;
  if (s.cfg != nullptr) {  // grouped solve: this start's request
    if (s.cfg[j].kind != KIND) return;
    param = s.cfg[j].param;
    tol = s.cfg[j].tol;
    maxit = s.cfg[j].maxit;
  }
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const float* vg = V + j * ldv;
  if (STAGED) {
    for (int i = tid; i < p; i += kXT) vstage[i] = vg[i];
    __syncthreads();
  }
  auto val = [&](int i) -> float { return STAGED ? vstage[i] : vg[i]; };

  const int chunk = (int)ceil_div(p, kXT);
  const int cb = tid * chunk < p ? tid * chunk : p;
  const int ce = cb + chunk < p ? cb + chunk : p;

  // ---------------- threshold ----------------
  uint32_t thr_key = 0;   // T_s: keys above are kept; equal keys up to cut
  int64_t cut = -1;
  double lam = 0.0;       // V_l: kept iff |v| > lam;  U_g: kept iff v^2 > g
  if (KIND == kTopS || KIND == kLambdaS) {
    uint32_t mk = 0;
    for (int i = tid; i < p; i += kXT) {
      uint32_t k = key_of(val(i));
      mk = k > mk ? k : mk;
    }
    mk = block_max(mk, sm.ured);
    const double s_par = param;
    const double rs = sqrt(s_par);
    if (KIND == kTopS) {
      const int64_t s_int = (int64_t)s_par < (int64_t)p ? (int64_t)s_par : (int64_t)p;
      // #{key >= 0} = p >= s and #{key >= mk + 1} = 0 < s
      thr_key = search_count(val, p, 0u, mk + 1, s_int, sm.ired);
      // ties at thr_key: keep the first (s - #{key > thr_key}) in index order
      if (tid == 0) sm.cut = -1;
      const int gt = count_ge1(thr_key + 1, p, vstage, vg, STAGED, sm.ired);
      int eq = 0;
      for (int i = cb; i < ce; ++i) eq += key_of(val(i)) == thr_key;
      int eq_total;
      int eq_off = block_exclusive_scan(eq, sm.scan, &eq_total);
      const int need = (int)s_int - gt;  // >= 1
      if (eq_off < need && need <= eq_off + eq) {
        int seen = eq_off;
        for (int i = cb; i < ce; ++i) {
          if (key_of(val(i)) == thr_key) {
            ++seen;
            if (seen == need) {
              sm.cut = i;
              break;
            }
          }
        }
      }
      __syncthreads();
      cut = sm.cut;
    }
    if (KIND == kLambdaS) {
      // constraint inactive when ||v||_1 <= sqrt(s) ||v||_2: lambda = 0
      double a0[2] = {0.0, 0.0};
      for (int i = tid; i < p; i += kXT) {
        double a = fabs((double)val(i));
        a0[0] += a;
        a0[1] += a * a;
      }
      block_sum_n<double, 2>(a0, sm.dred);
      const bool active = a0[0] > rs * sqrt(a0[1]);
      bool done = !active;
      if (active) {
        // ---- fast path: the M largest entries ----
        int64_t m0 = full ? 2 * (int64_t)s.nnz[j] + 32 : 4 * (int64_t)ceil(s_par) + 64;
        const int64_t smin = (int64_t)floor(s_par) + 2;
        m0 = m0 < smin ? smin : m0;
        m0 = m0 > kMaxCand ? kMaxCand : m0;
        m0 = m0 > p ? p : m0;
        uint32_t t0 = search_count(val, p, 0u, mk + 1, m0, sm.ired);
        t0 = t0 < 1u ? 1u : t0;  // zeros never enter
        const double t0f = (double)__uint_as_float(t0);
        double a1[2] = {0.0, 0.0};
        int mine = 0;
        for (int i = tid; i < p; i += kXT) {
          double a = fabs((double)val(i));
          if (key_of(val(i)) >= t0) ++mine;
          double d = a - t0f;
          d = d > 0.0 ? d : 0.0;
          a1[0] += d;
          a1[1] += d * d;
        }
        block_sum_n<double, 2>(a1, sm.dred);
        const int ncand = block_sum(mine, sm.ired);
        // rho(t0) >= sqrt(s): the root is >= t0 and only candidates matter
        const bool ok = ncand <= kMaxCand && a1[1] > 0.0 && a1[0] >= rs * sqrt(a1[1]);
        if (ok) {
          if (tid == 0) sm.ncand = 0;
          __syncthreads();
          for (int base = (tid / kWave) * kWave; base < p; base += kXT) {
            const int i = base + lane;
            const float v = i < p ? val(i) : 0.f;
            const bool in = i < p && key_of(v) >= t0;
            const unsigned long long mask = __ballot(in);
            int wbase = 0;
            if (lane == 0 && mask) wbase = atomicAdd(&sm.ncand, (int)__popcll(mask));
            wbase = __shfl(wbase, 0, kWave);
            if (in) {
              const unsigned long long below = mask & ((1ull << lane) - 1ull);
              sm.cand[wbase + __popcll(below)] = fabsf(v);
            }
          }
          __syncthreads();
          int np2 = 2;
          while (np2 < ncand) np2 <<= 1;
          for (int i = ncand + tid; i < np2; i += kXT) sm.cand[i] = -1.f;
          // bitonic sort, descending
          for (int size = 2; size <= np2; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
              __syncthreads();
              for (int t = tid; t < np2 / 2; t += kXT) {
                const int pos = 2 * stride * (t / stride) + (t % stride);
                const int partner = pos + stride;
                const bool desc = (pos & size) == 0;
                const float x0 = sm.cand[pos], x1 = sm.cand[partner];
                if ((x0 < x1) == desc) {
                  sm.cand[pos] = x1;
                  sm.cand[partner] = x0;
                }
              }
            }
          }
          __syncthreads();
          // prefix sums of c and c^2; thread t owns sorted positions 2t, 2t+1
          const int q0 = 2 * tid, q1 = 2 * tid + 1;
          const double c0 = q0 < ncand ? (double)sm.cand[q0] : 0.0;
          const double c1 = q1 < ncand ? (double)sm.cand[q1] : 0.0;
          double pre[2] = {c0 + c1, c0 * c0 + c1 * c1};
          double tot[2];
          block_exclusive_scan2(pre, sm.dscan, tot);
          if (tid == 0) sm.kbest = INT32_MAX;
          __syncthreads();
          double S1 = pre[0], S2 = pre[1];
          int myk = INT32_MAX;
          double seg[4] = {0, 0, 0, 0};
          for (int e = 0; e < 2; ++e) {
            const int q = q0 + e;
            if (q >= ncand) break;
            const double c = e == 0 ? c0 : c1;
            S1 += c;
            S2 += c * c;
            const int k = q + 1;  // top-k prefix
            if ((double)k <= s_par) continue;
            const double lo = k < ncand ? (double)sm.cand[k] : t0f;
            const double l1 = S1 - (double)k * lo;
            const double l2 = S2 - 2.0 * lo * S1 + (double)k * lo * lo;
            if (l2 > 0.0 && l1 >= rs * sqrt(l2) && k < myk) {
              myk = k;
              seg[0] = S1;
              seg[1] = S2;
              seg[2] = lo;
              seg[3] = c;
            }
          }
          if (myk != INT32_MAX) atomicMin(&sm.kbest, myk);
          __syncthreads();
          const int kb = sm.kbest;
          if (myk == kb && kb != INT32_MAX) {
            sm.seg[0] = seg[0];
            sm.seg[1] = seg[1];
            sm.seg[2] = seg[2];
            sm.seg[3] = seg[3];
          }
          __syncthreads();
          if (kb != INT32_MAX) {
            const double k = (double)kb, S1b = sm.seg[0], S2b = sm.seg[1];
            double disc = k * S2b - S1b * S1b;
            disc = disc > 0.0 ? disc : 0.0;
            double l = (S1b - sqrt(s_par * disc / (k - s_par))) / k;
            l = l < sm.seg[2] ? sm.seg[2] : l;
            l = l > sm.seg[3] ? sm.seg[3] : l;
            lam = l;
            done = true;
          }
          __syncthreads();
        }
      }
      if (!done) {
        // ---- fallback: FP64 search of the float interval holding the root ----
        uint32_t lo = 0, hi = mk;  // rho(0) > sqrt(s); nothing exceeds mk
        while (hi - lo > 1) {
          uint32_t t[kNCd];
          spread<kNCd>(lo, hi, t);
          double acc[2 * kNCd];
#pragma unroll
          for (int c = 0; c < 2 * kNCd; ++c) acc[c] = 0.0;
          double tf[kNCd];
#pragma unroll
          for (int c = 0; c < kNCd; ++c) tf[c] = (double)__uint_as_float(t[c]);
          for (int i = tid; i < p; i += kXT) {
            double a = fabs((double)val(i));
#pragma unroll
            for (int c = 0; c < kNCd; ++c) {
              double d = a - tf[c];
              d = d > 0.0 ? d : 0.0;
              acc[2 * c] += d;
              acc[2 * c + 1] += d * d;
            }
          }
          block_sum_n<double, 2 * kNCd>(acc, sm.dred);
          uint32_t nlo = lo, nhi = hi;
#pragma unroll
          for (int c = 0; c < kNCd; ++c) {
            if (t[c] >= hi) continue;
            bool pred = acc[2 * c + 1] > 0.0 && acc[2 * c] >= rs * sqrt(acc[2 * c + 1]);
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
        for (int i = tid; i < p; i += kXT) {
          double a = fabs((double)val(i));
          if (a > tl) {
            ks[0] += 1.0;
            ks[1] += a;
            ks[2] += a * a;
          }
        }
        block_sum_n<double, 3>(ks, sm.dred);
        const double k = ks[0], S1 = ks[1], S2 = ks[2];
        double l = tl;
        if (k > s_par) {
          double disc = k * S2 - S1 * S1;
          disc = disc > 0.0 ? disc : 0.0;
          l = (S1 - sqrt(s_par * disc / (k - s_par))) / k;
        }
        l = l < tl ? tl : l;
        l = l > th ? th : l;
        lam = l;
      }
    }
  } else {
    lam = param;  // gamma
  }

  // keep test and kept value w_i for entry i
  auto kept = [&](int i, float v, double* w) -> bool {
    if (KIND == kTopS) {
      uint32_t k = key_of(v);
      *w = (double)v;
      return k != 0 && (k > thr_key || (k == thr_key && (int64_t)i <= cut));
    } else if (KIND == kHardGamma) {
      *w = (double)v;
      return (double)v * (double)v > lam;
    } else {
      double a = fabs((double)v);
      *w = v > 0.f ? a - lam : lam - a;
      return a > lam;
    }
  };

  // ---------------- norms, phi and counts ----------------
  int cnt = 0;
  double acc[2] = {0.0, 0.0};  // sum w^2, sum (v^2 - g) over kept
  for (int i = cb; i < ce; ++i) {
    float v = val(i);
    double w;
    if (kept(i, v, &w)) {
      ++cnt;
      acc[0] += w * w;
      if (KIND == kHardGamma) acc[1] += w * w - lam;
    }
  }
  block_sum_n<double, 2>(acc, sm.dred);
  int total;
  int off = block_exclusive_scan(cnt, sm.scan, &total);
  const double nrm = sqrt(acc[0]);
  double phi;
  if (KIND == kHardGamma)
    phi = acc[1];
  else if (KIND == kLambdaS)
    phi = lam * sqrt(param) + nrm;
  else
    phi = nrm;
  const bool zero = !(nrm > 0.0);
  const double inv = zero ? 0.0 : 1.0 / nrm;

  // ---------------- write x (list and dense row) ----------------
  if (list_idx != nullptr && !zero && total <= list_cap) {
    int32_t* li = list_idx + j * ldl;
    float* lv = list_val + j * ldl;
    for (int i = cb; i < ce; ++i) {
      float v = val(i);
      double w;
      if (kept(i, v, &w)) {
        li[off] = i;
        lv[off] = (float)(w * inv);
        ++off;
      }
    }
  }
  float* x = X + j * ldx;
  const bool marking = colmark != nullptr && !zero && plan->mark != 0;
  const int32_t epoch = marking ? plan->epoch : 0;
  for (int i = tid; i < p; i += kXT) {
    float v = val(i);
    double w;
    bool k = kept(i, v, &w);
    x[i] = (k && !zero) ? (float)(w * inv) : 0.f;
    if (k && marking) colmark[i] = epoch;
  }

  // ---------------- state and stop test (Section 2.2) ----------------
  if (tid == 0) {
    if (!full) {
      // operator-only mode: phi and nnz are plain outputs in s.phi / s.nnz
      s.phi[j] = phi;
      s.nnz[j] = zero ? 0 : total;
    } else {
      const int it = s.iters[j] + 1;
      const double prev = s.phi[j];
      s.iters[j] = it;
      s.phi_prev[j] = prev;
      s.phi[j] = phi;
      s.nnz[j] = zero ? 0 : total;
      if (zero)
        s.status[j] = SPCA_ZERO;
      else if (it >= 2 && tol >= 0.0 && phi <= (1.0 + tol) * prev)
        s.status[j] = SPCA_CONVERGED;
      else if (it >= maxit)
        s.status[j] = SPCA_MAXIT;
    }
  }
}


// ---------------------------------------------------------------------------
// Register-resident variant for p <= 256 * NPT.  A 256-thread block per
// start, thread t holding the contiguous entries [t NPT, (t+1) NPT) of the
// row (16-byte loads), so that every pass is register arithmetic, index
// order is thread order for the prefix counts, and all starts of a batch
// are resident on the chip at once.  Keys are selected by radix select:
// three histogram passes over 11, 11 and 9 bits of the 31-bit key with
// integer LDS atomics (exact and order-independent).
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kRT = 256;  // threads per start
constexpr int kRW = kRT / kWave;
constexpr int kBins = 2048;

struct RSmem {
  uint32_t hist[kBins];
  double dred[2 * kNCd * (kRW + 1)];
  int32_t ired[16 * (kRW + 1)];
  uint32_t ured[kRW + 1];
  int scan[kRW + 1];
  double dscan[2 * (kRW + 1)];
  float cand[kMaxCand];
  int ncand;
  int kbest;
  int64_t cut;
  uint32_t sel[2];  // selected bin, count above it
  double seg[4];
  uint64_t pscan[3 * (kRW + 1)];  // packed per-row counts (rank_rows)
};

// Index-order ranks over the striped row layout of the one-workgroup
// x-update: thread t holds elements 4 (q kRT + t) + e, e < 4, for rows q <
// R.  Given per-thread counts c[q] <= 4 of the elements that satisfy a
// predicate, returns in base[q] the number of such elements at a lower
// index than this thread's row-q group (earlier rows of the whole block,
// then lower threads of the same row), and the block total.  Four 16-bit
// fields per 64-bit word hold row counts up to 4 kRT without carries.
template <int R>
__device__ __forceinline__ int rank_rows(const int (&c)[R], int (&base)[R], uint64_t* scratch) {
  constexpr int W = (R + 3) / 4;
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  uint64_t in[W], inc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) in[w] = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) in[q / 4] |= (uint64_t)c[q] << (16 * (q % 4));
#pragma unroll
  for (int w = 0; w < W; ++w) inc[w] = in[w];
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t o = __shfl_up(inc[w], off, kWave);
      if (lane >= off) inc[w] += o;
    }
  }
  if (lane == kWave - 1) {
#pragma unroll
    for (int w = 0; w < W; ++w) scratch[wave * W + w] = inc[w];
  }
  __syncthreads();
  uint64_t before[W], tot[W];
#pragma unroll
  for (int w = 0; w < W; ++w) before[w] = tot[w] = 0;
#pragma unroll
  for (int u = 0; u < kRW; ++u) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t x = scratch[u * W + w];
      if (u < wave) before[w] += x;
      tot[w] += x;
    }
  }
  __syncthreads();
  int run = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int sh = 16 * (q % 4);
    const int mine = (int)(((before[q / 4] + inc[q / 4] - in[q / 4]) >> sh) & 0xffffu);
    base[q] = run + mine;
    run += (int)((tot[q / 4] >> sh) & 0xffffu);
  }
  return run;
}

// Exclusive prefix sums of two doubles per thread in thread order (kRT).
__device__ __forceinline__ void rscan2(double (&v)[2], double* scratch) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  double inc[2] = {v[0], v[1]};
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double o = __shfl_up(inc[c], off, kWave);
      if (lane >= off) inc[c] += o;
    }
  }
  if (lane == kWave - 1) {
    scratch[2 * wave] = inc[0];
    scratch[2 * wave + 1] = inc[1];
  }
  __syncthreads();
  double b0 = 0.0, b1 = 0.0;
  for (int w = 0; w < wave; ++w) {
    b0 += scratch[2 * w];
    b1 += scratch[2 * w + 1];
  }
  v[0] = b0 + inc[0] - v[0];
  v[1] = b1 + inc[1] - v[1];
  __syncthreads();
}

// The need-th largest key (1 <= need <= number of entries) and the number of
// keys strictly above it.  Entries beyond p are zero keys.
// Marks a register value as changed, so that the compiler recomputes what
// it derives from it (keys, bins) instead of holding copies across passes.
__device__ __forceinline__ void reload(float& x) { asm volatile("" : "+v"(x)); }

template <int NPT>
__device__ void radix_select(float (&v)[NPT], uint32_t need, RSmem& sm,
                             uint32_t* key_out, uint32_t* above_out) {
  const int tid = threadIdx.x;
  uint32_t prefix = 0;      // selected high bits so far
  uint32_t above = 0;       // keys strictly above the selected prefix range
  // (shift, bits) of the three passes over the 31-bit key
  const int shifts[3] = {20, 9, 0};
  const int widths[3] = {11, 11, 9};
#pragma unroll 1
  for (int pass = 0; pass < 3; ++pass) {
    const int sh = shifts[pass];
    const uint32_t nb = 1u << widths[pass];
    const uint32_t hi_mask = pass == 0 ? 0u : (0x7fffffffu >> (sh + widths[pass])) << (sh + widths[pass]);
    for (int i = tid; i < kBins; i += kRT) sm.hist[i] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      reload(v[k]);
      const uint32_t key = key_of(v[k]);
      if ((key & hi_mask) == prefix) atomicAdd(&sm.hist[(key >> sh) & (nb - 1)], 1u);
    }
    __syncthreads();
    // bins from the top: thread t owns bins nb-1-8t .. nb-8-8t
    constexpr int kPer = kBins / kRT;  // 8
    uint32_t local = 0;
    int first = (int)nb - 1 - kPer * tid;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      int bin = first - q;
      local += bin >= 0 ? sm.hist[bin] : 0u;
    }
    int total;
    const uint32_t before = (uint32_t)block_exclusive_scan((int)local, sm.scan, &total);
    const uint32_t rem = need - above;
    if (before < rem && rem <= before + local) {
      uint32_t run = before;
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        int bin = first - q;
        uint32_t h = bin >= 0 ? sm.hist[bin] : 0u;
        if (run < rem && rem <= run + h) {
          sm.sel[0] = (uint32_t)bin;
          sm.sel[1] = run;
        }
        run += h;
      }
    }
    __syncthreads();
    prefix |= sm.sel[0] << sh;
    above += sm.sel[1];
    __syncthreads();
  }
  *key_out = prefix;
  *above_out = above;
}

// Register budget: the top-s kernel keeps its keys live across the radix
// passes and is left at 2 waves per SIMD; the others fit 4.
// WARM: the sparsity-targeted warm-up (Section 4.1) of the parameter.
template <int KIND, int NPT, bool WARM>
__global__ __launch_bounds__(kRT, (KIND == kTopS || WARM) ? 2 : 4) void x_update_reg_kernel(
    const float* __restrict__ V, int64_t ldv, int p, double param,
    float* __restrict__ X, int64_t ldx, int32_t* __restrict__ list_idx,
    float* __restrict__ list_val, int64_t ldl, int list_cap, StartState s,
    double tol, int maxit, int32_t* __restrict__ colmark, const Plan* plan,
    Warm wm) {
  static_assert(NPT % 4 == 0, "NPT must be a multiple of 4");
  __shared__ RSmem sm;
  const int64_t j = blockIdx.x;
  const bool full = s.status != nullptr;
  if (full && s.status[j] != kRunning) return;
  if (s.cfg != nullptr) {  // grouped solve: this start's request
    if (s.cfg[j].kind != KIND) return;
    param = s.cfg[j].param;
    tol = s.cfg[j].tol;
    maxit = s.cfg[j].maxit;
  }
  // after the candidate kernel: only the rows it could not settle
  if (s.redo != nullptr && s.redo[j] == 0) return;
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  // Striped rows: element 4 (q kRT + tid) + e is v[4 q + e], so that each
  // 16-byte load and store instruction covers 1 KB of contiguous memory.
  constexpr int R = NPT / 4;
  auto gidx = [&](int k) { return 4 * ((k / 4) * kRT + tid) + k % 4; };
  const float* vg = V + j * ldv;
  float v[NPT];
#pragma unroll
  for (int q = 0; q < NPT; q += 4) {
    const int i = gidx(q);
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

  uint32_t thr_key = 0;
  int64_t cut = -1;
  double lam = 0.0;
  const int itc = full ? s.iters[j] + 1 : 1;  // this x-update's number
  const bool warming = WARM && itc <= wm.K;
  if (KIND == kTopS) {
    const uint32_t s_int = (uint32_t)((int64_t)param < (int64_t)p ? (int64_t)param : (int64_t)p);
    uint32_t above;
    radix_select<NPT>(v, s_int, sm, &thr_key, &above);
    // ties at thr_key: keep the first (s - #{key > thr_key}) in index order
    if (tid == 0) sm.cut = -1;
    int eq[R], eq_base[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      eq[q] = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        reload(v[4 * q + e]);
        eq[q] += key_of(v[4 * q + e]) == thr_key && gidx(4 * q + e) < p;
      }
    }
    rank_rows<R>(eq, eq_base, sm.pscan);
    const int need = (int)s_int - (int)above;  // >= 1
#pragma unroll
    for (int q = 0; q < R; ++q) {
      int seen = eq_base[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * q + e;
        if (key_of(v[k]) == thr_key && gidx(k) < p) {
          ++seen;
          if (seen == need) sm.cut = gidx(k);
        }
      }
    }
    __syncthreads();
    cut = sm.cut;
  } else if (KIND == kLambdaS && WARM && !warming) {
    lam = wm.gam[j];  // frozen after the warm-up
  } else if (KIND == kLambdaS) {
    const double s_par = param;
    const double rs = sqrt(s_par);
    double a0[2] = {0.0, 0.0};
    uint32_t mk = 0;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      double a = fabs((double)v[k]);
      a0[0] += a;
      a0[1] += a * a;
      uint32_t key = key_of(v[k]);
      mk = key > mk ? key : mk;
    }
    block_sum_n<double, 2>(a0, sm.dred);
    const bool active = a0[0] > rs * sqrt(a0[1]);
    bool done = !active;
    if (active) {
      mk = block_max(mk, sm.ured);
      int64_t m0 = full ? 2 * (int64_t)s.nnz[j] + 32 : 4 * (int64_t)ceil(s_par) + 64;
      const int64_t smin = (int64_t)floor(s_par) + 2;
      m0 = m0 < smin ? smin : m0;
      m0 = m0 > kMaxCand ? kMaxCand : m0;
      m0 = m0 > p ? p : m0;
      uint32_t t0, above0;
      radix_select<NPT>(v, (uint32_t)m0, sm, &t0, &above0);
      t0 = t0 < 1u ? 1u : t0;  // zeros never enter
      const double t0f = (double)__uint_as_float(t0);
      double a1[2] = {0.0, 0.0};
      int mine = 0;
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        mine += key_of(v[k]) >= t0;
        double d = fabs((double)v[k]) - t0f;
        d = d > 0.0 ? d : 0.0;
        a1[0] += d;
        a1[1] += d * d;
      }
      block_sum_n<double, 2>(a1, sm.dred);
      const int ncand = block_sum(mine, sm.ired);
      // rho(t0) >= sqrt(s): the root is >= t0 and only candidates matter
      const bool ok = ncand <= kMaxCand && a1[1] > 0.0 && a1[0] >= rs * sqrt(a1[1]);
      if (ok) {
        if (tid == 0) sm.ncand = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
          const bool in = key_of(v[k]) >= t0;
          const unsigned long long mask = __ballot(in);
          int wbase = 0;
          if (lane == 0 && mask) wbase = atomicAdd(&sm.ncand, (int)__popcll(mask));
          wbase = __shfl(wbase, 0, kWave);
          if (in) {
            const unsigned long long below = mask & ((1ull << lane) - 1ull);
            sm.cand[wbase + __popcll(below)] = fabsf(v[k]);
          }
        }
        __syncthreads();
        int np2 = 2;
        while (np2 < ncand) np2 <<= 1;
        for (int i = ncand + tid; i < np2; i += kRT) sm.cand[i] = -1.f;
        // bitonic sort, descending
        for (int size = 2; size <= np2; size <<= 1) {
          for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int t = tid; t < np2 / 2; t += kRT) {
              const int pos = 2 * stride * (t / stride) + (t % stride);
              const int partner = pos + stride;
              const bool desc = (pos & size) == 0;
              const float x0 = sm.cand[pos], x1 = sm.cand[partner];
              if ((x0 < x1) == desc) {
                sm.cand[pos] = x1;
                sm.cand[partner] = x0;
              }
            }
          }
        }
        __syncthreads();
        // prefix sums of c and c^2; thread t owns sorted positions [8t, 8t+8)
        constexpr int kCP = kMaxCand / kRT;
        double cv[kCP];
        double pre[2] = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < kCP; ++e) {
          const int q = kCP * tid + e;
          cv[e] = q < ncand ? (double)sm.cand[q] : 0.0;
          pre[0] += cv[e];
          pre[1] += cv[e] * cv[e];
        }
        rscan2(pre, sm.dscan);
        if (tid == 0) sm.kbest = INT32_MAX;
        __syncthreads();
        double S1 = pre[0], S2 = pre[1];
        int myk = INT32_MAX;
        double seg[4] = {0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < kCP; ++e) {
          const int q = kCP * tid + e;
          S1 += cv[e];
          S2 += cv[e] * cv[e];
          const int k = q + 1;  // top-k prefix
          if (q >= ncand || (double)k <= s_par || myk != INT32_MAX) continue;
          const double lo = k < ncand ? (double)sm.cand[k] : t0f;
          const double l1 = S1 - (double)k * lo;
          const double l2 = S2 - 2.0 * lo * S1 + (double)k * lo * lo;
          if (l2 > 0.0 && l1 >= rs * sqrt(l2)) {
            myk = k;
            seg[0] = S1;
            seg[1] = S2;
            seg[2] = lo;
            seg[3] = cv[e];
          }
        }
        if (myk != INT32_MAX) atomicMin(&sm.kbest, myk);
        __syncthreads();
        const int kb = sm.kbest;
        if (myk == kb && kb != INT32_MAX) {
          sm.seg[0] = seg[0];
          sm.seg[1] = seg[1];
          sm.seg[2] = seg[2];
          sm.seg[3] = seg[3];
        }
        __syncthreads();
        if (kb != INT32_MAX) {
          const double k = (double)kb, S1b = sm.seg[0], S2b = sm.seg[1];
          double disc = k * S2b - S1b * S1b;
          disc = disc > 0.0 ? disc : 0.0;
          double l = (S1b - sqrt(s_par * disc / (k - s_par))) / k;
          l = l < sm.seg[2] ? sm.seg[2] : l;
          l = l > sm.seg[3] ? sm.seg[3] : l;
          lam = l;
          done = true;
        }
        __syncthreads();
      }
    }
    if (!done) {
      // fallback: FP64 search of the float interval holding the root; reads
      // the row from memory so that the fast path keeps its registers
      uint32_t lo = 0, hi = mk;
      while (hi - lo > 1) {
        uint32_t t[kNCd];
        spread<kNCd>(lo, hi, t);
        double acc[2 * kNCd];
#pragma unroll
        for (int c = 0; c < 2 * kNCd; ++c) acc[c] = 0.0;
        double tf[kNCd];
#pragma unroll
        for (int c = 0; c < kNCd; ++c) tf[c] = (double)__uint_as_float(t[c]);
#pragma unroll 1
        for (int i = tid; i < p; i += kRT) {
          const double a = fabs((double)vg[i]);
#pragma unroll
          for (int c = 0; c < kNCd; ++c) {
            double d = a - tf[c];
            d = d > 0.0 ? d : 0.0;
            acc[2 * c] += d;
            acc[2 * c + 1] += d * d;
          }
        }
        block_sum_n<double, 2 * kNCd>(acc, sm.dred);
        uint32_t nlo = lo, nhi = hi;
#pragma unroll
        for (int c = 0; c < kNCd; ++c) {
          if (t[c] >= hi) continue;
          bool pred = acc[2 * c + 1] > 0.0 && acc[2 * c] >= rs * sqrt(acc[2 * c + 1]);
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
#pragma unroll 1
      for (int i = tid; i < p; i += kRT) {
        const double a = fabs((double)vg[i]);
        if (a > tl) {
          ks[0] += 1.0;
          ks[1] += a;
          ks[2] += a * a;
        }
      }
      block_sum_n<double, 3>(ks, sm.dred);
      const double k = ks[0], S1 = ks[1], S2 = ks[2];
      double l = tl;
      if (k > s_par) {
        double disc = k * S2 - S1 * S1;
        disc = disc > 0.0 ? disc : 0.0;
        l = (S1 - sqrt(s_par * disc / (k - s_par))) / k;
      }
      l = l < tl ? tl : l;
      l = l > th ? th : l;
      lam = l;
    }
  } else if (WARM && warming) {
    // gamma for target nonzeros: the (target + 1)-th largest |v_i| (or its
    // square for U_gamma), which the strict threshold then excludes
    if ((int64_t)wm.target >= (int64_t)p) {
      lam = 0.0;
    } else {
      uint32_t tk, above;
      radix_select<NPT>(v, (uint32_t)wm.target + 1u, sm, &tk, &above);
      const double t = (double)__uint_as_float(tk);
      lam = KIND == kHardGamma ? t * t : t;
    }
  } else if (WARM) {
    lam = wm.gam[j];
  } else {
    lam = param;
  }

  auto kept = [&](int i, float vv, double* w) -> bool {
    if (KIND == kTopS) {
      uint32_t k = key_of(vv);
      *w = (double)vv;
      return k != 0 && (k > thr_key || (k == thr_key && (int64_t)i <= cut));
    } else if (KIND == kHardGamma) {
      *w = (double)vv;
      return (double)vv * (double)vv > lam;
    } else {
      double a = fabs((double)vv);
      *w = vv > 0.f ? a - lam : lam - a;
      return a > lam;
    }
  };

  int cnt[R], off[R];
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int q = 0; q < R; ++q) {
    cnt[q] = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * q + e;
      double w;
      reload(v[k]);
      if (kept(gidx(k), v[k], &w)) {
        ++cnt[q];
        acc[0] += w * w;
        if (KIND == kHardGamma) acc[1] += w * w - lam;
      }
    }
  }
  block_sum_n<double, 2>(acc, sm.dred);
  const int total = rank_rows<R>(cnt, off, sm.pscan);
  const double nrm = sqrt(acc[0]);
  double phi;
  if (KIND == kHardGamma)
    phi = acc[1];
  else if (KIND == kLambdaS)
    phi = lam * sqrt(param) + nrm;
  else
    phi = nrm;
  const bool zero = !(nrm > 0.0);
  const double inv = zero ? 0.0 : 1.0 / nrm;

  // the list is written only when it can serve the list-based product
  const bool listed = list_idx != nullptr && !zero && total <= list_cap;
  const bool marking = colmark != nullptr && !zero && plan->mark != 0;
  const int32_t epoch = marking ? plan->epoch : 0;
  int32_t* li = listed ? list_idx + j * ldl : nullptr;
  float* lv = listed ? list_val + j * ldl : nullptr;
  float* x = X + j * ldx;
#pragma unroll
  for (int q = 0; q < NPT; q += 4) {
    float xo[4];
    int o = off[q / 4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double w;
      const int gi = gidx(q + e);
      reload(v[q + e]);  // recompute w here rather than hold it since the count pass
      const bool kp = kept(gi, v[q + e], &w) && !zero;
      xo[e] = kp ? (float)(w * inv) : 0.f;
      if (kp && li != nullptr) {
        li[o] = gi;
        lv[o] = xo[e];
        ++o;
      }
      if (kp && marking) colmark[gi] = epoch;
    }
    const int i = gidx(q);
    if (i + 3 < p) {
      floatx4 t = {xo[0], xo[1], xo[2], xo[3]};
      *reinterpret_cast<floatx4*>(x + i) = t;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i + e < p) x[i + e] = xo[e];
    }
  }

  if (tid == 0) {
    if (WARM && warming && KIND != kTopS) wm.gam[j] = lam;
    // the selection threshold, a first guess for the next x-update
    if (full && s.thr != nullptr) {
      if (KIND == kTopS) s.thr[j] = zero ? 0.f : __uint_as_float(thr_key);
      if (KIND == kLambdaS) s.thr[j] = zero ? 0.f : (float)lam;
    }
    if (!full) {
      s.phi[j] = phi;
      s.nnz[j] = zero ? 0 : total;
    } else {
      const int it = s.iters[j] + 1;
      const double prev = s.phi[j];
      s.iters[j] = it;
      s.phi_prev[j] = prev;
      s.phi[j] = phi;
      s.nnz[j] = zero ? 0 : total;
      if (zero)
        s.status[j] = SPCA_ZERO;
      else if (it >= 2 && tol >= 0.0 && (!WARM || it >= wm.K + 1) &&
               phi <= (1.0 + tol) * prev)
        s.status[j] = SPCA_CONVERGED;
      else if (it >= maxit)
        s.status[j] = SPCA_MAXIT;
    }
  }
}

// ---------------------------------------------------------------------------
// Candidate x-update for T_s and V_{lambda_s} (register-resident rows,
// inside a solve).  Near convergence the selection threshold moves little
// between x-updates, so the entries with |v_i| at least 90% of the last
// threshold (the s-th largest |v_i|, or lambda) are few, and they contain
// every entry the operator keeps:
//   T_s       when at least s of them exist, the s largest |v_i| (ties to
//             the lower index) are the s first candidates in (|v| desc,
//             index asc) order;
//   lambda_s  when rho(t) = ||(|v| - t)_+||_1 / ||(|v| - t)_+||_2 >= sqrt(s)
//             at the guess t, the root lies above t (rho is non-increasing),
//             and the segment scan over the sorted candidates finds it.
// The candidates (at most kCandCap) are sorted in registers (a bitonic
// network: shuffles within a wave, LDS across waves, register swaps within
// a thread), and the norm, phi, list (sorted again, by index) and column
// marks all come from them; one more pass over the registers writes x.  A
// row whose guess does not hold (the first x-update, or a threshold that
// moved by more than 10%) is flagged in s.redo and left to
// x_update_reg_kernel, launched right after.  Reductions run in a fixed
// order, so results are deterministic.
// lambda_s first tries the last x-update's kept set S = {|v_i| > lambda'}:
// restricted to S, the root condition sum (|v| - l) = sqrt(s) ||(|v| - l)||_2
// is a quadratic in l whose smaller root is (S1 - sqrt(s (k S2 - S1^2) /
// (k - s))) / k (k = |S|, S1 = sum |v|, S2 = sum v^2 over S); when exactly
// the entries of S lie above that l, it is the root of the whole row, and
// the row is finished from registers without candidates or sorts.
// ---------------------------------------------------------------------------
constexpr int kCandCap = 1024;
constexpr int kCandPer = kCandCap / kRT;  // sorted positions per thread
constexpr float kGuessLow = 0.9f;
constexpr float kGuessRetry = 0.7f;  // the next guesses: this factor lower
constexpr int kLamRounds = 6;        // closed-form rounds of lambda_s before the candidates
constexpr uint32_t kIdxMask = 0x3fffu;    // row indices below 16384

struct CSmem {
  // candidate sort keys, (|v| bits) << 32 | (kIdxMask - index) << 1 | sign:
  // descending order is |v| descending, then index ascending
  uint64_t k64[kCandCap];
  int scan[kRW + 1];
  double dscan[2 * (kRW + 1)];
  double red[2];
  int kbest;
  double seg[4];
};

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)x, m, kWave);
  const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), m, kWave);
  return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of kRT E keys: x[e] is element tid + kRT e.
// Partners fewer than 64 apart are in the same wave (shuffles), 64 and 128
// apart in another wave (through buf, kRT E keys of LDS), kRT and more
// apart in the same thread.
template <int E>
__device__ __forceinline__ void block_sort_asc(uint64_t (&x)[E], uint64_t* buf) {
  const int tid = threadIdx.x;
  constexpr int N = kRT * E;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= kRT) {
        const int d = stride / kRT;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int e2 = e ^ d;
          if (e2 > e) {
            const bool asc = ((tid + kRT * e) & size) == 0;
            const uint64_t a = x[e], b = x[e2];
            const bool sw = asc ? a > b : a < b;
            x[e] = sw ? b : a;
            x[e2] = sw ? a : b;
          }
        }
      } else {
        if (stride >= kWave) {
#pragma unroll
          for (int e = 0; e < E; ++e) buf[tid + kRT * e] = x[e];
          __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int i = tid + kRT * e;
          const uint64_t b = stride >= kWave ? buf[i ^ stride] : shfl_xor_u64(x[e], stride);
          const bool lower = (i & stride) == 0;
          const bool asc = (i & size) == 0;
          const uint64_t mn = x[e] < b ? x[e] : b;
          const uint64_t mx = x[e] < b ? b : x[e];
          x[e] = lower == asc ? mn : mx;
        }
        if (stride >= kWave) __syncthreads();
      }
    }
  }
}

// Sorts arr[0, n) ascending in place (n <= kCandCap), padding with pad.
// Entries may have been written by any thread before the call.
template <int E>
__device__ __forceinline__ void sort_in_lds(uint64_t* arr, int n, uint64_t pad) {
  __syncthreads();
  uint64_t x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = threadIdx.x + kRT * e;
    x[e] = i < n ? arr[i] : pad;
  }
  __syncthreads();
  block_sort_asc<E>(x, arr);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = threadIdx.x + kRT * e;
    if (i < n) arr[i] = x[e];
  }
  __syncthreads();
}

// The same for n <= 64: the first wave sorts with shuffles alone.
__device__ __forceinline__ void sort_wave_lds(uint64_t* arr, int n, uint64_t pad) {
  __syncthreads();
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    uint64_t x = lane < n ? arr[lane] : pad;
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        const uint64_t b = shfl_xor_u64(x, stride);
        const bool lower = (lane & stride) == 0;
        const bool asc = (lane & size) == 0;
        const uint64_t mn = x < b ? x : b;
        const uint64_t mx = x < b ? b : x;
        x = lower == asc ? mn : mx;
      }
    }
    if (lane < n) arr[lane] = x;
  }
  __syncthreads();
}

__device__ __forceinline__ void sort_lds(uint64_t* arr, int n, uint64_t pad) {
  if (n <= kWave)
    sort_wave_lds(arr, n, pad);
  else if (n <= kRT)
    sort_in_lds<1>(arr, n, pad);
  else if (n <= 2 * kRT)
    sort_in_lds<2>(arr, n, pad);
  else
    sort_in_lds<4>(arr, n, pad);
}

// Sum over positions [0, m) of f(q), FP64, in a fixed order: lane l of the
// first wave adds positions l, l + 64, ..., then an xor butterfly.  The
// result is returned to every thread of the block.
template <typename F>
__device__ __forceinline__ double fixed_sum(int m, F f, double* slot) {
  if (threadIdx.x < kWave) {
    double a = 0.0;
    for (int q = threadIdx.x; q < m; q += kWave) a += f(q);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, kWave);
    if (threadIdx.x == 0) *slot = a;
  }
  __syncthreads();
  const double r = *slot;
  __syncthreads();
  return r;
}

template <int KIND, int NPT>
__global__ __launch_bounds__(kRT, 4) void x_update_cand_kernel(
    const float* __restrict__ V, int64_t ldv, int p, double param,
    float* __restrict__ X, int64_t ldx, int32_t* __restrict__ list_idx,
    float* __restrict__ list_val, int64_t ldl, int list_cap, StartState s,
    double tol, int maxit, int32_t* __restrict__ colmark, const Plan* plan) {
  static_assert(KIND == kTopS || KIND == kLambdaS, "T_s and lambda_s only");
  static_assert(kRT * NPT <= (int)kIdxMask + 1, "row indices must fit the sort key");
  __shared__ CSmem sm;
  const int64_t j = blockIdx.x;
  if (s.status[j] != kRunning) return;
  if (s.cfg != nullptr) {  // grouped solve: this start's request
    if (s.cfg[j].kind != KIND) return;
    param = s.cfg[j].param;
    tol = s.cfg[j].tol;
    maxit = s.cfg[j].maxit;
  }
  const int tid = threadIdx.x;
  const uint32_t t0 = key_of(s.thr[j] * kGuessLow);
  if (t0 == 0u) {  // no guess yet
    if (tid == 0) s.redo[j] = 1;
    return;
  }
  auto gidx = [&](int k) { return 4 * ((k / 4) * kRT + tid) + k % 4; };
  const float* vg = V + j * ldv;
  float v[NPT];
#pragma unroll
  for (int q = 0; q < NPT; q += 4) {
    const int i = gidx(q);
    if (i + 3 < p) {
      const floatx4 w4 = *reinterpret_cast<const floatx4*>(vg + i);
      v[q] = w4.x;
      v[q + 1] = w4.y;
      v[q + 2] = w4.z;
      v[q + 3] = w4.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[q + e] = i + e < p ? vg[i + e] : 0.f;
    }
  }
  if constexpr (KIND == kLambdaS) {
    // closed-form root on the last kept set (every branch below depends on
    // block totals only, so all threads take it together)
    constexpr int R = NPT / 4;
    // S_0 = {|v| > lambda'}; each round takes the root l of S_t's quadratic
    // and S_{t+1} = {|v| > l}, until S_{t+1} = S_t (l is then the root of the
    // row) or kLamRounds rounds; a row that does not settle takes the
    // candidate path below
    const double lprev = (double)s.thr[j];
    double set3[3] = {0.0, 0.0, 0.0};  // |S|, sum |v| and sum v^2 over S
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      reload(v[k]);  // each pass derives its doubles afresh (no copies held across passes)
      const double a = fabs((double)v[k]);
      if (a > lprev) {
        set3[0] += 1.0;
        set3[1] += a;
        set3[2] += a * a;
      }
    }
    block_sum_n<double, 3>(set3, reinterpret_cast<double*>(sm.k64));
    double lam = -1.0;
    int cnt[R], off[R];
    double acc[2] = {0.0, 0.0};
    bool settled = false;
#pragma unroll 1
    for (int round = 0; round < kLamRounds; ++round) {
      const double kk = set3[0];
      if (!(kk > param)) break;
      double disc = kk * set3[2] - set3[1] * set3[1];
      disc = disc > 0.0 ? disc : 0.0;
      lam = (set3[1] - sqrt(param * disc / (kk - param))) / kk;
      if (!(lam > 0.0)) break;
      // the set above lam: its size and sums (the next round's), and the
      // squared distances to lam (the norm, if the set is unchanged)
      double b4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < R; ++q) {
        cnt[q] = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          reload(v[4 * q + e]);
          const double a = fabs((double)v[4 * q + e]);
          if (a > lam) {
            ++cnt[q];
            b4[0] += 1.0;
            b4[1] += a;
            b4[2] += a * a;
            b4[3] += (a - lam) * (a - lam);
          }
        }
      }
      block_sum_n<double, 4>(b4, reinterpret_cast<double*>(sm.k64));
      if (b4[0] == kk) {  // nested sets of equal size: unchanged
        acc[0] = b4[3];
        acc[1] = b4[0];
        settled = true;
        break;
      }
      set3[0] = b4[0];
      set3[1] = b4[1];
      set3[2] = b4[2];
    }
    if (settled) {  // {|v| > lam} is the set lam came from: lam is the root
      const int total = rank_rows<R>(cnt, off, sm.k64);
      const double nrm = sqrt(acc[0]);
      const double phi = lam * sqrt(param) + nrm;
      const bool zero = !(nrm > 0.0);
      const double inv = zero ? 0.0 : 1.0 / nrm;
      const bool listed = list_idx != nullptr && !zero && total <= list_cap;
      const bool marking = colmark != nullptr && !zero && plan->mark != 0;
      const int32_t epoch = marking ? plan->epoch : 0;
      int32_t* li = listed ? list_idx + j * ldl : nullptr;
      float* lv = listed ? list_val + j * ldl : nullptr;
      float* x = X + j * ldx;
#pragma unroll
      for (int q = 0; q < NPT; q += 4) {
        float xo[4];
        int o = off[q / 4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          reload(v[q + e]);
          const float vv = v[q + e];
          const double a = fabs((double)vv);
          const bool kp = a > lam && !zero;
          const double w = vv > 0.f ? a - lam : lam - a;
          xo[e] = kp ? (float)(w * inv) : 0.f;
          const int gi = gidx(q + e);
          if (kp && li != nullptr) {
            li[o] = gi;
            lv[o] = xo[e];
            ++o;
          }
          if (kp && marking) colmark[gi] = epoch;
        }
        const int i = gidx(q);
        if (i + 3 < p) {
          floatx4 w4 = {xo[0], xo[1], xo[2], xo[3]};
          *reinterpret_cast<floatx4*>(x + i) = w4;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (i + e < p) x[i + e] = xo[e];
        }
      }
      if (tid == 0) {
        s.redo[j] = 0;
        s.thr[j] = zero ? 0.f : (float)lam;
        const int it = s.iters[j] + 1;
        const double prev = s.phi[j];
        s.iters[j] = it;
        s.phi_prev[j] = prev;
        s.phi[j] = phi;
        s.nnz[j] = zero ? 0 : total;
        if (zero)
          s.status[j] = SPCA_ZERO;
        else if (it >= 2 && tol >= 0.0 && phi <= (1.0 + tol) * prev)
          s.status[j] = SPCA_CONVERGED;
        else if (it >= maxit)
          s.status[j] = SPCA_MAXIT;
      }
      return;
    }
  }
  // the candidate at sorted position q
  auto cval = [&](int q) -> float {  // signed value
    const uint64_t k = ~sm.k64[q];
    const uint32_t bits = (uint32_t)(k >> 32) | ((uint32_t)k << 31);
    return __uint_as_float(bits);
  };
  auto cidx = [&](int q) -> int {
    return (int)(kIdxMask - (((uint32_t)~sm.k64[q] >> 1) & kIdxMask));
  };
  const uint32_t s_int =
      (uint32_t)((int64_t)param < (int64_t)p ? (int64_t)param : (int64_t)p);

  // the guess t: accepted when it brackets the threshold (at least s keys
  // at or above it for T_s; for lambda_s more than s keys and
  // rho(t) >= sqrt(s), i.e. the root at or above t) with at most kCandCap
  // candidates; otherwise lowered twice by a factor 0.7 (too many
  // candidates leave the row to the full kernel at once)
  const double rs = sqrt(param);
  uint32_t t = t0;
  bool ok = false;
  int mine = 0;
#pragma unroll 1
  for (int attempt = 0; attempt < 3; ++attempt) {
    if (attempt > 0) t = key_of(__uint_as_float(t) * kGuessRetry);
    if (t == 0u) break;
    // (the rho test only picks the guess, so FP32 sums do: a guess
    // accepted by rounding finds no root segment below and is left to the
    // full kernel)
    mine = 0;
    float a[2] = {0.f, 0.f};
    const float tf = __uint_as_float(t);
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const bool in = key_of(v[k]) >= t;
      mine += in;
      if (KIND == kLambdaS) {
        const float d = in ? fabsf(v[k]) - tf : 0.f;
        a[0] += d;
        a[1] += d * d;
      }
    }
    const int n_in = block_sum(mine, sm.scan);
    if (KIND == kLambdaS) block_sum_n<float, 2>(a, reinterpret_cast<float*>(sm.dscan));
    if (n_in > kCandCap) break;
    if (KIND == kTopS ? n_in >= (int)s_int
                      : (double)n_in > param && a[1] > 0.f &&
                            (double)a[0] >= rs * sqrt((double)a[1])) {
      ok = true;
      break;
    }
  }
  if (!ok) {
    if (tid == 0) s.redo[j] = 1;
    return;
  }
  int nc;
  int off = block_exclusive_scan(mine, sm.scan, &nc);
  // sort keys, complemented so that an ascending sort gives (|v| desc,
  // index asc); the pads (all ones) go last
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const uint32_t key = key_of(v[k]);
    if (key >= t) {
      const uint32_t lo = ((kIdxMask - (uint32_t)gidx(k)) << 1) | (__float_as_uint(v[k]) >> 31);
      sm.k64[off++] = ~(((uint64_t)key << 32) | lo);
    }
  }
  sort_lds(sm.k64, nc, ~0ull);

  uint32_t thr_key = 0;
  int64_t cut = -1;
  double lam = 0.0;
  int nkept;
  if (KIND == kTopS) {
    thr_key = key_of(cval(s_int - 1));
    cut = cidx(s_int - 1);
    nkept = (int)s_int;
  } else {
    const double s_par = param;
    const double tf = (double)__uint_as_float(t);
    // prefix sums of c and c^2 over the sorted candidates; thread t owns
    // positions kCandPer t onward; the segment holding the root
    double cv[kCandPer], pre[2] = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kCandPer; ++e) {
      const int q = kCandPer * tid + e;
      cv[e] = q < nc ? fabs((double)cval(q)) : 0.0;
      pre[0] += cv[e];
      pre[1] += cv[e] * cv[e];
    }
    rscan2(pre, sm.dscan);
    if (tid == 0) sm.kbest = INT32_MAX;
    __syncthreads();
    double S1 = pre[0], S2 = pre[1];
    int myk = INT32_MAX;
    double seg[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kCandPer; ++e) {
      const int q = kCandPer * tid + e;
      S1 += cv[e];
      S2 += cv[e] * cv[e];
      const int k = q + 1;
      if (q >= nc || (double)k <= s_par || myk != INT32_MAX) continue;
      const double lo = k < nc ? fabs((double)cval(k)) : tf;
      const double l1 = S1 - (double)k * lo;
      const double l2 = S2 - 2.0 * lo * S1 + (double)k * lo * lo;
      if (l2 > 0.0 && l1 >= rs * sqrt(l2)) {
        myk = k;
        seg[0] = S1;
        seg[1] = S2;
        seg[2] = lo;
        seg[3] = cv[e];
      }
    }
    if (myk != INT32_MAX) atomicMin(&sm.kbest, myk);
    __syncthreads();
    const int kb = sm.kbest;
    if (myk == kb && kb != INT32_MAX) {
      sm.seg[0] = seg[0];
      sm.seg[1] = seg[1];
      sm.seg[2] = seg[2];
      sm.seg[3] = seg[3];
    }
    __syncthreads();
    if (kb == INT32_MAX) {  // rounding at the lower end: leave it to the full kernel
      if (tid == 0) s.redo[j] = 1;
      return;
    }
    const double k = (double)kb, S1b = sm.seg[0], S2b = sm.seg[1];
    double disc = k * S2b - S1b * S1b;
    disc = disc > 0.0 ? disc : 0.0;
    double l = (S1b - sqrt(s_par * disc / (k - s_par))) / k;
    l = l < sm.seg[2] ? sm.seg[2] : l;
    l = l > sm.seg[3] ? sm.seg[3] : l;
    lam = l;
    // kept: |v| > lambda, a prefix of the sorted candidates
    int cnt = 0;
    for (int q = tid; q < nc; q += kRT) cnt += fabs((double)cval(q)) > lam;
    nkept = block_sum(cnt, sm.scan);
  }
  // w of the kept candidate at sorted position q
  auto wsorted = [&](int q) -> double {
    const float x = cval(q);
    if (KIND == kTopS) return (double)x;
    const double a = fabs((double)x);
    return x > 0.f ? a - lam : lam - a;
  };
  const double nrm2 = fixed_sum(nkept, [&](int q) {
    const double w = wsorted(q);
    return w * w;
  }, &sm.red[0]);
  const double nrm = sqrt(nrm2);
  const double phi = KIND == kLambdaS ? lam * sqrt(param) + nrm : nrm;
  const bool zero = !(nrm > 0.0);
  const double inv = zero ? 0.0 : 1.0 / nrm;
  // list (index order) and column marks, from the kept candidates: their
  // (index, x value) pairs sorted by index
  const bool listed = list_idx != nullptr && !zero && nkept <= list_cap;
  const bool marking = colmark != nullptr && !zero && plan->mark != 0;
  const int32_t epoch = marking ? plan->epoch : 0;
  if (listed || marking) {
    uint64_t pr[kCandPer];
#pragma unroll
    for (int e = 0; e < kCandPer; ++e) {
      const int q = tid + kRT * e;
      pr[e] = q < nkept ? ((uint64_t)(uint32_t)cidx(q) << 32) |
                              __float_as_uint((float)(wsorted(q) * inv))
                        : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kCandPer; ++e) {
      const int q = tid + kRT * e;
      if (q < nkept) sm.k64[q] = pr[e];
    }
    sort_lds(sm.k64, nkept, ~0ull);
    for (int q = tid; q < nkept; q += kRT) {
      const uint64_t k = sm.k64[q];
      const int iq = (int)(k >> 32);
      if (listed) {
        list_idx[j * ldl + q] = iq;
        list_val[j * ldl + q] = __uint_as_float((uint32_t)k);
      }
      if (marking) colmark[iq] = epoch;
    }
  }
  // x, from the registers
  float* x = X + j * ldx;
#pragma unroll
  for (int q = 0; q < NPT; q += 4) {
    float xo[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float vv = v[q + e];
      const uint32_t kk = key_of(vv);
      bool kp;
      double w;
      if (KIND == kTopS) {
        w = (double)vv;
        kp = kk != 0u && (kk > thr_key || (kk == thr_key && (int64_t)gidx(q + e) <= cut));
      } else {
        const double a = fabs((double)vv);
        w = vv > 0.f ? a - lam : lam - a;
        kp = a > lam;
      }
      xo[e] = (kp && !zero) ? (float)(w * inv) : 0.f;
    }
    const int i = gidx(q);
    if (i + 3 < p) {
      floatx4 w4 = {xo[0], xo[1], xo[2], xo[3]};
      *reinterpret_cast<floatx4*>(x + i) = w4;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i + e < p) x[i + e] = xo[e];
    }
  }
  if (tid == 0) {
    s.redo[j] = 0;
    s.thr[j] = zero ? 0.f : (KIND == kTopS ? __uint_as_float(thr_key) : (float)lam);
    const int it = s.iters[j] + 1;
    const double prev = s.phi[j];
    s.iters[j] = it;
    s.phi_prev[j] = prev;
    s.phi[j] = phi;
    s.nnz[j] = zero ? 0 : nkept;
    if (zero)
      s.status[j] = SPCA_ZERO;
    else if (it >= 2 && tol >= 0.0 && phi <= (1.0 + tol) * prev)
      s.status[j] = SPCA_CONVERGED;
    else if (it >= maxit)
      s.status[j] = SPCA_MAXIT;
  }
}

template <int KIND, int NPT>
void launch_reg(hipStream_t st, double param, const float* V, int64_t ldv,
                int64_t r, int64_t p, float* X, int64_t ldx, int32_t* li,
                float* lv, int64_t ldl, int list_cap, StartState s, double tol,
                int maxit, int32_t* colmark, const Plan* plan, Warm wm) {
  // inside a solve, T_s and lambda_s first try the candidate kernel; the
  // full kernel then takes only the rows it flagged
  constexpr bool kCand = KIND == kTopS || KIND == kLambdaS;
  const bool cand = kCand && wm.K == 0 && s.status != nullptr && s.thr != nullptr &&
                    s.redo != nullptr;
  if (!cand) s.redo = nullptr;
  if constexpr (kCand) {
    if (cand)
      hipLaunchKernelGGL((x_update_cand_kernel<KIND, NPT>), dim3((unsigned)r), dim3(kRT),
                         0, st, V, ldv, (int)p, param, X, ldx, li, lv, ldl, list_cap, s,
                         tol, maxit, colmark, plan);
  }
  if (KIND != kTopS && wm.K > 0)
    hipLaunchKernelGGL((x_update_reg_kernel<KIND, NPT, true>), dim3((unsigned)r),
                       dim3(kRT), 0, st, V, ldv, (int)p, param, X, ldx, li, lv,
                       ldl, list_cap, s, tol, maxit, colmark, plan, wm);
  else
    hipLaunchKernelGGL((x_update_reg_kernel<KIND, NPT, false>), dim3((unsigned)r),
                       dim3(kRT), 0, st, V, ldv, (int)p, param, X, ldx, li, lv,
                       ldl, list_cap, s, tol, maxit, colmark, plan, wm);
}

template <int KIND>
void launch_kind(hipStream_t st, double param, const float* V, int64_t ldv,
                 int64_t r, int64_t p, float* X, int64_t ldx, int32_t* li,
                 float* lv, int64_t ldl, int list_cap, StartState s, double tol,
                 int maxit, int32_t* colmark, const Plan* plan, Warm wm) {
  const bool aligned = ldv % 4 == 0 && ldx % 4 == 0 &&
                       (uintptr_t)V % 16 == 0 && (uintptr_t)X % 16 == 0;
  const int64_t per = ceil_div(p, kRT);
  if (aligned && per <= 48) {
    if (per <= 8)
      launch_reg<KIND, 8>(st, param, V, ldv, r, p, X, ldx, li, lv, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
    else if (per <= 16)
      launch_reg<KIND, 16>(st, param, V, ldv, r, p, X, ldx, li, lv, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
    else if (per <= 24)
      launch_reg<KIND, 24>(st, param, V, ldv, r, p, X, ldx, li, lv, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
    else if (per <= 32)
      launch_reg<KIND, 32>(st, param, V, ldv, r, p, X, ldx, li, lv, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
    else if (per <= 40)
      launch_reg<KIND, 40>(st, param, V, ldv, r, p, X, ldx, li, lv, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
    else
      launch_reg<KIND, 48>(st, param, V, ldv, r, p, X, ldx, li, lv, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
    return;
  }
  if (p <= kStageMax) {
    size_t shm = (size_t)p * sizeof(float);
    hipLaunchKernelGGL((x_update_kernel<KIND, true>), dim3((unsigned)r),
                       dim3(kXT), shm, st, V, ldv, (int)p, param, X, ldx, li,
                       lv, ldl, list_cap, s, tol, maxit, colmark, plan);
  } else {
    hipLaunchKernelGGL((x_update_kernel<KIND, false>), dim3((unsigned)r),
                       dim3(kXT), 0, st, V, ldv, (int)p, param, X, ldx, li, lv,
                       ldl, list_cap, s, tol, maxit, colmark, plan);
  }
}

}  // namespace

void x_update(hipStream_t st, int fid, double s_or_gamma, const float* V,
              int64_t ldv, int64_t r, int64_t p, float* X, int64_t ldx,
              int32_t* list_idx, float* list_val, int64_t ldl, int list_cap,
              StartState s, double tol, int32_t maxit, int32_t* colmark,
              const Plan* plan, void* wide, Warm wm) {
  if (wide != nullptr &&
      x_update_wide(st, fid, s_or_gamma, V, ldv, r, p, X, ldx, list_idx, list_val,
                    ldl, list_cap, s, tol, maxit, colmark, plan, wide, wm))
    return;
  switch (xkind_of(fid)) {
    case kTopS:
      launch_kind<kTopS>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                         list_val, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
      break;
    case kLambdaS:
      launch_kind<kLambdaS>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                            list_val, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
      break;
    case kHardGamma:
      launch_kind<kHardGamma>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                              list_val, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
      break;
    case kSoftGamma:
      launch_kind<kSoftGamma>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                              list_val, ldl, list_cap, s, tol, maxit, colmark, plan, wm);
      break;
  }
}

}  // namespace spca
