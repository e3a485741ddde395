// x-update of Algorithm 2 (Table 3, rows S3-S6), one workgroup per start:
//   L0 constraint  x = T_s(v) / ||T_s(v)||             phi = ||T_s(v)||
//   L1 constraint  x = V_l(v) / ||V_l(v)||, l = lambda_s(v)
//                                                      phi = l sqrt(s) + ||V_l(v)||
//   L0 penalty     x = U_g(v) / ||U_g(v)||             phi = sum_kept (v_i^2 - g)
//   L1 penalty     x = V_g(v) / ||V_g(v)||             phi = ||V_g(v)||
// followed by the ratio stop test of Section 2.2.
//
// Selection without sorting.  The bit pattern of a non-negative float is
// monotone in its value, so thresholds are searched over the 31-bit keys of
// |v_i|.  Each step tests kNC thresholds at once with one deterministic
// block reduction (an 8-ary search, 11 steps for 31 bits):
//   T_s       largest key t with #{key >= t} >= s; ties at that key go to the
//             lowest indices (a block-wide prefix count finds the cut index).
//   lambda_s  the derivative of l sqrt(s) + ||V_l(v)|| is sqrt(s) - rho(l)
//             with rho = ||V_l||_1 / ||V_l||_2 non-increasing, so the search
//             finds the float interval [t, t+) holding the root; on it the
//             active set is fixed and the root has the closed form
//             l = (S1 - sqrt(s (k S2 - S1^2) / (k - s))) / k.
// Comparisons that decide membership use FP64 on the FP32 inputs (squares
// and differences of floats are exact or correctly rounded there).
#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr int kXT = 1024;  // threads per start
constexpr int kNW = kXT / kWave;
constexpr int kNC = 7;     // thresholds per search step
constexpr int64_t kStageMax = 12288;  // p staged in LDS up to this size

__device__ __forceinline__ uint32_t key_of(float v) {
  return __float_as_uint(v) & 0x7fffffffu;
}

struct XSmem {
  double dred[2 * kNC * (kNW + 1)];
  int32_t ired[kNC * (kNW + 1)];
  uint32_t ured[kNW + 1];
  int scan[kNW + 1];
  int64_t cut;  // last index kept among the ties (T_s)
};

template <int KIND, bool STAGED>
__global__ __launch_bounds__(kXT) void x_update_kernel(
    const float* __restrict__ V, int64_t ldv, int p, double param,
    float* __restrict__ X, int64_t ldx, int32_t* __restrict__ list_idx,
    float* __restrict__ list_val, int64_t ldl, StartState s, double tol,
    int maxit) {
  extern __shared__ __attribute__((aligned(16))) float vstage[];
  __shared__ XSmem sm;
  const int64_t j = blockIdx.x;
  const bool full = s.status != nullptr;
  if (full && s.status[j] != kRunning) return;
  const int tid = threadIdx.x;
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
    bool search = true;
    uint32_t lo = 0, hi = mk + 1;
    if (KIND == kTopS) {
      const int64_t s_int = (int64_t)s_par < (int64_t)p ? (int64_t)s_par : (int64_t)p;
      // pred(t) = #{key >= t} >= s ; pred(0) holds, pred(mk + 1) fails
      while (hi - lo > 1) {
        uint32_t t[kNC];
        const uint32_t span = hi - lo;
#pragma unroll
        for (int c = 0; c < kNC; ++c) {
          uint32_t d = span > kNC + 1
                           ? (uint32_t)(((uint64_t)span * (uint64_t)(c + 1)) / (kNC + 1))
                           : (uint32_t)(c + 1);
          t[c] = d < span ? lo + d : hi;
        }
        int cnt[kNC];
#pragma unroll
        for (int c = 0; c < kNC; ++c) cnt[c] = 0;
        for (int i = tid; i < p; i += kXT) {
          uint32_t k = key_of(val(i));
#pragma unroll
          for (int c = 0; c < kNC; ++c) cnt[c] += k >= t[c];
        }
        block_sum_n<int, kNC>(cnt, sm.ired);
        uint32_t nlo = lo, nhi = hi;
#pragma unroll
        for (int c = 0; c < kNC; ++c) {
          if (t[c] >= hi) continue;
          if (cnt[c] >= s_int) {
            nlo = t[c] > nlo ? t[c] : nlo;
          } else {
            nhi = t[c] < nhi ? t[c] : nhi;
          }
        }
        lo = nlo;
        hi = nhi;
      }
      thr_key = lo;
      // ties at thr_key: keep the first (s - #{key > thr_key}) in index order
      if (tid == 0) sm.cut = -1;
      int gt = 0, eq = 0;
      for (int i = tid; i < p; i += kXT) {
        uint32_t k = key_of(val(i));
        gt += k > thr_key;
      }
      for (int i = cb; i < ce; ++i) eq += key_of(val(i)) == thr_key;
      gt = block_sum(gt, sm.ired);
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
      search = false;
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
      search = a0[0] > rs * sqrt(a0[1]);
      if (!search) lam = 0.0;
      hi = mk;  // no entry exceeds max |v|: rho undefined, pred false
      while (search && hi - lo > 1) {
        uint32_t t[kNC];
        const uint32_t span = hi - lo;
#pragma unroll
        for (int c = 0; c < kNC; ++c) {
          uint32_t d = span > kNC + 1
                           ? (uint32_t)(((uint64_t)span * (uint64_t)(c + 1)) / (kNC + 1))
                           : (uint32_t)(c + 1);
          t[c] = d < span ? lo + d : hi;
        }
        double acc[2 * kNC];
#pragma unroll
        for (int c = 0; c < 2 * kNC; ++c) acc[c] = 0.0;
        double tf[kNC];
#pragma unroll
        for (int c = 0; c < kNC; ++c) tf[c] = (double)__uint_as_float(t[c]);
        for (int i = tid; i < p; i += kXT) {
          double a = fabs((double)val(i));
#pragma unroll
          for (int c = 0; c < kNC; ++c) {
            double d = a - tf[c];
            d = d > 0.0 ? d : 0.0;
            acc[2 * c] += d;
            acc[2 * c + 1] += d * d;
          }
        }
        block_sum_n<double, 2 * kNC>(acc, sm.dred);
        uint32_t nlo = lo, nhi = hi;
#pragma unroll
        for (int c = 0; c < kNC; ++c) {
          if (t[c] >= hi) continue;
          bool pred = acc[2 * c + 1] > 0.0 && acc[2 * c] >= rs * sqrt(acc[2 * c + 1]);
          if (pred) {
            nlo = t[c] > nlo ? t[c] : nlo;
          } else {
            nhi = t[c] < nhi ? t[c] : nhi;
          }
        }
        lo = nlo;
        hi = nhi;
      }
      if (search) {
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
  if (list_idx != nullptr && !zero) {
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
  for (int i = tid; i < p; i += kXT) {
    float v = val(i);
    double w;
    bool k = kept(i, v, &w);
    x[i] = (k && !zero) ? (float)(w * inv) : 0.f;
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

template <int KIND>
void launch_kind(hipStream_t st, double param, const float* V, int64_t ldv,
                 int64_t r, int64_t p, float* X, int64_t ldx, int32_t* li,
                 float* lv, int64_t ldl, StartState s, double tol, int maxit) {
  if (p <= kStageMax) {
    size_t shm = (size_t)p * sizeof(float);
    hipLaunchKernelGGL((x_update_kernel<KIND, true>), dim3((unsigned)r),
                       dim3(kXT), shm, st, V, ldv, (int)p, param, X, ldx, li,
                       lv, ldl, s, tol, maxit);
  } else {
    hipLaunchKernelGGL((x_update_kernel<KIND, false>), dim3((unsigned)r),
                       dim3(kXT), 0, st, V, ldv, (int)p, param, X, ldx, li, lv,
                       ldl, s, tol, maxit);
  }
}

}  // namespace

void x_update(hipStream_t st, int fid, double s_or_gamma, const float* V,
              int64_t ldv, int64_t r, int64_t p, float* X, int64_t ldx,
              int32_t* list_idx, float* list_val, int64_t ldl, StartState s,
              double tol, int32_t maxit) {
  switch (xkind_of(fid)) {
    case kTopS:
      launch_kind<kTopS>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                         list_val, ldl, s, tol, maxit);
      break;
    case kLambdaS:
      launch_kind<kLambdaS>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                            list_val, ldl, s, tol, maxit);
      break;
    case kHardGamma:
      launch_kind<kHardGamma>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                              list_val, ldl, s, tol, maxit);
      break;
    case kSoftGamma:
      launch_kind<kSoftGamma>(st, s_or_gamma, V, ldv, r, p, X, ldx, list_idx,
                              list_val, ldl, s, tol, maxit);
      break;
  }
}

}  // namespace spca
