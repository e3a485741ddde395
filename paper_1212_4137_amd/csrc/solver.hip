// C-ABI of libspca: argument checks, the per-device context and workspace,
// and the host driver of the batched AM iteration (Algorithm 2 run from r
// starts at once, Section 4).  One iteration is
//   [dense]  U = X A^T (MFMA GEMM)  ->  y-update kernel
//   [sparse] list-based A x fused with the y-update      (one of the two runs;
//                                                         the planner decides
//                                                         on the device)
//   V = Y A (MFMA GEMM)  ->  x-update + stop test  ->  planner
// The host only polls the count of running starts every check_every
// iterations; everything else stays on the device.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spca.h"
#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"

namespace spca {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

int check_problem(int64_t n, int64_t p, int64_t lda, int fid, double sg,
                  int64_t r, double tol, int32_t maxit) {
  (void)tol;
  SPCA_REQUIRE(n >= 1 && p >= 1, "n and p must be >= 1");
  SPCA_REQUIRE(r >= 1, "r (number of starts) must be >= 1");
  SPCA_REQUIRE(lda >= n, "lda must be >= n");
  SPCA_REQUIRE(fid >= 1 && fid <= 8, "formulation must be in 1..8 (Table 1)");
  SPCA_REQUIRE(maxit >= 1, "maxit must be >= 1");
  SPCA_REQUIRE(p <= INT32_MAX && n <= INT32_MAX && r <= INT32_MAX,
               "n, p and r must fit in int32");
  SPCA_REQUIRE(isfinite(sg), "s_or_gamma must be finite");
  if (fid <= 2) {
    SPCA_REQUIRE(sg >= 1.0 && sg <= (double)p && sg == floor(sg),
                 "L0 constraint needs an integral s in [1, p]");
  } else if (fid <= 4) {
    SPCA_REQUIRE(sg >= 1.0, "L1 constraint needs s >= 1");
  } else {
    SPCA_REQUIRE(sg >= 0.0, "penalty gamma must be >= 0");
  }
  return SPCA_OK;
}

namespace {

// The list-based A x is possible when every running start has at most
// max(32, p / 8) nonzeros; only those starts keep (index, value) lists.
constexpr double kSparseFraction = 0.125;
inline int list_cap_of(int64_t p) {
  int64_t c = (int64_t)(kSparseFraction * (double)p);
  return (int)(c < 32 ? (p < 32 ? p : 32) : c);
}

constexpr int kMaxSplits = 16;  // K splits of the dense A x product
static_assert(kMaxSplits <= kSplitsMax, "the y-update sums at most kSplitsMax partials");
constexpr int kTimeSample = 8;  // SPCA_FLAG_TIME_SAMPLED: events every 8th iteration

struct Layout {
  int64_t n, p, r;
  int64_t ldx, ldu, ldat, ldac;
  bool copy_a, bf16;
  int64_t ldab, ldatb, ldyb, ldxb;
  size_t off_Ab, off_Atb, off_Yb, off_Xb, off_Xp;
  GemmPlan plan_ax, plan_aty;
  int ax_split_cap, aty_split_cap;
  size_t off_At, off_Ac, off_X, off_U, off_Y, off_V, off_li, off_lv;
  size_t off_phi, off_phip, off_nnz, off_it, off_st, off_plan, off_part,
      off_f, off_ev, off_xn, off_best, off_xout, off_sup, off_colsq, off_bad, off_thr, off_redo;
  size_t off_mark, off_ulist, off_Xc, off_Qc, off_wide, off_gam;
  size_t wide_bytes;
  int64_t ucap;  // largest support union the union product can hold
  GemmPlan plan_union;
  size_t total;
  int nchunks;
};

size_t carve(size_t* cur, size_t bytes) {
  size_t o = (*cur + 255) / 256 * 256;
  *cur = o + bytes;
  return o;
}

Layout make_layout(int64_t n, int64_t p, int64_t r, bool copy_a, bool bf16) {
  Layout L;
  L.n = n;
  L.p = p;
  L.r = r;
  L.ldx = round_up(p, 4);
  L.ldu = round_up(n, 4);
  L.ldat = round_up(p, 4);
  L.ldac = round_up(n, 4);
  L.copy_a = copy_a;
  L.bf16 = bf16;
  L.ldab = round_up(n, 8);
  L.ldatb = round_up(p, 8);
  L.ldyb = round_up(n, 8);
  L.ldxb = round_up(p, 8);
  L.nchunks = (int)ceil_div(n, 64);  // partial pairs per start (64-row tiles at most)
  const int eb = bf16 ? 2 : 4;
  L.plan_ax = plan_gemm_nt(r, n, p, kMaxSplits, eb);   // U^T = X^T A^T, K = p
  L.plan_aty = plan_gemm_nt(r, p, n, kMaxSplits, eb);  // V^T = Y^T A,   K = n
  // union product (FP32 only): K = u <= ucap columns, gathered A is
  // n x ucap (<= 256 MB)
  L.ucap = bf16 ? 0 : p;
  const int64_t mem_cap = (int64_t)(64LL << 20) / (n > 0 ? n : 1);
  if (L.ucap > mem_cap) L.ucap = mem_cap < 1024 ? (p < 1024 ? p : 1024) : mem_cap;
  L.plan_union = plan_gemm_nt(r, n, L.ucap < 256 ? (L.ucap > 0 ? L.ucap : 1) : 256, 1);
  size_t c = 0;
  L.off_At = carve(&c, bf16 ? 0 : sizeof(float) * (size_t)n * L.ldat);
  L.off_Ab = carve(&c, bf16 ? sizeof(uint16_t) * (size_t)p * L.ldab : 0);
  L.off_Atb = carve(&c, bf16 ? sizeof(uint16_t) * (size_t)n * L.ldatb : 0);
  L.off_Yb = carve(&c, bf16 ? sizeof(uint16_t) * (size_t)r * L.ldyb : 0);
  L.off_Xb = carve(&c, bf16 ? sizeof(uint16_t) * (size_t)r * L.ldxb : 0);
  L.off_Xp = carve(&c, bf16 ? sizeof(float) * (size_t)r * p : 0);

  L.off_Ac = carve(&c, copy_a ? sizeof(float) * (size_t)p * L.ldac : 0);
  L.off_X = carve(&c, sizeof(float) * (size_t)r * L.ldx);
  // room for the largest split count a tuned plan may pick
  L.ax_split_cap = max_feasible_splits(p, kMaxSplits, eb);
  if (L.ax_split_cap < L.plan_ax.splits) L.ax_split_cap = L.plan_ax.splits;
  L.off_U = carve(&c, sizeof(float) * (size_t)L.ax_split_cap * r * L.ldu);
  L.off_Y = carve(&c, sizeof(float) * (size_t)r * L.ldu);
  // V and the partials of a K-split A^T Y (summed into V before the x-update)
  L.aty_split_cap = max_feasible_splits(n, kMaxSplits, eb);
  if (L.aty_split_cap < L.plan_aty.splits) L.aty_split_cap = L.plan_aty.splits;
  L.off_V = carve(&c, sizeof(float) * (size_t)L.aty_split_cap * r * L.ldx);
  L.off_li = carve(&c, sizeof(int32_t) * (size_t)r * L.ldx);
  L.off_lv = carve(&c, sizeof(float) * (size_t)r * L.ldx);
  L.off_phi = carve(&c, sizeof(double) * r);
  L.off_phip = carve(&c, sizeof(double) * r);
  L.off_nnz = carve(&c, sizeof(int32_t) * r);
  L.off_it = carve(&c, sizeof(int32_t) * r);
  L.off_st = carve(&c, sizeof(int32_t) * r);
  L.off_thr = carve(&c, sizeof(float) * r);
  L.off_redo = carve(&c, sizeof(int32_t) * r);
  L.off_plan = carve(&c, sizeof(Plan));
  L.off_part = carve(&c, sizeof(double) * 2 * (size_t)r * L.nchunks);
  L.off_f = carve(&c, sizeof(double) * r);
  L.off_ev = carve(&c, sizeof(double) * r);
  L.off_xn = carve(&c, sizeof(double) * 2 * r);
  L.off_best = carve(&c, sizeof(int32_t) * 2);
  L.off_xout = carve(&c, sizeof(double) * p);
  L.off_gam = carve(&c, sizeof(double) * r);
  L.off_sup = carve(&c, sizeof(int32_t) * p);
  L.off_colsq = carve(&c, sizeof(double) * p);
  L.off_bad = carve(&c, sizeof(int32_t));
  L.off_mark = carve(&c, sizeof(int32_t) * p);
  L.off_ulist = carve(&c, sizeof(int32_t) * p);
  L.off_Xc = carve(&c, sizeof(float) * (size_t)r * round_up(L.ucap, 4));
  L.off_Qc = carve(&c, sizeof(float) * (size_t)n * round_up(L.ucap, 4));
  L.wide_bytes = x_update_wide_bytes(1, r, p);
  L.off_wide = carve(&c, L.wide_bytes);
  L.total = c;
  return L;
}

// Buffers of on-the-fly replacement (slots r, starts l).
size_t otf_bytes(int64_t r, int64_t p, int64_t l) {
  size_t c = 0;
  carve(&c, sizeof(int32_t) * 3 * r);
  carve(&c, sizeof(int32_t) * 4);
  carve(&c, sizeof(double));
  carve(&c, sizeof(float) * p);
  carve(&c, sizeof(double) * 3 * l);
  carve(&c, sizeof(int32_t) * 3 * l);
  return c;
}

Otf carve_otf(char* base, int64_t r, int64_t p, int64_t l) {
  size_t c = 0;
  Otf o;
  int32_t* slots = (int32_t*)(base + carve(&c, sizeof(int32_t) * 3 * r));
  o.slot_start = slots;
  o.retiring = slots + r;
  o.refill = slots + 2 * r;
  o.ctl = (int32_t*)(base + carve(&c, sizeof(int32_t) * 4));
  o.best_f = (double*)(base + carve(&c, sizeof(double)));
  o.best_x = (float*)(base + carve(&c, sizeof(float) * p));
  double* d = (double*)(base + carve(&c, sizeof(double) * 3 * l));
  o.f = d;
  o.ev = d + l;
  o.phi = d + 2 * l;
  int32_t* q = (int32_t*)(base + carve(&c, sizeof(int32_t) * 3 * l));
  o.iters = q;
  o.status = q + l;
  o.nnz = q + 2 * l;
  o.x_all = nullptr;
  o.total = l;
  return o;
}

}  // namespace
}  // namespace spca

static int ensure_capture_stream(spca_ctx* ctx) {
  if (ctx->capture == nullptr)
    SPCA_HIP_TRY(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
  return SPCA_OK;
}

using namespace spca;

// Times `launch` for every compiled shape and every power-of-two split up to
// split_cap (3 runs after 1 warm-up, HIP events on the stream) and records
// the fastest in the tuning table under (M, N, K, max_splits).  Shapes whose
// rows would be mostly padding are skipped, as in the model.
template <typename F>
static int autotune_product(hipStream_t st, int64_t M, int64_t N, int64_t K,
                            int split_cap, int max_splits, int eb, F launch) {
  hipEvent_t e0, e1;
  SPCA_HIP_TRY(hipEventCreate(&e0));
  hipError_t ce = hipEventCreate(&e1);
  if (ce != hipSuccess) {
    (void)hipEventDestroy(e0);
    SPCA_HIP_TRY(ce);
  }
  GemmPlan best = model_plan_gemm_nt(M, N, K, max_splits, eb);
  float best_ms = 3.4e38f;
  hipError_t err = hipSuccess;
  const int cap = max_feasible_splits(K, split_cap, eb);
  for (int shape = 0; shape < gemm_num_shapes() && err == hipSuccess; ++shape) {
    const int bm = gemm_shape_bm(shape);
    if (bm > 32 && M <= bm / 2) continue;
    for (int splits = 1; splits <= cap && err == hipSuccess; splits *= 2) {
      const GemmPlan g{shape, splits};
      launch(g);
      err = hipEventRecord(e0, st);
      for (int k = 0; k < 3 && err == hipSuccess; ++k) launch(g);
      if (err == hipSuccess) err = hipEventRecord(e1, st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipGetLastError();
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err == hipSuccess && ms < best_ms) {
        best_ms = ms;
        best = g;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  SPCA_HIP_TRY(err);
  record_tuned_plan(M, N, K, max_splits, eb, best);
  return SPCA_OK;
}

// Components one after another: component c is solved on A deflated by the
// loadings 1 .. c - 1 (SOLVE: the dense or the sparse solve).
template <typename Prob, typename Solve>
static int components_loop(spca_ctx* ctx, void* stream, const Prob* prob,
                           const spca_solve_opts* opts, int32_t ncomp, double* X_out,
                           spca_result* res, Solve solve) {
  SPCA_REQUIRE(ctx && prob && opts && X_out && res,
               "ctx, prob, opts, X_out and res must not be NULL");
  SPCA_REQUIRE(ncomp >= 1 && ncomp <= kMaxDefl, "ncomp must be in 1..16");
  SPCA_REQUIRE(opts->deflate_X == nullptr && opts->deflate_k == 0,
               "deflate_X / deflate_k are set by the component loop");
  SPCA_REQUIRE(prob->p >= 1, "p must be >= 1");
  const int64_t p = prob->p;
  hipStream_t st = (hipStream_t)stream;
  double* Xd = nullptr;
  {
    DeviceGuard g(ctx->device);
    SPCA_HIP_TRY(hipMalloc(&Xd, sizeof(double) * (size_t)ncomp * p));
  }
  std::vector<int32_t> sup(p);
  int rc = SPCA_OK;
  for (int32_t c = 0; c < ncomp && rc == SPCA_OK; ++c) {
    spca_solve_opts o = *opts;
    o.deflate_X = c > 0 ? Xd : nullptr;
    o.deflate_k = c;
    spca_outputs out{};
    out.x = X_out + (int64_t)c * p;
    out.support = sup.data();
    out.res = &res[c];
    rc = solve(ctx, stream, prob, &o, &out);
    if (rc == SPCA_OK && c + 1 < ncomp) {
      DeviceGuard g(ctx->device);
      hipError_t e = hipMemcpyAsync(Xd + (int64_t)c * p, X_out + (int64_t)c * p,
                                    sizeof(double) * p, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        set_error(std::string("component loadings: ") + hipGetErrorString(e));
        rc = SPCA_EHIP;
      }
    }
  }
  {
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(st);
    (void)hipFree(Xd);
  }
  return rc;
}

int ensure_workspace(spca_ctx* ctx, hipStream_t st, size_t bytes) {
  if (ctx->budget != 0 && bytes > ctx->budget) {
    set_error("workspace of " + std::to_string(bytes) +
              " bytes exceeds the context budget of " +
              std::to_string(ctx->budget));
    return SPCA_ENOMEM;
  }
  if (bytes <= ctx->ws_cap) return SPCA_OK;
  if (ctx->ws_external) {
    set_error("workspace of " + std::to_string(bytes) +
              " bytes exceeds the caller-provided " + std::to_string(ctx->ws_cap));
    return SPCA_ENOMEM;
  }
  if (ctx->ws) {
    SPCA_HIP_TRY(hipStreamSynchronize(st));
    SPCA_HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
  }
  hipError_t e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes: " +
              hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SPCA_ENOMEM : SPCA_EHIP;
  }
  ctx->ws_cap = bytes;
  return SPCA_OK;
}

// The solve-wide warning from the final per-start statuses (spca_result
// .warning): all starts degenerate, all ended with x = 0, or (with the stop
// test on) none converged.
int32_t solve_warning(const std::vector<int32_t>& st, int64_t l, double tol) {
  int64_t deg = 0, zero = 0, conv = 0;
  for (int64_t j = 0; j < l; ++j) {
    deg += st[j] == SPCA_DEGENERATE;
    zero += st[j] == SPCA_ZERO;
    conv += st[j] == SPCA_CONVERGED;
  }
  if (l > 0 && deg == l) return SPCA_WARN_ALL_DEGENERATE;
  if (l > 0 && deg + zero == l) return SPCA_WARN_ALL_ZERO;
  if (tol >= 0.0 && conv == 0) return SPCA_WARN_NO_CONVERGED;
  return SPCA_WARN_NONE;
}

extern "C" {

const char* spca_last_error(void) { return spca::last_error(); }

// Workspace of one solve: its layout, and for BF16 storage the layout of the
// FP32 polish sub-solve of all r starts after it.
static size_t solve_bytes(const Layout& L, int64_t n, int64_t p, int64_t r) {
  size_t b = L.total;
  if (L.bf16) b = (size_t)round_up((int64_t)b, 256) + make_layout(n, p, r, true, false).total;
  return b;
}

size_t spca_workspace_bytes(int64_t n, int64_t p, int32_t r, int precision) {
  if (n < 1 || p < 1 || r < 1) return 0;
  const Layout L = make_layout(n, p, r, true, precision == SPCA_PREC_BF16_POLISH);
  return solve_bytes(L, n, p, r);
}

int spca_ctx_set_workspace(spca_ctx* ctx, void* dev_ptr, size_t bytes) {
  SPCA_REQUIRE(ctx != nullptr, "ctx must not be NULL");
  SPCA_REQUIRE((dev_ptr == nullptr) == (bytes == 0),
               "dev_ptr and bytes must be both set or both zero");
  SPCA_REQUIRE((uintptr_t)dev_ptr % 256 == 0, "dev_ptr must be 256-byte aligned");
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (ctx->ws && !ctx->ws_external) {
    DeviceGuard g(ctx->device);
    SPCA_HIP_TRY(hipDeviceSynchronize());
    SPCA_HIP_TRY(hipFree(ctx->ws));
  }
  ctx->ws = dev_ptr;
  ctx->ws_cap = bytes;
  ctx->ws_external = dev_ptr != nullptr;
  return SPCA_OK;
}

int spca_ctx_create(spca_ctx** ctx, int device, size_t hbm_budget_bytes) {
  SPCA_REQUIRE(ctx != nullptr, "ctx must not be NULL");
  int ndev = 0;
  SPCA_HIP_TRY(hipGetDeviceCount(&ndev));
  SPCA_REQUIRE(device >= 0 && device < ndev, "device ordinal out of range");
  spca_ctx* c = new spca_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  {
    DeviceGuard g(device);
    hipError_t e = hipHostMalloc((void**)&c->host_poll, sizeof(int32_t) * 4,
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
      set_error(std::string("hipHostMalloc: ") + hipGetErrorString(e));
      delete c;
      return SPCA_EHIP;
    }
  }
  *ctx = c;
  return SPCA_OK;
}

int spca_ctx_destroy(spca_ctx* ctx) {
  if (ctx == nullptr) return SPCA_OK;
  if (ctx->polish) spca_ctx_destroy(ctx->polish);
  {
    DeviceGuard g(ctx->device);
    if (ctx->ws && !ctx->ws_external) {
      (void)hipDeviceSynchronize();
      (void)hipFree(ctx->ws);
    }
    if (ctx->host_poll) (void)hipHostFree(ctx->host_poll);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    ctx->t_aty.destroy();
    ctx->t_xup.destroy();
    ctx->t_ax.destroy();
  }
  delete ctx;
  return SPCA_OK;
}


// a7 polish: FP32 AM of the same formulation on the caller's FP32 A,
// continued from the BF16-phase iterates, in two batched sub-solves with the
// same stop test:
//   1. every start, for at most kPolishRank iterations: BF16 rounding moves
//      each trajectory by up to about 1e-3 relative, enough to reorder the
//      starts' objectives, so the starts are ranked only after some FP32
//      iterations;
//   2. the kPolishKeep best starts of that ranking (FP64 objective), for the
//      remaining polish_maxit - kPolishRank iterations.
// Working on all of A lets a column that BF16 rounding moved across a
// selection threshold come back.  The sub-solves' results (per start and
// best) are the solve's results.
constexpr int kPolishRank = 4;   // FP32 iterations of every start
constexpr int kPolishKeep = 16;  // starts polished to the end


static int polish_subsolve(spca_ctx* ctx, hipStream_t st, const spca_problem* prob,
                           const spca_solve_opts* opts, const float* Xp, int32_t r,
                           int32_t maxit, size_t ws_off, spca_outputs* sub_out) {
  if (ctx->polish == nullptr) {
    int rc = spca_ctx_create(&ctx->polish, ctx->device, 0);
    if (rc != SPCA_OK) return rc;
  }
  // the sub-solve works in the tail of this solve's workspace
  {
    int rc = spca_ctx_set_workspace(ctx->polish, (char*)ctx->ws + ws_off,
                                    ctx->ws_cap - ws_off);
    if (rc != SPCA_OK) return rc;
  }
  spca_problem sub = *prob;
  spca_solve_opts so{Xp, r, opts->tol, maxit, SPCA_PREC_FP32, 0, opts->check_every,
                     opts->flags & ~SPCA_FLAG_TIME_SAMPLED};
  return spca_am_solve_ex(ctx->polish, st, &sub, &so, sub_out);
}

int spca_am_solve_ex(spca_ctx* ctx, void* stream, const spca_problem* prob,
                     const spca_solve_opts* opts, spca_outputs* out) {
  SPCA_REQUIRE(ctx && prob && opts && out && out->res,
               "ctx, prob, opts, out and out->res must not be NULL");
  SPCA_REQUIRE(prob->A != nullptr, "A must not be NULL");
  const int64_t n = prob->n, p = prob->p, lda = prob->lda;
  const int fid = prob->formulation;
  const double sg = prob->s_or_gamma;
  const int64_t r = opts->r;
  int rc = check_problem(n, p, lda, fid, sg, r, opts->tol, opts->maxit);
  if (rc != SPCA_OK) return rc;
  SPCA_REQUIRE(opts->X0 != nullptr || r == 1,
               "X0 may be NULL only with r == 1 (start e_i at the largest column)");
  SPCA_REQUIRE(opts->precision == SPCA_PREC_FP32 ||
                   opts->precision == SPCA_PREC_BF16_POLISH,
               "precision must be SPCA_PREC_FP32 or SPCA_PREC_BF16_POLISH");
  SPCA_REQUIRE(opts->polish_maxit >= 0, "polish_maxit must be >= 0");
  SPCA_REQUIRE(opts->check_every >= 1, "check_every must be >= 1");
  const bool bf16 = opts->precision == SPCA_PREC_BF16_POLISH;
  SPCA_REQUIRE(opts->total_starts >= 0, "total_starts must be >= 0");
  const int64_t l = opts->total_starts > r ? opts->total_starts : r;
  const bool otf = l > r;
  SPCA_REQUIRE(opts->warmup_iters >= 0, "warmup_iters must be >= 0");
  const bool warm = opts->warmup_iters > 0;
  if (warm) {
    SPCA_REQUIRE(fid >= 3, "the warm-up applies to formulations 3..8");
    SPCA_REQUIRE(!bf16 && !otf, "the warm-up runs in FP32 without total_starts > r");
    if (fid >= 5)
      SPCA_REQUIRE(opts->target_nnz >= 1 && opts->target_nnz <= p,
                   "target_nnz must be in 1..p for the penalty warm-up");
  }
  SPCA_REQUIRE(opts->deflate_k >= 0 && opts->deflate_k <= kMaxDefl,
               "deflate_k must be in 0..16");
  const int dk = opts->deflate_k;
  if (dk > 0) {
    SPCA_REQUIRE(opts->deflate_X != nullptr, "deflate_X must be set when deflate_k > 0");
    SPCA_REQUIRE(!bf16 && !otf, "deflation runs in FP32 without total_starts > r");
  }
  if (otf) {
    SPCA_REQUIRE(!bf16, "on-the-fly replacement runs in FP32 only");
    SPCA_REQUIRE(opts->X0 != nullptr, "on-the-fly replacement needs X0 (total_starts rows)");
  }

  std::lock_guard<std::mutex> lock(ctx->mu);
  DeviceGuard g(ctx->device);
  hipStream_t st = (hipStream_t)stream;

  const bool copy_a = (lda % 4) != 0 || ((uintptr_t)prob->A % 16) != 0;
  Layout L = make_layout(n, p, r, copy_a, bf16);
  const size_t otf_off = (size_t)round_up((int64_t)solve_bytes(L, n, p, r), 256);
  rc = ensure_workspace(ctx, st, otf ? otf_off + otf_bytes(r, p, l)
                                : otf_off + deflate_bytes(n, p, r, dk));
  if (rc != SPCA_OK) return rc;
  char* base = (char*)ctx->ws;
  float* At = (float*)(base + L.off_At);
  float* X = (float*)(base + L.off_X);
  float* U = (float*)(base + L.off_U);
  float* Y = (float*)(base + L.off_Y);
  float* V = (float*)(base + L.off_V);
  int32_t* li = (int32_t*)(base + L.off_li);
  float* lv = (float*)(base + L.off_lv);
  Plan* plan = (Plan*)(base + L.off_plan);
  StartState s{(double*)(base + L.off_phi), (double*)(base + L.off_phip),
               (int32_t*)(base + L.off_nnz), (int32_t*)(base + L.off_it),
               (int32_t*)(base + L.off_st), (float*)(base + L.off_thr),
               (int32_t*)(base + L.off_redo)};
  double* partial = (double*)(base + L.off_part);
  double* fj = (double*)(base + L.off_f);
  double* evj = (double*)(base + L.off_ev);
  double* xnorm = (double*)(base + L.off_xn);
  int32_t* best = (int32_t*)(base + L.off_best);
  double* xout = (double*)(base + L.off_xout);
  int32_t* sup = (int32_t*)(base + L.off_sup);
  double* colsq = (double*)(base + L.off_colsq);
  int32_t* bad = (int32_t*)(base + L.off_bad);
  int32_t* colmark = (int32_t*)(base + L.off_mark);
  int32_t* ulist = (int32_t*)(base + L.off_ulist);
  float* Xc = (float*)(base + L.off_Xc);
  float* Qc = (float*)(base + L.off_Qc);
  const int64_t ldc_u = round_up(L.ucap, 4);
  uint16_t* Ab = (uint16_t*)(base + L.off_Ab);
  uint16_t* Atb = (uint16_t*)(base + L.off_Atb);
  uint16_t* Yb = (uint16_t*)(base + L.off_Yb);
  uint16_t* Xb = (uint16_t*)(base + L.off_Xb);
  void* wide = L.wide_bytes ? (void*)(base + L.off_wide) : nullptr;
  Otf o{};
  if (otf) {
    o = carve_otf(base + otf_off, r, p, l);
    o.x_all = out->X_final;  // l x p, filed as each start finishes
  }
  Defl defl{};
  if (dk > 0) defl = carve_deflate(base + otf_off, n, p, r, dk);
  double* gam = (double*)(base + L.off_gam);
  Warm wm;
  if (warm) {
    wm.K = opts->warmup_iters;
    wm.target = fid >= 5 ? opts->target_nnz : 0;
    wm.gam = gam;
  }

  // a0: stage A (aligned column-major copy only when needed) and its
  // row-major twin used by the dense A x.
  const float* A = prob->A;
  int64_t ldA = lda;
  if (copy_a) {
    float* Ac = (float*)(base + L.off_Ac);
    copy_columns_f32(st, prob->A, lda, Ac, L.ldac, n, p);
    A = Ac;
    ldA = L.ldac;
  }
  if (opts->flags & SPCA_FLAG_CHECK_FINITE) {
    SPCA_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
    count_nonfinite(st, A, ldA, n, p, bad);
    SPCA_HIP_TRY(hipMemcpyAsync(ctx->host_poll, bad, sizeof(int32_t),
                                hipMemcpyDeviceToHost, st));
    SPCA_HIP_TRY(hipStreamSynchronize(st));
    SPCA_REQUIRE(ctx->host_poll[0] == 0, "A holds NaN or Inf entries");
  }
  if (bf16) {
    // a7: A in BF16, column-major (for A^T Y) and row-major (for A X)
    to_bf16_colmajor(st, A, ldA, n, p, Ab, L.ldab);
    to_bf16_rowmajor(st, A, ldA, n, p, Atb, L.ldatb);
  } else {
    transpose_f32(st, A, ldA, At, L.ldat, n, p);
  }
  SPCA_LAUNCH_CHECK("layout copies of A");
  if (dk > 0) {
    deflate_setup(st, opts->deflate_X, A, ldA, n, p, defl);
    SPCA_LAUNCH_CHECK("deflation setup");
  }

  // starting points
  if (opts->X0 != nullptr) {
    SPCA_HIP_TRY(hipMemcpy2DAsync(X, sizeof(float) * L.ldx, opts->X0,
                                  sizeof(float) * p, sizeof(float) * p, r,
                                  hipMemcpyDeviceToDevice, st));
  } else {
    max_norm_column_start(st, A, ldA, n, p, colsq, X, L.ldx);
  }
  if (opts->flags & SPCA_FLAG_AUTOTUNE) {
    // a8: measure every tile shape and split on this solve's own operands
    // for the products that have no entry in the tuning table yet.  Y holds
    // the leading entries of the starts (zero beyond p): with Y = 0 the chip
    // draws less power and clocks higher than on real operands (2.4 against
    // 1.9 GHz for the 16 GB instance's A^T Y), which would time every plan
    // too fast.
    SPCA_HIP_TRY(hipMemsetAsync(Y, 0, sizeof(float) * r * L.ldu, st));
    SPCA_HIP_TRY(hipMemcpy2DAsync(Y, sizeof(float) * L.ldu, X, sizeof(float) * L.ldx,
                                  sizeof(float) * (size_t)(n < p ? n : p), r,
                                  hipMemcpyDeviceToDevice, st));
    if (bf16) rows_to_bf16(st, Y, L.ldu, r, n, Yb, L.ldyb, nullptr);
    const int eb = bf16 ? 2 : 4;
    GemmPlan tmp;
    if (!tuned_plan(r, n, p, kMaxSplits, eb, &tmp)) {
      if (bf16) rows_to_bf16(st, X, L.ldx, r, p, Xb, L.ldxb, nullptr);
      auto run_ax = [&](GemmPlan g) {
        if (bf16)
          gemm_nt_bf16(st, Xb, L.ldxb, Atb, L.ldatb, U, L.ldu, r, n, p, nullptr, 0, g,
                       r * L.ldu);
        else
          gemm_nt_f32(st, X, L.ldx, At, L.ldat, U, L.ldu, r, n, p, nullptr, 0, g,
                      r * L.ldu);
      };
      rc = autotune_product(st, r, n, p, L.ax_split_cap, kMaxSplits, eb, run_ax);
      if (rc != SPCA_OK) return rc;
    }
    if (!tuned_plan(r, p, n, kMaxSplits, eb, &tmp)) {
      auto run_aty = [&](GemmPlan g) {
        if (bf16)
          gemm_nt_bf16(st, Yb, L.ldyb, Ab, L.ldab, V, L.ldx, r, p, n, nullptr, 0, g,
                       r * L.ldx);
        else
          gemm_nt_f32(st, Y, L.ldu, A, ldA, V, L.ldx, r, p, n, nullptr, 0, g, r * L.ldx);
      };
      rc = autotune_product(st, r, p, n, L.aty_split_cap, kMaxSplits, eb, run_aty);
      if (rc != SPCA_OK) return rc;
    }
    L.plan_ax = plan_gemm_nt(r, n, p, kMaxSplits, eb);
    L.plan_aty = plan_gemm_nt(r, p, n, kMaxSplits, eb);
  }
  init_state(st, s, r);
  if (otf) otf_init(st, o, r);
  init_plan(st, plan, L.plan_ax.splits);
  if (wide) SPCA_HIP_TRY(x_update_wide_reset(st, wide, r));
  SPCA_HIP_TRY(hipMemsetAsync(colmark, 0, sizeof(int32_t) * p, st));
  compact_rows(st, X, L.ldx, r, p, li, lv, L.ldx, s.nnz, s.status, colmark, plan);
  const int dense_only = (opts->flags & SPCA_FLAG_DENSE_ONLY) ? 1 : 0;
  // the union product is offered only when allowed and while the union
  // fits its buffers (at most ucap columns)
  const int64_t ucap_eff = (opts->flags & SPCA_FLAG_NO_UNION) ? 0 : L.ucap;
  const int list_cap = list_cap_of(p);
  // union_on: the union gather and product are launched and the planner may
  // pick them.  At each poll the host keeps them while the planner reports
  // the union product picked or within 1.25x of the best product at its latest
  // probe, and drops them otherwise (never while the plan of the next
  // iteration is the union product); the probes go on, so a union that
  // becomes cheap brings them back at the next poll.
  bool union_on = ucap_eff > 0;
  auto plan_iter = [&]() {
    plan_next(st, s, r, n, p, list_cap, dense_only, L.plan_ax.splits, ucap_eff,
              colmark, ulist, plan, dk > 0 ? 1 : 0, union_on ? 1 : 0);
  };
  plan_iter();
  if (bf16) rows_to_bf16(st, X, L.ldx, r, p, Xb, L.ldxb, plan);
  SPCA_LAUNCH_CHECK("staging");

  const int32_t maxit = opts->maxit;
  const bool timed = out->kernel_times != nullptr;
  const bool sampled = (opts->flags & SPCA_FLAG_TIME_SAMPLED) != 0;
  ctx->t_aty.reset();
  ctx->t_xup.reset();
  ctx->t_ax.reset();
  // One AM iteration (Algorithm 2, one pass of its loop), enqueued on `q`.
  // Every launch reads its control data (mode, active starts, sizes) from
  // the device-side plan, so the same sequence serves every iteration and
  // can be captured once into a graph.
  auto iteration = [&](hipStream_t q, bool tm) -> int {
    // u = A x and the y-update
    if (tm) SPCA_HIP_TRY(ctx->t_ax.mark(q));
    if (bf16)
      gemm_nt_bf16(q, Xb, L.ldxb, Atb, L.ldatb, U, L.ldu, r, n, p, &plan->mode,
                   kAxDense, L.plan_ax, r * L.ldu);
    else
      gemm_nt_f32(q, X, L.ldx, At, L.ldat, U, L.ldu, r, n, p, &plan->mode,
                  kAxDense, L.plan_ax, r * L.ldu);
    if (tm) SPCA_HIP_TRY(ctx->t_ax.mark(q));
    if (!bf16 && union_on) {  // the planner can pick the union product
      union_gather(q, X, L.ldx, r, A, ldA, n, ulist, plan, Xc, ldc_u, Qc, ldc_u);
      gemm_nt_f32(q, Xc, ldc_u, Qc, ldc_u, U, L.ldu, r, n, L.ucap, &plan->mode,
                  kAxUnion, L.plan_union, 0, &plan->union_size);
    }
    if (!rows_product_possible(n, dk > 0 ? 1 : 0)) {
      // the planner never picks the row-block product here
    } else if (bf16) {
      sparse_ax_rows_bf16(q, Ab, L.ldab, n, li, lv, L.ldx, U, L.ldu, r, s, plan);
    } else {
      sparse_ax_rows(q, A, ldA, n, li, lv, L.ldx, U, L.ldu, r, s, plan);
    }
    if (dk > 0) deflate_u(q, X, L.ldx, p, U, L.ldu, n, r, s, plan, defl);
    y_update(q, fid, U, r * L.ldu, Y, L.ldu, r, n, s, plan, bf16 ? Yb : nullptr,
             L.ldyb);
    if (bf16)
      sparse_ax_y_update_bf16(q, fid, Ab, L.ldab, n, li, lv, L.ldx, Y, L.ldu, Yb,
                              L.ldyb, r, s, plan);
    else
      sparse_ax_y_update(q, fid, A, ldA, n, li, lv, L.ldx, Y, L.ldu, r, s, plan);
    // v = A^T y and the x-update with the stop test
    if (tm) SPCA_HIP_TRY(ctx->t_aty.mark(q));
    if (bf16)
      gemm_nt_bf16(q, Yb, L.ldyb, Ab, L.ldab, V, L.ldx, r, p, n, nullptr, 0,
                   L.plan_aty, r * L.ldx);
    else
      gemm_nt_f32(q, Y, L.ldu, A, ldA, V, L.ldx, r, p, n, nullptr, 0,
                  L.plan_aty, r * L.ldx);
    sum_splits(q, V, r * L.ldx, L.plan_aty.splits, r * L.ldx);
    if (tm) SPCA_HIP_TRY(ctx->t_aty.mark(q));
    if (dk > 0) deflate_v(q, V, L.ldx, p, r, s, defl);
    if (tm) SPCA_HIP_TRY(ctx->t_xup.mark(q));
    x_update(q, fid, sg, V, L.ldx, r, p, X, L.ldx, li, lv, L.ldx, list_cap, s,
             opts->tol, maxit, colmark, plan, wide, wm);
    if (tm) SPCA_HIP_TRY(ctx->t_xup.mark(q));
    if (otf)
      otf_step(q, fid, sg, A, ldA, n, p, X, L.ldx, opts->X0, li, lv, L.ldx, s, r,
               partial, fj, evj, xnorm, o, 0);
    plan_next(q, s, r, n, p, list_cap, dense_only, L.plan_ax.splits, ucap_eff,
              colmark, ulist, plan, dk > 0 ? 1 : 0, union_on ? 1 : 0);
    if (bf16) rows_to_bf16(q, X, L.ldx, r, p, Xb, L.ldxb, plan);
    SPCA_LAUNCH_CHECK("AM iteration");
    return SPCA_OK;
  };
  // the host reads the number of active starts after every check_every
  // iterations and stops once none is left
  // (and updates union_on from the plan's mode and union evidence)
  auto none_active = [&](bool* done) -> int {
    static_assert(offsetof(Plan, active) == 4 && offsetof(Plan, union_close) == 8,
                  "mode, active and union_close lead the plan");
    SPCA_HIP_TRY(hipMemcpyAsync(ctx->host_poll, plan, 3 * sizeof(int32_t),
                                hipMemcpyDeviceToHost, st));
    SPCA_HIP_TRY(hipStreamSynchronize(st));
    *done = ctx->host_poll[1] == 0;
    if (ucap_eff > 0) {
      if (union_on && ctx->host_poll[2] == 0 && ctx->host_poll[0] != kAxUnion)
        union_on = false;
      else if (!union_on && ctx->host_poll[2] != 0)
        union_on = true;
    }
    return SPCA_OK;
  };
  const int32_t every = opts->check_every;
  // with replacement every slot runs its starts back to back, and all slots
  // stay busy while starts remain, so maxit (l / r + 1) iterations suffice
  const int64_t loop_max64 = otf ? (int64_t)maxit * (ceil_div(l, r) + 1) : maxit;
  const int32_t loop_max = loop_max64 > INT32_MAX ? INT32_MAX : (int32_t)loop_max64;
  int32_t it = 0;
  bool done = false;
  if ((opts->flags & SPCA_FLAG_GRAPH) && !timed && loop_max >= every) {
    // a8: capture check_every iterations once (on the context's own stream,
    // since the legacy default stream cannot be captured) and replay the
    // graph on the caller's stream.  The captured sequence holds kernel
    // launches only.
    rc = ensure_capture_stream(ctx);
    if (rc != SPCA_OK) return rc;
    // one graph per union_on state, captured when first needed
    hipGraphExec_t execs[2] = {nullptr, nullptr};
    auto capture = [&](hipGraphExec_t* exec) -> int {
      hipGraph_t graph = nullptr;
      SPCA_HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
      int body_rc = SPCA_OK;
      for (int32_t k = 0; k < every && body_rc == SPCA_OK; ++k)
        body_rc = iteration(ctx->capture, false);
      hipError_t end_rc = hipStreamEndCapture(ctx->capture, &graph);
      if (body_rc != SPCA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return body_rc;
      }
      SPCA_HIP_TRY(end_rc);
      hipError_t inst_rc = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      SPCA_HIP_TRY(inst_rc);
      return SPCA_OK;
    };
    int loop_rc = SPCA_OK;
    while (!done && it + every <= loop_max) {
      hipGraphExec_t& exec = execs[union_on ? 1 : 0];
      if (exec == nullptr) {
        loop_rc = capture(&exec);
        if (loop_rc != SPCA_OK) break;
      }
      hipError_t e = hipGraphLaunch(exec, st);
      if (e != hipSuccess) {
        set_error(std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        loop_rc = SPCA_EHIP;
        break;
      }
      it += every;
      if (it < loop_max) {
        loop_rc = none_active(&done);
        if (loop_rc != SPCA_OK) break;
      }
    }
    for (hipGraphExec_t e : execs)
      if (e != nullptr) (void)hipGraphExecDestroy(e);
    if (loop_rc != SPCA_OK) return loop_rc;
  }
  for (; !done && it < loop_max; ++it) {
    rc = iteration(st, timed && (!sampled || it % kTimeSample == 0));
    if (rc != SPCA_OK) return rc;
    if ((it + 1) % every == 0 && it + 1 < loop_max) {
      rc = none_active(&done);
      if (rc != SPCA_OK) return rc;
    }
  }

  // a6: FP64 objective, explained variance, best start, output vector; the
  // lists are rebuilt from the final dense iterates (dense starts keep none)
  if (otf) {
    // close what is still running, then the best start's vector
    otf_step(st, fid, sg, A, ldA, n, p, X, L.ldx, opts->X0, li, lv, L.ldx, s, r,
             partial, fj, evj, xnorm, o, 1);
    otf_output(st, o, p, best, xout, sup);
  }
  // the FP64 product of the evaluation may split its columns over the
  // V buffer, free once the loop is done
  double* upart = (double*)(base + L.off_V);
  // BF16 + polish: the polish re-evaluates every start after its FP32
  // iterations, so the BF16 phase's own result is needed for one start only
  // (objective_pre_polish): the one with the largest in-loop objective phi
  int32_t pre_best = -1;
  if (!otf) {
    compact_rows(st, X, L.ldx, r, p, li, lv, L.ldx, s.nnz, nullptr, nullptr, nullptr);
    // under the penalty warm-up every start has its own gamma: f uses it,
    // and the best start is the one with the largest explained variance
    const bool per_start_gamma = warm && fid >= 5;
    if (dk > 0) deflate_final_alpha(st, X, L.ldx, p, r, defl);
    std::vector<int32_t> nnz_h(r), st_h(r);
    std::vector<double> phi_h(r);
    SPCA_HIP_TRY(hipMemcpyAsync(nnz_h.data(), s.nnz, sizeof(int32_t) * r,
                                hipMemcpyDeviceToHost, st));
    SPCA_HIP_TRY(hipMemcpyAsync(st_h.data(), s.status, sizeof(int32_t) * r,
                                hipMemcpyDeviceToHost, st));
    SPCA_HIP_TRY(hipMemcpyAsync(phi_h.data(), s.phi, sizeof(double) * r,
                                hipMemcpyDeviceToHost, st));
    SPCA_HIP_TRY(hipStreamSynchronize(st));
    if (bf16 && opts->polish_maxit > 0) {
      for (int64_t j = 0; j < r; ++j) {
        const bool live = st_h[j] != SPCA_DEGENERATE && st_h[j] != SPCA_ZERO && nnz_h[j] > 0;
        if (live && (pre_best < 0 || phi_h[j] > phi_h[pre_best])) pre_best = (int32_t)j;
      }
    }
    if (pre_best >= 0) {
      const int64_t jp = pre_best;
      StartState s1{s.phi + jp, s.phi_prev + jp, s.nnz + jp, s.iters + jp, s.status + jp,
                    s.thr + jp, s.redo + jp};
      const bool dense1 = (double)nnz_h[jp] * 4.0 >= (double)p;
      finalize(st, fid, sg, A, ldA, n, p, li + jp * L.ldx, lv + jp * L.ldx, L.ldx, s1, 1,
               partial, fj + jp, evj + jp, xnorm, best, xout, sup, nullptr, false, defl,
               dense1 ? X + jp * L.ldx : nullptr, L.ldx, upart);
    } else {
      // mostly dense iterates (a quarter of all entries or more): one FP64
      // product on the matrix cores instead of per-start sums over the lists
      double tot_nnz = 0.0;
      for (int64_t j = 0; j < r; ++j) tot_nnz += nnz_h[j];
      const bool dense_eval = r >= 16 && tot_nnz * 4.0 >= (double)r * (double)p;
      finalize(st, fid, sg, A, ldA, n, p, li, lv, L.ldx, s, r, partial, fj, evj,
               xnorm, best, xout, sup, per_start_gamma ? gam : nullptr, per_start_gamma,
               defl, dense_eval ? X : nullptr, L.ldx, upart);
    }
  }
  SPCA_LAUNCH_CHECK("finalize");

  int32_t hb[2];
  Plan hplan;
  SPCA_HIP_TRY(hipMemcpyAsync(hb, best, sizeof(hb), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(&hplan, plan, sizeof(Plan), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  const int32_t jb = pre_best >= 0 ? pre_best : hb[0], nnzb = hb[1];
  // per-start results: the slots themselves, or with replacement the
  // records of all l starts
  std::vector<double> f_all(l), ev_all(l), phi_all(l);
  std::vector<int32_t> it_all(l), st_all(l), nnz_all(l);
  SPCA_HIP_TRY(hipMemcpyAsync(f_all.data(), otf ? o.f : fj, sizeof(double) * l,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(ev_all.data(), otf ? o.ev : evj, sizeof(double) * l,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(phi_all.data(), otf ? o.phi : s.phi, sizeof(double) * l,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(it_all.data(), otf ? o.iters : s.iters,
                              sizeof(int32_t) * l, hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(st_all.data(), otf ? o.status : s.status,
                              sizeof(int32_t) * l, hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(nnz_all.data(), otf ? o.nnz : s.nnz,
                              sizeof(int32_t) * l, hipMemcpyDeviceToHost, st));
  if (out->x)
    SPCA_HIP_TRY(hipMemcpyAsync(out->x, xout, sizeof(double) * p,
                                hipMemcpyDeviceToHost, st));
  if (out->support && nnzb > 0)
    SPCA_HIP_TRY(hipMemcpyAsync(out->support, sup, sizeof(int32_t) * nnzb,
                                hipMemcpyDeviceToHost, st));
  if (out->param_per_start && warm)
    SPCA_HIP_TRY(hipMemcpyAsync(out->param_per_start, gam, sizeof(double) * r,
                                hipMemcpyDeviceToHost, st));
  if (out->X_final && !otf)
    SPCA_HIP_TRY(hipMemcpy2DAsync(out->X_final, sizeof(float) * p, X,
                                  sizeof(float) * L.ldx, sizeof(float) * p, r,
                                  hipMemcpyDeviceToDevice, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));

  if (timed) {
    double* kt = out->kernel_times;
    SPCA_HIP_TRY(ctx->t_aty.total_ms(&kt[0]));
    kt[1] = (double)(ctx->t_aty.used / 2);
    SPCA_HIP_TRY(ctx->t_xup.total_ms(&kt[2]));
    kt[3] = (double)(ctx->t_xup.used / 2);
    SPCA_HIP_TRY(ctx->t_ax.total_ms(&kt[4]));
    kt[5] = (double)(ctx->t_ax.used / 2);
    kt[6] = hplan.mode_count[kAxDense];
    kt[7] = hplan.mode_count[kAxList];
    kt[8] = hplan.mode_count[kAxUnion];
    kt[7] += hplan.mode_count[kAxListRows];
    kt[9] = hplan.mode_count[kAxListRows];
    kt[10] = hplan.active_sum;
    kt[11] = hplan.nnz_sum;
  }
  double total_iters = 0.0;
  for (int64_t j = 0; j < l; ++j) total_iters += it_all[j];
  spca_result* res = out->res;
  res->objective = f_all[jb];
  res->objective_pre_polish = f_all[jb];
  res->polish_iters = 0;
  res->explained_var = ev_all[jb];
  res->phi = phi_all[jb];
  res->iters_x_starts = total_iters;
  res->best_start = jb;
  res->nnz = nnzb;
  res->iters = it_all[jb];
  res->status = st_all[jb];
  if (bf16 && opts->polish_maxit > 0 && nnzb > 0) {
    // 1. every start, kPolishRank FP32 iterations from its BF16-phase iterate
    float* Xp = (float*)(base + L.off_Xp);
    SPCA_HIP_TRY(hipMemcpy2DAsync(Xp, sizeof(float) * p, X, sizeof(float) * L.ldx,
                                  sizeof(float) * p, r, hipMemcpyDeviceToDevice, st));
    const size_t ws_off = (size_t)round_up((int64_t)L.total, 256);
    const int32_t m1 = opts->polish_maxit < kPolishRank ? opts->polish_maxit : kPolishRank;
    std::vector<double> pf(r), pev(r), pphi(r), xa(p);
    std::vector<int32_t> pit(r), pst(r), pnnz(r), sa(p);
    spca_result r1{};
    spca_outputs so{};
    so.x = xa.data();
    so.support = sa.data();
    so.res = &r1;
    so.f_per_start = pf.data();
    so.ev_per_start = pev.data();
    so.phi_per_start = pphi.data();
    so.iters_per_start = pit.data();
    so.status_per_start = pst.data();
    so.nnz_per_start = pnnz.data();
    so.X_final = Xp;  // the ranked iterates, read again by the second sub-solve
    // the context lock is held, so the workspace stays valid meanwhile
    rc = polish_subsolve(ctx, st, prob, opts, Xp, (int32_t)r, m1, ws_off, &so);
    if (rc != SPCA_OK) return rc;
    std::vector<int32_t> polish_it(r);
    for (int64_t j = 0; j < r; ++j) {
      f_all[j] = pf[j];
      ev_all[j] = pev[j];
      phi_all[j] = pphi[j];
      polish_it[j] = pit[j];
      st_all[j] = pst[j];
      nnz_all[j] = pnnz[j];
    }
    double polish_work = r1.iters_x_starts;
    // 2. the kPolishKeep best still-running starts of that ranking, to the end
    std::vector<int32_t> keep;
    if (opts->polish_maxit > m1) {
      for (int64_t j = 0; j < r; ++j)
        if (pst[j] == SPCA_MAXIT && pnnz[j] > 0) keep.push_back((int32_t)j);
      std::stable_sort(keep.begin(), keep.end(),
                       [&](int32_t a, int32_t b) { return pf[a] > pf[b]; });
      if ((int)keep.size() > kPolishKeep) keep.resize(kPolishKeep);
      std::sort(keep.begin(), keep.end());
    }
    // the result: stage 1's best, unless stage 2 improves on it
    int32_t jbest = r1.best_start;
    spca_result rb = r1;
    const double* xbest = xa.data();
    const int32_t* sbest = sa.data();
    bool best_kept = false;
    for (int32_t k : keep) best_kept = best_kept || k == jbest;
    std::vector<double> xb(keep.empty() ? 0 : p);
    std::vector<int32_t> sb(keep.empty() ? 0 : p);
    if (!keep.empty()) {
      // gather the kept rows to the front of Xp (ascending indices, so no
      // source row is overwritten before it is read)
      for (size_t c = 0; c < keep.size(); ++c)
        if ((int32_t)c != keep[c])
          SPCA_HIP_TRY(hipMemcpyAsync(Xp + c * p, Xp + (int64_t)keep[c] * p,
                                      sizeof(float) * p, hipMemcpyDeviceToDevice, st));
      const int32_t mk = (int32_t)keep.size();
      std::vector<double> qf(mk), qev(mk), qphi(mk);
      std::vector<int32_t> qit(mk), qst(mk), qnnz(mk);
      spca_result r2{};
      spca_outputs o2{};
      o2.x = xb.data();
      o2.support = sb.data();
      o2.res = &r2;
      o2.f_per_start = qf.data();
      o2.ev_per_start = qev.data();
      o2.phi_per_start = qphi.data();
      o2.iters_per_start = qit.data();
      o2.status_per_start = qst.data();
      o2.nnz_per_start = qnnz.data();
      rc = polish_subsolve(ctx, st, prob, opts, Xp, mk, opts->polish_maxit - m1, ws_off, &o2);
      if (rc != SPCA_OK) return rc;
      for (int32_t c = 0; c < mk; ++c) {
        const int32_t j = keep[c];
        f_all[j] = qf[c];
        ev_all[j] = qev[c];
        phi_all[j] = qphi[c];
        polish_it[j] += qit[c];
        st_all[j] = qst[c];
        nnz_all[j] = qnnz[c];
      }
      polish_work += r2.iters_x_starts;
      const int32_t jb2 = keep[r2.best_start];
      // stage 1's best stands only if it was not continued and is not
      // beaten (ties to the lower start index)
      if (best_kept || r2.objective > rb.objective ||
          (r2.objective == rb.objective && jb2 < jbest)) {
        jbest = jb2;
        rb = r2;
        xbest = xb.data();
        sbest = sb.data();
      }
    }
    res->objective = rb.objective;
    res->explained_var = rb.explained_var;
    res->phi = rb.phi;
    res->iters_x_starts = total_iters + polish_work;
    res->best_start = jbest;
    res->nnz = rb.nnz;
    res->iters = it_all[jbest] + polish_it[jbest];
    res->status = rb.status;
    res->polish_iters = polish_it[jbest];
    for (int64_t j = 0; j < r; ++j) it_all[j] += polish_it[j];
    if (out->x) std::copy(xbest, xbest + p, out->x);
    if (out->support) std::copy(sbest, sbest + rb.nnz, out->support);
  }
  for (int64_t j = 0; j < l; ++j) {
    if (out->f_per_start) out->f_per_start[j] = f_all[j];
    if (out->ev_per_start) out->ev_per_start[j] = ev_all[j];
    if (out->phi_per_start) out->phi_per_start[j] = phi_all[j];
    if (out->iters_per_start) out->iters_per_start[j] = it_all[j];
    if (out->status_per_start) out->status_per_start[j] = st_all[j];
    if (out->nnz_per_start) out->nnz_per_start[j] = nnz_all[j];
  }
  out->res->warning = solve_warning(st_all, l, opts->tol);
  return SPCA_OK;
}

int spca_am_solve_sparse(spca_ctx* ctx, void* stream, const spca_sparse_problem* prob,
                         const spca_solve_opts* opts, spca_outputs* out) {
  SPCA_REQUIRE(ctx && prob && opts && out && out->res,
               "ctx, prob, opts, out and out->res must not be NULL");
  const int64_t n = prob->n, p = prob->p, r = opts->r;
  const int fid = prob->formulation;
  const double sg = prob->s_or_gamma;
  int rc = check_problem(n, p, n, fid, sg, r, opts->tol, opts->maxit);
  if (rc != SPCA_OK) return rc;
  SPCA_REQUIRE(prob->col_ptr && prob->row_idx && prob->col_val && prob->row_ptr &&
                   prob->col_idx && prob->row_val,
               "every array of the sparse matrix must be set");
  SPCA_REQUIRE(((uintptr_t)prob->row_idx | (uintptr_t)prob->col_val | (uintptr_t)prob->col_idx |
                (uintptr_t)prob->row_val | (uintptr_t)prob->col_ptr |
                (uintptr_t)prob->row_ptr) % 16 == 0,
               "the arrays of the sparse matrix must be 16-byte aligned");
  SPCA_REQUIRE(opts->X0 != nullptr, "the sparse solve needs X0");
  SPCA_REQUIRE(opts->precision == SPCA_PREC_FP32, "the sparse solve runs in FP32");
  SPCA_REQUIRE(opts->total_starts <= r, "the sparse solve takes no total_starts > r");
  SPCA_REQUIRE(opts->deflate_k >= 0 && opts->deflate_k <= kMaxDefl,
               "deflate_k must be in 0..16");
  const int dk = opts->deflate_k;
  SPCA_REQUIRE(dk == 0 || opts->deflate_X != nullptr,
               "deflate_X must be set when deflate_k > 0");
  SPCA_REQUIRE(opts->check_every >= 1, "check_every must be >= 1");
  SPCA_REQUIRE(opts->warmup_iters >= 0, "warmup_iters must be >= 0");
  const bool warm = opts->warmup_iters > 0;
  if (warm) {
    SPCA_REQUIRE(fid >= 3, "the warm-up applies to formulations 3..8");
    if (fid >= 5)
      SPCA_REQUIRE(opts->target_nnz >= 1 && opts->target_nnz <= p,
                   "target_nnz must be in 1..p for the penalty warm-up");
  }
  std::lock_guard<std::mutex> lock(ctx->mu);
  DeviceGuard g(ctx->device);
  hipStream_t st = (hipStream_t)stream;

  // nnz from the two pointer arrays (their first entries must be 0 and
  // their last ones equal)
  int64_t ends[4];
  SPCA_HIP_TRY(hipMemcpyAsync(&ends[0], prob->col_ptr, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(&ends[1], prob->col_ptr + p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(&ends[2], prob->row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(&ends[3], prob->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  SPCA_REQUIRE(ends[0] == 0 && ends[2] == 0 && ends[1] == ends[3] && ends[1] >= 0,
               "col_ptr and row_ptr must start at 0 and end at the same nnz");
  const int64_t nnz = ends[1];

  // workspace: the iterates of the dense path, the transposed operands and
  // products, the chunk tables and partials of the balanced products, and
  // the partials of the final evaluation
  const int64_t ldx = round_up(p, 4), ldu = round_up(n, 4), ldt = sparse_ld(r);
  const int64_t nch = sparse_chunks(nnz), nfin = sparse_final_parts(n);
  const int force = (opts->flags & SPCA_FLAG_SPARSE_PANELS)      ? 1
                    : (opts->flags & SPCA_FLAG_SPARSE_NO_PANELS) ? -1
                                                                 : 0;
  const int32_t npan = sparse_panels(n, p, nnz, ldt, force);
  size_t c = 0;
  const size_t o_X = carve(&c, sizeof(float) * r * ldx);
  const size_t o_XT = carve(&c, sizeof(float) * p * ldt);
  const size_t o_U = carve(&c, sizeof(float) * r * ldu);
  const size_t o_UT = carve(&c, sizeof(float) * n * ldt);
  const size_t o_ypart = carve(&c, sizeof(double) * r * sparse_y_parts(n));
  const size_t o_YT = carve(&c, sizeof(float) * n * ldt);
  const size_t o_V = carve(&c, sizeof(float) * r * ldx);
  const size_t o_VT = carve(&c, sizeof(float) * (npan > 0 ? npan : 1) * p * ldt);
  const size_t o_pptr = carve(&c, sizeof(int64_t) * (npan * p + 1));
  const size_t o_pidx = carve(&c, npan > 0 ? sizeof(int32_t) * nnz : 0);
  const size_t o_pval = carve(&c, npan > 0 ? sizeof(float) * nnz : 0);
  const size_t o_pfirst = carve(&c, npan > 0 ? sizeof(int32_t) * nch : 0);
  const size_t o_ptmp = carve(&c, npan > 0 ? sizeof(int64_t) * sparse_panel_tmp(npan, p) : 0);
  const size_t o_carry = carve(&c, sizeof(float) * 2 * nch * ldt);
  const size_t o_cf = carve(&c, sizeof(int32_t) * nch);
  const size_t o_rf = carve(&c, sizeof(int32_t) * nch);
  const size_t o_cs = carve(&c, sizeof(int32_t) * nch);
  const size_t o_rs = carve(&c, sizeof(int32_t) * nch);
  const size_t o_bad = carve(&c, sizeof(int32_t) * 4);
  const size_t o_li = carve(&c, sizeof(int32_t) * r * ldx);
  const size_t o_lv = carve(&c, sizeof(float) * r * ldx);
  const size_t o_phi = carve(&c, sizeof(double) * r);
  const size_t o_phip = carve(&c, sizeof(double) * r);
  const size_t o_nnz = carve(&c, sizeof(int32_t) * r);
  const size_t o_it = carve(&c, sizeof(int32_t) * r);
  const size_t o_st = carve(&c, sizeof(int32_t) * r);
  const size_t o_thr = carve(&c, sizeof(float) * r);
  const size_t o_redo = carve(&c, sizeof(int32_t) * r);
  const size_t o_plan = carve(&c, sizeof(Plan));
  const size_t o_part = carve(&c, sizeof(double) * 2 * r * nfin);
  const size_t o_f = carve(&c, sizeof(double) * r);
  const size_t o_ev = carve(&c, sizeof(double) * r);
  const size_t o_xn = carve(&c, sizeof(double) * 2 * r);
  const size_t o_best = carve(&c, sizeof(int32_t) * 2);
  const size_t o_xout = carve(&c, sizeof(double) * p);
  const size_t o_sup = carve(&c, sizeof(int32_t) * p);
  const size_t o_mark = carve(&c, sizeof(int32_t) * p);
  const size_t o_ul = carve(&c, sizeof(int32_t) * p);
  const size_t o_gam = carve(&c, sizeof(double) * r);
  const size_t wide_bytes = x_update_wide_bytes(1, r, p);
  const size_t o_wide = carve(&c, wide_bytes);
  const size_t o_defl = carve(&c, deflate_bytes(n, p, r, dk));
  rc = ensure_workspace(ctx, st, c);
  if (rc != SPCA_OK) return rc;
  char* base = (char*)ctx->ws;
  float* X = (float*)(base + o_X);
  float* XT = (float*)(base + o_XT);
  float* U = (float*)(base + o_U);
  float* UT = (float*)(base + o_UT);
  double* ypart = (double*)(base + o_ypart);
  float* YT = (float*)(base + o_YT);
  float* V = (float*)(base + o_V);
  float* VT = (float*)(base + o_VT);
  float* carry = (float*)(base + o_carry);
  int32_t* bad = (int32_t*)(base + o_bad);
  int32_t* li = (int32_t*)(base + o_li);
  float* lv = (float*)(base + o_lv);
  StartState s{(double*)(base + o_phi), (double*)(base + o_phip), (int32_t*)(base + o_nnz),
               (int32_t*)(base + o_it), (int32_t*)(base + o_st), (float*)(base + o_thr),
               (int32_t*)(base + o_redo)};
  Plan* plan = (Plan*)(base + o_plan);
  double* partial = (double*)(base + o_part);
  double* fj = (double*)(base + o_f);
  double* evj = (double*)(base + o_ev);
  double* xnorm = (double*)(base + o_xn);
  int32_t* best = (int32_t*)(base + o_best);
  double* xout = (double*)(base + o_xout);
  int32_t* sup = (int32_t*)(base + o_sup);
  int32_t* colmark = (int32_t*)(base + o_mark);
  int32_t* ulist = (int32_t*)(base + o_ul);
  double* gam = (double*)(base + o_gam);
  void* wide = wide_bytes ? (void*)(base + o_wide) : nullptr;
  Defl defl{};
  if (dk > 0) defl = carve_deflate(base + o_defl, n, p, r, dk);
  Warm wm;
  if (warm) {
    wm.K = opts->warmup_iters;
    wm.target = fid >= 5 ? opts->target_nnz : 0;
    wm.gam = gam;
  }
  SparseA a{n, p, nnz, prob->col_ptr, prob->row_idx, prob->col_val, prob->row_ptr,
            prob->col_idx, prob->row_val, (int32_t*)(base + o_cf), (int32_t*)(base + o_rf)};

  // validation and chunk tables (every later kernel relies on them)
  SPCA_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
  sparse_prepare(st, a, bad);
  SPCA_LAUNCH_CHECK("sparse validation");
  int32_t hbad = 0;
  SPCA_HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  SPCA_REQUIRE(!(hbad & 1), "col_ptr or row_ptr decreases");
  SPCA_REQUIRE(!(hbad & 2), "a row or column index is out of range");
  SPCA_REQUIRE(!(hbad & 4), "the row indices of a column must be strictly increasing");
  if (npan > 0) {
    a.npan = npan;
    a.prow = ceil_div(n, (int64_t)npan);
    a.pptr = (int64_t*)(base + o_pptr);
    a.pidx = (int32_t*)(base + o_pidx);
    a.pval = (float*)(base + o_pval);
    a.pfirst = (int32_t*)(base + o_pfirst);
    a.ptmp = (int64_t*)(base + o_ptmp);
    sparse_build_panels(st, a);
    SPCA_LAUNCH_CHECK("sparse row panels");
  }
  // majors crossing chunk boundaries; products leave the rows of empty
  // majors alone, so the transposed products start at zero
  a.row_split = (int32_t*)(base + o_rs);
  a.col_split = (int32_t*)(base + o_cs);
  SPCA_HIP_TRY(hipMemsetAsync(bad + 1, 0, 2 * sizeof(int32_t), st));
  sparse_split_lists(st, a, bad + 1);
  SPCA_LAUNCH_CHECK("sparse split lists");
  SPCA_HIP_TRY(hipMemsetAsync(UT, 0, sizeof(float) * n * ldt, st));
  SPCA_HIP_TRY(hipMemsetAsync(VT, 0, sizeof(float) * (npan > 0 ? npan : 1) * p * ldt, st));
  int32_t nsplit[2];
  SPCA_HIP_TRY(hipMemcpyAsync(nsplit, bad + 1, sizeof(nsplit), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  a.nrow_split = nsplit[0];
  a.ncol_split = nsplit[1];

  if (dk > 0) {
    // deflation (further components): loadings, Gram matrix, FP64 scores
    deflate_loadings(st, opts->deflate_X, p, defl);
    sparse_deflate_scores(st, a, defl);
    SPCA_LAUNCH_CHECK("sparse deflation setup");
  }
  SPCA_HIP_TRY(hipMemcpy2DAsync(X, sizeof(float) * ldx, opts->X0, sizeof(float) * p,
                                sizeof(float) * p, r, hipMemcpyDeviceToDevice, st));
  init_state(st, s, r);
  init_plan(st, plan, 1);
  if (wide) SPCA_HIP_TRY(x_update_wide_reset(st, wide, r));
  SPCA_HIP_TRY(hipMemsetAsync(colmark, 0, sizeof(int32_t) * p, st));
  compact_rows(st, X, ldx, r, p, li, lv, ldx, s.nnz, s.status, colmark, plan);
  const int list_cap = list_cap_of(p);
  // the planner of the dense path, without the union product and with the
  // list product always followed by the separate y-update: its mode picks
  // the row gather (dense) or the support-column scatter (lists)
  plan_next(st, s, r, n, p, list_cap, 0, 1, 0, colmark, ulist, plan, 1);
  SPCA_LAUNCH_CHECK("sparse staging");
  const int32_t maxit = opts->maxit;
  const bool timed = out->kernel_times != nullptr;
  const bool sampled = (opts->flags & SPCA_FLAG_TIME_SAMPLED) != 0;
  ctx->t_aty.reset();
  ctx->t_xup.reset();
  ctx->t_ax.reset();
  auto iteration = [&](hipStream_t q, bool tm) -> int {
    transpose_f32(q, X, ldx, XT, ldt, p, r);
    if (tm) SPCA_HIP_TRY(ctx->t_ax.mark(q));
    sparse_ax_dense(q, a, XT, ldt, r, UT, carry, U, ldu, s, plan);
    if (tm) SPCA_HIP_TRY(ctx->t_ax.mark(q));
    sparse_ax_list(q, a, li, lv, ldx, U, ldu, r, s, plan);
    if (dk > 0) deflate_u(q, X, ldx, p, U, ldu, n, r, s, plan, defl);
    sparse_y_update(q, fid, U, ldu, n, r, s, ypart, YT, ldt);
    if (tm) SPCA_HIP_TRY(ctx->t_aty.mark(q));
    sparse_aty(q, a, YT, ldt, r, VT, carry, V, ldx, s, plan);
    if (tm) SPCA_HIP_TRY(ctx->t_aty.mark(q));
    if (dk > 0) deflate_v(q, V, ldx, p, r, s, defl);
    if (tm) SPCA_HIP_TRY(ctx->t_xup.mark(q));
    x_update(q, fid, sg, V, ldx, r, p, X, ldx, li, lv, ldx, list_cap, s, opts->tol, maxit,
             colmark, plan, wide, wm);
    if (tm) SPCA_HIP_TRY(ctx->t_xup.mark(q));
    plan_next(q, s, r, n, p, list_cap, 0, 1, 0, colmark, ulist, plan, 1);
    SPCA_LAUNCH_CHECK("sparse AM iteration");
    return SPCA_OK;
  };
  auto none_active = [&](bool* done) -> int {
    SPCA_HIP_TRY(hipMemcpyAsync(ctx->host_poll, &plan->active, sizeof(int32_t),
                                hipMemcpyDeviceToHost, st));
    SPCA_HIP_TRY(hipStreamSynchronize(st));
    *done = ctx->host_poll[0] == 0;
    return SPCA_OK;
  };
  const int32_t every = opts->check_every;
  int32_t it = 0;
  bool done = false;
  if ((opts->flags & SPCA_FLAG_GRAPH) && maxit >= every && !timed) {
    rc = ensure_capture_stream(ctx);
    if (rc != SPCA_OK) return rc;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    SPCA_HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    int body_rc = SPCA_OK;
    for (int32_t k = 0; k < every && body_rc == SPCA_OK; ++k)
      body_rc = iteration(ctx->capture, false);
    hipError_t end_rc = hipStreamEndCapture(ctx->capture, &graph);
    if (body_rc != SPCA_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return body_rc;
    }
    SPCA_HIP_TRY(end_rc);
    hipError_t inst_rc = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    SPCA_HIP_TRY(inst_rc);
    int loop_rc = SPCA_OK;
    while (!done && it + every <= maxit) {
      hipError_t e = hipGraphLaunch(exec, st);
      if (e != hipSuccess) {
        set_error(std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        loop_rc = SPCA_EHIP;
        break;
      }
      it += every;
      if (it < maxit) {
        loop_rc = none_active(&done);
        if (loop_rc != SPCA_OK) break;
      }
    }
    (void)hipGraphExecDestroy(exec);
    if (loop_rc != SPCA_OK) return loop_rc;
  }
  for (; !done && it < maxit; ++it) {
    rc = iteration(st, timed && (!sampled || it % kTimeSample == 0));
    if (rc != SPCA_OK) return rc;
    if ((it + 1) % every == 0 && it + 1 < maxit) {
      rc = none_active(&done);
      if (rc != SPCA_OK) return rc;
    }
  }

  // FP64 evaluation on the sparse matrix
  compact_rows(st, X, ldx, r, p, li, lv, ldx, s.nnz, nullptr, nullptr, nullptr);
  x_norms(st, lv, ldx, s, r, xnorm);
  if (dk > 0) deflate_final_alpha(st, X, ldx, p, r, defl);
  sparse_final(st, a, li, lv, ldx, s, r, xnorm, partial, defl);
  const bool per_start_gamma = warm && fid >= 5;
  objective_and_best(st, fid, sg, s, r, p, partial, (int)nfin, li, lv, ldx, xnorm, fj, evj, best,
                     xout, sup, per_start_gamma ? gam : nullptr, per_start_gamma);
  SPCA_LAUNCH_CHECK("sparse finalize");

  int32_t hb[2];
  SPCA_HIP_TRY(hipMemcpyAsync(hb, best, sizeof(hb), hipMemcpyDeviceToHost, st));
  std::vector<double> f_all(r), ev_all(r), phi_all(r);
  std::vector<int32_t> it_all(r), st_all(r), nnz_all(r);
  SPCA_HIP_TRY(hipMemcpyAsync(f_all.data(), fj, sizeof(double) * r, hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(ev_all.data(), evj, sizeof(double) * r, hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(phi_all.data(), s.phi, sizeof(double) * r, hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(it_all.data(), s.iters, sizeof(int32_t) * r, hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(st_all.data(), s.status, sizeof(int32_t) * r, hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(nnz_all.data(), s.nnz, sizeof(int32_t) * r, hipMemcpyDeviceToHost, st));
  Plan hplan;
  SPCA_HIP_TRY(hipMemcpyAsync(&hplan, plan, sizeof(Plan), hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  if (timed) {
    // as in spca_am_solve_ex; [4] covers the row-gather A x (launches of list
    // iterations return at once)
    double* kt = out->kernel_times;
    SPCA_HIP_TRY(ctx->t_aty.total_ms(&kt[0]));
    kt[1] = (double)(ctx->t_aty.used / 2);
    SPCA_HIP_TRY(ctx->t_xup.total_ms(&kt[2]));
    kt[3] = (double)(ctx->t_xup.used / 2);
    SPCA_HIP_TRY(ctx->t_ax.total_ms(&kt[4]));
    kt[5] = (double)(ctx->t_ax.used / 2);
    kt[6] = hplan.mode_count[kAxDense];
    kt[7] = hplan.mode_count[kAxList] + hplan.mode_count[kAxListRows];
    kt[8] = hplan.mode_count[kAxUnion];
    kt[9] = hplan.mode_count[kAxListRows];
    kt[10] = hplan.active_sum;
    kt[11] = hplan.nnz_sum;
  }
  const int32_t jb = hb[0], nnzb = hb[1];
  if (out->x)
    SPCA_HIP_TRY(hipMemcpyAsync(out->x, xout, sizeof(double) * p, hipMemcpyDeviceToHost, st));
  if (out->support && nnzb > 0)
    SPCA_HIP_TRY(hipMemcpyAsync(out->support, sup, sizeof(int32_t) * nnzb,
                                hipMemcpyDeviceToHost, st));
  if (out->param_per_start && warm)
    SPCA_HIP_TRY(hipMemcpyAsync(out->param_per_start, gam, sizeof(double) * r,
                                hipMemcpyDeviceToHost, st));
  if (out->X_final)
    SPCA_HIP_TRY(hipMemcpy2DAsync(out->X_final, sizeof(float) * p, X, sizeof(float) * ldx,
                                  sizeof(float) * p, r, hipMemcpyDeviceToDevice, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  double total_iters = 0.0;
  for (int64_t j = 0; j < r; ++j) total_iters += it_all[j];
  spca_result* res = out->res;
  res->objective = f_all[jb];
  res->objective_pre_polish = f_all[jb];
  res->polish_iters = 0;
  res->explained_var = ev_all[jb];
  res->phi = phi_all[jb];
  res->iters_x_starts = total_iters;
  res->best_start = jb;
  res->nnz = nnzb;
  res->iters = it_all[jb];
  res->status = st_all[jb];
  for (int64_t j = 0; j < r; ++j) {
    if (out->f_per_start) out->f_per_start[j] = f_all[j];
    if (out->ev_per_start) out->ev_per_start[j] = ev_all[j];
    if (out->phi_per_start) out->phi_per_start[j] = phi_all[j];
    if (out->iters_per_start) out->iters_per_start[j] = it_all[j];
    if (out->status_per_start) out->status_per_start[j] = st_all[j];
    if (out->nnz_per_start) out->nnz_per_start[j] = nnz_all[j];
  }
  out->res->warning = solve_warning(st_all, r, opts->tol);
  return SPCA_OK;
}

int spca_am_components_sparse(spca_ctx* ctx, void* stream, const spca_sparse_problem* prob,
                              const spca_solve_opts* opts, int32_t ncomp, double* X_out,
                              spca_result* res) {
  return components_loop(ctx, stream, prob, opts, ncomp, X_out, res, spca_am_solve_sparse);
}

int spca_am_components(spca_ctx* ctx, void* stream, const spca_problem* prob,
                       const spca_solve_opts* opts, int32_t ncomp, double* X_out,
                       spca_result* res) {
  return components_loop(ctx, stream, prob, opts, ncomp, X_out, res, spca_am_solve_ex);
}

static std::mutex g_default_mu;
static std::vector<spca_ctx*> g_default_ctx;

int spca_am_solve(const float* A, int64_t n, int64_t p, int64_t lda,
                  int formulation, double s_or_gamma, const float* X0,
                  int32_t r, double tol, int32_t maxit, double* x_out,
                  int32_t* support_out, spca_result* res) {
  SPCA_REQUIRE(A && x_out && support_out && res,
               "A, x_out, support_out and res must not be NULL");
  int rc = check_problem(n, p, lda, formulation, s_or_gamma, r, tol, maxit);
  if (rc != SPCA_OK) return rc;
  int dev = 0;
  SPCA_HIP_TRY(hipGetDevice(&dev));
  spca_ctx* ctx = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_default_mu);
    if ((int)g_default_ctx.size() <= dev) g_default_ctx.resize(dev + 1, nullptr);
    if (g_default_ctx[dev] == nullptr) {
      rc = spca_ctx_create(&g_default_ctx[dev], dev, 0);
      if (rc != SPCA_OK) return rc;
    }
    ctx = g_default_ctx[dev];
  }
  spca_problem prob{A, n, p, lda, formulation, s_or_gamma};
  spca_solve_opts opts{X0, r, tol, maxit, SPCA_PREC_FP32, 0, 8, 0};
  spca_outputs out{};
  out.x = x_out;
  out.support = support_out;
  out.res = res;
  return spca_am_solve_ex(ctx, nullptr, &prob, &opts, &out);
}

int spca_gemm_nt_f32(void* stream, const float* P, int64_t ldp, const float* Q,
                     int64_t ldq, float* C, int64_t ldc, int64_t M, int64_t N,
                     int64_t K) {
  SPCA_REQUIRE(P && Q && C, "P, Q and C must not be NULL");
  SPCA_REQUIRE(M >= 0 && N >= 0 && K >= 0, "sizes must be >= 0");
  SPCA_REQUIRE(M <= INT32_MAX && N <= INT32_MAX && K <= INT32_MAX,
               "sizes must fit in int32");
  SPCA_REQUIRE(ldp >= K && ldq >= K && ldc >= N, "leading dimensions too small");
  SPCA_REQUIRE(ldp % 4 == 0 && ldq % 4 == 0,
               "ldp and ldq must be multiples of 4");
  SPCA_REQUIRE((uintptr_t)P % 16 == 0 && (uintptr_t)Q % 16 == 0,
               "P and Q must be 16-byte aligned");
  gemm_nt_f32((hipStream_t)stream, P, ldp, Q, ldq, C, ldc, M, N, K, nullptr, 0,
              plan_gemm_nt(M, N, K, 1), 0);
  SPCA_LAUNCH_CHECK("gemm_nt_f32");
  return SPCA_OK;
}

int spca_gemm_nt_f32_shape(void* stream, const float* P, int64_t ldp,
                           const float* Q, int64_t ldq, float* C, int64_t ldc,
                           int64_t M, int64_t N, int64_t K, int shape,
                           int splits) {
  SPCA_REQUIRE(P && Q && C, "P, Q and C must not be NULL");
  SPCA_REQUIRE(M >= 0 && N >= 0 && K >= 0, "sizes must be >= 0");
  SPCA_REQUIRE(M <= INT32_MAX && N <= INT32_MAX && K <= INT32_MAX,
               "sizes must fit in int32");
  SPCA_REQUIRE(ldp >= K && ldq >= K && ldc >= N, "leading dimensions too small");
  SPCA_REQUIRE(ldp % 4 == 0 && ldq % 4 == 0,
               "ldp and ldq must be multiples of 4");
  SPCA_REQUIRE((uintptr_t)P % 16 == 0 && (uintptr_t)Q % 16 == 0,
               "P and Q must be 16-byte aligned");
  SPCA_REQUIRE(shape >= 0 && shape < gemm_num_shapes(), "shape index out of range");
  SPCA_REQUIRE(splits >= 1 && splits <= 64, "splits must be in 1..64");
  gemm_nt_f32((hipStream_t)stream, P, ldp, Q, ldq, C, ldc, M, N, K, nullptr, 0,
              GemmPlan{shape, splits}, M * ldc);
  SPCA_LAUNCH_CHECK("gemm_nt_f32");
  return SPCA_OK;
}

int spca_gemm_nt_bf16_shape(void* stream, const uint16_t* P, int64_t ldp,
                            const uint16_t* Q, int64_t ldq, float* C, int64_t ldc,
                            int64_t M, int64_t N, int64_t K, int shape, int splits) {
  SPCA_REQUIRE(P && Q && C, "P, Q and C must not be NULL");
  SPCA_REQUIRE(M >= 0 && N >= 0 && K >= 0, "sizes must be >= 0");
  SPCA_REQUIRE(M <= INT32_MAX && N <= INT32_MAX && K <= INT32_MAX,
               "sizes must fit in int32");
  SPCA_REQUIRE(ldp >= K && ldq >= K && ldc >= N, "leading dimensions too small");
  SPCA_REQUIRE(ldp % 8 == 0 && ldq % 8 == 0, "ldp and ldq must be multiples of 8");
  SPCA_REQUIRE((uintptr_t)P % 16 == 0 && (uintptr_t)Q % 16 == 0,
               "P and Q must be 16-byte aligned");
  SPCA_REQUIRE(shape >= 0 && shape < gemm_num_shapes(), "shape index out of range");
  SPCA_REQUIRE(splits >= 1 && splits <= 64, "splits must be in 1..64");
  gemm_nt_bf16((hipStream_t)stream, P, ldp, Q, ldq, C, ldc, M, N, K, nullptr, 0,
               GemmPlan{shape, splits}, M * ldc);
  SPCA_LAUNCH_CHECK("gemm_nt_bf16");
  return SPCA_OK;
}

int spca_gemm_nt_bf16(void* stream, const uint16_t* P, int64_t ldp,
                      const uint16_t* Q, int64_t ldq, float* C, int64_t ldc,
                      int64_t M, int64_t N, int64_t K) {
  SPCA_REQUIRE(P && Q && C, "P, Q and C must not be NULL");
  SPCA_REQUIRE(M >= 0 && N >= 0 && K >= 0, "sizes must be >= 0");
  SPCA_REQUIRE(M <= INT32_MAX && N <= INT32_MAX && K <= INT32_MAX,
               "sizes must fit in int32");
  SPCA_REQUIRE(ldp >= K && ldq >= K && ldc >= N, "leading dimensions too small");
  SPCA_REQUIRE(ldp % 8 == 0 && ldq % 8 == 0,
               "ldp and ldq must be multiples of 8");
  SPCA_REQUIRE((uintptr_t)P % 16 == 0 && (uintptr_t)Q % 16 == 0,
               "P and Q must be 16-byte aligned");
  gemm_nt_bf16((hipStream_t)stream, P, ldp, Q, ldq, C, ldc, M, N, K, nullptr, 0,
               plan_gemm_nt(M, N, K, 1, 2), 0);
  SPCA_LAUNCH_CHECK("gemm_nt_bf16");
  return SPCA_OK;
}

int spca_tune_table_export(char* buf, size_t cap, size_t* len) {
  SPCA_REQUIRE(len != nullptr, "len must not be NULL");
  const std::string t = tune_table_text();
  *len = t.size();
  if (buf != nullptr && cap > 0) {
    const size_t k = t.size() < cap - 1 ? t.size() : cap - 1;
    std::memcpy(buf, t.data(), k);
    buf[k] = '\0';
    SPCA_REQUIRE(t.size() < cap, "buffer too small for the tuning table");
  }
  return SPCA_OK;
}

int spca_tune_table_import(const char* text) {
  SPCA_REQUIRE(text != nullptr, "text must not be NULL");
  std::string err;
  SPCA_REQUIRE(tune_table_load(text, &err), err.c_str());
  return SPCA_OK;
}

int spca_tune_table_clear(void) {
  tune_table_clear();
  return SPCA_OK;
}

int spca_gemm_nt_f32_plan(int64_t M, int64_t N, int64_t K, int max_splits,
                          int* shape, int* splits) {
  SPCA_REQUIRE(shape && splits, "shape and splits must not be NULL");
  SPCA_REQUIRE(M >= 1 && N >= 1 && K >= 1 && max_splits >= 1,
               "sizes and max_splits must be >= 1");
  GemmPlan g = plan_gemm_nt(M, N, K, max_splits);
  *shape = g.shape;
  *splits = g.splits;
  return SPCA_OK;
}

int spca_x_update(void* stream, int formulation, const float* V, int64_t ldv,
                  int64_t r, int64_t p, double s_or_gamma, float* X,
                  int64_t ldx, double* phi, int32_t* nnz) {
  SPCA_REQUIRE(V && X && phi && nnz, "V, X, phi and nnz must not be NULL");
  int rc = check_problem(1, p, 1, formulation, s_or_gamma, r, 0.0, 1);
  if (rc != SPCA_OK) return rc;
  SPCA_REQUIRE(ldv >= p && ldx >= p, "leading dimensions too small");
  StartState s{phi, nullptr, nnz, nullptr, nullptr};
  hipStream_t st = (hipStream_t)stream;
  // long rows: the chunked kernels need scratch, held for this call only
  const size_t wb = x_update_wide_bytes(formulation, r, p);
  void* wide = nullptr;
  if (wb) {
    SPCA_HIP_TRY(hipMalloc(&wide, wb));
    hipError_t e = x_update_wide_reset(st, wide, r);
    if (e != hipSuccess) {
      (void)hipFree(wide);
      SPCA_HIP_TRY(e);
    }
  }
  x_update(st, formulation, s_or_gamma, V, ldv, r, p, X, ldx, nullptr, nullptr, 0,
           0, s, -1.0, 1, nullptr, nullptr, wide);
  hipError_t le = hipGetLastError();
  if (wide) {
    hipError_t se = hipStreamSynchronize(st);
    (void)hipFree(wide);
    if (le == hipSuccess) le = se;
  }
  if (le != hipSuccess) {
    set_error(std::string("x_update: ") + hipGetErrorString(le));
    return SPCA_EHIP;
  }
  return SPCA_OK;
}

}  // extern "C"
