// Grouped solves: several independent requests (each with its own A,
// formulation, parameter, starts, tolerance and iteration limit) iterated
// together, one set of kernel launches per AM iteration for all of them
// (Algorithm 2 from every start of every request, Section 4).
//
// Layout: the starts of all requests are the rows of one batch (request q
// owns rows first[q] .. first[q+1]); X and V rows hold p_max entries and U
// and Y rows n_max, with the entries beyond a request's own p or n zero
// throughout.  Per iteration:
//   U = X A^T     one grouped MFMA launch over the tiles of every request
//                 (K split per request), reading each request's row-major A
//   y-update      one launch, variance type and partial count per start
//   V = Y A       one grouped MFMA launch (K split per request), then the
//                 partial sums in one launch
//   x-update      one launch sequence per operator kind present (T_s,
//                 lambda_s, U_gamma, V_gamma), each start taking its
//                 parameter, tolerance and limit from its request
//   count         running starts per request and in total (requests with
//                 none left are skipped by the products)
// The products are always dense: the groups are meant for small requests,
// whose cost is launch count rather than arithmetic.
//
// A request's result depends only on the request: its K splits follow from
// its own n and p, each product's tile computes the same sums in the same
// order whatever tile it lands in, and the zero padding adds exact zeros at
// the ends of the per-thread sums of the y- and x-updates.  So a request
// gives the same bits alone and in any group.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spca.h"
#include "common.hpp"
#include "context.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr int64_t kGroupSplitK = 1024;  // target K per split of a product
constexpr int kGroupMaxSplits = 12;
static_assert(kGroupMaxSplits <= kSplitsMax, "the grouped sums add at most kSplitsMax partials");

size_t gcarve(size_t* cur, size_t bytes) {
  size_t o = (*cur + 255) / 256 * 256;
  *cur = o + bytes;
  return o;
}

int32_t group_splits(int64_t K) {
  const int64_t s = ceil_div(K, kGroupSplitK);
  return (int32_t)(s < 1 ? 1 : s > kGroupMaxSplits ? kGroupMaxSplits : s);
}

struct GroupLayout {
  int32_t count = 0;
  int64_t R = 0, n_max = 0, p_max = 0, ldx = 0, ldu = 0;
  int32_t sax = 1, saty = 1;  // largest split counts
  std::vector<int64_t> first;
  std::vector<int32_t> ax_splits, aty_splits;
  std::vector<bool> copy_a;
  std::vector<int64_t> ldat, ldac;
  std::vector<size_t> off_At, off_Ac, off_part, off_xout, off_sup;
  size_t off_X, off_U, off_Y, off_V, off_li, off_lv, off_phi, off_phip, off_nnz, off_it,
      off_st, off_thr, off_redo, off_cfg, off_f, off_ev, off_xn, off_best, off_desc, off_first,
      off_run, off_colsq;
  size_t total = 0;
};

GroupLayout group_layout(int32_t count, const spca_problem* probs, const spca_solve_opts* opts) {
  GroupLayout L;
  L.count = count;
  L.first.assign(count + 1, 0);
  for (int32_t q = 0; q < count; ++q) {
    L.first[q + 1] = L.first[q] + opts[q].r;
    L.n_max = std::max<int64_t>(L.n_max, probs[q].n);
    L.p_max = std::max<int64_t>(L.p_max, probs[q].p);
    L.ax_splits.push_back(group_splits(probs[q].p));
    L.aty_splits.push_back(group_splits(probs[q].n));
    L.sax = std::max(L.sax, L.ax_splits.back());
    L.saty = std::max(L.saty, L.aty_splits.back());
    L.copy_a.push_back(probs[q].lda % 4 != 0 || (uintptr_t)probs[q].A % 16 != 0);
    L.ldat.push_back(round_up(probs[q].p, 4));
    L.ldac.push_back(round_up(probs[q].n, 4));
  }
  L.R = L.first[count];
  L.ldx = round_up(L.p_max, 4);
  L.ldu = round_up(L.n_max, 4);
  size_t c = 0;
  for (int32_t q = 0; q < count; ++q) {
    const spca_problem& pr = probs[q];
    L.off_At.push_back(gcarve(&c, sizeof(float) * (size_t)pr.n * L.ldat[q]));
    L.off_Ac.push_back(gcarve(&c, L.copy_a[q] ? sizeof(float) * (size_t)pr.p * L.ldac[q] : 0));
    L.off_part.push_back(
        gcarve(&c, sizeof(double) * 2 * (size_t)opts[q].r * (size_t)ceil_div(pr.n, 64)));
    L.off_xout.push_back(gcarve(&c, sizeof(double) * (size_t)pr.p));
    L.off_sup.push_back(gcarve(&c, sizeof(int32_t) * (size_t)pr.p));
  }
  const size_t R = (size_t)L.R;
  L.off_X = gcarve(&c, sizeof(float) * R * L.ldx);
  L.off_U = gcarve(&c, sizeof(float) * (size_t)L.sax * R * L.ldu);
  L.off_Y = gcarve(&c, sizeof(float) * R * L.ldu);
  L.off_V = gcarve(&c, sizeof(float) * (size_t)L.saty * R * L.ldx);
  L.off_li = gcarve(&c, sizeof(int32_t) * R * L.ldx);
  L.off_lv = gcarve(&c, sizeof(float) * R * L.ldx);
  L.off_phi = gcarve(&c, sizeof(double) * R);
  L.off_phip = gcarve(&c, sizeof(double) * R);
  L.off_nnz = gcarve(&c, sizeof(int32_t) * R);
  L.off_it = gcarve(&c, sizeof(int32_t) * R);
  L.off_st = gcarve(&c, sizeof(int32_t) * R);
  L.off_thr = gcarve(&c, sizeof(float) * R);
  L.off_redo = gcarve(&c, sizeof(int32_t) * R);
  L.off_cfg = gcarve(&c, sizeof(RowCfg) * R);
  L.off_f = gcarve(&c, sizeof(double) * R);
  L.off_ev = gcarve(&c, sizeof(double) * R);
  L.off_xn = gcarve(&c, sizeof(double) * 2 * R);
  L.off_best = gcarve(&c, sizeof(int32_t) * 2 * (size_t)count);
  L.off_desc = gcarve(&c, sizeof(GemmGroupDesc) * 2 * (size_t)count);
  L.off_first = gcarve(&c, sizeof(int64_t) * (size_t)(count + 1));
  L.off_run = gcarve(&c, sizeof(int32_t) * (size_t)(count + 1));
  L.off_colsq = gcarve(&c, sizeof(double) * (size_t)L.p_max);
  L.total = c;
  return L;
}

// The arguments every request of a group must satisfy.
int check_group(int32_t count, const spca_problem* probs, const spca_solve_opts* opts) {
  SPCA_REQUIRE(count >= 1 && count <= SPCA_GROUP_MAX_REQUESTS,
               "count must be in 1..SPCA_GROUP_MAX_REQUESTS");
  SPCA_REQUIRE(probs != nullptr && opts != nullptr, "probs and opts must not be NULL");
  int64_t R = 0;
  for (int32_t q = 0; q < count; ++q) {
    const spca_problem& pr = probs[q];
    const spca_solve_opts& o = opts[q];
    const std::string at = " (request " + std::to_string(q) + ")";
    if (pr.A == nullptr) {
      set_error("A must not be NULL" + at);
      return SPCA_EINVAL;
    }
    int rc = check_problem(pr.n, pr.p, pr.lda, pr.formulation, pr.s_or_gamma, o.r, o.tol,
                           o.maxit);
    if (rc != SPCA_OK) {
      set_error(std::string(spca_last_error()) + at);
      return rc;
    }
    if (pr.p > SPCA_GROUP_MAX_P) {
      set_error("p above SPCA_GROUP_MAX_P" + at);
      return SPCA_EINVAL;
    }
    if (o.X0 == nullptr && o.r != 1) {
      set_error("X0 may be NULL only with r == 1" + at);
      return SPCA_EINVAL;
    }
    if (o.precision != SPCA_PREC_FP32 || o.total_starts > o.r || o.warmup_iters != 0 ||
        o.deflate_k != 0) {
      set_error("grouped solves run FP32 without replacement, warm-up or deflation" + at);
      return SPCA_EINVAL;
    }
    if (o.check_every < 1) {
      set_error("check_every must be >= 1" + at);
      return SPCA_EINVAL;
    }
    R += o.r;
  }
  SPCA_REQUIRE(R <= SPCA_GROUP_MAX_STARTS, "more than SPCA_GROUP_MAX_STARTS starts in the group");
  return SPCA_OK;
}

}  // namespace
}  // namespace spca

using namespace spca;

extern "C" {

size_t spca_group_workspace_bytes(int32_t count, const spca_problem* probs,
                                  const spca_solve_opts* opts) {
  if (count < 1 || probs == nullptr || opts == nullptr) return 0;
  for (int32_t q = 0; q < count; ++q)
    if (probs[q].n < 1 || probs[q].p < 1 || opts[q].r < 1) return 0;
  return group_layout(count, probs, opts).total;
}

int spca_am_solve_group(spca_ctx* ctx, void* stream, int32_t count, const spca_problem* probs,
                        const spca_solve_opts* opts, spca_outputs* outs) {
  int rc = check_group(count, probs, opts);
  if (rc != SPCA_OK) return rc;
  SPCA_REQUIRE(ctx != nullptr && outs != nullptr, "ctx and outs must not be NULL");
  for (int32_t q = 0; q < count; ++q)
    SPCA_REQUIRE(outs[q].res != nullptr, "every outs[q].res must be set");
  std::lock_guard<std::mutex> lock(ctx->mu);
  DeviceGuard g(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  GroupLayout L = group_layout(count, probs, opts);
  rc = ensure_workspace(ctx, st, L.total);
  if (rc != SPCA_OK) return rc;
  char* base = (char*)ctx->ws;
  const int64_t R = L.R, ldx = L.ldx, ldu = L.ldu;
  float* X = (float*)(base + L.off_X);
  float* U = (float*)(base + L.off_U);
  float* Y = (float*)(base + L.off_Y);
  float* V = (float*)(base + L.off_V);
  int32_t* li = (int32_t*)(base + L.off_li);
  float* lv = (float*)(base + L.off_lv);
  RowCfg* cfg = (RowCfg*)(base + L.off_cfg);
  StartState s{(double*)(base + L.off_phi), (double*)(base + L.off_phip),
               (int32_t*)(base + L.off_nnz), (int32_t*)(base + L.off_it),
               (int32_t*)(base + L.off_st),  (float*)(base + L.off_thr),
               (int32_t*)(base + L.off_redo)};
  double* fj = (double*)(base + L.off_f);
  double* evj = (double*)(base + L.off_ev);
  double* xnorm = (double*)(base + L.off_xn);
  int32_t* best = (int32_t*)(base + L.off_best);
  GemmGroupDesc* desc = (GemmGroupDesc*)(base + L.off_desc);
  int64_t* first_d = (int64_t*)(base + L.off_first);
  int32_t* running = (int32_t*)(base + L.off_run);
  double* colsq = (double*)(base + L.off_colsq);

  // a0: the padding of every operand stays zero for the whole solve
  SPCA_HIP_TRY(hipMemsetAsync(X, 0, sizeof(float) * (size_t)R * ldx, st));
  SPCA_HIP_TRY(hipMemsetAsync(U, 0, sizeof(float) * (size_t)L.sax * R * ldu, st));
  SPCA_HIP_TRY(hipMemsetAsync(Y, 0, sizeof(float) * (size_t)R * ldu, st));
  SPCA_HIP_TRY(hipMemsetAsync(V, 0, sizeof(float) * (size_t)L.saty * R * ldx, st));

  // per request: aligned A, its row-major twin, the starts, the per-start
  // settings and the two product descriptors
  std::vector<const float*> Aq(count);
  std::vector<int64_t> ldAq(count);
  std::vector<RowCfg> hcfg((size_t)R);
  std::vector<GemmGroupDesc> hdesc(2 * (size_t)count);
  bool kinds[4] = {false, false, false, false};
  int fid_of_kind[4] = {0, 0, 0, 0};
  int32_t maxit_all = 0, every = INT32_MAX;
  for (int32_t q = 0; q < count; ++q) {
    const spca_problem& pr = probs[q];
    const spca_solve_opts& o = opts[q];
    const int64_t n = pr.n, p = pr.p, r = o.r, f0 = L.first[q];
    const float* A = pr.A;
    int64_t ldA = pr.lda;
    if (L.copy_a[q]) {
      float* Ac = (float*)(base + L.off_Ac[q]);
      copy_columns_f32(st, pr.A, pr.lda, Ac, L.ldac[q], n, p);
      A = Ac;
      ldA = L.ldac[q];
    }
    Aq[q] = A;
    ldAq[q] = ldA;
    float* At = (float*)(base + L.off_At[q]);
    transpose_f32(st, A, ldA, At, L.ldat[q], n, p);
    float* Xq = X + f0 * ldx;
    if (o.X0 != nullptr)
      SPCA_HIP_TRY(hipMemcpy2DAsync(Xq, sizeof(float) * ldx, o.X0, sizeof(float) * p,
                                    sizeof(float) * p, r, hipMemcpyDeviceToDevice, st));
    else
      max_norm_column_start(st, A, ldA, n, p, colsq, Xq, ldx);
    const XKind kind = xkind_of(pr.formulation);
    kinds[kind] = true;
    fid_of_kind[kind] = pr.formulation;
    for (int64_t j = 0; j < r; ++j)
      hcfg[f0 + j] = RowCfg{pr.s_or_gamma, o.tol, o.maxit, (int32_t)kind,
                            l1_variance(pr.formulation) ? 1 : 0, L.ax_splits[q],
                            L.aty_splits[q]};
    maxit_all = std::max(maxit_all, o.maxit);
    every = std::min(every, o.check_every);
    // U rows (r x n) = X rows (r x p) A^T: Q = A row-major (n x p)
    GemmGroupDesc& d1 = hdesc[q];
    d1 = GemmGroupDesc{};
    d1.P = Xq;
    d1.ldp = ldx;
    d1.Q = At;
    d1.ldq = L.ldat[q];
    d1.C = U + f0 * ldu;
    d1.ldc = ldu;
    d1.split_stride = R * ldu;
    d1.M = (int32_t)r;
    d1.N = (int32_t)n;
    d1.K = (int32_t)p;
    d1.splits = L.ax_splits[q];
    d1.req = q;
    // V rows (r x p) = Y rows (r x n) A: Q = A column-major (p x n)
    GemmGroupDesc& d2 = hdesc[count + q];
    d2 = GemmGroupDesc{};
    d2.P = Y + f0 * ldu;
    d2.ldp = ldu;
    d2.Q = A;
    d2.ldq = ldA;
    d2.C = V + f0 * ldx;
    d2.ldc = ldx;
    d2.split_stride = R * ldx;
    d2.M = (int32_t)r;
    d2.N = (int32_t)p;
    d2.K = (int32_t)n;
    d2.splits = L.aty_splits[q];
    d2.req = q;
  }
  int tiles_ax = 0, tiles_aty = 0;
  gemm_group_tiles(hdesc.data(), count, &tiles_ax);
  gemm_group_tiles(hdesc.data() + count, count, &tiles_aty);
  SPCA_HIP_TRY(hipMemcpyAsync(cfg, hcfg.data(), sizeof(RowCfg) * (size_t)R,
                              hipMemcpyHostToDevice, st));
  SPCA_HIP_TRY(hipMemcpyAsync(desc, hdesc.data(), sizeof(GemmGroupDesc) * 2 * (size_t)count,
                              hipMemcpyHostToDevice, st));
  SPCA_HIP_TRY(hipMemcpyAsync(first_d, L.first.data(), sizeof(int64_t) * (size_t)(count + 1),
                              hipMemcpyHostToDevice, st));
  init_state(st, s, R);
  // nonzeros of the starts (the x-update sizes its first lambda_s
  // candidate count from them)
  compact_rows(st, X, ldx, R, L.p_max, li, lv, ldx, s.nnz, s.status, nullptr, nullptr);
  group_count(st, s.status, first_d, count, running);
  SPCA_LAUNCH_CHECK("group staging");

  StartState sg = s;
  sg.cfg = cfg;
  auto iteration = [&]() -> int {
    gemm_nt_f32_group(st, desc, count, tiles_ax, running);
    group_y_update(st, U, R * ldu, Y, ldu, R, L.n_max, sg);
    gemm_nt_f32_group(st, desc + count, count, tiles_aty, running);
    if (L.saty > 1) group_sum_splits(st, V, R * ldx, ldx, R, L.p_max, sg);
    for (int k = 0; k < 4; ++k)
      if (kinds[k])
        x_update(st, fid_of_kind[k], 1.0, V, ldx, R, L.p_max, X, ldx, nullptr, nullptr, 0, 0,
                 sg, 0.0, 1, nullptr, nullptr, nullptr);
    group_count(st, s.status, first_d, count, running);
    SPCA_LAUNCH_CHECK("group iteration");
    return SPCA_OK;
  };
  for (int32_t it = 0; it < maxit_all; ++it) {
    rc = iteration();
    if (rc != SPCA_OK) return rc;
    if ((it + 1) % every == 0 && it + 1 < maxit_all) {
      SPCA_HIP_TRY(hipMemcpyAsync(ctx->host_poll, running + count, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, st));
      SPCA_HIP_TRY(hipStreamSynchronize(st));
      if (ctx->host_poll[0] == 0) break;
    }
  }

  // a6 per request: lists of the final iterates, FP64 objective and
  // explained variance, best start, output vector (the FP64 product may
  // split its columns over the V buffer: at most r p floats per request,
  // and the requests' evaluations run one after another on the stream)
  compact_rows(st, X, ldx, R, L.p_max, li, lv, ldx, s.nnz, nullptr, nullptr, nullptr);
  std::vector<int32_t> nnz_h((size_t)R);
  SPCA_HIP_TRY(hipMemcpyAsync(nnz_h.data(), s.nnz, sizeof(int32_t) * (size_t)R,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  for (int32_t q = 0; q < count; ++q) {
    const spca_problem& pr = probs[q];
    const int64_t r = opts[q].r, f0 = L.first[q];
    double tot_nnz = 0.0;
    for (int64_t j = 0; j < r; ++j) tot_nnz += nnz_h[f0 + j];
    const bool dense_eval = r >= 16 && tot_nnz * 4.0 >= (double)r * (double)pr.p;
    StartState sq{s.phi + f0, s.phi_prev + f0, s.nnz + f0, s.iters + f0, s.status + f0,
                  s.thr + f0, s.redo + f0};
    finalize(st, pr.formulation, pr.s_or_gamma, Aq[q], ldAq[q], pr.n, pr.p, li + f0 * ldx,
             lv + f0 * ldx, ldx, sq, r, (double*)(base + L.off_part[q]), fj + f0, evj + f0,
             xnorm + 2 * f0, best + 2 * q, (double*)(base + L.off_xout[q]),
             (int32_t*)(base + L.off_sup[q]), nullptr, false, Defl{},
             dense_eval ? X + f0 * ldx : nullptr, ldx, (double*)V);
  }
  SPCA_LAUNCH_CHECK("group finalize");
  std::vector<int32_t> hb(2 * (size_t)count), it_h((size_t)R), st_h((size_t)R);
  std::vector<double> f_h((size_t)R), ev_h((size_t)R), phi_h((size_t)R);
  SPCA_HIP_TRY(hipMemcpyAsync(hb.data(), best, sizeof(int32_t) * 2 * (size_t)count,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(f_h.data(), fj, sizeof(double) * (size_t)R,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(ev_h.data(), evj, sizeof(double) * (size_t)R,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(phi_h.data(), s.phi, sizeof(double) * (size_t)R,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(it_h.data(), s.iters, sizeof(int32_t) * (size_t)R,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(st_h.data(), s.status, sizeof(int32_t) * (size_t)R,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipMemcpyAsync(nnz_h.data(), s.nnz, sizeof(int32_t) * (size_t)R,
                              hipMemcpyDeviceToHost, st));
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  for (int32_t q = 0; q < count; ++q) {
    const spca_solve_opts& o = opts[q];
    spca_outputs& out = outs[q];
    const int64_t r = o.r, f0 = L.first[q], p = probs[q].p;
    const int32_t jb = hb[2 * q], nnzb = hb[2 * q + 1];
    if (out.x)
      SPCA_HIP_TRY(hipMemcpyAsync(out.x, base + L.off_xout[q], sizeof(double) * p,
                                  hipMemcpyDeviceToHost, st));
    if (out.support && nnzb > 0)
      SPCA_HIP_TRY(hipMemcpyAsync(out.support, base + L.off_sup[q], sizeof(int32_t) * nnzb,
                                  hipMemcpyDeviceToHost, st));
    if (out.X_final)
      SPCA_HIP_TRY(hipMemcpy2DAsync(out.X_final, sizeof(float) * p, X + f0 * ldx,
                                    sizeof(float) * ldx, sizeof(float) * p, r,
                                    hipMemcpyDeviceToDevice, st));
    double total_iters = 0.0;
    std::vector<int32_t> stq((size_t)r);
    for (int64_t j = 0; j < r; ++j) {
      total_iters += it_h[f0 + j];
      stq[j] = st_h[f0 + j];
      if (out.f_per_start) out.f_per_start[j] = f_h[f0 + j];
      if (out.ev_per_start) out.ev_per_start[j] = ev_h[f0 + j];
      if (out.phi_per_start) out.phi_per_start[j] = phi_h[f0 + j];
      if (out.iters_per_start) out.iters_per_start[j] = it_h[f0 + j];
      if (out.status_per_start) out.status_per_start[j] = st_h[f0 + j];
      if (out.nnz_per_start) out.nnz_per_start[j] = nnz_h[f0 + j];
    }
    spca_result* res = out.res;
    *res = spca_result{};
    res->objective = f_h[f0 + jb];
    res->objective_pre_polish = res->objective;
    res->explained_var = ev_h[f0 + jb];
    res->phi = phi_h[f0 + jb];
    res->iters_x_starts = total_iters;
    res->best_start = jb;
    res->nnz = nnzb;
    res->iters = it_h[f0 + jb];
    res->status = st_h[f0 + jb];
    res->warning = solve_warning(stq, r, o.tol);
  }
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  return SPCA_OK;
}

}  // extern "C"
