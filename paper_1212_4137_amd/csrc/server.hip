// Request server: continuous batching of independent sparse PCA solves on
// one GPU.  Requests of any shape, formulation and precision queue in
// arrival order; a request is admitted as soon as a worker is free and its
// HBM footprint (its A when the server generates it, its starts, the spike
// factors and the solve workspace) fits in what is left of the server's
// arena.  Each worker owns a stream and a context, so admitted requests run
// concurrently on the device, and a finished request's memory and worker go
// to the next one at once.  The arena is one device allocation made when
// the server starts; requests take first-fit blocks of it, so serving never
// calls the device allocator (whose release synchronizes the device).
// Small FP32 requests (p <= SPCA_GROUP_MAX_P and n p r at most kGroupWork)
// are served in groups: a worker that admits such a request also admits the
// small requests queued right behind it (up to kGroupMax of them, as far as
// the arena allows) and iterates them together with spca_am_solve_group, so
// that every kernel launch of an iteration serves all of them.  A small
// request always takes that path, also alone.
// A result depends only on its request: every kernel of the solve is
// deterministic, each solve runs on its own workspace, and a grouped
// request gives the same bits in any group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/spca.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spca {
namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, cap) with coalescing of free neighbours.
class Arena {
 public:
  explicit Arena(size_t cap) : cap_(cap) {
    if (cap > 0) free_[0] = cap;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t roff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t cap() const { return cap_; }

 private:
  size_t cap_;
  std::map<size_t, size_t> free_;
};

constexpr int kGroupMax = 32;           // requests per group
constexpr int64_t kGroupStarts = 4096;  // starts per group
constexpr double kGroupWork = 5.4e8;    // n p r of a request served in groups

// Served in groups: FP32, rows short enough for the grouped x-update, small
// products, no flag beyond SPCA_FLAG_GRAPH, and arguments the solve accepts
// (a request that fails its checks runs alone and reports the error).
bool groupable(const spca_request* q) {
  if (q->precision != SPCA_PREC_FP32 || q->p > SPCA_GROUP_MAX_P) return false;
  if ((double)q->n * (double)q->p * (double)q->r > kGroupWork) return false;
  if ((q->flags & ~SPCA_FLAG_GRAPH) != 0 || q->check_every < 0) return false;
  const double par = q->gamma_rel > 0.0 && q->formulation >= 5 ? 0.0 : q->s_or_gamma;
  const int64_t lda = q->A ? q->lda : round_up(q->n, 4);
  return check_problem(q->n, q->p, lda, q->formulation, par, q->r, q->tol, q->maxit) == SPCA_OK;
}

// Parts of a request's block, in order.  A grouped request's block holds
// no workspace (ws = 0); its group's workspace is a block of its own, and
// `group_ws` is that of the request alone (what admission needs at least).
struct Footprint {
  size_t a, uv, x0, gamma, ws, total;
  size_t group_ws;
  int64_t lda;
  bool grouped;
};

// The grouped-solve arguments of a request whose A and starts sit at the
// given device addresses (the sizes are what spca_group_workspace_bytes
// reads; the pointers only decide whether A needs an aligned copy).
void group_args(const spca_request* q, int64_t lda, const float* A, const float* X0,
                double param, spca_problem* pr, spca_solve_opts* o) {
  *pr = spca_problem{A, q->n, q->p, lda, q->formulation, param};
  *o = spca_solve_opts{};
  o->X0 = X0;
  o->r = q->r;
  o->tol = q->tol;
  o->maxit = q->maxit;
  o->precision = SPCA_PREC_FP32;
  o->check_every = q->check_every > 0 ? q->check_every : 8;
}

Footprint footprint_of(const spca_request* q, bool grouping) {
  Footprint f{};
  const bool gen = q->A == nullptr;
  f.lda = gen ? round_up(q->n, 4) : q->lda;
  f.a = gen ? align_up(sizeof(float) * (size_t)f.lda * q->p) : 0;
  f.uv = gen && q->k > 0 ? align_up(sizeof(double) * (size_t)q->k * (q->n + q->p)) : 0;
  f.x0 = align_up(sizeof(float) * (size_t)q->r * q->p);
  f.gamma = kAlign;
  f.grouped = grouping && groupable(q);
  if (f.grouped) {
    spca_problem pr;
    spca_solve_opts o;
    group_args(q, f.lda, q->A ? q->A : (const float*)kAlign, (const float*)kAlign, 1.0, &pr, &o);
    f.group_ws = align_up(spca_group_workspace_bytes(1, &pr, &o));
    f.ws = 0;
    f.total = f.a + f.uv + f.x0 + f.gamma + f.group_ws;
  } else {
    f.ws = align_up(spca_workspace_bytes(q->n, q->p, q->r, q->precision));
    f.total = f.a + f.uv + f.x0 + f.gamma + f.ws;
  }
  return f;
}

// the request's own block (A, spike factors, starts, gamma, workspace of an
// ungrouped solve)
size_t block_of(const Footprint& f) { return f.a + f.uv + f.x0 + f.gamma + f.ws; }

// max_i ||a_i||_2^2 over the columns (non-negative doubles order like their
// bit patterns, so an integer max gives the exact result in any order)
__global__ __launch_bounds__(256) void col_sq_max_kernel(
    const float* __restrict__ A, int64_t lda, int64_t n, int64_t p,
    unsigned long long* out) {
  __shared__ double red[8];
  for (int64_t k = blockIdx.x; k < p; k += gridDim.x) {
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
      const double a = A[i + k * lda];
      acc += a * a;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(acc));
  }
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Job {
  int64_t id;
  spca_request q;
  std::vector<double> thetas, U, V;
  Footprint fp;
  double t_submit;
};

}  // namespace
}  // namespace spca

using namespace spca;

struct spca_server {
  int device = 0;
  char* base = nullptr;
  Arena* arena = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job> queue;
  std::deque<spca_completion> done;
  std::vector<std::thread> workers;
  bool stop = false;
  int64_t next_id = 0;
  size_t in_use = 0, peak_in_use = 0;
  int32_t running = 0, peak_running = 0;
  int64_t completed = 0;
  int32_t group_limit = kGroupMax;  // requests per group; 0: no groups
};

namespace {

// Generates an admitted request's inputs in its block (A when the server
// generates it, the starts, gamma) on the worker's stream; the caller
// synchronizes.  A and X0 of the solve and its parameter are returned.
int prepare_job(spca_server* srv, Job& job, size_t off, hipStream_t st, const float** A_out,
                float** X0_out, double* param_out, bool* param_ready) {
  const spca_request& q = job.q;
  const Footprint& f = job.fp;
  char* blk = srv->base + off;
  float* A = q.A ? const_cast<float*>(q.A) : (float*)blk;
  double* Ud = (double*)(blk + f.a);
  double* Vd = Ud + (size_t)q.k * q.n;
  float* X0 = (float*)(blk + f.a + f.uv);
  unsigned long long* gbits = (unsigned long long*)(blk + f.a + f.uv + f.x0);
  int rc;
  if (q.A == nullptr) {
    if (q.k > 0) {
      SPCA_HIP_TRY(hipMemcpyAsync(Ud, job.U.data(), sizeof(double) * q.k * q.n,
                                  hipMemcpyHostToDevice, st));
      SPCA_HIP_TRY(hipMemcpyAsync(Vd, job.V.data(), sizeof(double) * q.k * q.p,
                                  hipMemcpyHostToDevice, st));
    }
    rc = spca_generate_spiked(st, q.seed, q.n, q.p, A, f.lda, q.k,
                              job.thetas.data(), Ud, q.n, Vd, q.p);
    if (rc != SPCA_OK) return rc;
  }
  // starts: r rows of p entries from the same counter generator
  rc = spca_generate_spiked(st, q.start_seed, q.p, q.r, X0, q.p, 0, nullptr,
                            nullptr, 0, nullptr, 0);
  if (rc != SPCA_OK) return rc;
  *param_out = q.s_or_gamma;
  *param_ready = true;
  if (q.gamma_rel > 0.0 && q.formulation >= 5) {
    // gamma = gamma_rel max_i ||a_i||_2, read back once the inputs are ready
    SPCA_HIP_TRY(hipMemsetAsync(gbits, 0, sizeof(unsigned long long), st));
    const unsigned g = (unsigned)(q.p < 4096 ? q.p : 4096);
    hipLaunchKernelGGL(col_sq_max_kernel, dim3(g), dim3(256), 0, st, A, f.lda, q.n,
                       q.p, gbits);
    SPCA_LAUNCH_CHECK("column norms");
    *param_ready = false;
  }
  *A_out = A;
  *X0_out = X0;
  return SPCA_OK;
}

// gamma from the column norms prepare_job left in the request's block (the
// stream has been synchronized)
double gamma_of(spca_server* srv, const Job& job, size_t off, hipStream_t st) {
  const Footprint& f = job.fp;
  unsigned long long hb = 0;
  if (hipMemcpyAsync(&hb, srv->base + off + f.a + f.uv + f.x0, sizeof(hb),
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return NAN;  // the solve then rejects gamma
  double m2;
  std::memcpy(&m2, &hb, sizeof(m2));
  return job.q.gamma_rel * sqrt(m2);
}

// runs one admitted request on the worker's stream and context
int run_job(spca_server* srv, Job& job, size_t off, hipStream_t st, spca_ctx* ctx,
            spca_completion* c) {
  const spca_request& q = job.q;
  const Footprint& f = job.fp;
  const float* A = nullptr;
  float* X0 = nullptr;
  double param = 0.0;
  bool ready = false;
  int rc = prepare_job(srv, job, off, st, &A, &X0, &param, &ready);
  if (rc != SPCA_OK) return rc;
  // inputs are ready: what follows is the solve alone
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  if (!ready) param = gamma_of(srv, job, off, st);
  c->s_or_gamma = param;
  c->t_solve = now_s();
  void* ws = srv->base + off + f.a + f.uv + f.x0 + f.gamma;
  rc = spca_ctx_set_workspace(ctx, ws, f.ws);
  if (rc != SPCA_OK) return rc;
  spca_problem prob{A, q.n, q.p, f.lda, q.formulation, param};
  spca_solve_opts opts{X0, q.r, q.tol, q.maxit, q.precision, q.polish_maxit,
                       q.check_every > 0 ? q.check_every : 8, q.flags};
  spca_outputs out{};
  out.x = q.x_out;
  out.support = q.support_out;
  out.res = &c->res;
  return spca_am_solve_ex(ctx, st, &prob, &opts, &out);
}

// Requests admitted together: one ungrouped request, or a group.
struct Batch {
  std::vector<Job> jobs;
  std::vector<size_t> offs;
  size_t ws_off = 0, ws_bytes = 0;
  bool group = false;
};

// Admits the queue head if memory allows, and with a grouped head also the
// grouped requests queued right behind it (as many as the limits and the
// arena allow); called with srv->mu held.  false: nothing admitted.
bool admit(spca_server* srv, Batch* b) {
  if (srv->queue.empty()) return false;
  if (!srv->queue.front().fp.grouped) {
    size_t off = 0;
    if (!srv->arena->alloc(srv->queue.front().fp.total, &off)) return false;
    b->offs.assign(1, off);
    b->jobs.push_back(std::move(srv->queue.front()));
    srv->queue.pop_front();
    b->group = false;
    return true;
  }
  std::vector<size_t> offs;
  std::vector<spca_problem> probs;
  std::vector<spca_solve_opts> opts;
  int64_t starts = 0;
  for (size_t k = 0; k < srv->queue.size() && (int)k < srv->group_limit; ++k) {
    const Job& j = srv->queue[k];
    if (!j.fp.grouped || starts + j.q.r > kGroupStarts) break;
    size_t off = 0;
    if (!srv->arena->alloc(block_of(j.fp), &off)) break;
    offs.push_back(off);
    spca_problem pr;
    spca_solve_opts o;
    group_args(&j.q, j.fp.lda, j.q.A ? j.q.A : (const float*)kAlign, (const float*)kAlign, 1.0,
               &pr, &o);
    probs.push_back(pr);
    opts.push_back(o);
    starts += j.q.r;
  }
  // the group's workspace; requests leave from the back until it fits
  while (!offs.empty()) {
    const size_t ws =
        align_up(spca_group_workspace_bytes((int32_t)offs.size(), probs.data(), opts.data()));
    size_t woff = 0;
    if (srv->arena->alloc(ws, &woff)) {
      b->ws_off = woff;
      b->ws_bytes = ws;
      break;
    }
    srv->arena->release(offs.back(), block_of(srv->queue[offs.size() - 1].fp));
    offs.pop_back();
    probs.pop_back();
    opts.pop_back();
  }
  if (offs.empty()) return false;
  for (size_t k = 0; k < offs.size(); ++k) {
    b->jobs.push_back(std::move(srv->queue.front()));
    srv->queue.pop_front();
  }
  b->offs = offs;
  b->group = true;
  return true;
}

size_t batch_bytes(const Batch& b) {
  if (!b.group) return align_up(b.jobs[0].fp.total);
  size_t t = b.ws_bytes;
  for (const Job& j : b.jobs) t += align_up(block_of(j.fp));
  return t;
}

void release_batch(spca_server* srv, const Batch& b) {
  if (!b.group) {
    srv->arena->release(b.offs[0], b.jobs[0].fp.total);
    return;
  }
  for (size_t k = 0; k < b.jobs.size(); ++k) srv->arena->release(b.offs[k], block_of(b.jobs[k].fp));
  srv->arena->release(b.ws_off, b.ws_bytes);
}

// runs an admitted group: inputs of every request, then one grouped solve;
// a request whose inputs fail is left out with its error
void run_group(spca_server* srv, Batch& b, hipStream_t st, spca_ctx* ctx,
               std::vector<spca_completion>& cs) {
  const size_t m = b.jobs.size();
  std::vector<const float*> As(m);
  std::vector<float*> X0s(m);
  std::vector<double> params(m);
  std::vector<char> ready(m), ok(m);
  for (size_t k = 0; k < m; ++k) {
    bool rdy = false;
    cs[k].rc = prepare_job(srv, b.jobs[k], b.offs[k], st, &As[k], &X0s[k], &params[k], &rdy);
    ready[k] = rdy;
    ok[k] = cs[k].rc == SPCA_OK;
    if (!ok[k]) std::strncpy(cs[k].error, spca_last_error(), sizeof(cs[k].error) - 1);
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    for (size_t k = 0; k < m; ++k) {
      cs[k].rc = SPCA_EHIP;
      std::strncpy(cs[k].error, "stream synchronization failed", sizeof(cs[k].error) - 1);
    }
    return;
  }
  std::vector<spca_problem> probs;
  std::vector<spca_solve_opts> opts;
  std::vector<spca_outputs> outs;
  std::vector<size_t> idx;
  const double t_solve = now_s();
  for (size_t k = 0; k < m; ++k) {
    if (!ok[k]) continue;
    if (!ready[k]) params[k] = gamma_of(srv, b.jobs[k], b.offs[k], st);
    cs[k].s_or_gamma = params[k];
    cs[k].t_solve = t_solve;
    const spca_request& q = b.jobs[k].q;
    spca_problem pr;
    spca_solve_opts o;
    group_args(&q, b.jobs[k].fp.lda, As[k], X0s[k], params[k], &pr, &o);
    spca_outputs out{};
    out.x = q.x_out;
    out.support = q.support_out;
    out.res = &cs[k].res;
    probs.push_back(pr);
    opts.push_back(o);
    outs.push_back(out);
    idx.push_back(k);
  }
  if (idx.empty()) return;
  int rc = spca_ctx_set_workspace(ctx, srv->base + b.ws_off, b.ws_bytes);
  if (rc == SPCA_OK)
    rc = spca_am_solve_group(ctx, st, (int32_t)idx.size(), probs.data(), opts.data(),
                             outs.data());
  if (rc != SPCA_OK) {
    for (size_t k : idx) {
      cs[k].rc = rc;
      std::strncpy(cs[k].error, spca_last_error(), sizeof(cs[k].error) - 1);
    }
    (void)hipStreamSynchronize(st);
  }
}

void worker_main(spca_server* srv) {
  (void)hipSetDevice(srv->device);
  hipStream_t st = nullptr;
  spca_ctx* ctx = nullptr;
  const bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
                  spca_ctx_create(&ctx, srv->device, 0) == SPCA_OK;
  for (;;) {
    Batch b;
    {
      std::unique_lock<std::mutex> lock(srv->mu);
      // admission in arrival order: the head request waits for memory
      srv->cv_work.wait(lock, [&] {
        return (srv->stop && srv->queue.empty()) || admit(srv, &b);
      });
      if (b.jobs.empty()) break;
      srv->in_use += batch_bytes(b);
      srv->peak_in_use = std::max(srv->peak_in_use, srv->in_use);
      srv->running += (int32_t)b.jobs.size();
      srv->peak_running = std::max(srv->peak_running, srv->running);
    }
    const double t_admit = now_s();
    std::vector<spca_completion> cs(b.jobs.size());
    for (size_t k = 0; k < b.jobs.size(); ++k) {
      cs[k] = spca_completion{};
      cs[k].id = b.jobs[k].id;
      cs[k].t_submit = b.jobs[k].t_submit;
      cs[k].t_admit = t_admit;
      cs[k].footprint = b.jobs[k].fp.total;
    }
    if (!ok) {
      for (auto& c : cs) c.rc = SPCA_EHIP;
    } else if (!b.group) {
      cs[0].rc = run_job(srv, b.jobs[0], b.offs[0], st, ctx, &cs[0]);
      if (cs[0].rc != SPCA_OK) {
        std::strncpy(cs[0].error, spca_last_error(), sizeof(cs[0].error) - 1);
        (void)hipStreamSynchronize(st);
      }
    } else {
      run_group(srv, b, st, ctx, cs);
    }
    const double t_done = now_s();
    for (auto& c : cs) c.t_done = t_done;
    {
      std::lock_guard<std::mutex> lock(srv->mu);
      release_batch(srv, b);
      srv->in_use -= batch_bytes(b);
      srv->running -= (int32_t)b.jobs.size();
      srv->completed += (int64_t)b.jobs.size();
      for (auto& c : cs) srv->done.push_back(c);
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
  }
  if (ctx) spca_ctx_destroy(ctx);
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

size_t spca_request_footprint(const spca_request* q) {
  if (q == nullptr || q->n < 1 || q->p < 1 || q->r < 1) return 0;
  return footprint_of(q, true).total;
}

int spca_server_create(spca_server** out, int device, size_t hbm_bytes,
                       int32_t workers) {
  SPCA_REQUIRE(out != nullptr, "server must not be NULL");
  SPCA_REQUIRE(hbm_bytes >= kAlign, "the arena needs at least 256 bytes");
  SPCA_REQUIRE(workers >= 1 && workers <= 64, "workers must be in 1..64");
  int ndev = 0;
  SPCA_HIP_TRY(hipGetDeviceCount(&ndev));
  SPCA_REQUIRE(device >= 0 && device < ndev, "device ordinal out of range");
  SPCA_HIP_TRY(hipSetDevice(device));
  spca_server* srv = new spca_server();
  srv->device = device;
  hipError_t e = hipMalloc((void**)&srv->base, hbm_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete srv;
    set_error(std::string("server arena hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SPCA_ENOMEM : SPCA_EHIP;
  }
  srv->arena = new Arena(hbm_bytes);
  for (int w = 0; w < workers; ++w) srv->workers.emplace_back(worker_main, srv);
  *out = srv;
  return SPCA_OK;
}

int spca_server_set_group_limit(spca_server* srv, int32_t max_requests) {
  SPCA_REQUIRE(srv != nullptr, "server must not be NULL");
  SPCA_REQUIRE(max_requests >= 0 && max_requests <= SPCA_GROUP_MAX_REQUESTS,
               "max_requests must be in 0..SPCA_GROUP_MAX_REQUESTS");
  std::lock_guard<std::mutex> lock(srv->mu);
  SPCA_REQUIRE(srv->queue.empty() && srv->running == 0,
               "the group limit is set while no request is queued or running");
  srv->group_limit = max_requests;
  return SPCA_OK;
}

int spca_server_submit(spca_server* srv, const spca_request* q, int64_t* id) {
  SPCA_REQUIRE(srv && q && id, "server, request and id must not be NULL");
  SPCA_REQUIRE(q->n >= 1 && q->p >= 1 && q->r >= 1, "n, p and r must be >= 1");
  SPCA_REQUIRE(q->A != nullptr || (q->k >= 0 && q->k <= 16),
               "a generated A takes 0..16 spikes");
  SPCA_REQUIRE(q->A == nullptr || q->lda >= q->n, "lda must be >= n");
  SPCA_REQUIRE(q->A != nullptr || q->k == 0 || (q->thetas && q->U && q->V),
               "spikes need thetas, U and V");
  Job job;
  job.q = *q;
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    job.fp = footprint_of(q, srv->group_limit > 0);
  }
  SPCA_REQUIRE(job.fp.total <= srv->arena->cap(),
               "request footprint exceeds the server's HBM arena");
  if (q->A == nullptr && q->k > 0) {
    job.thetas.assign(q->thetas, q->thetas + q->k);
    job.U.assign(q->U, q->U + (size_t)q->k * q->n);
    job.V.assign(q->V, q->V + (size_t)q->k * q->p);
  }
  job.q.thetas = job.q.U = job.q.V = nullptr;
  job.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    SPCA_REQUIRE(!srv->stop, "server is shutting down");
    job.id = srv->next_id++;
    *id = job.id;
    srv->queue.push_back(std::move(job));
  }
  srv->cv_work.notify_all();
  return SPCA_OK;
}

int spca_server_poll(spca_server* srv, spca_completion* out, int32_t max,
                     int32_t* count, int32_t wait_ms) {
  SPCA_REQUIRE(srv && count && (out || max == 0), "server, out and count must be set");
  std::unique_lock<std::mutex> lock(srv->mu);
  if (srv->done.empty() && wait_ms != 0) {
    auto ready = [&] { return !srv->done.empty(); };
    if (wait_ms < 0)
      srv->cv_done.wait(lock, ready);
    else
      srv->cv_done.wait_for(lock, std::chrono::milliseconds(wait_ms), ready);
  }
  int32_t k = 0;
  while (k < max && !srv->done.empty()) {
    out[k++] = srv->done.front();
    srv->done.pop_front();
  }
  *count = k;
  return SPCA_OK;
}

int spca_server_stats(spca_server* srv, spca_server_stats_t* s) {
  SPCA_REQUIRE(srv && s, "server and stats must not be NULL");
  std::lock_guard<std::mutex> lock(srv->mu);
  s->arena_bytes = srv->arena->cap();
  s->in_use_bytes = srv->in_use;
  s->peak_in_use_bytes = srv->peak_in_use;
  s->queued = (int64_t)srv->queue.size();
  s->running = srv->running;
  s->peak_running = srv->peak_running;
  s->completed = srv->completed;
  s->now = now_s();
  return SPCA_OK;
}

int spca_server_destroy(spca_server* srv) {
  if (srv == nullptr) return SPCA_OK;
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();
  (void)hipSetDevice(srv->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(srv->base);
  delete srv->arena;
  delete srv;
  return SPCA_OK;
}

}  // extern "C"
