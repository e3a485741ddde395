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
// A result depends only on its request: every kernel of the solve is
// deterministic and each solve runs on its own workspace.
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

// Parts of a request's block, in order.
struct Footprint {
  size_t a, uv, x0, gamma, ws, total;
  int64_t lda;
};

Footprint footprint_of(const spca_request* q) {
  Footprint f{};
  const bool gen = q->A == nullptr;
  f.lda = gen ? round_up(q->n, 4) : q->lda;
  f.a = gen ? align_up(sizeof(float) * (size_t)f.lda * q->p) : 0;
  f.uv = gen && q->k > 0 ? align_up(sizeof(double) * (size_t)q->k * (q->n + q->p)) : 0;
  f.x0 = align_up(sizeof(float) * (size_t)q->r * q->p);
  f.gamma = kAlign;
  f.ws = align_up(spca_workspace_bytes(q->n, q->p, q->r, q->precision));
  f.total = f.a + f.uv + f.x0 + f.gamma + f.ws;
  return f;
}

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
};

namespace {

// runs one admitted request on the worker's stream and context
int run_job(spca_server* srv, Job& job, size_t off, hipStream_t st, spca_ctx* ctx,
            spca_completion* c) {
  const spca_request& q = job.q;
  const Footprint& f = job.fp;
  char* blk = srv->base + off;
  float* A = q.A ? const_cast<float*>(q.A) : (float*)blk;
  const int64_t lda = f.lda;
  double* Ud = (double*)(blk + f.a);
  double* Vd = Ud + (size_t)q.k * q.n;
  float* X0 = (float*)(blk + f.a + f.uv);
  unsigned long long* gbits = (unsigned long long*)(blk + f.a + f.uv + f.x0);
  void* ws = blk + f.a + f.uv + f.x0 + f.gamma;
  int rc;
  if (q.A == nullptr) {
    if (q.k > 0) {
      SPCA_HIP_TRY(hipMemcpyAsync(Ud, job.U.data(), sizeof(double) * q.k * q.n,
                                  hipMemcpyHostToDevice, st));
      SPCA_HIP_TRY(hipMemcpyAsync(Vd, job.V.data(), sizeof(double) * q.k * q.p,
                                  hipMemcpyHostToDevice, st));
    }
    rc = spca_generate_spiked(st, q.seed, q.n, q.p, A, lda, q.k,
                              job.thetas.data(), Ud, q.n, Vd, q.p);
    if (rc != SPCA_OK) return rc;
  }
  // starts: r rows of p entries from the same counter generator
  rc = spca_generate_spiked(st, q.start_seed, q.p, q.r, X0, q.p, 0, nullptr,
                            nullptr, 0, nullptr, 0);
  if (rc != SPCA_OK) return rc;
  double param = q.s_or_gamma;
  if (q.gamma_rel > 0.0 && q.formulation >= 5) {
    SPCA_HIP_TRY(hipMemsetAsync(gbits, 0, sizeof(unsigned long long), st));
    const unsigned g = (unsigned)(q.p < 4096 ? q.p : 4096);
    hipLaunchKernelGGL(col_sq_max_kernel, dim3(g), dim3(256), 0, st, A, lda, q.n,
                       q.p, gbits);
    SPCA_LAUNCH_CHECK("column norms");
    unsigned long long hb = 0;
    SPCA_HIP_TRY(hipMemcpyAsync(&hb, gbits, sizeof(hb), hipMemcpyDeviceToHost, st));
    SPCA_HIP_TRY(hipStreamSynchronize(st));
    double m2;
    std::memcpy(&m2, &hb, sizeof(m2));
    param = q.gamma_rel * sqrt(m2);
  }
  c->s_or_gamma = param;
  // inputs are ready: what follows is the solve alone
  SPCA_HIP_TRY(hipStreamSynchronize(st));
  c->t_solve = now_s();
  rc = spca_ctx_set_workspace(ctx, ws, f.ws);
  if (rc != SPCA_OK) return rc;
  spca_problem prob{A, q.n, q.p, lda, q.formulation, param};
  spca_solve_opts opts{X0, q.r, q.tol, q.maxit, q.precision, q.polish_maxit,
                       q.check_every > 0 ? q.check_every : 8, q.flags};
  spca_outputs out{};
  out.x = q.x_out;
  out.support = q.support_out;
  out.res = &c->res;
  return spca_am_solve_ex(ctx, st, &prob, &opts, &out);
}

void worker_main(spca_server* srv) {
  (void)hipSetDevice(srv->device);
  hipStream_t st = nullptr;
  spca_ctx* ctx = nullptr;
  const bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
                  spca_ctx_create(&ctx, srv->device, 0) == SPCA_OK;
  for (;;) {
    Job job;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lock(srv->mu);
      // admission in arrival order: the head request waits for memory
      srv->cv_work.wait(lock, [&] {
        return (srv->stop && srv->queue.empty()) ||
               (!srv->queue.empty() &&
                srv->arena->alloc(srv->queue.front().fp.total, &off));
      });
      if (srv->queue.empty()) break;
      job = std::move(srv->queue.front());
      srv->queue.pop_front();
      srv->in_use += align_up(job.fp.total);
      srv->peak_in_use = std::max(srv->peak_in_use, srv->in_use);
      ++srv->running;
      srv->peak_running = std::max(srv->peak_running, srv->running);
    }
    spca_completion c{};
    c.id = job.id;
    c.t_submit = job.t_submit;
    c.t_admit = now_s();
    c.footprint = job.fp.total;
    c.rc = ok ? run_job(srv, job, off, st, ctx, &c) : SPCA_EHIP;
    if (c.rc != SPCA_OK) {
      std::strncpy(c.error, spca_last_error(), sizeof(c.error) - 1);
      (void)hipStreamSynchronize(st);
    }
    c.t_done = now_s();
    {
      std::lock_guard<std::mutex> lock(srv->mu);
      srv->arena->release(off, job.fp.total);
      srv->in_use -= align_up(job.fp.total);
      --srv->running;
      ++srv->completed;
      srv->done.push_back(c);
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
  return footprint_of(q).total;
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
  job.fp = footprint_of(q);
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
