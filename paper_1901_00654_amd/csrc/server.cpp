// Serving loop declared in include/tsmg.h: a queue of independent smoothing
// requests, admitted by their estimated peak device memory (shortest
// estimated work first, or first in first out) and solved by worker threads
// that each own a HIP stream, so the
// kernels of concurrent requests overlap on the GPU. A request's points,
// hierarchy and solver vectors live on the device from admission to the end
// of its solve; its solution then waits in host memory for ts_server_wait.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "api_util.h"
#include "problem.h"

namespace tsmg {

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int d = 0;
  int32_t intervals[kMaxDim] = {};
  double lo[kMaxDim] = {}, hi[kMaxDim] = {};
  int64_t n = 0;
  std::vector<double> x, y;   // host copies, released once on the device
  double lam = 0.0;
  ts_options opt{};
  int64_t K = 0;
  size_t footprint = 0;
  double work = 0.0;          // estimated cost of one operator apply (admission order)
  bool done = false;
  bool claimed = false;       // a thread is in ts_server_wait for it
  ts_result res{};
  std::vector<double> alpha;
};

void set_result_error(ts_result& r, ts_status code, const std::string& msg) {
  r.status = code;
  std::snprintf(r.error, sizeof(r.error), "%s", msg.c_str());
}

}  // namespace

struct Server {
  int device = 0;
  size_t budget = 0;
  int policy = TS_ADMIT_SHORTEST;
  double max_wait_s = 5.0;
  double stencil_budget = 0.0;
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_id = 1;
  bool stopping = false;
  size_t in_use = 0;
  int active = 0;
  ts_server_stats stats{};
  std::vector<std::thread> workers;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // The queued request a free worker admits next (queue.end(): none yet).
  // FIFO: the oldest, once it fits in what the memory budget has left (it
  // holds back the ones behind it). Shortest first: the oldest request that
  // has waited max_wait_s and fits, else the fitting request with the least
  // estimated work per operator apply (ties: the older), so that short
  // requests are not held behind long ones and none waits indefinitely.
  std::deque<Request*>::iterator choose() {
    if (queue.empty()) return queue.end();
    if (policy == TS_ADMIT_FIFO)
      return in_use + queue.front()->footprint <= budget ? queue.begin() : queue.end();
    const double t = now();
    auto best = queue.end();
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      Request* q = *it;
      if (in_use + q->footprint > budget) continue;
      if (t - q->res.t_submit >= max_wait_s) return it;   // the oldest overdue one
      if (best == queue.end() || q->work < (*best)->work) best = it;
    }
    return best;
  }

  void worker() {
    hipStream_t st = nullptr;
    std::string init_error;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      st = nullptr;
      init_error = "worker could not set up its device stream";
    }
    for (;;) {
      Request* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        std::deque<Request*>::iterator pick;
        cv_work.wait(lk, [&] {
          pick = choose();
          return pick != queue.end() || (stopping && queue.empty());
        });
        if (queue.empty()) break;   // stopping and drained
        r = *pick;
        queue.erase(pick);
        in_use += r->footprint;
        ++active;
        stats.max_active = std::max(stats.max_active, active);
        stats.max_in_use = std::max(stats.max_in_use, in_use);
        r->res.t_start = now();
      }
      if (st) run(r, st);
      else set_result_error(r->res, TS_EDEVICE, init_error);
      {
        std::lock_guard<std::mutex> lk(mu);
        in_use -= r->footprint;
        --active;
        r->res.t_done = now();
        r->done = true;
        if (r->res.status < 0) ++stats.failed;
        else ++stats.completed;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
  }

  // Setup and solve of one request on stream st (ts_create + ts_solve from a
  // zero start), then the solution to host memory.
  void run(Request* r, hipStream_t st) {
    try {
      const int64_t xy_bytes = r->n * (r->d + 1) * int64_t(sizeof(double));
      std::unique_ptr<Problem> P;
      {
        DevBuf<double> xd, yd;
        xd.alloc(size_t(r->n) * r->d);
        yd.alloc(size_t(r->n));
        hip_check(hipMemcpyAsync(xd.p, r->x.data(), size_t(r->n) * r->d * sizeof(double), hipMemcpyHostToDevice, st),
                  "upload x");
        hip_check(hipMemcpyAsync(yd.p, r->y.data(), size_t(r->n) * sizeof(double), hipMemcpyHostToDevice, st),
                  "upload y");
        ts_options o = r->opt;
        o.stream = st;
        P.reset(create_problem(r->d, kDeg, r->intervals, r->lo, r->hi, r->n, xd.p, yd.p, r->lam, &o, stencil_budget));
      }   // create_problem synchronised the stream: the device copies of x, y can go
      std::vector<double>().swap(r->x);
      std::vector<double>().swap(r->y);
      DevBuf<double> alpha;
      alpha.alloc(size_t(r->K));
      ts_solve_info info{};
      const ts_status s = solve(P.get(), alpha.p, 0, &info);
      r->alpha.resize(size_t(r->K));
      hip_check(hipMemcpyAsync(r->alpha.data(), alpha.p, size_t(r->K) * sizeof(double), hipMemcpyDeviceToHost, st),
                "download");
      hip_check(hipStreamSynchronize(st), "sync");
      r->res.status = s;
      r->res.info = info;
      r->res.peak_bytes = size_t(P->mem_peak + xy_bytes);
    } catch (const Error& e) {
      set_result_error(r->res, e.code, e.msg);
    } catch (const std::exception& e) {
      set_result_error(r->res, TS_EDEVICE, e.what());
    } catch (...) {
      set_result_error(r->res, TS_EDEVICE, "unknown internal error");
    }
  }
};

}  // namespace tsmg

struct ts_server {
  tsmg::Server impl;
};

namespace {

void need(bool ok, const char* msg) {
  if (!ok) throw tsmg::Error{TS_EINVAL, msg};
}

}  // namespace

extern "C" {

void ts_server_default_options(ts_server_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->memory_budget = 0;
  o->slots = 4;
  o->policy = TS_ADMIT_SHORTEST;
  o->max_wait_s = 5.0;
}

ts_status ts_server_create(const ts_server_options* opt, ts_server** out) {
  TS_API_BEGIN
  need(out != nullptr, "out must not be null");
  *out = nullptr;
  ts_server_options o;
  ts_server_default_options(&o);
  if (opt) o = *opt;
  need(o.slots >= 1 && o.slots <= 64, "slots must be in 1..64");
  need(o.policy == TS_ADMIT_FIFO || o.policy == TS_ADMIT_SHORTEST, "unknown admission policy");
  need(o.max_wait_s >= 0.0, "max_wait_s must be >= 0");
  std::unique_ptr<ts_server> s(new ts_server());
  tsmg::Server& S = s->impl;
  tsmg::hip_check(hipGetDevice(&S.device), "hipGetDevice");
  size_t free_b = 0, total_b = 0;
  tsmg::hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
  S.budget = o.memory_budget ? o.memory_budget : free_b / 2;
  S.policy = o.policy;
  S.max_wait_s = o.max_wait_s;
  // per-level stencil cap of every request: a quarter of the budget, at most 16 GB
  S.stencil_budget = std::min(16e9, 0.25 * double(S.budget));
  S.stats.memory_budget = S.budget;
  S.t0 = tsmg::Clock::now();
  try {
    for (int i = 0; i < o.slots; ++i) S.workers.emplace_back([&S] { S.worker(); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S.mu);
      S.stopping = true;
    }
    S.cv_work.notify_all();
    for (auto& t : S.workers) t.join();
    throw;
  }
  *out = s.release();
  return TS_OK;
  TS_API_END
}

ts_status ts_server_submit(ts_server* s, const ts_request* q, uint64_t* ticket) {
  TS_API_BEGIN
  need(s != nullptr && q != nullptr && ticket != nullptr, "null argument");
  tsmg::Server& S = s->impl;
  need(q->q == 3, "only cubic splines (q = 3) are supported");
  need(q->d >= 1 && q->d <= tsmg::kMaxDim, "d must be in 1..5");
  need(q->intervals && q->lo && q->hi && q->x && q->y, "null array in request");
  need(q->n >= 1, "n must be >= 1");
  need(q->lambda > 0.0 && std::isfinite(q->lambda), "lambda must be finite and > 0");
  const int d = q->d, N = q->intervals[0];
  need(N >= 2 && (N & (N - 1)) == 0, "intervals must be a power of two >= 2");
  int G = 0;
  while ((1 << G) < N) ++G;
  need(int64_t(G) * d <= 30, "N^d must not exceed 2^30 cells");
  std::unique_ptr<tsmg::Request> r(new tsmg::Request());
  r->d = d;
  r->K = 1;
  for (int p = 0; p < d; ++p) {
    need(q->intervals[p] == N, "all dimensions must have the same number of intervals");
    need(q->lo[p] < q->hi[p] && std::isfinite(q->lo[p]) && std::isfinite(q->hi[p]),
         "box must satisfy lo < hi with finite bounds");
    r->intervals[p] = q->intervals[p];
    r->lo[p] = q->lo[p];
    r->hi[p] = q->hi[p];
    r->K *= N + tsmg::kDeg;
  }
  need(r->K < 2147483647LL, "(N+3)^d must be < 2^31");
  ts_default_options(&r->opt);
  if (q->opt) r->opt = *q->opt;
  r->opt.stream = nullptr;
  need(tsmg::precision_available(r->opt.precision), "unknown or unavailable precision");
  need(r->opt.tol > 0.0, "tol must be > 0");
  r->n = q->n;
  r->lam = q->lambda;
  r->footprint = size_t(tsmg::footprint_bytes(d, N, q->n, r->opt, S.stencil_budget) +
                        q->n * (d + 1) * int64_t(sizeof(double)) + r->K * int64_t(sizeof(double)));
  r->res.footprint = r->footprint;
  {   // points x patch entries plus coefficients x stencil entries
    double patch = 1.0, stencil = 1.0;
    for (int p = 0; p < d; ++p) { patch *= 4.0; stencil *= 7.0; }
    r->work = double(q->n) * patch + double(r->K) * stencil;
  }
  r->res.K = r->K;
  if (r->footprint > S.budget)
    throw tsmg::Error{TS_ENOMEM, "request needs about " + std::to_string(r->footprint) +
                                     " bytes of device memory, more than the server budget of " +
                                     std::to_string(S.budget)};
  r->x.assign(q->x, q->x + size_t(q->n) * d);
  r->y.assign(q->y, q->y + size_t(q->n));
  {
    std::lock_guard<std::mutex> lk(S.mu);
    need(!S.stopping, "server is shutting down");
    const uint64_t id = S.next_id++;
    r->res.t_submit = S.now();
    S.queue.push_back(r.get());
    S.reqs.emplace(id, std::move(r));
    ++S.stats.submitted;
    *ticket = id;
  }
  S.cv_work.notify_one();
  return TS_OK;
  TS_API_END
}

ts_status ts_server_poll(ts_server* s, uint64_t ticket, int* done) {
  TS_API_BEGIN
  need(s != nullptr && done != nullptr, "null argument");
  tsmg::Server& S = s->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.reqs.find(ticket);
  need(it != S.reqs.end(), "unknown or released ticket");
  *done = it->second->done ? 1 : 0;
  return TS_OK;
  TS_API_END
}

ts_status ts_server_wait(ts_server* s, uint64_t ticket, double* alpha, int64_t capacity, ts_result* result) {
  TS_API_BEGIN
  need(s != nullptr, "null server");
  tsmg::Server& S = s->impl;
  std::unique_lock<std::mutex> lk(S.mu);
  auto it = S.reqs.find(ticket);
  need(it != S.reqs.end(), "unknown or released ticket");
  tsmg::Request* r = it->second.get();
  // one waiter per ticket: the waiter that claims it is the only one that
  // releases it, so no other thread can hold a pointer to it afterwards
  need(!r->claimed, "ticket is already being waited for by another thread");
  need(!(alpha && capacity < r->K), "alpha buffer is smaller than K");
  r->claimed = true;
  S.cv_done.wait(lk, [&] { return r->done; });
  if (alpha && r->res.status >= 0) std::memcpy(alpha, r->alpha.data(), size_t(r->K) * sizeof(double));
  if (result) *result = r->res;
  S.reqs.erase(S.reqs.find(ticket));
  return TS_OK;
  TS_API_END
}

ts_status ts_server_get_stats(ts_server* s, ts_server_stats* out) {
  TS_API_BEGIN
  need(s != nullptr && out != nullptr, "null argument");
  tsmg::Server& S = s->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  *out = S.stats;
  out->queued = int64_t(S.queue.size());
  out->active = S.active;
  out->in_use = S.in_use;
  return TS_OK;
  TS_API_END
}

void ts_server_destroy(ts_server* s) {
  if (!s) return;
  tsmg::Server& S = s->impl;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stopping = true;
  }
  S.cv_work.notify_all();
  for (auto& t : S.workers)
    if (t.joinable()) t.join();
  delete s;
}

}  // extern "C"
