// Continuous-batching serving loop behind flr_server_* (include/flr.h).
//
// Requests wait in a FIFO.  A dispatcher admits the oldest request whose
// problem is idle as soon as a slot is free and the device bytes of the
// problems in flight plus its own stay within the budget; a request that
// does not fit blocks the ones behind it, so large requests are not starved.
// Each slot is a worker thread driving its problem's own stream, so requests
// that arrive while others run are admitted as slots free up and their
// kernels overlap on the GPU.  A result depends only on its own problem's
// buffers and fixed reduction trees, so it is the same alone and in the mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/flr.h"

namespace flr {
flr_status solve_locked(flr_problem h, double l1, double l2, double tol, const flr_solve_opts* o, double* beta_out,
                        flr_result* res);
std::mutex& problem_mutex(flr_problem h);
size_t problem_footprint(flr_problem h);
int problem_device(flr_problem h);
void set_last_error(const std::string& s);
}  // namespace flr

struct flr_ctx_s;

namespace {
struct Request {
  uint64_t ticket = 0;
  flr_problem h = nullptr;
  double l1 = 0, l2 = 0, tol = 0;
  flr_solve_opts opts{};
  bool has_opts = false;
  size_t bytes = 0;
  std::chrono::steady_clock::time_point t_submit;
};
struct Done {
  flr_status st = FLR_OK;
  flr_result res{};
  std::vector<double> beta;
};
}  // namespace

struct flr_server_s {
  size_t budget = 0;
  int slots = 1;
  std::mutex mu;
  std::condition_variable cv;       // dispatcher / workers wake-up
  std::condition_variable done_cv;  // pollers
  std::deque<Request> queue;
  std::map<uint64_t, Done> done;
  std::map<uint64_t, int> state;  // 0 queued, 1 running, 2 done
  std::map<flr_problem, int> busy;
  size_t in_use = 0;
  int running = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  std::deque<Request> ready;  // admitted, waiting for a worker
};

static void worker_loop(flr_server s) {
  for (;;) {
    Request rq;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop) return;
        // admission: oldest request that fits; an oversized head blocks the rest
        if (!s->ready.empty()) break;
        bool admitted = false;
        for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
          if (s->busy[it->h]) continue;
          if (s->running >= s->slots) break;
          if (s->in_use + it->bytes > s->budget && s->running > 0) break;
          s->in_use += it->bytes;
          s->running += 1;
          s->busy[it->h] = 1;
          s->state[it->ticket] = 1;
          s->ready.push_back(*it);
          s->queue.erase(it);
          admitted = true;
          break;
        }
        if (admitted) break;
        s->cv.wait(lk);
      }
      rq = s->ready.front();
      s->ready.pop_front();
    }
    Done d;
    d.beta.resize((size_t)flr_problem_p(rq.h));
    {
      std::lock_guard<std::mutex> pl(flr::problem_mutex(rq.h));
      d.st = flr::solve_locked(rq.h, rq.l1, rq.l2, rq.tol, rq.has_opts ? &rq.opts : nullptr, d.beta.data(), &d.res);
    }
    d.res.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - rq.t_submit).count();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->in_use -= rq.bytes;
      s->running -= 1;
      s->busy[rq.h] = 0;
      s->state[rq.ticket] = 2;
      s->done[rq.ticket] = std::move(d);
    }
    s->cv.notify_all();
    s->done_cv.notify_all();
  }
}

extern "C" {

flr_status flr_server_create(flr_ctx ctx, size_t hbm_budget_bytes, int32_t max_slots, flr_server* out) {
  if (!ctx || !out || max_slots < 1 || hbm_budget_bytes == 0) {
    flr::set_last_error("flr_server_create: need a context, a budget > 0 and max_slots >= 1");
    return FLR_ERR_INVALID_ARG;
  }
  flr_server s = new flr_server_s;
  s->budget = hbm_budget_bytes;
  s->slots = max_slots;
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker_loop, s);
  *out = s;
  return FLR_OK;
}

flr_status flr_server_submit(flr_server s, flr_problem h, double l1, double l2, double tol, const flr_solve_opts* opts,
                             uint64_t* ticket) {
  if (!s || !h || !ticket) {
    flr::set_last_error("flr_server_submit: NULL argument");
    return FLR_ERR_INVALID_ARG;
  }
  if (!(l1 >= 0.0) || !(l2 >= 0.0) || !(tol > 0.0)) {
    flr::set_last_error("flr_server_submit: lambda must be >= 0 and tol > 0");
    return FLR_ERR_INVALID_ARG;
  }
  Request rq;
  rq.h = h;
  rq.l1 = l1;
  rq.l2 = l2;
  rq.tol = tol;
  if (opts) {
    rq.opts = *opts;
    rq.has_opts = true;
    rq.opts.warm_start = nullptr;  // a caller buffer may not outlive the call; use_last still applies
  }
  rq.bytes = flr::problem_footprint(h);
  if (rq.bytes > s->budget) {
    flr::set_last_error("flr_server_submit: problem footprint exceeds the server budget");
    return FLR_ERR_BUSY;
  }
  rq.t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rq.ticket = s->next_ticket++;
    s->state[rq.ticket] = 0;
    s->queue.push_back(rq);
  }
  s->cv.notify_all();
  *ticket = rq.ticket;
  return FLR_OK;
}

flr_status flr_server_poll(flr_server s, uint64_t ticket, int blocking, double* beta_out_host, flr_result* res) {
  if (!s) return FLR_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto st = s->state.find(ticket);
  if (st == s->state.end()) {
    flr::set_last_error("flr_server_poll: unknown ticket");
    return FLR_ERR_INVALID_ARG;
  }
  if (st->second != 2) {
    if (!blocking) return FLR_ERR_NOT_READY;
    s->done_cv.wait(lk, [&] { return s->state[ticket] == 2; });
  }
  Done d = std::move(s->done[ticket]);
  s->done.erase(ticket);
  s->state.erase(ticket);
  lk.unlock();
  if (beta_out_host) std::copy(d.beta.begin(), d.beta.end(), beta_out_host);
  if (res) *res = d.res;
  return d.st;
}

flr_status flr_server_stats(flr_server s, int32_t* queued, int32_t* running, size_t* bytes_in_use) {
  if (!s) return FLR_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int32_t)(s->queue.size() + s->ready.size());
  if (running) *running = s->running;
  if (bytes_in_use) *bytes_in_use = s->in_use;
  return FLR_OK;
}

void flr_server_destroy(flr_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  delete s;
}

}  // extern "C"
