// Host engine behind the C ABI of include/flr.h: problem residency, the
// captured launch rotation, the solve driver and the status plumbing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/flr.h"
#include "flr_band.h"
#include "flr_internal.h"
#include "flr_problem.h"

namespace flr {
hipError_t launch_rotation(const Dims& D, const Bufs& B, int par, int which, hipStream_t st, bool mixed);
hipError_t launch_setup(const Dims& D, const void* X, const double* y, double* cpart, double* spart, double* c,
                        double* s, hipStream_t st);
hipError_t launch_init(const Dims& D, const Bufs& B, const double* warm, int use_warm, hipStream_t st);
hipError_t launch_grouped(int dtype, bool mixed, const GroupEntry* e, int count, int wgs, int par, int which,
                          hipStream_t st);
hipError_t launch_gather_states(const GroupEntry* e, int count, State* out, hipStream_t st);
hipError_t launch_check_finite(const void* X, int dtype, int64_t count, int* flag, hipStream_t st);
}  // namespace flr

using namespace flr;

static thread_local std::string g_last_error;

static flr_status fail(flr_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_OR_FAIL(expr)                                                                                   \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) {                                                                                 \
      (void)hipGetLastError(); /* a failed call also leaves its error for the next check */                 \
      return fail(e_ == hipErrorOutOfMemory ? FLR_ERR_OUT_OF_MEMORY : FLR_ERR_DEVICE,                       \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                                       \
    }                                                                                                       \
  } while (0)

namespace {

template <typename T>
hipError_t dalloc(flr_problem h, T** p, size_t count) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e == hipSuccess) {
    h->allocs.push_back(*p);
    h->footprint += bytes;
    e = hipMemsetAsync(*p, 0, bytes, h->stream);
  }
  return e;
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

Dims choose_dims(int64_t n, int64_t p, int dtype, bool flsa) {
  Dims D{};
  D.n = n;
  D.p = p;
  D.dtype = dtype;
  D.flsa = flsa ? 1 : 0;
  const int V = dtype == FLR_F64 ? 2 : dtype == FLR_F32 ? 4 : 8;
  D.c1 = 256 * V;
  D.c2 = 64 * V;
  D.p_pad = round_up(p, D.c1);
  D.ldx = D.p_pad;
  D.cb1 = (int32_t)(D.p_pad / D.c1);
  const char* ta = getenv("FLR_TARGET_WG_A");
  const char* tb = getenv("FLR_TARGET_WG_B");
  // 512 workgroups per GEMV launch (two per CU): measured best on the
  // n = 1000, p = 10^4 f32 workload (A 9.1 us, B 10.8 us per launch, and
  // fewer column-panel partials for the block kernel to sum) over 256..2048
  const int target = ta ? atoi(ta) : 512;
  const int target_b = tb ? atoi(tb) : 512;
  int64_t rb1 = std::max<int64_t>(1, (target + D.cb1 - 1) / D.cb1);
  rb1 = std::min<int64_t>(rb1, std::max<int64_t>(1, n / 4));
  D.r1 = (int32_t)((n + rb1 - 1) / rb1);
  D.rb1 = (int32_t)((n + D.r1 - 1) / D.r1);
  D.cb2 = (int32_t)(D.p_pad / D.c2);
  int64_t rb2 = std::max<int64_t>(1, (target_b + D.cb2 - 1) / D.cb2);
  rb2 = std::min<int64_t>(rb2, std::max<int64_t>(1, n / 4));
  int64_t r2 = (n + rb2 - 1) / rb2;
  if (r2 > kMaxR2) r2 = kMaxR2;
  D.r2 = (int32_t)r2;
  D.rb2 = (int32_t)((n + r2 - 1) / r2);
  if (flsa) {  // X = I: one row panel per column panel, nothing streamed
    D.rb1 = 1;
    D.r1 = (int32_t)std::min<int64_t>(n, INT32_MAX);
    D.rb2 = 1;
    D.r2 = 0;
  }
  D.nblk = (int32_t)(D.p_pad / kBlk);
  D.gridB = std::max(D.cb2 * D.rb2, D.nblk);
  D.nloss = flsa ? D.cb2 : D.rb2;
  return D;
}

bool is_device_ptr(const void* ptr) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

flr_status build_graph(flr_problem h, bool mixed, bool band) {
  hipGraphExec_t& ge = h->gexec[mixed][band];
  hipGraph_t& gr = h->graph[mixed][band];
  if (ge) return FLR_OK;
  HIP_OR_FAIL(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  const int per = band ? 4 : 3;  // A, B, C (, K)
  for (int i = 0; i < per * kRounds && err == hipSuccess; ++i)
    err = launch_rotation(h->D, h->B, i & 1, i % per, h->stream, mixed);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(h->stream, &g);
  if (err != hipSuccess) return fail(FLR_ERR_DEVICE, std::string("capture launch: ") + hipGetErrorString(err));
  HIP_OR_FAIL(e2);
  gr = g;
  HIP_OR_FAIL(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  return FLR_OK;
}

flr_status validate_lambdas(double l1, double l2, double tol) {
  if (!(std::isfinite(l1) && l1 >= 0.0) || !(std::isfinite(l2) && l2 >= 0.0))
    return fail(FLR_ERR_INVALID_ARG, "lambda1 and lambda2 must be finite and >= 0");
  if (!(std::isfinite(tol) && tol > 0.0)) return fail(FLR_ERR_INVALID_ARG, "tol must be finite and > 0");
  return FLR_OK;
}

// One solve in flight: the problem, its captured rotation and the launch count.
struct SolveRun {
  flr_problem h = nullptr;
  hipGraphExec_t gexec = nullptr;
  int64_t max_launches = 0, launched = 0;
  int in_flight = 0;
  bool done = false;
  std::chrono::steady_clock::time_point t0;
};

// Parameters, warm start and initial state of a solve (solve_begin adds the
// captured rotation; the ragged batch captures grouped launches instead).
flr_status solve_prepare(flr_problem h, double l1, double l2, double tol, const flr_solve_opts* o, SolveRun& run) {
  run.t0 = std::chrono::steady_clock::now();
  run.h = h;
  flr_solve_opts dflt;
  flr_default_opts(&dflt);
  if (!o) o = &dflt;
  if (!(o->eps >= 0.0) || !(o->inner_tol >= 0.0) || o->max_iter < 0 || o->max_cg < 0)
    return fail(FLR_ERR_INVALID_ARG, "options out of range");
  const Dims& D = h->D;
  Params& P = *h->h_prm;
  P.lam1 = l1;
  P.lam2 = l2;
  P.eps = o->eps > 0.0 ? o->eps : 1e-8;
  P.tol = tol;
  P.inner_tol = o->inner_tol > 0.0 ? o->inner_tol : tol;
  P.cnorm = h->cnorm > 0.0 ? h->cnorm : 1.0;
  P.max_iter = o->max_iter > 0 ? o->max_iter : 10000;
  P.max_cg = o->max_cg > 0 ? o->max_cg : (int32_t)std::min<int64_t>(D.p, INT32_MAX);
  int pre = o->preconditioner;
  if (pre < FLR_PRECOND_AUTO || pre > FLR_PRECOND_BAND) return fail(FLR_ERR_INVALID_ARG, "unknown preconditioner");
  if (pre == FLR_PRECOND_AUTO)
    pre = !(l1 > 0.0) ? FLR_PRECOND_JACOBI : h->band_w ? FLR_PRECOND_BAND : FLR_PRECOND_TRIDIAG;
  if ((pre == FLR_PRECOND_TRIDIAG || pre == FLR_PRECOND_BAND) && !(l1 > 0.0))
    return fail(FLR_ERR_INVALID_ARG, "the tridiagonal and banded preconditioners need lambda1 > 0 (M is singular otherwise)");
  if (pre == FLR_PRECOND_BAND && !h->band_w)
    return fail(FLR_ERR_INVALID_ARG, "banded preconditioner: the edge set has bandwidth < 2 or its band is too wide");
  P.jacobi = pre == FLR_PRECOND_JACOBI ? 1 : 0;
  P.band = pre == FLR_PRECOND_BAND ? h->band_w : 0;
  P.mixed = o->precision == FLR_PREC_MIXED_FP32 ? 1 : 0;
  HIP_OR_FAIL(hipMemcpyAsync(h->d_prm, h->h_prm, sizeof(Params), hipMemcpyHostToDevice, h->stream));

  const double* warm = nullptr;
  int use_warm = 0;
  if (o->warm_start) {
    if (is_device_ptr(o->warm_start)) {
      warm = o->warm_start;
    } else {
      // staged in the residual buffer; k_init reads warm[j] before clearing r[j] in the same thread
      HIP_OR_FAIL(hipMemcpyAsync(h->B.r, o->warm_start, D.p * sizeof(double), hipMemcpyHostToDevice, h->stream));
      warm = h->B.r;
    }
    use_warm = 1;
  } else if (o->use_last && h->has_solution) {
    warm = h->B.x;
    use_warm = 1;
  }
  HIP_OR_FAIL(launch_init(D, h->B, warm, use_warm, h->stream));
  // every MM step takes at most max_cg PCG steps, as many FP64 residual
  // refreshes (mixed precision: each follows at least one PCG step) and its
  // boundary; one graph launch holds kRounds rotations
  run.max_launches = ((int64_t)P.max_iter * (2 * (int64_t)P.max_cg + 2) + 2) / kRounds + 4;
  run.launched = 0;
  run.in_flight = 0;
  run.done = false;
  return FLR_OK;
}

flr_status solve_begin(flr_problem h, double l1, double l2, double tol, const flr_solve_opts* o, SolveRun& run) {
  flr_status st = solve_prepare(h, l1, l2, tol, o, run);
  if (st != FLR_OK) return st;
  const bool mixed = h->h_prm->mixed != 0;
  const bool band = h->h_prm->band != 0;
  st = build_graph(h, mixed, band);
  if (st != FLR_OK) return st;
  run.gexec = h->gexec[mixed][band];
  return FLR_OK;
}

// Keeps two launches of the captured rotation in flight: launches one when
// fewer are, else looks at the older one (waiting for it when blocking) and
// marks the solve done once the state it left says so.  *progress: whether
// anything was launched or retired.
flr_status solve_advance(SolveRun& run, bool blocking, bool* progress) {
  flr_problem h = run.h;
  *progress = false;
  if (!run.done && run.in_flight < 2) {
    if (run.launched >= run.max_launches) return fail(FLR_ERR_DEVICE, "solve did not terminate within its launch bound");
    const int slot = (int)(run.launched & 1);
    HIP_OR_FAIL(hipGraphLaunch(run.gexec, h->stream));
    HIP_OR_FAIL(hipMemcpyAsync(&h->h_state[slot], &h->B.st[0], sizeof(State), hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(hipEventRecord(h->ev[slot], h->stream));
    ++run.launched;
    ++run.in_flight;
    *progress = true;
    if (run.in_flight < 2) return FLR_OK;
  }
  if (run.in_flight == 0) return FLR_OK;
  const int oldest = (int)((run.launched - run.in_flight) & 1);
  if (blocking) {
    HIP_OR_FAIL(hipEventSynchronize(h->ev[oldest]));
  } else {
    const hipError_t q = hipEventQuery(h->ev[oldest]);
    if (q == hipErrorNotReady) return FLR_OK;
    HIP_OR_FAIL(q);
  }
  --run.in_flight;
  *progress = true;
  if (h->h_state[oldest].phase == PH_DONE) run.done = true;
  return FLR_OK;
}

// After the solve is done: outputs and status.
flr_status solve_end(SolveRun& run, double* beta_out, flr_result* res) {
  flr_problem h = run.h;
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  const State fin = h->h_state[(run.launched - 1) & 1];
  if (beta_out) HIP_OR_FAIL(hipMemcpy(beta_out, h->B.x, h->D.p * sizeof(double), hipMemcpyDefault));
  h->has_solution = true;
  flr_status st = fin.status == ST_OK ? FLR_OK : fin.status == ST_MAX_ITER ? FLR_ERR_MAX_ITER : FLR_ERR_NUMERICAL;
  if (res) {
    res->objective = fin.f_new;
    res->rel_change = fin.rel_change;
    res->rel_residual = fin.rel_res;
    res->cg_iters = fin.cg_total;
    res->mm_iters = fin.mm_iter;
    res->status = st;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - run.t0).count();
  }
  if (st == FLR_ERR_NUMERICAL) g_last_error = "non-finite value or CG breakdown inside the solve";
  if (st == FLR_ERR_MAX_ITER) g_last_error = "MM iteration cap reached";
  return st;
}

// One solve on the problem's stream; beta_out host or device (or nullptr).
flr_status run_solve(flr_problem h, double l1, double l2, double tol, const flr_solve_opts* o, double* beta_out,
                     flr_result* res) {
  if (o && o->method != FLR_METHOD_PCG) {
    if (o->method != FLR_METHOD_CHOLESKY) return fail(FLR_ERR_INVALID_ARG, "unknown method");
    if (!(o->eps >= 0.0) || o->max_iter < 0) return fail(FLR_ERR_INVALID_ARG, "options out of range");
    return dense_run(h, l1, l2, tol, o, beta_out, res);
  }
  SolveRun run;
  flr_status st = solve_begin(h, l1, l2, tol, o, run);
  if (st != FLR_OK) return st;
  // FLR_PROGRESS=1: a line on stderr every few seconds from the polling loop
  const char* prog_env = std::getenv("FLR_PROGRESS");
  const bool progress = prog_env && prog_env[0] && prog_env[0] != '0';
  auto t_prog = std::chrono::steady_clock::now();
  while (!run.done) {
    bool moved = false;
    st = solve_advance(run, true, &moved);
    if (st != FLR_OK) return st;
    if (progress && std::chrono::steady_clock::now() - t_prog > std::chrono::seconds(5)) {
      t_prog = std::chrono::steady_clock::now();
      const State& hs = h->h_state[(run.launched - run.in_flight - 1) & 1];
      std::fprintf(stderr, "flr solve: MM %d, PCG steps %lld, f %.12g\n", hs.mm_iter, (long long)hs.cg_total,
                   hs.f_new);
    }
  }
  return solve_end(run, beta_out, res);
}

// Device and host buffers of one ragged batch (released on every return).
struct BatchWork {
  GroupEntry* d_ent = nullptr;
  State* d_st = nullptr;
  State* h_st = nullptr;      // pinned, 2 slots of count states; the last states read are at h_st
  State* h_slot[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~BatchWork() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
    if (h_st) (void)hipHostFree(h_st);
    if (d_ent) (void)hipFree(d_ent);
  }
};

// The ragged batch in grouped launches: the problems are sorted into groups
// of one stored type and precision; one round is, per group, one launch each
// of A, B and C over every problem of the group and one banded-solve launch
// (the problems without a band only pass their state on, which keeps every
// problem's state parity that of the banded rotation).  kRounds rounds are
// captured in one graph on the first problem's stream and launched with two
// in flight, the states of all problems gathered into one copy per launch;
// the batch ends when every problem's state says done.
flr_status batch_run(const flr_problem* hs, int32_t count, std::vector<SolveRun>& runs, BatchWork& bw) {
  struct Group {
    int dtype;
    bool mixed;
    int first, count, wa, wb, wc;
  };
  std::vector<GroupEntry> ents;
  std::vector<Group> groups;
  std::vector<int> order;  // problem index of each entry
  int64_t max_launches = 0;
  for (int dt = 0; dt < 3; ++dt) {
    for (int mx = 0; mx < 2; ++mx) {
      Group g{dt, mx != 0, (int)ents.size(), 0, 0, 0, 0};
      for (int32_t i = 0; i < count; ++i) {
        flr_problem h = hs[i];
        if (h->D.dtype != dt || (h->h_prm->mixed != 0) != (mx != 0)) continue;
        GroupEntry e{};
        e.D = h->D;
        e.B = h->B;
        e.wg_a = g.wa;
        e.wg_b = g.wb;
        e.wg_c = g.wc;
        e.band = h->h_prm->band != 0 ? 1 : 0;
        g.wa += h->D.cb1 * h->D.rb1;
        g.wb += h->D.gridB;
        g.wc += h->D.nblk;
        ents.push_back(e);
        order.push_back(i);
        ++g.count;
        max_launches = std::max(max_launches, runs[(size_t)i].max_launches);
      }
      if (g.count) groups.push_back(g);
    }
  }
  // states are gathered in entry order
  const size_t nst = (size_t)count;
  HIP_OR_FAIL(hipMalloc(reinterpret_cast<void**>(&bw.d_ent), ents.size() * sizeof(GroupEntry) + nst * sizeof(State)));
  bw.d_st = reinterpret_cast<State*>(bw.d_ent + ents.size());
  HIP_OR_FAIL(hipHostMalloc(reinterpret_cast<void**>(&bw.h_st), 3 * nst * sizeof(State), hipHostMallocDefault));
  bw.h_slot[0] = bw.h_st + nst;
  bw.h_slot[1] = bw.h_st + 2 * nst;
  for (auto& e : bw.ev) HIP_OR_FAIL(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipStream_t st = hs[0]->stream;
  // the problems' initializations (on their own streams) come first
  for (int32_t i = 0; i < count; ++i) HIP_OR_FAIL(hipStreamSynchronize(hs[i]->stream));
  HIP_OR_FAIL(hipMemcpy(bw.d_ent, ents.data(), ents.size() * sizeof(GroupEntry), hipMemcpyHostToDevice));
  HIP_OR_FAIL(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  for (int r = 0; r < kRounds && err == hipSuccess; ++r)
    for (const Group& g : groups)
      for (int which = 0; which < 4 && err == hipSuccess; ++which) {
        const int wgs = which == 0 ? g.wa : which == 1 ? g.wb : which == 2 ? g.wc : g.count;
        err = launch_grouped(g.dtype, g.mixed, bw.d_ent + g.first, g.count, wgs, which & 1, which, st);
      }
  hipError_t e2 = hipStreamEndCapture(st, &bw.graph);
  if (err != hipSuccess) return fail(FLR_ERR_DEVICE, std::string("batch capture: ") + hipGetErrorString(err));
  HIP_OR_FAIL(e2);
  HIP_OR_FAIL(hipGraphInstantiate(&bw.exec, bw.graph, nullptr, nullptr, 0));
  int64_t launched = 0;
  int in_flight = 0;
  bool done = false;
  while (!done) {
    if (in_flight < 2) {
      if (launched >= max_launches) return fail(FLR_ERR_DEVICE, "batch did not terminate within its launch bound");
      const int slot = (int)(launched & 1);
      HIP_OR_FAIL(hipGraphLaunch(bw.exec, st));
      HIP_OR_FAIL(launch_gather_states(bw.d_ent, (int)ents.size(), bw.d_st, st));
      HIP_OR_FAIL(hipMemcpyAsync(bw.h_slot[slot], bw.d_st, nst * sizeof(State), hipMemcpyDeviceToHost, st));
      HIP_OR_FAIL(hipEventRecord(bw.ev[slot], st));
      ++launched;
      if (++in_flight < 2) continue;
    }
    const int oldest = (int)((launched - in_flight) & 1);
    HIP_OR_FAIL(hipEventSynchronize(bw.ev[oldest]));
    --in_flight;
    done = true;
    for (size_t k = 0; k < nst; ++k) done = done && bw.h_slot[oldest][k].phase == PH_DONE;
  }
  HIP_OR_FAIL(hipStreamSynchronize(st));
  const State* last = bw.h_slot[(launched - 1) & 1];
  for (size_t k = 0; k < nst; ++k) bw.h_st[order[k]] = last[k];
  return FLR_OK;
}

}  // namespace

namespace flr {
flr_status solve_locked(flr_problem h, double l1, double l2, double tol, const flr_solve_opts* o, double* beta_out,
                        flr_result* res) {
  flr_status v = validate_lambdas(l1, l2, tol);
  if (v != FLR_OK) return v;
  if (hipSetDevice(h->ctx->device) != hipSuccess) return fail(FLR_ERR_DEVICE, "hipSetDevice failed");
  return run_solve(h, l1, l2, tol, o, beta_out, res);
}
std::mutex& problem_mutex(flr_problem h) { return h->busy; }
bool is_device_pointer(const void* p) { return is_device_ptr(p); }
size_t problem_footprint(flr_problem h) { return h->footprint; }
int problem_device(flr_problem h) { return h->ctx->device; }
void set_last_error(const std::string& s) { g_last_error = s; }
}  // namespace flr

extern "C" {

void flr_default_opts(flr_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps = 1e-8;
  o->precision = FLR_PREC_FP64;
  o->preconditioner = FLR_PRECOND_AUTO;
}

const char* flr_status_string(flr_status st) {
  switch (st) {
    case FLR_OK: return "ok";
    case FLR_ERR_INVALID_ARG: return "invalid argument";
    case FLR_ERR_OUT_OF_MEMORY: return "out of device memory";
    case FLR_ERR_DEVICE: return "device error";
    case FLR_ERR_NUMERICAL: return "numerical failure";
    case FLR_ERR_MAX_ITER: return "iteration cap reached";
    case FLR_ERR_BUSY: return "busy";
    case FLR_ERR_NOT_READY: return "not ready";
  }
  return "unknown status";
}

const char* flr_last_error(void) { return g_last_error.c_str(); }

flr_status flr_ctx_create(int device, void* hip_stream, flr_ctx* out) {
  if (!out) return fail(FLR_ERR_INVALID_ARG, "out is NULL");
  int ndev = 0;
  HIP_OR_FAIL(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(FLR_ERR_INVALID_ARG, "no such device");
  HIP_OR_FAIL(hipSetDevice(device));
  flr_ctx c = new flr_ctx_s;
  c->device = device;
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return fail(FLR_ERR_DEVICE, hipGetErrorString(e));
    }
    c->own_stream = true;
  }
  *out = c;
  return FLR_OK;
}

void flr_ctx_destroy(flr_ctx c) {
  if (!c) return;
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

static void problem_free(flr_problem h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  flr::grid_free(h);
  flr::dense_free(h);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      if (h->gexec[a][b]) (void)hipGraphExecDestroy(h->gexec[a][b]);
      if (h->graph[a][b]) (void)hipGraphDestroy(h->graph[a][b]);
    }
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->h_prm) (void)hipHostFree(h->h_prm);
  if (h->h_state) (void)hipHostFree(h->h_state);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

// X == nullptr: the fused lasso signal approximation (X = I, n = p).
static flr_status create_impl(flr_ctx ctx, const void* X, flr_dtype x_dtype, int64_t n, int64_t p, int64_t ldx,
                              const double* y, const int64_t* edges, int64_t m, flr_problem* out) {
  const bool flsa = X == nullptr;
  if (!ctx || !y || !out) return fail(FLR_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || p < 1 || ldx < p) return fail(FLR_ERR_INVALID_ARG, "need n >= 1, p >= 1, ldx >= p");
  if (x_dtype != FLR_F64 && x_dtype != FLR_F32 && x_dtype != FLR_BF16)
    return fail(FLR_ERR_INVALID_ARG, "unknown x_dtype");
  if (m < 0 || (m > 0 && !edges)) return fail(FLR_ERR_INVALID_ARG, "bad edge list");
  if (n > (int64_t)1 << 31 || p > (int64_t)kMaxBlocks * kBlk - 2048)
    return fail(FLR_ERR_INVALID_ARG, "problem too large: n <= 2^31 and p <= 260096 (1024 solver blocks of 256, less one A panel)");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(y[i])) return fail(FLR_ERR_INVALID_ARG, "y has a non-finite value");
  // canonical unordered edge set
  std::vector<std::pair<int64_t, int64_t>> ev;
  ev.reserve((size_t)m);
  for (int64_t e = 0; e < m; ++e) {
    int64_t j = edges[2 * e], k = edges[2 * e + 1];
    if (j < 0 || k < 0 || j >= p || k >= p) return fail(FLR_ERR_INVALID_ARG, "edge index out of range");
    if (j == k) return fail(FLR_ERR_INVALID_ARG, "self-loop in the edge set");
    ev.emplace_back(std::min(j, k), std::max(j, k));
  }
  std::sort(ev.begin(), ev.end());
  ev.erase(std::unique(ev.begin(), ev.end()), ev.end());
  const int64_t mm = (int64_t)ev.size();
  if (2 * mm > (int64_t)INT32_MAX) return fail(FLR_ERR_INVALID_ARG, "too many edges");
  // symmetric CSR, columns sorted per row
  std::vector<int32_t> deg((size_t)p + 1, 0);
  for (auto& e : ev) {
    deg[(size_t)e.first + 1]++;
    deg[(size_t)e.second + 1]++;
  }
  std::vector<int32_t> rowptr((size_t)p + 1, 0);
  for (int64_t j = 0; j < p; ++j) rowptr[(size_t)j + 1] = rowptr[(size_t)j] + deg[(size_t)j + 1];
  std::vector<int32_t> col((size_t)std::max<int64_t>(2 * mm, 1)), fill(rowptr.begin(), rowptr.end() - 1);
  for (auto& e : ev) {
    col[(size_t)fill[(size_t)e.first]++] = (int32_t)e.second;
    col[(size_t)fill[(size_t)e.second]++] = (int32_t)e.first;
  }
  std::vector<int32_t> prevpos((size_t)p, -1);
  for (int64_t j = 0; j < p; ++j) {
    std::sort(col.begin() + rowptr[(size_t)j], col.begin() + rowptr[(size_t)j + 1]);
    for (int32_t q = rowptr[(size_t)j]; q < rowptr[(size_t)j + 1]; ++q)
      if (col[(size_t)q] == j - 1) prevpos[(size_t)j] = q;
  }

  HIP_OR_FAIL(hipSetDevice(ctx->device));
  flr_problem h = new flr_problem_s;
  h->ctx = ctx;
  h->m = mm;
  h->nnz = 2 * mm;
  h->D = choose_dims(n, p, x_dtype, flsa);
  const Dims& D = h->D;
  auto bail = [&](flr_status st) {
    problem_free(h);
    return st;
  };
#define CK(expr)                                                                                           \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess) {                                                                                \
      (void)hipGetLastError(); /* a failed call also leaves its error for the next check */                \
      return bail(fail(e_ == hipErrorOutOfMemory ? FLR_ERR_OUT_OF_MEMORY : FLR_ERR_DEVICE,                 \
                       std::string(#expr) + ": " + hipGetErrorString(e_)));                                \
    }                                                                                                      \
  } while (0)
  CK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
  CK(hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming));
  CK(hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming));
  CK(hipHostMalloc(reinterpret_cast<void**>(&h->h_prm), sizeof(Params), hipHostMallocDefault));
  CK(hipHostMalloc(reinterpret_cast<void**>(&h->h_state), 2 * sizeof(State), hipHostMallocDefault));
  const size_t xb = x_dtype == FLR_F64 ? 8 : x_dtype == FLR_F32 ? 4 : 2;
  void* Xd = nullptr;
  if (!flsa) {
    size_t bytes = (size_t)n * (size_t)D.ldx * xb;
    CK(hipMalloc(&Xd, bytes));
    h->allocs.push_back(Xd);
    h->footprint += bytes;
    CK(hipMemsetAsync(Xd, 0, bytes, h->stream));
    CK(hipMemcpy2DAsync(Xd, (size_t)D.ldx * xb, X, (size_t)ldx * xb, (size_t)p * xb, (size_t)n, hipMemcpyDefault,
                        h->stream));
  }
  Bufs& B = h->B;
  B.X = Xd;
  double *yd, *c, *s, *cpart, *spart;
  int32_t *rp, *cl, *pp;
  int* flag;
  CK(dalloc(h, &yd, (size_t)n));
  CK(dalloc(h, &rp, (size_t)p + 1));
  CK(dalloc(h, &cl, col.size()));
  CK(dalloc(h, &pp, (size_t)p));
  CK(dalloc(h, &c, (size_t)D.p_pad));
  CK(dalloc(h, &s, (size_t)D.p_pad));
  CK(dalloc(h, &B.x, (size_t)D.p_pad));
  CK(dalloc(h, &B.r, (size_t)D.p_pad));
  CK(dalloc(h, &B.yv, (size_t)D.p_pad));
  CK(dalloc(h, &B.pbuf, 2 * (size_t)D.p_pad));
  CK(dalloc(h, &B.a, (size_t)D.p_pad));
  CK(dalloc(h, &B.w, col.size()));
  CK(dalloc(h, &B.d, (size_t)D.p_pad));
  CK(dalloc(h, &B.e, (size_t)D.p_pad));
  CK(dalloc(h, &B.L, (size_t)D.p_pad));
  CK(dalloc(h, &B.invD, (size_t)D.p_pad));
  CK(dalloc(h, &B.sig, (size_t)D.p_pad));
  CK(dalloc(h, &B.psi, (size_t)D.p_pad));
  CK(dalloc(h, &B.upart, (size_t)D.cb1 * (size_t)n));
  CK(dalloc(h, &B.qpart, (size_t)D.rb2 * (size_t)D.p_pad));
  CK(dalloc(h, &B.pqpart, (size_t)D.gridB));
  CK(dalloc(h, &B.losspart, (size_t)std::max(D.rb2, D.cb2)));
  CK(dalloc(h, &B.penpart, (size_t)D.nblk));
  CK(dalloc(h, &B.blk, (size_t)BK_N * (size_t)D.nblk));
  CK(dalloc(h, &B.carry, 2 * (size_t)D.nblk));
  // banded factor of M for graphs of bandwidth >= 2 (lattice, all-pairs)
  {
    int64_t bw = 0;
    for (auto& e : ev) bw = std::max(bw, e.second - e.first);
    const int64_t W = bw + 1;
    if (bw >= 2 && W <= kBandMaxW && (double)p * (double)W * 8.0 <= 4.0 * (1 << 30)) {
      CK(dalloc(h, &B.Lb, (size_t)p * (size_t)W));
      CK(dalloc(h, &B.LbT, (size_t)p * (size_t)W));
      CK(dalloc(h, &B.invdb, (size_t)D.p_pad));
      CK(dalloc(h, &B.btmp, (size_t)D.p_pad));
      h->band_w = (int)W;
    }
  }
  CK(dalloc(h, &B.counter, 64));
  CK(dalloc(h, &B.st, 2));
  CK(dalloc(h, &h->d_prm, 1));
  CK(dalloc(h, &flag, 1));
  B.y = yd;
  B.rowptr = rp;
  B.col = cl;
  B.prevpos = pp;
  B.c = c;
  B.s = s;
  B.prm = h->d_prm;
  CK(hipMemcpyAsync(yd, y, (size_t)n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  CK(hipMemcpyAsync(rp, rowptr.data(), rowptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  CK(hipMemcpyAsync(cl, col.data(), col.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  CK(hipMemcpyAsync(pp, prevpos.data(), prevpos.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  int hflag = 0;
  std::vector<double> hc((size_t)D.p);
  if (!flsa) {
    CK(launch_check_finite(Xd, x_dtype, (int64_t)n * D.ldx, flag, h->stream));
    // setup partials reuse the q/u work areas: qpart holds rb2 x p_pad doubles
    cpart = B.qpart;
    double* tmp2 = nullptr;
    CK(hipMalloc(reinterpret_cast<void**>(&tmp2), (size_t)D.rb2 * (size_t)D.p_pad * sizeof(double)));
    spart = tmp2;
    CK(launch_setup(D, Xd, yd, cpart, spart, c, s, h->stream));
    CK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    CK(hipMemcpyAsync(hc.data(), c, (size_t)D.p * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    CK(hipStreamSynchronize(h->stream));
    (void)hipFree(tmp2);
  } else {
    // X = I: c = X^T y = y, ||X_j||^2 = 1 (the padding keeps zeros from dalloc)
    std::vector<double> ones((size_t)D.p, 1.0);
    CK(hipMemcpyAsync(c, y, (size_t)D.p * sizeof(double), hipMemcpyHostToDevice, h->stream));
    CK(hipMemcpyAsync(s, ones.data(), (size_t)D.p * sizeof(double), hipMemcpyHostToDevice, h->stream));
    CK(hipStreamSynchronize(h->stream));
    std::copy(y, y + D.p, hc.begin());
  }
  if (hflag) return bail(fail(FLR_ERR_INVALID_ARG, "X has a non-finite value"));
  double cn = 0.0;
  for (double v : hc) cn += v * v;
  h->cnorm = std::sqrt(cn);
#undef CK
  *out = h;
  return FLR_OK;
}

flr_status flr_create(flr_ctx ctx, const void* X, flr_dtype x_dtype, int64_t n, int64_t p, int64_t ldx,
                      const double* y, const int64_t* edges, int64_t m, flr_problem* out) {
  if (!X) return fail(FLR_ERR_INVALID_ARG, "NULL argument");
  return create_impl(ctx, X, x_dtype, n, p, ldx, y, edges, m, out);
}

flr_status flr_create_flsa(flr_ctx ctx, const double* y, int64_t p, const int64_t* edges, int64_t m,
                           flr_problem* out) {
  return create_impl(ctx, nullptr, FLR_F64, p, p, p, y, edges, m, out);
}

int32_t flr_problem_is_flsa(flr_problem h) { return h ? h->D.flsa : -1; }

void flr_destroy(flr_problem h) { problem_free(h); }

flr_status flr_problem_footprint(flr_problem h, size_t* bytes) {
  if (!h || !bytes) return fail(FLR_ERR_INVALID_ARG, "NULL argument");
  *bytes = h->footprint;
  return FLR_OK;
}
int64_t flr_problem_n(flr_problem h) { return h ? h->D.n : -1; }
int64_t flr_problem_p(flr_problem h) { return h ? h->D.p : -1; }
int64_t flr_problem_m(flr_problem h) { return h ? h->m : -1; }

flr_status flr_solve_ex(flr_problem h, double l1, double l2, double tol, const flr_solve_opts* opts, double* beta_out,
                        flr_result* res) {
  if (!h) return fail(FLR_ERR_INVALID_ARG, "NULL problem");
  flr_status v = validate_lambdas(l1, l2, tol);
  if (v != FLR_OK) return v;
  std::unique_lock<std::mutex> lk(h->busy, std::try_to_lock);
  if (!lk.owns_lock()) return fail(FLR_ERR_BUSY, "problem handle in use by another thread");
  if (hipSetDevice(h->ctx->device) != hipSuccess) return fail(FLR_ERR_DEVICE, "hipSetDevice failed");
  return run_solve(h, l1, l2, tol, opts, beta_out, res);
}

flr_status flr_solve(flr_problem h, double l1, double l2, double tol, double* beta_out_host, double* objective_out,
                     int32_t* iterations_out) {
  if (!beta_out_host) return fail(FLR_ERR_INVALID_ARG, "beta_out is NULL");
  flr_result r{};
  flr_status st = flr_solve_ex(h, l1, l2, tol, nullptr, beta_out_host, &r);
  if (st == FLR_OK || st == FLR_ERR_MAX_ITER || st == FLR_ERR_NUMERICAL) {
    if (objective_out) *objective_out = r.objective;
    if (iterations_out) *iterations_out = r.mm_iters;
  }
  return st;
}

flr_status flr_solve_batch(const flr_problem* hs, int32_t count, const double* l1, const double* l2, double tol,
                           const flr_solve_opts* opts, double* const* beta_out, flr_result* res) {
  if (!hs || !l1 || !l2 || count < 1) return fail(FLR_ERR_INVALID_ARG, "flr_solve_batch: bad arguments");
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i]) return fail(FLR_ERR_INVALID_ARG, "flr_solve_batch: NULL problem");
    for (int32_t k = 0; k < i; ++k)
      if (hs[k] == hs[i]) return fail(FLR_ERR_INVALID_ARG, "flr_solve_batch: a problem appears twice");
    if (hs[i]->ctx->device != hs[0]->ctx->device)
      return fail(FLR_ERR_INVALID_ARG, "flr_solve_batch: problems on different devices");
    flr_status v = validate_lambdas(l1[i], l2[i], tol);
    if (v != FLR_OK) return v;
  }
  std::vector<std::unique_lock<std::mutex>> locks;
  for (int32_t i = 0; i < count; ++i) {
    locks.emplace_back(hs[i]->busy, std::try_to_lock);
    if (!locks.back().owns_lock()) return fail(FLR_ERR_BUSY, "flr_solve_batch: a problem handle is in use");
  }
  if (hipSetDevice(hs[0]->ctx->device) != hipSuccess) return fail(FLR_ERR_DEVICE, "hipSetDevice failed");
  if (opts && opts->method != FLR_METHOD_PCG)
    return fail(FLR_ERR_INVALID_ARG, "flr_solve_batch runs Algorithm 2 (PCG) only");
  std::vector<SolveRun> runs((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    flr_status st = solve_prepare(hs[i], l1[i], l2[i], tol, opts, runs[(size_t)i]);
    if (st != FLR_OK) {
      for (int32_t k = 0; k < i; ++k) (void)hipStreamSynchronize(hs[k]->stream);
      return st;
    }
  }
  BatchWork bw;
  flr_status st = batch_run(hs, count, runs, bw);
  for (int32_t i = 0; i < count; ++i) (void)hipStreamSynchronize(hs[i]->stream);
  if (st != FLR_OK) return st;
  flr_status first = FLR_OK;
  for (int32_t i = 0; i < count; ++i) {
    flr_problem h = hs[i];
    const State fin = bw.h_st[i];
    if (beta_out && beta_out[i]) HIP_OR_FAIL(hipMemcpy(beta_out[i], h->B.x, h->D.p * sizeof(double), hipMemcpyDefault));
    h->has_solution = true;
    const flr_status si = fin.status == ST_OK ? FLR_OK : fin.status == ST_MAX_ITER ? FLR_ERR_MAX_ITER : FLR_ERR_NUMERICAL;
    if (res) {
      res[i].objective = fin.f_new;
      res[i].rel_change = fin.rel_change;
      res[i].rel_residual = fin.rel_res;
      res[i].cg_iters = fin.cg_total;
      res[i].mm_iters = fin.mm_iter;
      res[i].status = si;
      res[i].seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - runs[(size_t)i].t0).count();
    }
    if (si != FLR_OK && first == FLR_OK) {
      first = si;
      g_last_error = si == FLR_ERR_MAX_ITER ? "MM iteration cap reached" : "non-finite value or CG breakdown inside the solve";
    }
  }
  return first;
}

flr_status flr_solve_path(flr_problem h, const double* l1, const double* l2, const double* eps, int32_t count,
                          double tol, const flr_solve_opts* opts, double* beta_out, flr_result* res) {
  if (!h || !l1 || !l2 || count < 1) return fail(FLR_ERR_INVALID_ARG, "flr_solve_path: bad arguments");
  for (int32_t k = 0; k < count; ++k) {
    flr_status v = validate_lambdas(l1[k], l2[k], tol);
    if (v != FLR_OK) return v;
    if (eps && !(std::isfinite(eps[k]) && eps[k] > 0.0))
      return fail(FLR_ERR_INVALID_ARG, "flr_solve_path: every eps must be finite and > 0");
  }
  std::unique_lock<std::mutex> lk(h->busy, std::try_to_lock);
  if (!lk.owns_lock()) return fail(FLR_ERR_BUSY, "problem handle in use by another thread");
  if (hipSetDevice(h->ctx->device) != hipSuccess) return fail(FLR_ERR_DEVICE, "hipSetDevice failed");
  flr_solve_opts o;
  flr_default_opts(&o);
  if (opts) o = *opts;
  flr_status first = FLR_OK;
  for (int32_t k = 0; k < count; ++k) {
    if (eps) o.eps = eps[k];
    if (k > 0) {  // warm start at the previous point's solution (kept on the handle)
      o.warm_start = nullptr;
      o.use_last = 1;
    }
    double* bk = beta_out ? beta_out + (size_t)k * (size_t)h->D.p : nullptr;
    flr_result r{};
    flr_status st = run_solve(h, l1[k], l2[k], tol, &o, bk, &r);
    if (st != FLR_OK && st != FLR_ERR_MAX_ITER && st != FLR_ERR_NUMERICAL) return st;
    if (res) res[k] = r;
    if (st != FLR_OK && first == FLR_OK) first = st;
  }
  return first;
}

flr_status flr_profile_dense(flr_problem h, double lambda1, double lambda2, int32_t reps, double* avg_us) {
  if (!h || reps < 1 || !avg_us || !(lambda1 >= 0.0) || !(lambda2 >= 0.0))
    return fail(FLR_ERR_INVALID_ARG, "bad profiling arguments");
  std::unique_lock<std::mutex> lk(h->busy, std::try_to_lock);
  if (!lk.owns_lock()) return fail(FLR_ERR_BUSY, "problem handle in use by another thread");
  HIP_OR_FAIL(hipSetDevice(h->ctx->device));
  return dense_profile(h, lambda1, lambda2, reps, avg_us);
}

flr_status flr_profile_kernels(flr_problem h, int32_t reps, double* avg_us) {
  if (!h || reps < 1 || !avg_us) return fail(FLR_ERR_INVALID_ARG, "bad profiling arguments");
  if (!h->has_solution) return fail(FLR_ERR_INVALID_ARG, "profiling needs a completed solve");
  std::unique_lock<std::mutex> lk(h->busy, std::try_to_lock);
  if (!lk.owns_lock()) return fail(FLR_ERR_BUSY, "problem handle in use by another thread");
  HIP_OR_FAIL(hipSetDevice(h->ctx->device));
  State cg{};
  cg.phase = PH_CG;
  cg.first_cg = 1;
  cg.rz = 1.0;
  State* hs = h->h_state;
  hs[0] = cg;
  hs[1] = cg;
  hipEvent_t e0, e1, e2;
  HIP_OR_FAIL(hipEventCreate(&e0));
  HIP_OR_FAIL(hipEventCreate(&e1));
  HIP_OR_FAIL(hipEventCreate(&e2));
  HIP_OR_FAIL(hipMemcpyAsync(h->B.st, hs, 2 * sizeof(State), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(hipEventRecord(e0, h->stream));
  for (int i = 0; i < reps; ++i) HIP_OR_FAIL(launch_rotation(h->D, h->B, 0, 0, h->stream, false));
  HIP_OR_FAIL(hipEventRecord(e1, h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(h->B.st, hs, 2 * sizeof(State), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(hipEventRecord(e0, h->stream));
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  float ms_a = 0.f;
  // re-time A from its own start event
  HIP_OR_FAIL(hipEventRecord(e0, h->stream));
  for (int i = 0; i < reps; ++i) HIP_OR_FAIL(launch_rotation(h->D, h->B, 0, 0, h->stream, false));
  HIP_OR_FAIL(hipEventRecord(e1, h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(h->B.st, hs, 2 * sizeof(State), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  HIP_OR_FAIL(hipEventElapsedTime(&ms_a, e0, e1));
  float ms_b = 0.f;
  HIP_OR_FAIL(hipEventRecord(e1, h->stream));
  for (int i = 0; i < reps; ++i) HIP_OR_FAIL(launch_rotation(h->D, h->B, 1, 1, h->stream, false));
  HIP_OR_FAIL(hipEventRecord(e2, h->stream));
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  HIP_OR_FAIL(hipEventElapsedTime(&ms_b, e1, e2));
  // C in the same PCG-step state: it moves x and r, so both are saved first
  // and restored afterwards (the last solution stays intact)
  double* save = nullptr;
  const size_t vb = (size_t)h->D.p_pad * sizeof(double);
  HIP_OR_FAIL(hipMalloc(reinterpret_cast<void**>(&save), 2 * vb));
  HIP_OR_FAIL(hipMemcpyAsync(save, h->B.x, vb, hipMemcpyDeviceToDevice, h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(save + h->D.p_pad, h->B.r, vb, hipMemcpyDeviceToDevice, h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(h->B.st, hs, 2 * sizeof(State), hipMemcpyHostToDevice, h->stream));
  float ms_c = 0.f;
  HIP_OR_FAIL(hipEventRecord(e1, h->stream));
  for (int i = 0; i < reps; ++i) HIP_OR_FAIL(launch_rotation(h->D, h->B, 0, 2, h->stream, false));
  HIP_OR_FAIL(hipEventRecord(e2, h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(h->B.x, save, vb, hipMemcpyDeviceToDevice, h->stream));
  HIP_OR_FAIL(hipMemcpyAsync(h->B.r, save + h->D.p_pad, vb, hipMemcpyDeviceToDevice, h->stream));
  HIP_OR_FAIL(hipStreamSynchronize(h->stream));
  HIP_OR_FAIL(hipEventElapsedTime(&ms_c, e1, e2));
  (void)hipFree(save);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  avg_us[0] = 1000.0 * ms_a / reps;
  avg_us[1] = 1000.0 * ms_b / reps;
  avg_us[2] = 1000.0 * ms_c / reps;
  return FLR_OK;
}

}  // extern "C"
