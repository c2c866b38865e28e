// Host-side handle layouts shared by the engine, the grid solver and the
// serving loop.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/flr.h"
#include "flr_internal.h"

struct GridWork;  // batched-grid workspace (flr_grid.hip)
namespace flr {
struct DenseWork;  // Algorithm 1 workspace (flr_dense.hip)
}
using flr::Bufs;
using flr::Dims;
using flr::Params;
using flr::State;

struct flr_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
};

// Number of rotation rounds captured in one graph (3*S launches, or 4*S with
// the banded solve; S even keeps the state parity fixed per node).
static constexpr int kRounds = 16;

struct flr_problem_s {
  flr_ctx ctx = nullptr;
  Dims D{};
  Bufs B{};
  int64_t m = 0;
  int64_t nnz = 0;
  double cnorm = 0.0;
  hipStream_t stream = nullptr;
  Params* d_prm = nullptr;
  Params* h_prm = nullptr;  // pinned
  State* h_state = nullptr; // pinned, 2 slots
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraph_t graph[2][2] = {};         // [mixed][banded]
  hipGraphExec_t gexec[2][2] = {};
  int band_w = 0;                       // bandwidth + 1 of E when the banded factor is allocated, else 0
  std::vector<void*> allocs;
  size_t footprint = 0;
  bool has_solution = false;
  std::mutex busy;
  int64_t edges_m = 0;
  GridWork* grid = nullptr;  // workspace of the last grid solve (kept while large enough)
  flr::DenseWork* dense = nullptr;  // Algorithm 1: X^T X and the dense system (first use)
};


namespace flr {
void set_last_error(const std::string& s);
void grid_free(flr_problem h);
void dense_free(flr_problem h);
flr_status dense_run(flr_problem h, double l1, double l2, double tol, const flr_solve_opts* o, double* beta_out,
                     flr_result* res);
flr_status dense_profile(flr_problem h, double l1, double l2, int32_t reps, double* avg_us);
}  // namespace flr
