// Host engine of the multilevel W1 solver: per-precision batches of solves
// ("slots") advanced together, one iteration block per step.
#pragma once
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/w1.h"
#include "w1_internal.hpp"

namespace w1 {

double now_seconds();

// hipError_t -> status, with a message kept for w1_strerror-style reporting
int hip_status(hipError_t e, const char* what);
const char* last_error_text();

// A solve request (one pair) and its lifecycle.
struct Request {
  uint64_t ticket = 0;
  w1_params prm{};
  std::vector<int> sides;           // level sides, coarsest first
  int kind = K_PLAIN;               // K_PLAIN or K_PROX
  // device memory of the solve (all levels, staging, partials)
  char* mem = nullptr;
  size_t bytes = 0;
  // state
  enum { QUEUED, PREP, RUN, FINAL, DONE } state = QUEUED;
  int slot = -1;
  int level = 0;
  bool resident_level = false;
  w1_result res{};
  double t_submit = 0, t_admit = 0, t_level = 0;
  bool want_fields = true;
  // finest-level fields after completion (host, FP64), filled on demand
  std::vector<double> f_m1, f_m2, f_psi;
  bool fields_ready = false;
  int res_iters_seen = 0;           // profiling: iterations already counted
  // served mode: set under the handle's mutex after the worker's last
  // access; only then may w1_poll take the request (and free it)
  bool handed = false;
};

// Device bytes of one request.
size_t request_bytes(const w1_params& p);

// Side of the domain [0, c]^d the outputs refer to (w1_params.h): the solve
// runs on the unit square and W1 scales by c (unit masses), the flux by
// c^(1-d), the potential by c.
inline double domain_scale(const w1_params& p) { return p.h > 0 ? (double)p.n * p.h : 1.0; }

// Per-precision batch of in-flight requests.
class BatchBase {
 public:
  virtual ~BatchBase() {}
  // borrow (device inputs only): p0 / p1 stay valid and unchanged until the
  // request's preparation has run, so it reads them in place
  virtual int admit(Request* r, const double* p0, const double* p1, int on_device, bool borrow = false) = 0;
  virtual int step() = 0;                 // advance every slot by one block
  virtual int active() const = 0;
  virtual void collect(std::vector<Request*>& done) = 0;
  // after a failed step: every unfinished request ends as W1_SOLVE_FAILED
  virtual void abort_all() = 0;
  virtual int fetch_fields(Request* r) = 0;   // copy finest fields to host
  virtual int release(Request* r) = 0;        // free a finished slot
  // input preparation only: rho of every level to dense caller buffers
  virtual int prep_export(Request* r, void* const* rho_out) = 0;
  // per-family kernel timing (HIP events on the batch's stream)
  virtual void profile(int every) = 0;   // 0: off; k >= 1: time about one launch in k
  // device work a step queues per host synchronisation (microseconds, at
  // its own cost model) and the most iteration blocks in it: short steps
  // keep served requests' admission and completion prompt, long ones cut
  // the host synchronisations of a closed batch
  virtual void set_step_budget(double us, int max_blocks) = 0;
  virtual void kernel_stats(int family, double* out6) const = 0;
  // device memory that work already queued on the batch's stream may still
  // read: returned to the cache at the batch's next host synchronisation
  virtual void retire(size_t bytes, char* mem) = 0;
  // [0] host steps (one synchronisation each), [1] level starts,
  // [2] work-list uploads, [3] iteration blocks queued
  virtual void counters(int64_t* out5) const = 0;
};

std::unique_ptr<BatchBase> make_batch(bool fp64, int capacity, hipStream_t stream);

// step budgets: served mode (requests arrive while others run) and a
// closed batch (w1_solve: every request admitted up front)
constexpr double kServedStepUs = 2000.0;
constexpr int kServedStepBlocks = 64;
constexpr double kBatchStepUs = 16000.0;
constexpr int kBatchStepBlocks = 128;

// device staging memory for served requests (the solve-state block cache)
int stage_alloc(size_t bytes, char** out);
void stage_free(size_t bytes, char* mem);
// idle cached blocks back to the device (bytes released)
size_t cache_trim();
// hipMalloc that, when it fails, returns the cache's idle blocks to the
// device and tries once more
hipError_t dev_malloc(void** p, size_t bytes);

// Tuning choice for the plain tiled kernel.
struct TileChoice {
  int rh;      // region rows
  int steps;   // temporal block depth
  int nwv;     // wavefronts per workgroup (8 or 16)
  int rw;      // region columns (128, or 64 for launches that leave the device idle)
  // (rh: 64, or 32 with rw 64 and 8 wavefronts)
};
// launch-shape autotuner of the plain tiled kernel (process-wide)
std::string tuner_table();   // JSON array of the tuner's entries
void tuner_reset();

}  // namespace w1
