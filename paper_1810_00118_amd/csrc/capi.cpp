// extern "C" surface of the library (declared in include/w1.h): solver
// handles, batched solves, the continuous-batching server and the
// single-step entry points used to check each row of the method.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "engine.hpp"

using namespace w1;

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t _e = (x);                            \
    if (_e != hipSuccess) return hip_status(_e, #x); \
  } while (0)

// ---------------------------------------------------------------------------
// parameters
// ---------------------------------------------------------------------------
extern "C" void w1_params_default(w1_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->n = 64;
  p->levels = 1;
  p->metric = W1_METRIC_L1;
  p->algo = W1_ALGO_PROX;
  p->precision = W1_FP32;
  p->stop_rule = W1_STOP_FPR;
  p->tol = 0.0;
  p->alpha = -1.0;
  p->step_scale = 0.0;
  p->max_iters = 20000;
  p->check_every = 10;
  p->block_steps = 0;
  p->flags = 0;
}

extern "C" int w1_params_check(const w1_params* p) {
  if (!p) return W1_EINVAL;
  if (p->levels < 1 || p->levels > W1_MAX_LEVELS) return W1_EINVAL;
  if (p->n < 2 || p->n > 8192) return W1_EINVAL;
  if (p->n % (1 << (p->levels - 1)) != 0 || (p->n >> (p->levels - 1)) < 2) return W1_EINVAL;
  if (p->metric < W1_METRIC_L1 || p->metric > W1_METRIC_LINF) return W1_EINVAL;
  if (p->algo != W1_ALGO_PLAIN && p->algo != W1_ALGO_PROX) return W1_EINVAL;
  if (p->precision != W1_FP32 && p->precision != W1_FP64) return W1_EINVAL;
  if (p->stop_rule != W1_STOP_KKT && p->stop_rule != W1_STOP_FPR) return W1_EINVAL;
  if (!std::isfinite(p->tol) || !std::isfinite(p->alpha) || !std::isfinite(p->step_scale)) return W1_EINVAL;
  if (p->stop_rule == W1_STOP_KKT && p->tol < 0) return W1_EINVAL;
  if (p->max_iters < 1 || p->check_every < 1) return W1_EINVAL;
  // checks fall on multiples of check_every; the cap must be one of them
  if (p->max_iters % p->check_every != 0) return W1_EINVAL;
  if (p->block_steps < 0 || p->block_steps > TILED_MAX_STEPS) return W1_EINVAL;
  if (!std::isfinite(p->h)) return W1_EINVAL;
  for (int l = 0; l < W1_MAX_LEVELS; ++l) {
    const int c = p->level_caps[l];
    if (c < 0 || (c > 0 && (l >= p->levels || c % p->check_every != 0))) return W1_EINVAL;
  }
  if (p->diverge_window < 0 || p->reserved != 0) return W1_EINVAL;
  if (p->flags & ~(W1_FLAG_NO_RESIDENT | W1_FLAG_NO_CERT | W1_FLAG_LEVEL_COST | W1_FLAG_NO_FIELDS)) return W1_EINVAL;
  // plain: mu tau ||A||^2 < 1 holds up to step_scale 1 (the bound 2 sqrt 2 / h
  // exceeds ||A||); prox: mu tau <= 1, the practical choice of the paper.
  // Beyond, the fixed-point residual is no longer a norm of the iterate
  // change and can pass the stop test on a diverging iterate: larger steps
  // (up to 2) only with the FPR rule and the rise-window guard
  if (p->step_scale > 2.0) return W1_EINVAL;
  if (p->step_scale > 1.0 && (p->diverge_window < 1 || p->stop_rule != W1_STOP_FPR)) return W1_EINVAL;
  return W1_OK;
}

extern "C" size_t w1_bytes_per_solve(const w1_params* p) {
  if (w1_params_check(p)) return 0;
  return request_bytes(*p);
}

extern "C" const char* w1_version(void) { return "w1-mi355x 0.1 (gfx950)"; }

extern "C" const char* w1_strerror(int s) {
  switch (s) {
    case W1_OK: return "ok";
    case W1_EAGAIN: return "request still running";
    case W1_EINVAL: return "invalid argument";
    case W1_ENOMEM: return "out of device memory or budget";
    case W1_EBUSY: return "admission queue full";
    case W1_EDEVICE: return last_error_text()[0] ? last_error_text() : "HIP runtime error";
    case W1_ESTATE: return "call not valid in the current state";
    case W1_ENOTFOUND: return "unknown ticket";
    default: return "unknown status";
  }
}

static void fill_request(Request* r, const w1_params& p) {
  r->prm = p;
  r->sides.clear();
  for (int l = 0; l < p.levels; ++l) r->sides.push_back(p.n >> (p.levels - 1 - l));
  r->kind = p.algo == W1_ALGO_PLAIN ? K_PLAIN : K_PROX;
  r->want_fields = (p.flags & W1_FLAG_NO_FIELDS) == 0;
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct w1_ctx {
  w1_params prm{};
  int capacity = 1;
  size_t budget = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::unique_ptr<BatchBase> b32, b64;
  std::mutex run_mu;  // one thread drives the batches at a time
  std::mutex stage_mu;  // submit-side staging copies
  // w1_solve results kept for w1_fields
  std::vector<std::unique_ptr<Request>> last;
  // served mode
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  // masses of queued requests, in device staging memory (p0 then p1)
  struct Staged {
    char* mem = nullptr;
    size_t bytes = 0;
  };
  std::unordered_map<uint64_t, Staged> staged;
  hipStream_t stage_stream = nullptr;   // submit-side copies, synchronised there
  std::thread worker;
  bool stop = false;
  bool worker_started = false;
  int queue_limit = 4096;
  uint64_t next_ticket = 1;
  size_t in_use = 0, peak = 0;
  int64_t admitted = 0, finished = 0, running = 0;
  int worker_error = W1_OK;

  BatchBase* batch(int precision) {
    auto& b = precision == W1_FP64 ? b64 : b32;
    if (!b) b = make_batch(precision == W1_FP64, capacity, stream);
    return b.get();
  }
};

extern "C" int w1_plan(const w1_params* params, int32_t batch_capacity, size_t hbm_budget_bytes, void* hip_stream,
                       w1_handle* out) {
  if (!out || w1_params_check(params) || batch_capacity < 1) return W1_EINVAL;
  *out = nullptr;
  std::unique_ptr<w1_ctx> h(new w1_ctx());
  h->prm = *params;
  h->capacity = batch_capacity;
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    h->own_stream = true;
  }
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  h->budget = hbm_budget_bytes ? hbm_budget_bytes : fr / 2;
  const size_t need = request_bytes(*params) * (size_t)batch_capacity;
  if (need > h->budget) return W1_ENOMEM;
  *out = h.release();
  return W1_OK;
}

static void release_last(w1_ctx* h) {
  for (auto& r : h->last) {
    BatchBase* b = h->batch(r->prm.precision);
    if (b) b->release(r.get());
  }
  h->last.clear();
}

extern "C" int w1_solve(w1_handle h, int32_t count, const double* const* p0, const double* const* p1,
                        int32_t on_device, w1_result* out) {
  if (!h || count < 1 || count > h->capacity || !p0 || !p1 || !out) return W1_EINVAL;
  std::lock_guard<std::mutex> g(h->run_mu);
  release_last(h);
  BatchBase* b = h->batch(h->prm.precision);
  if (!b) return W1_EDEVICE;
  const double t0 = now_seconds();
  for (int k = 0; k < count; ++k) {
    if (!p0[k] || !p1[k]) return W1_EINVAL;
    std::unique_ptr<Request> r(new Request());
    fill_request(r.get(), h->prm);
    r->t_submit = t0;
    int st = b->admit(r.get(), p0[k], p1[k], on_device, on_device != 0);
    if (st) return st;
    h->last.push_back(std::move(r));
  }
  // a closed batch: long steps (fewer host synchronisations); the served
  // worker's short steps again afterwards
  b->set_step_budget(kBatchStepUs, kBatchStepBlocks);
  int st = W1_OK;
  while (true) {
    st = b->step();
    if (st) break;
    bool all_done = true;
    for (auto& r : h->last)
      if (r->state != Request::DONE) all_done = false;
    if (all_done) break;
  }
  b->set_step_budget(kServedStepUs, kServedStepBlocks);
  if (st) return st;
  for (int k = 0; k < count; ++k) out[k] = h->last[k]->res;
  return W1_OK;
}

extern "C" int w1_fields(w1_handle h, int32_t index, double* m1, double* m2, double* psi, int32_t on_device) {
  if (!h || index < 0 || index >= (int)h->last.size()) return W1_EINVAL;
  std::lock_guard<std::mutex> g(h->run_mu);
  Request* r = h->last[index].get();
  if (r->state != Request::DONE || r->res.status == W1_SOLVE_REJECTED) return W1_ESTATE;
  BatchBase* b = h->batch(r->prm.precision);
  int st = b->fetch_fields(r);
  if (st) return st;
  const size_t ne = r->f_m1.size();
  const hipMemcpyKind k = on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
  if (m1) HIPCHK(hipMemcpy(m1, r->f_m1.data(), ne * 8, k));
  if (m2) HIPCHK(hipMemcpy(m2, r->f_m2.data(), ne * 8, k));
  if (psi) HIPCHK(hipMemcpy(psi, r->f_psi.data(), ne * 8, k));
  return W1_OK;
}

// ---------------------------------------------------------------------------
// served mode: a worker thread admits queued requests while their state fits
// the budget and the slot capacity, and steps both precision batches; new
// requests join between iteration blocks (continuous batching)
// ---------------------------------------------------------------------------
static void worker_loop(w1_ctx* h) {
  (void)hipSetDevice(0);
  while (true) {
    std::vector<Request*> to_admit;
    {
      std::unique_lock<std::mutex> lk(h->mu);
      h->cv.wait_for(lk, std::chrono::milliseconds(20),
                     [&] { return h->stop || !h->queue.empty() || h->running > 0; });
      if (h->stop && h->queue.empty() && h->running == 0) return;
      while (!h->queue.empty()) {
        Request* r = h->queue.front();
        const size_t b = request_bytes(r->prm);
        if (h->running >= h->capacity || h->in_use + b > h->budget) break;
        h->queue.pop_front();
        h->in_use += b;
        h->peak = std::max(h->peak, h->in_use);
        h->running += 1;
        h->admitted += 1;
        to_admit.push_back(r);
      }
    }
    std::lock_guard<std::mutex> rg(h->run_mu);
    for (Request* r : to_admit) {
      w1_ctx::Staged in;
      {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = h->staged.find(r->ticket);
        in = it->second;
        h->staged.erase(it);
      }
      const size_t ne = (size_t)(r->prm.n + 1) * (r->prm.n + 1);
      const double* s0 = (const double*)in.mem;
      BatchBase* b = h->batch(r->prm.precision);
      int st = b ? b->admit(r, s0, s0 + ne, 1) : W1_EDEVICE;
      // the copies out of the staging memory are queued on the batch's
      // stream; the batch returns it to the cache after its next sync
      if (b) b->retire(in.bytes, in.mem);
      else stage_free(in.bytes, in.mem);
      if (st) {
        const size_t bytes = request_bytes(r->prm);
        std::lock_guard<std::mutex> lk(h->mu);
        r->res.status = W1_SOLVE_REJECTED;
        r->state = Request::DONE;
        h->worker_error = st;
        h->in_use -= bytes;
        h->running -= 1;
        h->finished += 1;
        r->handed = true;   // last access to r by the worker
        h->cv.notify_all();
      }
    }
    for (int prec = W1_FP32; prec <= W1_FP64; ++prec) {
      auto& bp = prec == W1_FP64 ? h->b64 : h->b32;
      if (!bp || bp->active() == 0) continue;
      int st = bp->step();
      if (st) {
        // the batch is unusable: its requests end as failed instead of
        // waiting for steps that no longer run
        bp->abort_all();
        std::lock_guard<std::mutex> lk(h->mu);
        h->worker_error = st;
      }
      std::vector<Request*> done;
      bp->collect(done);
      for (Request* r : done) {
        if (r->want_fields && r->res.status != W1_SOLVE_REJECTED && r->res.status != W1_SOLVE_FAILED)
          bp->fetch_fields(r);
        const size_t bytes = request_bytes(r->prm);
        bp->release(r);
        std::lock_guard<std::mutex> lk(h->mu);
        h->in_use -= bytes;
        h->running -= 1;
        h->finished += 1;
        r->handed = true;   // last access to r by the worker
      }
      if (!done.empty()) h->cv.notify_all();
    }
  }
}

extern "C" int w1_serve_config(w1_handle h, int32_t queue_limit) {
  if (!h || queue_limit < 1) return W1_EINVAL;
  std::lock_guard<std::mutex> lk(h->mu);
  h->queue_limit = queue_limit;
  return W1_OK;
}

extern "C" int w1_submit(w1_handle h, const w1_params* prm, const double* p0, const double* p1, int32_t on_device,
                         uint64_t* ticket) {
  if (!h || !p0 || !p1 || !ticket) return W1_EINVAL;
  const w1_params& p = prm ? *prm : h->prm;
  if (w1_params_check(&p)) return W1_EINVAL;
  if (request_bytes(p) > h->budget) return W1_ENOMEM;
  const size_t ne = (size_t)(p.n + 1) * (p.n + 1);
  // copy the masses into device staging memory on the handle's submit
  // stream and wait for that stream only: the caller may reuse its buffers
  // on return, and the solves in flight are not waited for
  w1_ctx::Staged sg;
  sg.bytes = 2 * ne * 8;
  {
    std::lock_guard<std::mutex> lk(h->stage_mu);
    if (!h->stage_stream) HIPCHK(hipStreamCreateWithFlags(&h->stage_stream, hipStreamNonBlocking));
    int st = stage_alloc(sg.bytes, &sg.mem);
    if (st) return st;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e1 = hipMemcpyAsync(sg.mem, p0, ne * 8, kind, h->stage_stream);
    hipError_t e2 = hipMemcpyAsync(sg.mem + ne * 8, p1, ne * 8, kind, h->stage_stream);
    hipError_t e3 = hipStreamSynchronize(h->stage_stream);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      if (e3 == hipSuccess) stage_free(sg.bytes, sg.mem);
      return hip_status(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3), "w1_submit copy");
    }
  }
  std::unique_ptr<Request> r(new Request());
  fill_request(r.get(), p);
  r->t_submit = now_seconds();
  {
    std::lock_guard<std::mutex> lk(h->mu);
    if ((int)h->queue.size() >= h->queue_limit) {
      stage_free(sg.bytes, sg.mem);
      return W1_EBUSY;
    }
    r->ticket = h->next_ticket++;
    *ticket = r->ticket;
    h->staged.emplace(r->ticket, sg);
    h->queue.push_back(r.get());
    h->all.emplace(r->ticket, std::move(r));
    if (!h->worker_started) {
      h->worker_started = true;
      h->worker = std::thread(worker_loop, h);
    }
  }
  h->cv.notify_all();
  return W1_OK;
}

extern "C" int w1_poll(w1_handle h, uint64_t ticket, w1_result* out, double* m1, double* m2, double* psi) {
  if (!h) return W1_EINVAL;
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    auto it = h->all.find(ticket);
    if (it == h->all.end()) return W1_ENOTFOUND;
    // fields asked of a request submitted without them: refused before the
    // ticket is consumed, so the result can still be polled
    if ((m1 || m2 || psi) && !it->second->want_fields) return W1_EINVAL;
    if (!it->second->handed) return W1_EAGAIN;
    r = std::move(it->second);
    h->all.erase(it);
  }
  if (out) *out = r->res;
  const size_t ne = (size_t)(r->prm.n + 1) * (r->prm.n + 1);
  if (r->fields_ready) {
    if (m1) std::memcpy(m1, r->f_m1.data(), ne * 8);
    if (m2) std::memcpy(m2, r->f_m2.data(), ne * 8);
    if (psi) std::memcpy(psi, r->f_psi.data(), ne * 8);
  }
  return W1_OK;
}

extern "C" int w1_drain(w1_handle h) {
  if (!h) return W1_EINVAL;
  std::unique_lock<std::mutex> lk(h->mu);
  h->cv.wait(lk, [&] { return h->queue.empty() && h->running == 0; });
  return h->worker_error;
}

extern "C" int w1_serve_stats(w1_handle h, int64_t* o) {
  if (!h || !o) return W1_EINVAL;
  std::lock_guard<std::mutex> lk(h->mu);
  o[0] = h->admitted;
  o[1] = h->finished;
  o[2] = (int64_t)h->queue.size();
  o[3] = h->running;
  o[4] = (int64_t)h->in_use;
  o[5] = (int64_t)h->peak;
  return W1_OK;
}

extern "C" int w1_engine_counters(w1_handle h, int64_t* o) {
  if (!h || !o) return W1_EINVAL;
  std::lock_guard<std::mutex> g(h->run_mu);
  for (int k = 0; k < 5; ++k) o[k] = 0;
  for (auto* b : {h->b32.get(), h->b64.get()}) {
    if (!b) continue;
    int64_t c[5];
    b->counters(c);
    for (int k = 0; k < 5; ++k) o[k] += c[k];
  }
  return W1_OK;
}

extern "C" int w1_trim_cache(size_t* released_bytes) {
  const size_t b = cache_trim();
  if (released_bytes) *released_bytes = b;
  return W1_OK;
}

extern "C" int w1_destroy(w1_handle h) {
  if (!h) return W1_EINVAL;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    h->stop = true;
  }
  h->cv.notify_all();
  if (h->worker.joinable()) h->worker.join();
  {
    std::lock_guard<std::mutex> g(h->run_mu);
    release_last(h);
    h->b32.reset();
    h->b64.reset();
  }
  for (auto& kv : h->staged) stage_free(kv.second.bytes, kv.second.mem);
  h->staged.clear();
  if (h->stage_stream) (void)hipStreamDestroy(h->stage_stream);
  if (h->own_stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return W1_OK;
}

extern "C" int w1_profile(w1_handle h, int32_t enable) {
  if (!h || enable < 0) return W1_EINVAL;
  std::lock_guard<std::mutex> g(h->run_mu);
  for (int prec = W1_FP32; prec <= W1_FP64; ++prec) {
    BatchBase* b = h->batch(prec);
    if (!b) return W1_EDEVICE;
    b->profile(enable);
  }
  return W1_OK;
}

extern "C" int w1_kernel_stats(w1_handle h, int32_t family, double* out6) {
  if (!h || !out6 || family < 0 || family >= W1_NFAM) return W1_EINVAL;
  std::lock_guard<std::mutex> g(h->run_mu);
  for (int k = 0; k < 6; ++k) out6[k] = 0;
  for (auto* b : {h->b32.get(), h->b64.get()}) {
    if (!b) continue;
    double o[6];
    b->kernel_stats(family, o);
    for (int k = 0; k < 6; ++k) out6[k] += o[k];
  }
  return W1_OK;
}

// ---------------------------------------------------------------------------
// single-step entry points: one level, caller buffers in dense layout
// ---------------------------------------------------------------------------
namespace {

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

template <typename T>
struct Op {
  hipStream_t st;
  int n, N;
  std::vector<void*> temps;
  SlotDesc<T> hd[2]{};
  SlotDesc<T>* dd = nullptr;
  SlotScalars* dsc = nullptr;
  double* part = nullptr;
  void* dbuf[8] = {};
  int nb = 0;

  Op(int n_, hipStream_t s) : st(s), n(n_), N(n_ + 1) {}
  ~Op() {
    (void)hipStreamSynchronize(st);
    for (void* p : temps) (void)hipFree(p);
  }
  int alloc(size_t bytes, void** p) {
    HIPCHK(dev_malloc(p, std::max<size_t>(bytes, 256)));
    temps.push_back(*p);
    return W1_OK;
  }
  T* plane() {
    void* p = nullptr;
    if (alloc((size_t)N * N * sizeof(T), &p)) return nullptr;
    (void)hipMemsetAsync(p, 0, (size_t)N * N * sizeof(T), st);
    return (T*)p;
  }
  int setup(int side, SlotDesc<T>& d, int metric, double mu, double tau) {
    d.n = side;
    d.pitch = side + 1;
    d.h = 1.0 / side;
    d.ih = (T)(double)side;
    d.mud = mu;
    d.taud = tau;
    d.mu = (T)mu;
    d.tau = (T)tau;
    d.metric = metric;
    d.rule = RULE_FPR;
    d.tol = -1.0;
    d.cap = 1 << 30;
    return W1_OK;
  }
  int dct(SlotDesc<T>& d) {
    // tables owned here: built from the same closed form as the engine's
    // (the FFT path needs no N x N matrices)
    const int M = d.n + 1;
    const bool fft = uses_fft(M, (int)sizeof(T));
    std::vector<double> s(M);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < M; ++k) {
      const double sn = std::sin(pi * k / (2.0 * M));
      s[k] = 4.0 * sn * sn;
    }
    void* c;
    if (alloc(M * 8, &c)) return W1_EDEVICE;
    HIPCHK(hipMemcpy(c, s.data(), M * 8, hipMemcpyHostToDevice));
    d.dcts = (const double*)c;
    std::vector<T> C, Ct;
    if (!fft) {
      C.resize((size_t)M * M);
      Ct.resize((size_t)M * M);
      for (int k = 0; k < M; ++k) {
        const double sk = k == 0 ? std::sqrt(1.0 / M) : std::sqrt(2.0 / M);
        for (int j = 0; j < M; ++j) {
          const double v = sk * std::cos(pi * k * (2.0 * j + 1.0) / (2.0 * M));
          C[(size_t)k * M + j] = (T)v;
          Ct[(size_t)j * M + k] = (T)v;
        }
      }
      void *a, *b;
      if (alloc(C.size() * sizeof(T), &a) | alloc(Ct.size() * sizeof(T), &b)) return W1_EDEVICE;
      HIPCHK(hipMemcpy(a, C.data(), C.size() * sizeof(T), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(b, Ct.data(), Ct.size() * sizeof(T), hipMemcpyHostToDevice));
      d.dctC = (const T*)a;
      d.dctCt = (const T*)b;
    }
    if (sizeof(T) == 4 && !fft) {
      void *a, *b;
      std::vector<T> Cp, Ctp;
      fold_order(M, C, &Cp, &Ctp);
      if (alloc(Cp.size() * sizeof(T), &a) | alloc(Ctp.size() * sizeof(T), &b)) return W1_EDEVICE;
      HIPCHK(hipMemcpy(a, Cp.data(), Cp.size() * sizeof(T), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(b, Ctp.data(), Ctp.size() * sizeof(T), hipMemcpyHostToDevice));
      d.dctCp = (const T*)a;
      d.dctCtp = (const T*)b;
    }
    if (fft) {
      std::vector<float> ch, fb, tw, mk;
      fft_tables(M, &ch, &fb, &tw, &mk);
      float2* tabs[4];
      int k = 0;
      for (auto* v : {&ch, &fb, &tw, &mk}) {
        void* q;
        if (alloc(v->size() * sizeof(float), &q)) return W1_EDEVICE;
        HIPCHK(hipMemcpy(q, v->data(), v->size() * sizeof(float), hipMemcpyHostToDevice));
        tabs[k++] = (float2*)q;
      }
      d.fft_chirp = tabs[0];
      d.fft_fb = tabs[1];
      d.fft_tw = tabs[2];
      d.fft_mk = tabs[3];
    }
    return W1_OK;
  }
  int commit(int count) {
    void* p;
    if (alloc(sizeof(SlotDesc<T>) * MAXL, &p)) return W1_EDEVICE;
    dd = (SlotDesc<T>*)p;
    if (alloc(sizeof(SlotScalars), &p)) return W1_EDEVICE;
    dsc = (SlotScalars*)p;
    HIPCHK(hipMemsetAsync(dsc, 0, sizeof(SlotScalars), st));
    SlotDesc<T> tab[MAXL]{};
    for (int i = 0; i < count; ++i) tab[i] = hd[i];
    HIPCHK(hipMemcpy(dd, tab, sizeof(tab), hipMemcpyHostToDevice));
    return W1_OK;
  }
  template <typename X>
  X* upload(const std::vector<X>& v) {
    void* p;
    if (alloc(v.size() * sizeof(X), &p)) return nullptr;
    if (hipMemcpy(p, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return (X*)p;
  }
  std::vector<Work> simple(int x, int side) {
    std::vector<Work> w;
    const int ti = cdiv(side + 1, ST_H), tj = cdiv(side + 1, ST_W);
    for (int a = 0; a < ti; ++a)
      for (int b = 0; b < tj; ++b) w.push_back(make_int4(x, a, b, a * tj + b));
    return w;
  }
  std::vector<Work> gemmw(int x, int side) {
    std::vector<Work> w;
    const int t = sizeof(T) == 4 && !uses_fft(side + 1, 4) ? fold_tiles(side + 1) : cdiv(side + 1, GEMM_T);
    for (int a = 0; a < t; ++a)
      for (int b = 0; b < t; ++b) w.push_back(make_int4(x, a, b, a * t + b));
    return w;
  }
  std::vector<Work> tiled(int x, int side, int rh, int rw, int S) {
    std::vector<Work> w;
    const int ti = cdiv(side + 1, rh - 2 * S), tj = cdiv(side + 1, rw - 2 * S);
    for (int a = 0; a < ti; ++a)
      for (int b = 0; b < tj; ++b) w.push_back(make_int4(x, a, b, a * tj + b));
    return w;
  }
  void poisson(Work* gw, int ng, int dst) {
    if constexpr (sizeof(T) == 4) {
      if (uses_fft(N, 4))
        poisson_fft(st, gw, ng, (const SlotDesc<float>*)dd, dsc, dst, 0, 1u << __builtin_ctz((unsigned)(2 * (N - 1))));
      else
        K<T>::poisson_fold(st, gw, ng, dd, dsc, dst, 0);
      return;
    }
    K<T>::gemm(st, gw, ng, dd, dsc, 0, 6, 7, 1, false, 0);
    K<T>::gemm(st, gw, ng, dd, dsc, 1, 7, 6, 0, true, 0);
    K<T>::gemm(st, gw, ng, dd, dsc, 1, 6, 7, 1, false, 0);
    K<T>::gemm(st, gw, ng, dd, dsc, 0, 7, dst, 0, false, 0);
  }
  int read_scalars(SlotScalars* h) {
    HIPCHK(hipMemcpyAsync(h, dsc, sizeof(SlotScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return W1_OK;
  }
};

int check_side(int n) { return (n >= 1 && n <= 8192) ? W1_OK : W1_EINVAL; }

template <typename T>
int op_plain_steps(int n, int metric, double scale, int steps, int block, int nwv, int rw, int rh, void* m1,
                   void* m2, void* phi, const void* rho, double* fpr, hipStream_t s) {
  Op<T> op(n, s);
  const double sc = scale > 0 ? scale : 0.5;
  const double mu = sc / (2.0 * std::sqrt(2.0) * n);
  SlotDesc<T>& d = op.hd[0];
  op.setup(n, d, metric, mu, mu);
  d.p[0] = (T*)m1;
  d.p[1] = (T*)m2;
  d.p[2] = (T*)phi;
  for (int k = 3; k < NPLANES; ++k)
    if (!(d.p[k] = op.plane())) return W1_ENOMEM;
  d.rho = (T*)rho;
  void* pp;
  // one partial per tile at the deepest temporal block (the most tiles)
  const int maxS = rh == TILED_RH_SHORT ? TILED_SHORT_MAX_STEPS
                                        : (rw == TILED_RW ? TILED_MAX_STEPS : TILED_NARROW_MAX_STEPS);
  const size_t ntile = (size_t)cdiv(n + 1, rh - 2 * maxS) * cdiv(n + 1, rw - 2 * maxS);
  if (op.alloc(sizeof(double) * NQ * ntile + 4096, &pp)) return W1_ENOMEM;
  d.part = (double*)pp;
  if (block < 0) {
    // resident kernel: the whole grid in one workgroup's LDS
    if (n + 1 > K<T>::plain_resident_max_side()) return W1_EINVAL;
    d.cap = steps;
    int st = op.commit(1);
    if (st) return st;
    std::vector<int> idx{0};
    int* di = op.upload(idx);
    if (!di) return W1_EDEVICE;
    K<T>::plain_resident(s, di, 1, op.dd, op.dsc, n + 1, steps, 0, metric);
    HIPCHK(hipGetLastError());
    SlotScalars h;
    st = op.read_scalars(&h);
    if (st) return st;
    if (fpr) *fpr = h.measure;
    return W1_OK;
  }
  int st = op.commit(1);
  if (st) return st;
  const int T_ = std::max(1, std::min(block > 0 ? block : 1, maxS));
  int done = 0, li = 0, lastS = 1;
  while (done < steps) {
    const int S = std::min(T_, steps - done);
    const bool chk = fpr && done + S == steps;
    auto w = op.tiled(0, n, rh, rw, S);
    Work* dw = op.upload(w);
    if (!dw) return W1_EDEVICE;
    K<T>::plain_tiled(s, dw, (int)w.size(), op.dd, op.dsc, li, S, rh, rw, chk, metric, nwv);
    ++li;
    done += S;
    lastS = S;
  }
  if (fpr) {
    std::vector<int> idx{0}, nt{(int)op.tiled(0, n, rh, rw, lastS).size()};
    int* di = op.upload(idx);
    int* dn = op.upload(nt);
    if (!di || !dn) return W1_EDEVICE;
    K<T>::check(s, di, dn, 1, op.dd, op.dsc, K_PLAIN, steps, li);
  }
  HIPCHK(hipGetLastError());
  if (li & 1) {  // the result is in set B: copy back to the caller's planes
    const size_t b = (size_t)(n + 1) * (n + 1) * sizeof(T);
    HIPCHK(hipMemcpyAsync(m1, d.p[3], b, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(m2, d.p[4], b, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(phi, d.p[5], b, hipMemcpyDeviceToDevice, s));
  }
  SlotScalars h;
  st = op.read_scalars(&h);
  if (st) return st;
  if (fpr) *fpr = h.measure;
  return W1_OK;
}

template <typename T>
int op_prox_steps(int n, int metric, double scale, int steps, int resident, void* m1, void* m2, void* w1, void* w2,
                  void* wb1, void* wb2, const void* rho, double* fpr, hipStream_t s) {
  Op<T> op(n, s);
  const double sc = scale > 0 ? scale : 0.5;
  SlotDesc<T>& d = op.hd[0];
  op.setup(n, d, metric, sc, sc);
  d.p[0] = (T*)m1;
  d.p[1] = (T*)m2;
  d.p[2] = (T*)w1;
  d.p[3] = (T*)w2;
  d.p[4] = (T*)wb1;
  d.p[5] = (T*)wb2;
  for (int k = 6; k < NPLANES; ++k)
    if (!(d.p[k] = op.plane())) return W1_ENOMEM;
  d.rho = (T*)rho;
  void* pp;
  if (op.alloc(sizeof(double) * NQ * (size_t)cdiv(n + 1, 16) * cdiv(n + 1, 64) + 4096, &pp)) return W1_ENOMEM;
  d.part = (double*)pp;
  int st = op.dct(d);
  if (st) return st;
  if (resident) {
    // every step in one launch; the stop-test sums of the last step give G^k
    d.cap = steps;
    st = op.commit(1);
    if (st) return st;
    std::vector<int> idx{0};
    int* di = op.upload(idx);
    if (!di) return W1_EDEVICE;
    K<T>::prox_resident(s, di, 1, op.dd, op.dsc, n + 1, steps, 0, metric);
    HIPCHK(hipGetLastError());
    SlotScalars h;
    st = op.read_scalars(&h);
    if (st) return st;
    if (fpr) *fpr = h.measure;
    return W1_OK;
  }
  st = op.commit(1);
  if (st) return st;
  auto sw = op.simple(0, n);
  auto gw = op.gemmw(0, n);
  Work* dsw = op.upload(sw);
  Work* dgw = op.upload(gw);
  if (!dsw || !dgw) return W1_EDEVICE;
  for (int it = 0; it < steps; ++it) {
    K<T>::div_pre(s, dsw, (int)sw.size(), op.dd, op.dsc, 0, K_PROX, 1);
    op.poisson(dgw, (int)gw.size(), 6);
    K<T>::prox_post(s, dsw, (int)sw.size(), op.dd, op.dsc, fpr && it == steps - 1);
  }
  if (fpr) {
    std::vector<int> idx{0}, nt{(int)sw.size()};
    int* di = op.upload(idx);
    int* dn = op.upload(nt);
    if (!di || !dn) return W1_EDEVICE;
    K<T>::check(s, di, dn, 1, op.dd, op.dsc, K_PROX, steps, 0);
  }
  HIPCHK(hipGetLastError());
  SlotScalars h;
  st = op.read_scalars(&h);
  if (st) return st;
  if (fpr) *fpr = h.measure;
  return W1_OK;
}

template <typename T>
int op_poisson(int n, const void* r, void* u, const void* w1, const void* w2, hipStream_t s) {
  Op<T> op(n, s);
  SlotDesc<T>& d = op.hd[0];
  op.setup(n, d, 1, 0.5, 0.5);
  for (int k = 0; k < NPLANES; ++k)
    if (!(d.p[k] = op.plane())) return W1_ENOMEM;
  if (w1) {
    d.p[2] = (T*)w1;
    d.p[3] = (T*)w2;
  }
  d.p[8] = (T*)u;
  int st = op.dct(d);
  if (st) return st;
  st = op.commit(1);
  if (st) return st;
  auto sw = op.simple(0, n);
  auto gw = op.gemmw(0, n);
  Work* dsw = op.upload(sw);
  Work* dgw = op.upload(gw);
  if (!dsw || !dgw) return W1_EDEVICE;
  if (w1) {
    K<T>::div_pre(s, dsw, (int)sw.size(), op.dd, op.dsc, 1, K_PROX, 0);
  } else {
    HIPCHK(hipMemcpyAsync(d.p[6], r, (size_t)(n + 1) * (n + 1) * sizeof(T), hipMemcpyDeviceToDevice, s));
  }
  op.poisson(dgw, (int)gw.size(), 8);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return W1_OK;
}

template <typename T>
int op_evaluate(int n, int metric, const void* m1, const void* m2, const void* psi, const void* rho, double* out,
                hipStream_t s) {
  Op<T> op(n, s);
  SlotDesc<T>& d = op.hd[0];
  op.setup(n, d, metric, 0.5, 0.5);
  for (int k = 0; k < NPLANES; ++k)
    if (!(d.p[k] = op.plane())) return W1_ENOMEM;
  d.p[0] = (T*)m1;
  d.p[1] = (T*)m2;
  d.p[8] = (T*)psi;
  d.rho = (T*)rho;
  void* pp;
  if (op.alloc(sizeof(double) * NQ * (size_t)cdiv(n + 1, 16) * cdiv(n + 1, 64) + 4096, &pp)) return W1_ENOMEM;
  d.part = (double*)pp;
  int st = op.dct(d);
  if (st) return st;
  st = op.commit(1);
  if (st) return st;
  auto sw = op.simple(0, n);
  auto gw = op.gemmw(0, n);
  Work* dsw = op.upload(sw);
  Work* dgw = op.upload(gw);
  std::vector<int> idx{0}, nt{(int)sw.size()};
  int* di = op.upload(idx);
  int* dn = op.upload(nt);
  if (!dsw || !dgw || !di || !dn) return W1_EDEVICE;
  K<T>::div_pre(s, dsw, (int)sw.size(), op.dd, op.dsc, 2, K_PROX, 0);
  op.poisson(dgw, (int)gw.size(), 6);
  K<T>::eval_sums(s, dsw, (int)sw.size(), op.dd, op.dsc, K_PROX, 1);
  K<T>::eval_final(s, di, dn, 1, op.dd, op.dsc, K_PROX, 1);
  HIPCHK(hipGetLastError());
  SlotScalars h;
  st = op.read_scalars(&h);
  if (st) return st;
  out[0] = h.eval[0];
  out[1] = h.eval[1];
  out[2] = h.eval[2];
  out[3] = h.eval[3];
  out[4] = h.eval[4];
  out[5] = h.eval[5];
  return W1_OK;
}

template <typename T>
int op_prolong(int nc, const void* c1, const void* c2, const void* cp, void* f1, void* f2, void* fp,
               hipStream_t s) {
  Op<T> op(2 * nc, s);
  SlotDesc<T>& c = op.hd[0];
  SlotDesc<T>& f = op.hd[1];
  op.setup(nc, c, 1, 0.5, 0.5);
  op.setup(2 * nc, f, 1, 0.5, 0.5);
  const int Nc = nc + 1;
  for (int k = 0; k < NPLANES; ++k) {
    void* p;
    if (op.alloc((size_t)Nc * Nc * sizeof(T), &p)) return W1_ENOMEM;
    c.p[k] = (T*)p;
    if (!(f.p[k] = op.plane())) return W1_ENOMEM;
  }
  const size_t cb = (size_t)Nc * Nc * sizeof(T);
  HIPCHK(hipMemsetAsync(c.p[0], 0, cb, s));
  HIPCHK(hipMemsetAsync(c.p[1], 0, cb, s));
  HIPCHK(hipMemsetAsync(c.p[2], 0, cb, s));
  if (c1) HIPCHK(hipMemcpyAsync(c.p[0], c1, cb, hipMemcpyDeviceToDevice, s));
  if (c2) HIPCHK(hipMemcpyAsync(c.p[1], c2, cb, hipMemcpyDeviceToDevice, s));
  if (cp) HIPCHK(hipMemcpyAsync(c.p[2], cp, cb, hipMemcpyDeviceToDevice, s));
  int st = op.commit(2);
  if (st) return st;
  auto w = op.simple(1, 2 * nc);
  Work* dw = op.upload(w);
  if (!dw) return W1_EDEVICE;
  K<T>::prolong(s, dw, (int)w.size(), op.dd, op.dsc, K_PLAIN);
  HIPCHK(hipGetLastError());
  const size_t fb = (size_t)(2 * nc + 1) * (2 * nc + 1) * sizeof(T);
  if (f1) HIPCHK(hipMemcpyAsync(f1, f.p[0], fb, hipMemcpyDeviceToDevice, s));
  if (f2) HIPCHK(hipMemcpyAsync(f2, f.p[1], fb, hipMemcpyDeviceToDevice, s));
  if (fp) HIPCHK(hipMemcpyAsync(fp, f.p[2], fb, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return W1_OK;
}

}  // namespace

#define DISPATCH(prec, call_f, call_d) \
  ((prec) == W1_FP32 ? (call_f) : (prec) == W1_FP64 ? (call_d) : W1_EINVAL)

extern "C" int w1_op_prepare(int32_t n, int32_t levels, int32_t precision, const double* p0, const double* p1,
                             void* const* rho_out, void* hip_stream) {
  w1_params p;
  w1_params_default(&p);
  p.n = n;
  p.levels = levels;
  p.precision = precision;
  p.algo = W1_ALGO_PLAIN;
  if (w1_params_check(&p) || !p0 || !p1 || !rho_out) return W1_EINVAL;
  for (int l = 0; l < levels; ++l)
    if (!rho_out[l]) return W1_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  std::unique_ptr<BatchBase> b = make_batch(precision == W1_FP64, 1, s);
  Request r;
  fill_request(&r, p);
  r.t_submit = now_seconds();
  int st = b->admit(&r, p0, p1, 1);
  if (st) return st;
  st = b->prep_export(&r, rho_out);
  b->release(&r);
  return st;
}

extern "C" int w1_op_prolong(int32_t nc, int32_t precision, const void* c_m1, const void* c_m2, const void* c_phi,
                             void* f_m1, void* f_m2, void* f_phi, void* hip_stream) {
  if (check_side(nc)) return W1_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  return DISPATCH(precision, op_prolong<float>(nc, c_m1, c_m2, c_phi, f_m1, f_m2, f_phi, s),
                  op_prolong<double>(nc, c_m1, c_m2, c_phi, f_m1, f_m2, f_phi, s));
}

extern "C" int w1_op_plain_steps(int32_t n, int32_t metric, int32_t precision, double step_scale, int32_t steps,
                                 int32_t block_steps, int32_t waves, int32_t region_width, int32_t region_height,
                                 void* m1, void* m2, void* phi, const void* rho, double* fpr_out,
                                 void* hip_stream) {
  if (check_side(n) || steps < 1 || metric < W1_METRIC_L1 || metric > W1_METRIC_LINF || !m1 || !m2 || !phi || !rho)
    return W1_EINVAL;
  if (step_scale > 1.0 || block_steps > TILED_MAX_STEPS || (waves != 0 && waves != 8 && waves != 16))
    return W1_EINVAL;
  const int rw = region_width ? region_width : TILED_RW;
  const int rh = region_height ? region_height : TILED_RH;
  if ((rw != TILED_RW && rw != TILED_RW_NARROW) || (rw == TILED_RW_NARROW && block_steps > TILED_NARROW_MAX_STEPS))
    return W1_EINVAL;
  if (rh != TILED_RH && (rh != TILED_RH_SHORT || rw != TILED_RW_NARROW || (waves != 0 && waves != 8) ||
                         block_steps > TILED_SHORT_MAX_STEPS))
    return W1_EINVAL;
  const int nwv = waves ? waves : 8;
  hipStream_t s = (hipStream_t)hip_stream;
  return DISPATCH(
      precision,
      op_plain_steps<float>(n, metric, step_scale, steps, block_steps, nwv, rw, rh, m1, m2, phi, rho, fpr_out, s),
      op_plain_steps<double>(n, metric, step_scale, steps, block_steps, nwv, rw, rh, m1, m2, phi, rho, fpr_out, s));
}

extern "C" int w1_tuner_table(char* buf, size_t len) {
  const std::string t = tuner_table();
  if (buf && len) {
    const size_t k = std::min(len - 1, t.size());
    std::memcpy(buf, t.data(), k);
    buf[k] = 0;
  }
  return (int)t.size();
}

extern "C" int w1_tuner_reset(void) {
  tuner_reset();
  return W1_OK;
}

extern "C" int w1_op_prox_steps(int32_t n, int32_t metric, int32_t precision, double step_scale, int32_t steps,
                                int32_t resident, void* m1, void* m2, void* w1, void* w2, void* wb1, void* wb2,
                                const void* rho, double* fpr_out, void* hip_stream) {
  if (check_side(n) || steps < 1 || metric < W1_METRIC_L1 || metric > W1_METRIC_LINF) return W1_EINVAL;
  if (!m1 || !m2 || !w1 || !w2 || !wb1 || !wb2 || !rho || step_scale > 1.0) return W1_EINVAL;
  if (resident && (precision != W1_FP32 || n + 1 > K<float>::prox_resident_max_side())) return W1_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  return DISPATCH(precision,
                  op_prox_steps<float>(n, metric, step_scale, steps, resident, m1, m2, w1, w2, wb1, wb2, rho,
                                       fpr_out, s),
                  op_prox_steps<double>(n, metric, step_scale, steps, 0, m1, m2, w1, w2, wb1, wb2, rho, fpr_out,
                                        s));
}

extern "C" int w1_op_poisson(int32_t n, int32_t precision, const void* r, void* u, void* hip_stream) {
  if (check_side(n) || !r || !u) return W1_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  return DISPATCH(precision, op_poisson<float>(n, r, u, nullptr, nullptr, s),
                  op_poisson<double>(n, r, u, nullptr, nullptr, s));
}

extern "C" int w1_op_potential(int32_t n, int32_t precision, const void* w1, const void* w2, void* psi,
                               void* hip_stream) {
  if (check_side(n) || !w1 || !w2 || !psi) return W1_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  return DISPATCH(precision, op_poisson<float>(n, nullptr, psi, w1, w2, s),
                  op_poisson<double>(n, nullptr, psi, w1, w2, s));
}

extern "C" int w1_op_evaluate(int32_t n, int32_t metric, int32_t precision, const void* m1, const void* m2,
                              const void* psi, const void* rho, double* out, void* hip_stream) {
  if (check_side(n) || metric < W1_METRIC_L1 || metric > W1_METRIC_LINF || !m1 || !m2 || !psi || !rho || !out)
    return W1_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  return DISPATCH(precision, op_evaluate<float>(n, metric, m1, m2, psi, rho, out, s),
                  op_evaluate<double>(n, metric, m1, m2, psi, rho, out, s));
}
