// Host engine: per-precision batches of W1 solves advanced one iteration
// block at a time (Algorithms 3 and 4 of arXiv 1810.00118).
//
// A step launches, for every in-flight solve, the work of its current level:
//   - plain levels whose grid fits one workgroup's LDS: the resident kernel
//     runs the whole level (to its stop test or cap) in one launch;
//   - other plain levels: `check_every` iterations in temporally blocked
//     tiled launches, then the stop test;
//   - prox levels: `check_every` iterations of (divergence, four DCT passes,
//     update), then the stop test.
// One host synchronisation per step reads the per-slot status; finished
// levels are prolonged to the next level (Sec. 3.3) or evaluated.  Every
// launch covers all slots of its kind through a device work list, so pairs
// of different sizes and metrics share launches.
#include "engine.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <tuple>

namespace w1 {

static thread_local std::string g_err;
const char* last_error_text() { return g_err.c_str(); }

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return W1_OK;
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? W1_ENOMEM : W1_EDEVICE;
}

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t _e = (x);                            \
    if (_e != hipSuccess) return hip_status(_e, #x); \
  } while (0)

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
static inline int cdiv(int a, int b) { return (a + b - 1) / b; }
static inline int pitch_of(int n) { return cdiv(n + 1, 32) * 32; }
static inline size_t plane_elems(int n) { return (size_t)(n + 1) * pitch_of(n); }
static inline int simple_ti(int n) { return cdiv(n + 1, ST_H); }
static inline int simple_tj(int n) { return cdiv(n + 1, ST_W); }
static inline int simple_tiles(int n) { return simple_ti(n) * simple_tj(n); }
static inline int gemm_t(int n) { return cdiv(n + 1, GEMM_T); }
// tiles per side of the DCT work list: the folded FP32 passes may need more
template <typename T>
static inline int dct_t(int n) {
  if (uses_fft(n + 1, (int)sizeof(T))) return gemm_t(n);   // 64 x 64 transpose tiles
  return sizeof(T) == 4 ? fold_tiles(n + 1) : gemm_t(n);
}
static inline int tiled_ti(int n, int rh, int S) { return cdiv(n + 1, rh - 2 * S); }
static inline int tiled_tj(int n, int rw, int S) { return cdiv(n + 1, rw - 2 * S); }
// nodes of a side-n grid that the tiled kernel's regions (rh x rw, origins
// at multiples of the interior size minus the S-node halo) cover, counted
// with multiplicity: the node updates one of its S-step launches computes
// per step, halo recomputation included, outside the grid not
static double tiled_computed(int n, int rh, int rw, int S) {
  auto covered = [n](int tiles, int inner, int width, int S_) {
    double tot = 0;
    for (int t = 0; t < tiles; ++t) {
      const int lo = std::max(t * inner - S_, 0), hi = std::min(t * inner - S_ + width - 1, n);
      tot += hi >= lo ? hi - lo + 1 : 0;
    }
    return tot;
  };
  return covered(tiled_ti(n, rh, S), rh - 2 * S, rh, S) * covered(tiled_tj(n, rw, S), rw - 2 * S, rw, S);
}
static inline int max_tiles(int n) {
  // the tiled kernel has the most tiles at its deepest temporal block
  const int tiled = std::max({tiled_ti(n, TILED_RH, TILED_MAX_STEPS) * tiled_tj(n, TILED_RW, TILED_MAX_STEPS),
                              tiled_ti(n, TILED_RH, TILED_NARROW_MAX_STEPS) *
                                  tiled_tj(n, TILED_RW_NARROW, TILED_NARROW_MAX_STEPS),
                              tiled_ti(n, TILED_RH_SHORT, TILED_SHORT_MAX_STEPS) *
                                  tiled_tj(n, TILED_RW_NARROW, TILED_SHORT_MAX_STEPS)});
  const int g = std::max(gemm_t(n), fold_tiles(n + 1));
  return std::max(simple_tiles(n), std::max(g * g, tiled));
}
// a slot's stop-test partials: room for two blocks of the most tiles, so
// that blocks of any launch shape can take their stop tests in pairs
static inline int part_tiles(int n) { return 2 * max_tiles(n); }
static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static double paper_eps(int algo, int n, bool multilevel) {
  const double s = (1.0 / n) / (1.0 / 512.0);
  if (algo == W1_ALGO_PLAIN) return multilevel ? 1e-6 / 128.0 * s * s : 1e-6 / 512.0 * s * s * s;
  return multilevel ? std::min(2e-4, 1e-4 / 32.0 * s * s) : std::min(2e-4, 1e-4 / 16.0 * s * s);
}

size_t request_bytes(const w1_params& p) {
  const size_t es = p.precision == W1_FP64 ? 8 : 4;
  size_t b = 0;
  for (int l = 0; l < p.levels; ++l) {
    const int nl = p.n >> (p.levels - 1 - l);
    const size_t pe = plane_elems(nl);
    b += (NPLANES + 1) * align256(pe * es) + 2 * align256(pe * 8);
  }
  b += align256((size_t)part_tiles(p.n) * NQ * 8);
  b += 3 * align256((size_t)(p.n + 1) * (p.n + 1) * 8);
  return b;
}

// ---------------------------------------------------------------------------
// Launch-shape autotuner for the plain tiled kernel.
// Every shape (temporal depth T dividing check_every, 8 or 16 wavefronts per
// workgroup) computes bit-identical iterates, so shapes can be tried on live
// work: per (precision, check_every, requested depth, size class of the
// active set) each candidate runs a few iteration blocks, timed with HIP
// events (tiled launches of the block only), and the one with the lowest
// time per node update is kept from then on.  Shared by all handles of the
// process.
// ---------------------------------------------------------------------------
class Tuner {
 public:
  static constexpr int kTrials = 3;   // timed blocks per candidate (first one discarded)

  TileChoice pick(int precision, double active_nodes, int check_every, int requested, int* arm_out,
                  long* entry_out) {
    std::lock_guard<std::mutex> g(mu_);
    const int cls = size_class(active_nodes);
    const auto key = std::make_tuple(precision, check_every, requested, cls);
    auto it = tab_.find(key);
    if (it == tab_.end()) {
      Entry e;
      e.key = key;
      for (int nwv : {8, 16}) {
        if (requested > 0) {
          e.arms.push_back(Arm{nwv, depth_for(requested, check_every), TILED_RW, TILED_RH});
          continue;
        }
        // depth 1 only when nothing deeper divides the cadence
        for (int t = 2; t <= std::min(check_every, TILED_MAX_STEPS); ++t)
          if (check_every % t == 0) e.arms.push_back(Arm{nwv, t, TILED_RW, TILED_RH});
        if (e.arms.empty() || e.arms.back().nwv != nwv)
          e.arms.push_back(Arm{nwv, depth_for(1, check_every), TILED_RW, TILED_RH});
      }
      // the narrow region at its deepest offered block: for active sets that
      // leave compute units idle, twice the workgroups at a larger halo
      // share (the size class decides, as for the other shapes)
      const int tn = depth_for(requested > 0 ? std::min(requested, TILED_NARROW_MAX_STEPS) : TILED_NARROW_MAX_STEPS,
                               check_every);
      for (int nwv : {8, 16}) e.arms.push_back(Arm{nwv, tn, TILED_RW_NARROW, TILED_RH});
      // the short narrow region (32 x 64, 8 wavefronts): twice the
      // workgroups again, for the few slots still running late in a batch
      const int ts = depth_for(requested > 0 ? std::min(requested, TILED_SHORT_MAX_STEPS) : TILED_SHORT_MAX_STEPS,
                               check_every);
      e.arms.push_back(Arm{8, ts, TILED_RW_NARROW, TILED_RH_SHORT});
      it = tab_.emplace(key, e).first;
      order_.push_back(key);
    }
    Entry& e = it->second;
    int a = e.best;
    if (a < 0) {
      bool measured = true;
      for (auto& A : e.arms) measured = measured && A.done >= kTrials;
      if (measured) {
        a = 0;
        for (size_t c = 1; c < e.arms.size(); ++c)
          if (e.arms[c].cost() < e.arms[a].cost()) a = (int)c;
        e.best = a;
      } else {
        // round robin, preferring candidates with the fewest blocks issued
        int least = 1 << 30;
        for (auto& A : e.arms) least = std::min(least, A.seen);
        for (size_t k = 0; k < e.arms.size(); ++k) {
          const int c = (int)((e.rr + k) % e.arms.size());
          if (e.arms[c].seen == least) {
            a = c;
            break;
          }
        }
        e.rr = (a + 1) % (int)e.arms.size();
        e.arms[a].seen++;
      }
    }
    TileChoice c;
    c.rh = e.arms[a].rh;
    c.steps = e.arms[a].T;
    c.nwv = e.arms[a].nwv;
    c.rw = e.arms[a].rw;
    *arm_out = e.best < 0 ? a : -1;   // only exploration blocks are timed
    *entry_out = (long)(std::find(order_.begin(), order_.end(), key) - order_.begin());
    return c;
  }

  // the entry of this active set has chosen its shape (no block of it is
  // an exploration block any more)
  bool settled(int precision, double active_nodes, int check_every, int requested) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = tab_.find(std::make_tuple(precision, check_every, requested, size_class(active_nodes)));
    return it != tab_.end() && it->second.best >= 0;
  }

  void report(long entry, int arm, double ms, double node_updates) {
    if (arm < 0 || node_updates <= 0) return;
    std::lock_guard<std::mutex> g(mu_);
    if (entry < 0 || entry >= (long)order_.size()) return;
    Entry& e = tab_[order_[entry]];
    if (arm >= (int)e.arms.size()) return;
    Arm& A = e.arms[arm];
    A.done++;
    if (A.done == 1) return;   // first block of a shape: cold caches, not counted
    A.ms += ms;
    A.units += node_updates;
  }

  // "precision/check_every/requested/class: best nwv x T (ns per node update)"
  std::string table() {
    std::lock_guard<std::mutex> g(mu_);
    std::string out = "[";
    for (size_t i = 0; i < order_.size(); ++i) {
      const Entry& e = tab_[order_[i]];
      char buf[256];
      std::snprintf(buf, sizeof buf, "%s{\"precision\":%d,\"check_every\":%d,\"requested\":%d,\"class\":%d,",
                    i ? "," : "", std::get<0>(e.key), std::get<1>(e.key), std::get<2>(e.key), std::get<3>(e.key));
      out += buf;
      out += "\"arms\":[";
      for (size_t a = 0; a < e.arms.size(); ++a) {
        const Arm& A = e.arms[a];
        std::snprintf(buf, sizeof buf,
                      "%s{\"waves\":%d,\"T\":%d,\"width\":%d,\"height\":%d,\"blocks\":%d,\"ns_per_update\":%.6g}",
                      a ? "," : "", A.nwv, A.T, A.rw, A.rh, A.done, A.units > 0 ? A.ms * 1e6 / A.units : -1.0);
        out += buf;
      }
      std::snprintf(buf, sizeof buf, "],\"best\":%d}", e.best);
      out += buf;
    }
    return out + "]";
  }

  void reset() {
    std::lock_guard<std::mutex> g(mu_);
    tab_.clear();
    order_.clear();
  }

 private:
  struct Arm {
    int nwv, T, rw, rh;
    int seen = 0, done = 0;
    double ms = 0, units = 0;
    double cost() const { return units > 0 ? ms / units : 1e300; }
  };
  using Key = std::tuple<int, int, int, int>;
  struct Entry {
    Key key;
    std::vector<Arm> arms;
    int rr = 0, best = -1;
  };
  // size classes of the active set: factors of 4 in node count
  static int size_class(double nodes) {
    int c = 0;
    for (double x = nodes / 16384.0; x >= 4.0 && c < 12; x /= 4.0) ++c;
    return c;
  }
  // the deepest depth dividing check_every that is not above `want`
  static int depth_for(int want, int check_every) {
    want = std::min(want, TILED_MAX_STEPS);
    for (int t = std::min(want, check_every); t >= 1; --t)
      if (check_every % t == 0) return t;
    return 1;
  }
  std::mutex mu_;
  std::map<Key, Entry> tab_;
  std::vector<Key> order_;
};

static Tuner& g_tuner() {
  static Tuner* t = new Tuner();
  return *t;
}

std::string tuner_table() { return g_tuner().table(); }
void tuner_reset() { g_tuner().reset(); }

// ---------------------------------------------------------------------------
// caching device allocator for solve state (exact-size reuse)
// ---------------------------------------------------------------------------
// Idle blocks are kept up to a cap (W1_BLOCK_CACHE_BYTES in the
// environment, default 4 GiB); a block that would exceed it goes back to
// the device at once.  A failed hipMalloc releases every idle block and
// retries once.
class BlockCache {
 public:
  BlockCache() {
    if (const char* e = std::getenv("W1_BLOCK_CACHE_BYTES")) cap_ = (size_t)std::strtoull(e, nullptr, 10);
  }
  int get(size_t bytes, char** out) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = free_.find(bytes);
    if (it != free_.end()) {
      *out = it->second;
      free_.erase(it);
      cached_ -= bytes;
      return W1_OK;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim_locked();
      e = hipMalloc(&p, bytes);
      if (e != hipSuccess) return hip_status(e, "hipMalloc(solve state)");
    }
    *out = (char*)p;
    return W1_OK;
  }
  void put(size_t bytes, char* p) {
    std::lock_guard<std::mutex> g(mu_);
    if (cached_ + bytes > cap_) {
      (void)hipFree(p);
      return;
    }
    free_.emplace(bytes, p);
    cached_ += bytes;
  }
  // every idle block back to the device; returns the bytes released
  size_t trim() {
    std::lock_guard<std::mutex> g(mu_);
    return trim_locked();
  }
  ~BlockCache() { trim_locked(); }

 private:
  size_t trim_locked() {
    for (auto& kv : free_) (void)hipFree(kv.second);
    free_.clear();
    const size_t b = cached_;
    cached_ = 0;
    return b;
  }
  std::mutex mu_;
  std::multimap<size_t, char*> free_;
  size_t cached_ = 0;
  size_t cap_ = (size_t)4 << 30;
};

// ---------------------------------------------------------------------------
// DCT-II tables per length and precision (process lifetime)
// ---------------------------------------------------------------------------
struct DctTab {
  void* C = nullptr;
  void* Ct = nullptr;
  void* Cp = nullptr;    // FP32 only: rows of C in even / odd order
  void* Ctp = nullptr;   // FP32 only: transpose of Cp
  double* s = nullptr;
  float2* chirp = nullptr;   // FP32, uses_fft(N): the FFT path's tables
  float2* fb = nullptr;
  float2* tw = nullptr;
  float2* mk = nullptr;
};
static std::mutex g_dct_mu;
static std::map<std::pair<int, int>, DctTab> g_dct;

template <typename T>
static int dct_tables(int N, DctTab* out) {
  std::lock_guard<std::mutex> g(g_dct_mu);
  auto key = std::make_pair(N, (int)sizeof(T));
  auto it = g_dct.find(key);
  if (it != g_dct.end()) {
    *out = it->second;
    return W1_OK;
  }
  std::vector<T> C((size_t)N * N), Ct((size_t)N * N);
  std::vector<double> s(N);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < N; ++k) {
    const double sk = k == 0 ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N);
    for (int j = 0; j < N; ++j) {
      const double v = sk * std::cos(pi * k * (2.0 * j + 1.0) / (2.0 * N));
      C[(size_t)k * N + j] = (T)v;
      Ct[(size_t)j * N + k] = (T)v;
    }
    const double sn = std::sin(pi * k / (2.0 * N));
    s[k] = 4.0 * sn * sn;
  }
  DctTab t;
  HIPCHK(dev_malloc((void**)&t.C, C.size() * sizeof(T)));
  HIPCHK(dev_malloc((void**)&t.Ct, Ct.size() * sizeof(T)));
  HIPCHK(dev_malloc((void**)&t.s, N * sizeof(double)));
  HIPCHK(hipMemcpy(t.C, C.data(), C.size() * sizeof(T), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(t.Ct, Ct.data(), Ct.size() * sizeof(T), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(t.s, s.data(), N * sizeof(double), hipMemcpyHostToDevice));
  if (uses_fft(N, (int)sizeof(T))) {
    std::vector<float> ch, fb, tw, mk;
    fft_tables(N, &ch, &fb, &tw, &mk);
    for (auto pr : {std::make_pair(&ch, &t.chirp), std::make_pair(&fb, &t.fb), std::make_pair(&tw, &t.tw),
                    std::make_pair(&mk, &t.mk)}) {
      HIPCHK(dev_malloc((void**)pr.second, pr.first->size() * sizeof(float)));
      HIPCHK(hipMemcpy(*pr.second, pr.first->data(), pr.first->size() * sizeof(float), hipMemcpyHostToDevice));
    }
  }
  if (sizeof(T) == 4) {
    std::vector<T> Cp, Ctp;
    fold_order(N, C, &Cp, &Ctp);
    HIPCHK(dev_malloc((void**)&t.Cp, Cp.size() * sizeof(T)));
    HIPCHK(dev_malloc((void**)&t.Ctp, Ctp.size() * sizeof(T)));
    HIPCHK(hipMemcpy(t.Cp, Cp.data(), Cp.size() * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(t.Ctp, Ctp.data(), Ctp.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  g_dct[key] = t;
  *out = t;
  return W1_OK;
}

// ---------------------------------------------------------------------------
// upload arena: pinned staging + device copy, reset once per step (after the
// step's synchronisation), so staged bytes are never rewritten while a copy
// may still read them
// ---------------------------------------------------------------------------
class Arena {
 public:
  explicit Arena(hipStream_t s) : st_(s) {}
  ~Arena() {
    for (auto& c : chunks_) {
      (void)hipHostFree(c.h);
      (void)hipFree(c.d);
    }
  }
  void reset() {
    for (auto& c : chunks_) c.used = 0;
    cur_ = 0;
  }
  template <typename X>
  X* put(const std::vector<X>& v, int* status) {
    return (X*)put_bytes(v.data(), v.size() * sizeof(X), status);
  }
  void* put_bytes(const void* src, size_t nbytes, int* status) {
    const size_t bytes = std::max<size_t>(align256(nbytes), 256);
    while (cur_ < chunks_.size() && chunks_[cur_].used + bytes > chunks_[cur_].cap) ++cur_;
    if (cur_ == chunks_.size()) {
      Chunk c;
      c.cap = std::max<size_t>(bytes, (size_t)4 << 20);
      if (hipHostMalloc((void**)&c.h, c.cap, hipHostMallocDefault) != hipSuccess ||
          dev_malloc((void**)&c.d, c.cap) != hipSuccess) {
        *status = W1_ENOMEM;
        g_err = "upload arena allocation failed";
        return nullptr;
      }
      chunks_.push_back(c);
    }
    Chunk& c = chunks_[cur_];
    char* h = c.h + c.used;
    char* d = c.d + c.used;
    if (nbytes) std::memcpy(h, src, nbytes);
    c.used += bytes;
    hipError_t e = hipMemcpyAsync(d, h, nbytes ? nbytes : 1, hipMemcpyHostToDevice, st_);
    if (e != hipSuccess) {
      *status = hip_status(e, "hipMemcpyAsync(upload)");
      return nullptr;
    }
    return d;
  }

 private:
  struct Chunk {
    char* h = nullptr;
    char* d = nullptr;
    size_t cap = 0, used = 0;
  };
  hipStream_t st_;
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
};

// never destroyed: freeing device memory from a static destructor would race
// the HIP runtime's own teardown at process exit
static BlockCache& g_blocks_ref() {
  static BlockCache* b = new BlockCache();
  return *b;
}
#define g_blocks g_blocks_ref()
int stage_alloc(size_t bytes, char** out) { return g_blocks.get(bytes, out); }
void stage_free(size_t bytes, char* mem) { g_blocks.put(bytes, mem); }
size_t cache_trim() { return g_blocks.trim(); }
hipError_t dev_malloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) return e;
  (void)hipGetLastError();
  g_blocks.trim();
  return hipMalloc(p, bytes);
}

// ---------------------------------------------------------------------------
// per-family launch timing with HIP events on the batch's stream
// ---------------------------------------------------------------------------
class Prof {
 public:
  explicit Prof(hipStream_t s) : st_(s) {}
  ~Prof() {
    for (auto& p : pend_) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool_) (void)hipEventDestroy(e);
  }
  bool on = false;
  int every = 1;
  void reset() {
    for (int f = 0; f < W1_NFAM; ++f) tot_[f][0] = tot_[f][1] = tot_[f][2] = tot_[f][3] = tot_[f][4] = 0;
    for (int f = 0; f < W1_NFAM; ++f) issued_[f] = 0;
    drawn_ = 0;
  }
  // returns the pending index (or -1 when off); `s`: the launch's stream
  // when it is not the batch's own
  // sample: subject to the 1-in-`every` draw (whole-level resident
  // launches, one per step, are always timed)
  int begin(int fam, hipStream_t s = nullptr, bool sample = true) {
    if (!on) return -1;
    issued_[fam] += 1;
    if (sample && every > 1 && mix64(++drawn_) % (uint64_t)every != 0) return -1;
    Pend p;
    p.a = ev();
    p.b = ev();
    (void)hipEventRecord(p.a, s ? s : st_);
    pend_.push_back(p);
    return (int)pend_.size() - 1;
  }
  // the same pair of events, not recorded here: the launch itself takes
  // them (hipExtLaunchKernel), so they carry the dispatch's own start and
  // end times and add no marker packets between dependent launches
  // With `every` = k > 1 only a sample of about one launch in k is timed
  // (a fixed pseudo-random sequence, so no period of the launch pattern
  // aliases with it): timed dispatches end with a cache flush that the
  // untimed ones skip.
  int begin_ext(int fam, hipEvent_t* a, hipEvent_t* b) {
    *a = *b = nullptr;
    if (!on) return -1;
    issued_[fam] += 1;
    if (every > 1 && mix64(++drawn_) % (uint64_t)every != 0) return -1;
    Pend p;
    p.a = ev();
    p.b = ev();
    p.ext = true;
    *a = p.a;
    *b = p.b;
    pend_.push_back(p);
    return (int)pend_.size() - 1;
  }
  void end(int i, int fam, double units, double bytes, double flops, hipStream_t s = nullptr) {
    if (i < 0) return;
    Pend& p = pend_[i];
    if (!p.ext) (void)hipEventRecord(p.b, s ? s : st_);
    p.fam = fam;
    p.units = units;
    p.bytes = bytes;
    p.flops = flops;
  }
  void set_units(int i, double units, double bytes) {
    if (i < 0 || i >= (int)pend_.size()) return;
    pend_[i].units = units;
    pend_[i].bytes = bytes;
  }
  // after the stream has been synchronised
  // (launches whose end event has not completed yet stay pending)
  void harvest() {
    std::vector<Pend> keep;
    for (auto& p : pend_) {
      if (hipEventQuery(p.b) == hipErrorNotReady) {
        keep.push_back(p);
        continue;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        tot_[p.fam][0] += 1;
        tot_[p.fam][1] += ms;
        tot_[p.fam][2] += p.units;
        tot_[p.fam][3] += p.bytes;
        tot_[p.fam][4] += p.flops;
      }
      pool_.push_back(p.a);
      pool_.push_back(p.b);
    }
    pend_.swap(keep);
  }
  void stats(int f, double* o) const {
    for (int k = 0; k < 5; ++k) o[k] = tot_[f][k];
    o[5] = issued_[f];
  }

 private:
  struct Pend {
    hipEvent_t a, b;
    bool ext = false;
    int fam = W1_FAM_OTHER;
    double units = 0, bytes = 0, flops = 0;
  };
  hipEvent_t ev() {
    if (!pool_.empty()) {
      hipEvent_t e = pool_.back();
      pool_.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  // SplitMix64's output function (Steele, Lea and Flood, 2014)
  static uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
  }
  hipStream_t st_;
  std::vector<Pend> pend_;
  std::vector<hipEvent_t> pool_;
  uint64_t drawn_ = 0;
  double tot_[W1_NFAM][5] = {};
  double issued_[W1_NFAM] = {};   // launches while timing was on, timed or not
};

// ---------------------------------------------------------------------------
// Batch<T>
// ---------------------------------------------------------------------------
template <typename T>
class Batch : public BatchBase {
 public:
  Batch(int capacity, hipStream_t s) : cap_(capacity), st_(s), arena_(s), prof_(s) {
    slots_.assign(cap_, nullptr);
    hdesc_.assign((size_t)cap_ * MAXL, SlotDesc<T>{});
    ok_ = dev_malloc((void**)&ddesc_, sizeof(SlotDesc<T>) * cap_ * MAXL) == hipSuccess &&
          dev_malloc((void**)&dsc_, sizeof(SlotScalars) * cap_) == hipSuccess &&
          hipHostMalloc((void**)&hsc_, sizeof(SlotScalars) * cap_, hipHostMallocDefault) == hipSuccess;
    if (ok_) ok_ = hipMemsetAsync(dsc_, 0, sizeof(SlotScalars) * cap_, st_) == hipSuccess;
    if (ok_) ok_ = hipStreamSynchronize(st_) == hipSuccess;
    // side stream for LDS-resident levels (default priority), so that their
    // few busy compute units overlap the batched launches of other levels
    if (ok_) ok_ = hipStreamCreateWithFlags(&rs_, hipStreamNonBlocking) == hipSuccess;
    if (ok_) ok_ = hipEventCreateWithFlags(&ev_up_, hipEventDisableTiming) == hipSuccess &&
                   hipEventCreateWithFlags(&ev_res_, hipEventDisableTiming) == hipSuccess &&
                   hipEventCreateWithFlags(&ev_sc_, hipEventDisableTiming) == hipSuccess &&
                   hipEventCreateWithFlags(&ev_arena_, hipEventDisableTiming) == hipSuccess;
    // W1_SPECULATE=0 turns the speculative iteration blocks off
    if (const char* e = std::getenv("W1_SPECULATE")) speculate_ = std::atoi(e) != 0;
    // W1_SIDE_STREAM=0 keeps every launch on the batch's stream (no
    // cross-stream event waits): the mode for counter collection, whose
    // per-dispatch serialisation must not meet a wait on another queue
    if (const char* e = std::getenv("W1_SIDE_STREAM")) side_stream_ = std::atoi(e) != 0;
    // W1_PAIRED_CHECK=0: the plain path's stop test after every block (the
    // paired form gives the same bits)
    if (const char* e = std::getenv("W1_PAIRED_CHECK")) pairs_ = std::atoi(e) != 0;
    // W1_GRAPH=1: plain-only steps replay their block sequence from a
    // captured HIP graph (same launches, same bits)
    if (const char* e = std::getenv("W1_GRAPH")) graph_ = std::atoi(e) != 0;
    // failure injection for tests of the error paths: W1_FAIL_AT_STEP=k
    // makes the k-th step of every batch of the process fail from the host
    // (no device work is affected)
    if (const char* e = std::getenv("W1_FAIL_AT_STEP")) fail_at_ = std::atol(e);
  }
  ~Batch() override {
    (void)hipStreamSynchronize(st_);
    if (rs_) (void)hipStreamSynchronize(rs_);
    drop_graphs();
    free_retired();
    for (auto& t : tune_pending_) {
      tune_pool_.push_back(t.a);
      tune_pool_.push_back(t.b);
    }
    for (auto e : tune_pool_) (void)hipEventDestroy(e);
    for (auto* r : slots_)
      if (r && r->mem) g_blocks.put(r->bytes, r->mem);
    for (auto& kv : lists_) {
      (void)hipFree(kv.second.d);
      (void)hipHostFree(kv.second.h);
      if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
    }
    (void)hipFree(ddesc_);
    (void)hipFree(dsc_);
    (void)hipHostFree(hsc_);
    if (ev_up_) (void)hipEventDestroy(ev_up_);
    if (ev_res_) (void)hipEventDestroy(ev_res_);
    if (ev_sc_) (void)hipEventDestroy(ev_sc_);
    if (ev_arena_) (void)hipEventDestroy(ev_arena_);
    if (rs_) (void)hipStreamDestroy(rs_);
  }

  int active() const override {
    int a = 0;
    for (auto* r : slots_)
      if (r && r->state != Request::DONE) ++a;
    return a;
  }

  int admit(Request* r, const double* p0, const double* p1, int on_device, bool borrow) override {
    if (!ok_) return W1_EDEVICE;
    int slot = -1;
    for (int i = 0; i < cap_; ++i)
      if (!slots_[i]) {
        slot = i;
        break;
      }
    if (slot < 0) return W1_EBUSY;
    r->bytes = request_bytes(r->prm);
    int st = g_blocks.get(r->bytes, &r->mem);
    if (st) return st;
    r->slot = slot;
    slots_[slot] = r;
    const int L = r->prm.levels;
    char* p = r->mem;
    for (int l = 0; l < L; ++l) {
      const int nl = r->sides[l];
      const size_t pe = plane_elems(nl);
      SlotDesc<T>& d = hdesc_[(size_t)slot * MAXL + l];
      d = SlotDesc<T>{};
      for (int k = 0; k < NPLANES; ++k) {
        d.p[k] = (T*)p;
        p += align256(pe * sizeof(T));
      }
      d.rho = (T*)p;
      p += align256(pe * sizeof(T));
      d.r0 = (double*)p;
      p += align256(pe * 8);
      d.r1 = (double*)p;
      p += align256(pe * 8);
      d.n = nl;
      d.pitch = pitch_of(nl);
      d.h = 1.0 / nl;
      d.ih = (T)((double)nl);
      set_steps(r, d);
      d.metric = r->prm.metric;
      d.rule = r->prm.stop_rule == W1_STOP_FPR ? RULE_FPR : RULE_KKT;
      double tolL = r->prm.tol;
      if (d.rule == RULE_FPR && tolL <= 0) tolL = paper_eps(r->prm.algo, r->prm.n, L > 1);
      d.tol = tolL * std::pow(2.0, (double)(L - 1 - l) * r->prm.alpha);
      d.cap = r->prm.level_caps[l] > 0 ? r->prm.level_caps[l] : r->prm.max_iters;
      d.divwin = d.rule == RULE_FPR ? r->prm.diverge_window : 0;
      // the Poisson solves of Algorithm 2, of the KKT test and of the
      // finest level's certificate
      if (r->kind == K_PROX || l == L - 1 || d.rule == RULE_KKT) {
        DctTab t;
        st = dct_tables<T>(nl + 1, &t);
        if (st) return st;
        d.dctC = (const T*)t.C;
        d.dctCt = (const T*)t.Ct;
        d.dctCp = (const T*)t.Cp;
        d.dctCtp = (const T*)t.Ctp;
        d.dcts = t.s;
        d.fft_chirp = t.chirp;
        d.fft_fb = t.fb;
        d.fft_tw = t.tw;
        d.fft_mk = t.mk;
      }
    }
    double* part = (double*)p;
    p += align256((size_t)part_tiles(r->prm.n) * NQ * 8);
    const size_t ne = (size_t)(r->prm.n + 1) * (r->prm.n + 1);
    double* in0 = (double*)p;
    p += align256(ne * 8);
    double* in1 = (double*)p;
    p += align256(ne * 8);
    double* psi = (double*)p;
    for (int l = 0; l < L; ++l) hdesc_[(size_t)slot * MAXL + l].part = part;
    SlotDesc<T>& fin = hdesc_[(size_t)slot * MAXL + L - 1];
    fin.in0 = in0;
    fin.in1 = in1;
    // the inputs are consumed by the preparation, so the fields reuse them
    fin.out_m1 = in0;
    fin.out_m2 = in1;
    fin.out_psi = psi;
    if (borrow && on_device) {
      // read in place by the preparation (w1_solve's caller buffers)
      fin.in0 = p0;
      fin.in1 = p1;
    } else {
      // queued on the batch's stream: the sources stay valid until the next
      // synchronisation (staging retired then)
      const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
      HIPCHK(hipMemcpyAsync(in0, p0, ne * 8, kind, st_));
      HIPCHK(hipMemcpyAsync(in1, p1, ne * 8, kind, st_));
    }
    r->state = Request::PREP;
    r->level = 0;
    r->res = w1_result{};
    for (int l = 0; l < W1_MAX_LEVELS; ++l) r->res.level_w1[l] = std::numeric_limits<double>::quiet_NaN();
    r->t_admit = now_seconds();
    dirty_.push_back(slot);
    ++gen_;
    return W1_OK;
  }

  // step sizes of a level (R4): plain mu = tau = scale / (2 sqrt 2 / h), the
  // Gershgorin bound of ||A||; prox mu = tau = scale
  static void set_steps(const Request* r, SlotDesc<T>& d) {
    const double sc = r->prm.step_scale > 0 ? r->prm.step_scale : 0.5;
    const double mu = r->kind == K_PLAIN ? sc / (2.0 * std::sqrt(2.0) / d.h) : sc;
    d.mud = d.taud = mu;
    d.mu = d.tau = (T)mu;
  }

  int step() override {
    if (!ok_) return W1_EDEVICE;
    ++n_steps_;
    if (fail_at_ > 0 && n_steps_ == fail_at_) {
      g_err = "step failure injected by W1_FAIL_AT_STEP";
      return fail(W1_EDEVICE);
    }
    // the previous step's uploads may still be queued behind its
    // speculative blocks: their staging bytes are rewritten only after
    if (arena_pending_) {
      HIPCHK(hipEventSynchronize(ev_arena_));
      arena_pending_ = false;
    }
    arena_.reset();
    int st = W1_OK;
    std::vector<Request*> prep;
    for (auto* r : slots_)
      if (r && r->state == Request::PREP) prep.push_back(r);
    if (!prep.empty()) {
      st = run_prep(prep);
      if (st) return fail(st);
    }
    std::vector<Request*> R;
    // grouped by (check_every, rule, metric, size class): one launch sequence
    // per group.  Plain levels share one class (one launch covers every
    // size); prox levels are classed by log2 of the side, so each class
    // advances at its own pace instead of every small level waiting for the
    // O(N^3) transforms of the largest one.
    std::map<std::tuple<int, int, int, int>, std::vector<Request*>> P, X;
    for (auto* r : slots_) {
      if (!r || r->state != Request::RUN) continue;
      int cls = 0;
      if (r->kind == K_PROX)
        for (int s = r->sides[r->level]; s > 1; s >>= 1) ++cls;
      const auto key = std::make_tuple(r->prm.check_every, r->prm.stop_rule, r->prm.metric, cls);
      if (r->resident_level) R.push_back(r);
      else if (r->kind == K_PROX) X[key].push_back(r);
      else P[key].push_back(r);
    }
    if (R.empty() && P.empty() && X.empty()) return W1_OK;
    st = flush_desc();
    if (st) return fail(st);
    // Several iteration blocks per host synchronisation (slots that stop
    // inside the pipeline are skipped by the gated kernels), sized so each
    // group gets the step budget of device work per step (2 ms in served
    // mode, up to 16 ms for a closed batch).  Beside running tiled or prox levels,
    // LDS-resident levels run in chunks of about that length.
    struct Grp {
      std::vector<Request*>* v;
      bool prox;
      int nb;
      double us;
    };
    std::vector<Grp> groups;
    // A long budget only pays for a group of many slots: the blocks queued
    // past a slot's stop run empty for it, which a lone slot pays in full
    // at every level (and a large set hardly at all, as its slots stop
    // spread over the blocks).  A group of k slots gets the served budget
    // scaled by k / 8, up to the batch's own.
    auto budget = [&](size_t k, double* us, int* cap) {
      const double f = std::max(1.0, (double)k / 8.0);
      *us = std::min(step_budget_us_, kServedStepUs * f);
      *cap = std::min(nb_cap_, (int)(kServedStepBlocks * f));
    };
    double plain_nodes = 0;
    size_t plain_slots = 0;
    for (auto& kv : P) {
      plain_slots += kv.second.size();
      for (auto* r : kv.second) plain_nodes += node_count(r->sides[r->level]) * r->prm.check_every;
    }
    // plain: ~3e11 node updates / s; one block count for all plain groups
    const double plain_us = std::max(30.0, plain_nodes / 3.0e5);
    double pb_us;
    int pb_cap;
    budget(plain_slots, &pb_us, &pb_cap);
    const int plain_nb = std::max(8, std::min(pb_cap, (int)(pb_us / plain_us)));
    for (auto& kv : P) groups.push_back(Grp{&kv.second, false, plain_nb, plain_us});
    for (auto& kv : X) {
      // per iteration: ~42 us of launch latency for the group, the DCT
      // passes at ~40 TFLOP/s (8 N^3 flops) and the node-wise kernels
      double it_us = 42.0;
      for (auto* r : kv.second) {
        const double N = r->sides[r->level] + 1.0;
        it_us += N * N * N / 5.0e6 + N * N / 5.0e4;
      }
      const double us = it_us * std::get<0>(kv.first);
      double xb_us;
      int xb_cap;
      budget(kv.second.size(), &xb_us, &xb_cap);
      groups.push_back(Grp{&kv.second, true, std::max(1, std::min(xb_cap, (int)(xb_us / us))), us});
    }
    int maxnb = 0;
    double step_us = 0;
    for (auto& g : groups) {
      maxnb = std::max(maxnb, g.nb);
      step_us = std::max(step_us, g.nb * g.us);
    }
    if (!R.empty()) {
      // alone (no other level running) the launch runs to its stop tests:
      // chunking a uniform batch spreads the next level over many small
      // launches, which costs more than the wait for the slowest pair
      const bool alone = groups.empty();
      // beside other levels, a few resident slots (each holds one compute
      // unit) run on the side stream; a large set fills the device anyway
      const bool side = side_stream_ && !alone && (int)R.size() <= 64;
      st = launch_resident(R, alone ? 0 : step_us, side);
      if (st) return fail(st);
    }
    n_blocks_ += maxnb;
    auto blocks = [&](int from, int to, bool spec) {
      for (int b = from; b < to; ++b) {
        int gp = 0, gx = 0;
        for (auto& g : groups) {
          const int gi = g.prox ? gx++ : gp++;
          if (b >= g.nb) continue;
          // plain groups take their blocks in pairs (from, from + 1), ...:
          // the pair's first block runs without a stop test of its own
          int pair = -1;
          if (!g.prox) {
            const int r = b - from, last = std::min(to, g.nb);
            if (r % 2 == 0 && b + 1 < last) pair = 0;
            else if (r % 2 == 1) pair = 1;
          }
          const int e = g.prox ? launch_prox_block(*g.v, gi) : launch_tiled_block(*g.v, gi, spec, pair);
          if (e) return e;
        }
      }
      return (int)W1_OK;
    };
    // plain-only steps may replay a captured graph of the same launches: the
    // work lists are those of the last eager step of this generation (the
    // same device buffers), the autotuner has settled on every group's
    // shape, and no launch is timed
    bool graphable = graph_ && R.empty() && X.empty() && !prof_.on && lists_gen_ == gen_;
    if (graphable)
      for (auto& kv : P) {
        double nodes = 0;
        for (auto* r : kv.second) nodes += node_count(r->sides[r->level]);
        const auto& r0 = kv.second[0]->prm;
        if (r0.stop_rule != W1_STOP_FPR ||
            !g_tuner().settled(sizeof(T) == 8 ? W1_FP64 : W1_FP32, nodes, r0.check_every, r0.block_steps))
          graphable = false;
      }
    st = graphable ? graph_blocks(0, maxnb, false, blocks) : blocks(0, maxnb, false);
    if (st) return fail(st);
    lists_gen_ = gen_;
    // The stop state after these blocks is copied back while a quarter as
    // many blocks more are queued behind the copy: slots still running keep
    // the device busy while the host handles the ones that stopped (the
    // gated kernels skip a slot once it has stopped, and level transitions
    // queued below run after these blocks)
    st = queue_scalars();
    if (st) return fail(st);
    if (speculate_ && !groups.empty()) {
      const int spec = std::max(1, maxnb / 4);
      n_blocks_ += spec;
      st = graphable ? graph_blocks(0, spec, true, blocks) : blocks(0, spec, true);
      if (st) return fail(st);
    }
    st = wait_scalars();
    if (st) return fail(st);
    std::vector<Request*> up, fin;
    auto consider = [&](Request* r) {
      const SlotScalars& s = hsc_[r->slot];
      if (s.status == ST_RUN) return;
      const int l = r->level;
      r->res.iters[l] = s.iters;
      r->res.measure[l] = s.measure;
      r->res.levels_run = l + 1;
      r->res.level_seconds[l] = now_seconds() - r->t_admit;
      if (s.status == ST_DIVERGED) {
        r->res.status = W1_SOLVE_DIVERGED;
        fin.push_back(r);
        return;
      }
      if (s.status == ST_CAP) r->res.status = W1_SOLVE_MAXITER;
      if (l + 1 < r->prm.levels) up.push_back(r);
      else fin.push_back(r);
    };
    for (auto* r : R) consider(r);
    for (auto& kv : P)
      for (auto* r : kv.second) consider(r);
    for (auto& kv : X)
      for (auto* r : kv.second) consider(r);
    if (!up.empty()) {
      st = advance_levels(up);
      if (st) return fail(st);
    }
    if (!fin.empty()) {
      st = finalize(fin);
      if (st) return fail(st);
    }
    HIPCHK(hipEventRecord(ev_arena_, st_));
    arena_pending_ = true;
    return W1_OK;
  }

  void collect(std::vector<Request*>& done) override {
    for (auto* r : slots_)
      if (r && r->state == Request::DONE) done.push_back(r);
  }

  void abort_all() override {
    for (auto* r : slots_) {
      if (!r || r->state == Request::DONE) continue;
      r->res.status = W1_SOLVE_FAILED;
      r->res.w1 = r->res.dual = r->res.lo = r->res.hi = r->res.kkt = NAN;
      r->state = Request::DONE;
      r->res.seconds = now_seconds() - r->t_submit;
    }
    ++gen_;
  }

  int fetch_fields(Request* r) override {
    if (r->fields_ready) return W1_OK;
    const size_t ne = (size_t)(r->prm.n + 1) * (r->prm.n + 1);
    r->f_m1.resize(ne);
    r->f_m2.resize(ne);
    r->f_psi.resize(ne);
    const SlotDesc<T>& fin = hdesc_[didx(r, r->prm.levels - 1)];
    HIPCHK(hipMemcpyAsync(r->f_m1.data(), fin.out_m1, ne * 8, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipMemcpyAsync(r->f_m2.data(), fin.out_m2, ne * 8, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipMemcpyAsync(r->f_psi.data(), fin.out_psi, ne * 8, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    const double c = domain_scale(r->prm);
    if (c != 1.0)
      for (size_t e = 0; e < ne; ++e) {
        r->f_m1[e] /= c;
        r->f_m2[e] /= c;
        r->f_psi[e] *= c;
      }
    r->fields_ready = true;
    return W1_OK;
  }

  int release(Request* r) override {
    if (r->slot >= 0 && r->slot < cap_ && slots_[r->slot] == r) {
      // after a failed step the stream may report the error again: the
      // slot is released all the same (its memory is not reused then)
      if (hipStreamSynchronize(st_) != hipSuccess) {
        (void)hipGetLastError();
        slots_[r->slot] = nullptr;
        r->mem = nullptr;
        r->slot = -1;
        ++gen_;
        return W1_EDEVICE;
      }
      g_blocks.put(r->bytes, r->mem);
      r->mem = nullptr;
      slots_[r->slot] = nullptr;
      r->slot = -1;
      ++gen_;
    }
    return W1_OK;
  }

  int prep_export(Request* r, void* const* rho_out) override {
    arena_.reset();
    std::vector<Request*> one{r};
    int st = run_prep(one);
    if (st) return fail(st);
    if (r->state == Request::DONE) return W1_EINVAL;
    for (int l = 0; l < r->prm.levels; ++l) {
      std::vector<std::pair<Request*, int>> lv{{r, l}};
      auto w = simple_work(lv);
      Work* dw = arena_.put(w, &st);
      if (st) return st;
      K<T>::export_dense(st_, dw, (int)w.size(), ddesc_, NPLANES, (T*)rho_out[l]);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st_));
    r->state = Request::DONE;
    return W1_OK;
  }

  void set_step_budget(double us, int max_blocks) override {
    step_budget_us_ = us;
    nb_cap_ = max_blocks;
  }
  void profile(int every) override {
    prof_.on = every > 0;
    prof_.every = every > 1 ? every : 1;
    prof_.reset();
  }
  void retire(size_t bytes, char* mem) override { retire_.emplace_back(bytes, mem); }
  void counters(int64_t* o) const override {
    o[0] = n_steps_;
    o[1] = n_levels_;
    o[2] = n_uploads_;
    o[3] = n_blocks_;
    o[4] = n_graphs_;
  }
  void kernel_stats(int f, double* o) const override {
    (void)hipStreamSynchronize(st_);   // the last step's speculative blocks
    prof_.harvest();
    prof_.stats(f, o);
  }

 private:
  int fail(int st) {
    ok_ = false;
    return st;
  }
  size_t didx(const Request* r, int l) const { return (size_t)r->slot * MAXL + l; }
  int dx(const Request* r, int l) const { return r->slot * MAXL + l; }
  static double node_count(int n) { return (double)(n + 1) * (double)(n + 1); }

  // descriptors of the changed slots to the device: the span from the lowest
  // to the highest changed slot in one staged copy (slots in between are
  // rewritten with their unchanged host copy), so a step costs two copies
  // however many slots changed
  int flush_desc() {
    if (dirty_.empty()) return W1_OK;
    int st = W1_OK;
    const auto mm = std::minmax_element(dirty_.begin(), dirty_.end());
    const size_t lo = (size_t)*mm.first * MAXL, hi = (size_t)(*mm.second + 1) * MAXL;
    SlotDesc<T>* src = (SlotDesc<T>*)arena_.put_bytes(hdesc_.data() + lo, sizeof(SlotDesc<T>) * (hi - lo), &st);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(ddesc_ + lo, src, sizeof(SlotDesc<T>) * (hi - lo), hipMemcpyDeviceToDevice, st_));
    dirty_.clear();
    return W1_OK;
  }

  // after a synchronisation of the stream: staging copies have completed
  void free_retired() {
    for (auto& m : retire_) g_blocks.put(m.first, m.second);
    retire_.clear();
  }

  // the slot scalars after the work queued so far: copy queued, event
  // recorded; wait_scalars() waits for that event only, so work queued in
  // between (speculative iteration blocks) overlaps the host's processing
  int queue_scalars() {
    if (res_side_) {
      // resident levels launched on the side stream finish before the copy
      HIPCHK(hipStreamWaitEvent(st_, ev_res_, 0));
      res_side_ = false;
    }
    HIPCHK(hipMemcpyAsync(hsc_, dsc_, sizeof(SlotScalars) * cap_, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipEventRecord(ev_sc_, st_));
    return W1_OK;
  }
  int read_scalars() {
    int st = queue_scalars();
    if (st) return st;
    return wait_scalars();
  }
  int wait_scalars() {
    HIPCHK(hipEventSynchronize(ev_sc_));
    free_retired();
    for (auto& t : tune_pending_) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) g_tuner().report(t.entry, t.arm, ms, t.units);
      tune_pool_.push_back(t.a);
      tune_pool_.push_back(t.b);
    }
    tune_pending_.clear();
    if (prof_.on) {
      for (auto& ru : resident_pending_) {
        double u = 0;
        for (auto* r : ru.second) {
          const int it = hsc_[r->slot].iters;
          u += (double)(it - r->res_iters_seen) * node_count(r->sides[r->level]);
          r->res_iters_seen = it;
        }
        prof_.set_units(ru.first, u, 0.0);
      }
      prof_.harvest();
    }
    resident_pending_.clear();
    return W1_OK;
  }

  // -- work lists --------------------------------------------------------
  // XCD-aware order: a launch's workgroup i normally runs on XCD i mod 8
  // (the dispatcher's round robin; not guaranteed when launches follow
  // each other closely), so each XCD mostly receives spatially contiguous
  // tiles (a slot's row band, or whole slots when there are many) and halo
  // re-reads hit its own L2.  Only locality depends on it, not results.
  static std::vector<Work> order_xcd(std::vector<std::vector<Work>>& q) {
    size_t mx = 0;
    for (auto& v : q) mx = std::max(mx, v.size());
    std::vector<Work> out;
    out.reserve(mx * 8);
    for (size_t k = 0; k < mx; ++k)
      for (int x = 0; x < 8; ++x) out.push_back(k < q[x].size() ? q[x][k] : make_int4(-1, 0, 0, 0));
    // trailing padding carries no work: drop it
    while (!out.empty() && out.back().x < 0) out.pop_back();
    return out;
  }
  template <typename F>
  std::vector<Work> make_work(const std::vector<std::pair<Request*, int>>& lv, F tiles) {
    std::vector<std::vector<Work>> q(8);
    int rank = 0;
    for (auto& e : lv) {
      int ti, tj;
      tiles(e.first->sides[e.second], &ti, &tj);
      for (int a = 0; a < ti; ++a)
        for (int b = 0; b < tj; ++b) {
          const int x = lv.size() >= 8 ? rank % 8 : (a * 8) / ti;
          q[x].push_back(make_int4(dx(e.first, e.second), a, b, a * tj + b));
        }
      ++rank;
    }
    return order_xcd(q);
  }
  std::vector<Work> simple_work(const std::vector<std::pair<Request*, int>>& lv) {
    return make_work(lv, [](int n, int* ti, int* tj) {
      *ti = simple_ti(n);
      *tj = simple_tj(n);
    });
  }
  std::vector<Work> gemm_work(const std::vector<std::pair<Request*, int>>& lv) {
    return make_work(lv, [](int n, int* ti, int* tj) { *ti = *tj = dct_t<T>(n); });
  }
  std::vector<Work> tiled_work(const std::vector<std::pair<Request*, int>>& lv, int rh, int rw, int S) {
    return make_work(lv, [rh, rw, S](int n, int* ti, int* tj) {
      *ti = tiled_ti(n, rh, S);
      *tj = tiled_tj(n, rw, S);
    });
  }
  static std::vector<std::pair<Request*, int>> at_level(const std::vector<Request*>& rs) {
    std::vector<std::pair<Request*, int>> v;
    for (auto* r : rs) v.emplace_back(r, r->level);
    return v;
  }
  static std::vector<std::pair<Request*, int>> at_finest(const std::vector<Request*>& rs) {
    std::vector<std::pair<Request*, int>> v;
    for (auto* r : rs) v.emplace_back(r, r->prm.levels - 1);
    return v;
  }

  // device lists cached until the set of running slots or their levels
  // change (generation counter); each list has its own pinned staging copy,
  // rewritten only after the previous upload from it has completed
  struct DevList {
    void* d = nullptr;
    void* h = nullptr;
    size_t cap = 0;
    int n = 0;
    std::vector<size_t> off, cnt;   // packed lists: offsets and counts
    uint64_t gen = ~0ull;
    hipEvent_t ev = nullptr;
  };
  // upload into a list's device buffer from its own pinned copy (grown as
  // needed); the copy is rewritten only after its previous upload completed
  int upload_list(DevList& L, const void* src, size_t nbytes) {
    const size_t bytes = std::max<size_t>(nbytes, 16);
    if (L.ev && hipEventSynchronize(L.ev) != hipSuccess) return W1_EDEVICE;
    if (bytes > L.cap) {
      // kernels queued earlier may still read the old list
      if (L.d && hipStreamSynchronize(st_) != hipSuccess) return W1_EDEVICE;
      (void)hipFree(L.d);
      (void)hipHostFree(L.h);
      L.d = L.h = nullptr;
      L.cap = bytes * 2;
      if (dev_malloc(&L.d, L.cap) != hipSuccess || hipHostMalloc(&L.h, L.cap, hipHostMallocDefault) != hipSuccess) {
        L.cap = 0;
        g_err = "work list allocation failed";
        return W1_ENOMEM;
      }
    }
    if (!L.ev && hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess) return W1_EDEVICE;
    if (nbytes) std::memcpy(L.h, src, nbytes);
    if (hipMemcpyAsync(L.d, L.h, std::max<size_t>(nbytes, 1), hipMemcpyHostToDevice, st_) != hipSuccess ||
        hipEventRecord(L.ev, st_) != hipSuccess)
      return W1_EDEVICE;
    L.gen = gen_;
    ++n_uploads_;
    return W1_OK;
  }
  template <typename X, typename F>
  X* cached(const std::string& key, F build, int* count, int* status) {
    DevList& L = lists_[key];
    if (L.gen != gen_) {
      std::vector<X> v = build();
      *status = upload_list(L, v.data(), v.size() * sizeof(X));
      if (*status) return nullptr;
      L.n = (int)v.size();
    }
    *count = L.n;
    return (X*)L.d;
  }
  // several lists of one launch sequence in one buffer: one upload per group
  struct Packed {
    std::vector<char> b;
    std::vector<size_t> off, cnt;
    template <typename X>
    void add(const std::vector<X>& v) {
      const size_t o = align256(b.size());
      b.resize(o + std::max<size_t>(v.size() * sizeof(X), 1));
      if (!v.empty()) std::memcpy(b.data() + o, v.data(), v.size() * sizeof(X));
      off.push_back(o);
      cnt.push_back(v.size());
    }
  };
  template <typename F>
  char* cached_packed(const std::string& key, F build, std::vector<size_t>* off, std::vector<size_t>* cnt,
                      int* status) {
    DevList& L = lists_[key];
    if (L.gen != gen_) {
      if (capturing_) {
        // a list that is not on the device yet cannot be uploaded inside a
        // capture: the step runs its blocks eagerly instead
        *status = kNotCaptured;
        return nullptr;
      }
      Packed p = build();
      *status = upload_list(L, p.b.data(), p.b.size());
      if (*status) return nullptr;
      L.off = p.off;
      L.cnt = p.cnt;
    }
    *off = L.off;
    *cnt = L.cnt;
    return (char*)L.d;
  }

  int reduce_lists(const std::vector<std::pair<Request*, int>>& lv, int (*tiles)(int), int** didx_out,
                   int** dnt_out) {
    int st = W1_OK;
    std::vector<int> idx, nt;
    for (auto& e : lv) {
      idx.push_back(dx(e.first, e.second));
      nt.push_back(tiles(e.first->sides[e.second]));
    }
    *didx_out = arena_.put(idx, &st);
    if (st) return st;
    *dnt_out = arena_.put(nt, &st);
    return st;
  }
  static int simple_tiles_f(int n) { return simple_tiles(n); }

  // -- preparation: masses -> rho pyramid (Sec. 2.2, restriction) --------
  int run_prep(std::vector<Request*>& prep) {
    int st = W1_OK;
    st = flush_desc();
    if (st) return st;
    auto fin = at_finest(prep);
    {
      auto w = simple_work(fin);
      Work* dw = arena_.put(w, &st);
      if (st) return st;
      K<T>::prep_stats(st_, dw, (int)w.size(), ddesc_);
      int *di, *dn;
      st = reduce_lists(fin, simple_tiles_f, &di, &dn);
      if (st) return st;
      K<T>::reduce(st_, di, dn, (int)fin.size(), ddesc_, dsc_, 3, 0, 0u);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(hsc_, dsc_, sizeof(SlotScalars) * cap_, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    free_retired();
    std::vector<Request*> good;
    for (auto* r : prep) {
      const SlotScalars& s = hsc_[r->slot];
      const double a = s.sums[0], b = s.sums[1];
      const bool bad = s.sums[2] > 0 || !(a > 0) || !(std::fabs(a - b) <= 1e-9 * a);
      if (bad) {
        r->res.status = W1_SOLVE_REJECTED;
        r->res.w1 = r->res.dual = r->res.lo = r->res.hi = r->res.kkt = NAN;
        r->state = Request::DONE;
        r->res.seconds = now_seconds() - r->t_submit;
        ++gen_;
      } else {
        good.push_back(r);
      }
    }
    if (good.empty()) return W1_OK;
    auto gfin = at_finest(good);
    {
      auto w = simple_work(gfin);
      Work* dw = arena_.put(w, &st);
      if (st) return st;
      K<T>::prep_scale(st_, dw, (int)w.size(), ddesc_, dsc_);
    }
    int maxL = 0;
    for (auto* r : good) maxL = std::max(maxL, r->prm.levels);
    // depth 0 is the finest level of every request, depth k its k-th coarser
    for (int depth = 0; depth < maxL; ++depth) {
      std::vector<std::pair<Request*, int>> lv;
      for (auto* r : good)
        if (r->prm.levels - 1 - depth >= 0) lv.emplace_back(r, r->prm.levels - 1 - depth);
      if (lv.empty()) continue;
      auto w = simple_work(lv);
      Work* dw = arena_.put(w, &st);
      if (st) return st;
      int *di, *dn;
      st = reduce_lists(lv, simple_tiles_f, &di, &dn);
      if (st) return st;
      if (depth > 0) {
        K<T>::restrict_level(st_, dw, (int)w.size(), ddesc_);
        K<T>::reduce(st_, di, dn, (int)lv.size(), ddesc_, dsc_, 2, 0, 0u);
        K<T>::scale_level(st_, dw, (int)w.size(), ddesc_, dsc_);
      }
      K<T>::rho_diff(st_, dw, (int)w.size(), ddesc_);
      K<T>::reduce(st_, di, dn, (int)lv.size(), ddesc_, dsc_, 1, 0, 0u);
      K<T>::rho_write(st_, dw, (int)w.size(), ddesc_, dsc_);
    }
    HIPCHK(hipGetLastError());
    return start_first_level(good);
  }

  // level 1 starts from zero (Algorithms 3 and 4)
  int start_first_level(const std::vector<Request*>& rs) {
    int st = W1_OK;
    for (auto* r : rs) start_level(r, 0);
    st = flush_desc();
    if (st) return st;
    auto lv = at_level(rs);
    auto w = simple_work(lv);
    Work* dw = arena_.put(w, &st);
    if (st) return st;
    unsigned mask = 0;
    for (auto* r : rs) mask |= r->kind == K_PLAIN ? 0x7u : 0x3Fu;
    K<T>::zero(st_, dw, (int)w.size(), ddesc_, mask);
    K<T>::reset_scalars(st_, dw, (int)w.size(), dsc_);
    HIPCHK(hipGetLastError());
    return W1_OK;
  }

  void start_level(Request* r, int l) {
    r->level = l;
    r->res_iters_seen = 0;
    r->state = Request::RUN;
    r->t_level = now_seconds();
    const bool allow = !(r->prm.flags & W1_FLAG_NO_RESIDENT);
    const int side = r->sides[l] + 1;
    r->resident_level = allow && (r->kind == K_PLAIN ? side <= K<T>::plain_resident_max_side()
                                                     : side <= K<T>::prox_resident_max_side());
    // descriptors are fixed at admission; only the work lists change
    ++gen_;
    ++n_levels_;
  }

  // -- resident levels (both algorithms) -----------------------------------
  // `budget_us` bounds a launch to about that much device time (0: run to
  // the stop test); one launch per (kind, check_every, metric).  With
  // `side`, the launches run on the side stream (after this step's uploads)
  // and the next read of the slot scalars waits for them: resident levels
  // and the batched launches touch disjoint slots, descriptors are not
  // rewritten before that read, and the upload arena is reset only after it.
  int launch_resident(std::vector<Request*>& R, double budget_us, bool side) {
    int st = W1_OK;
    std::map<std::tuple<int, int, int>, std::vector<Request*>> groups;
    for (auto* r : R) groups[std::make_tuple(r->kind, r->prm.check_every, r->prm.metric)].push_back(r);
    std::vector<int*> lists;
    for (auto& kv : groups) {
      std::vector<int> ids;
      for (auto* r : kv.second) ids.push_back(dx(r, r->level));
      lists.push_back(arena_.put(ids, &st));
      if (st) return st;
    }
    hipStream_t ls = st_;
    if (side) {
      HIPCHK(hipEventRecord(ev_up_, st_));
      HIPCHK(hipStreamWaitEvent(rs_, ev_up_, 0));
      ls = rs_;
    }
    size_t gi = 0;
    for (auto& kv : groups) {
      const int kind = std::get<0>(kv.first), ce = std::get<1>(kv.first), metric = std::get<2>(kv.first);
      int* di = lists[gi++];
      int maxside = 0;
      for (auto* r : kv.second) maxside = std::max(maxside, r->sides[r->level] + 1);
      const int nids = (int)kv.second.size();
      // rough cost of one iteration of the largest level in the group
      const double s3 = std::pow(maxside / 65.0, kind == K_PLAIN ? 2.0 : 3.0);
      const double it_us = kind == K_PLAIN ? 3.6 * s3 : 8.0 * s3 + 0.5;
      int chunk = 0;
      if (budget_us > 0) chunk = std::max(1, (int)(budget_us / it_us));
      const int c = chunk > 0 ? ((chunk + ce - 1) / ce) * ce : 0;
      const int pi = prof_.begin(kind == K_PLAIN ? W1_FAM_PLAIN_RESIDENT : W1_FAM_PROX_RESIDENT, ls, false);
      if (kind == K_PLAIN)
        K<T>::plain_resident(ls, di, nids, ddesc_, dsc_, maxside, ce, c, metric);
      else
        K<T>::prox_resident(ls, di, nids, ddesc_, dsc_, maxside, ce, c, metric);
      prof_.end(pi, kind == K_PLAIN ? W1_FAM_PLAIN_RESIDENT : W1_FAM_PROX_RESIDENT, 0, 0, 0, ls);
      if (pi >= 0) resident_pending_.emplace_back(pi, kv.second);
    }
    HIPCHK(hipGetLastError());
    if (side) {
      HIPCHK(hipEventRecord(ev_res_, rs_));
      res_side_ = true;
    }
    return W1_OK;
  }

  // -- plain: one block of check_every iterations, tiled -------------------
  // spec: a speculative block (never timed by the autotuner)
  // pair: -1 a block with its stop test; 0 the first of two blocks whose
  // stop tests run together after the second (1).  A pair needs one launch
  // per block: the second launch then reads the first's output set and
  // leaves it intact, so a slot that stops after the first block stops on
  // that block's iterate, as with a test per block; the partials of the
  // two blocks sit side by side in the slot's partial buffer.
  int launch_tiled_block(std::vector<Request*>& P, int group, bool spec = false, int pair = -1) {
    int st = W1_OK;
    const int ce = P[0]->prm.check_every;
    const bool fpr = P[0]->prm.stop_rule == W1_STOP_FPR;
    double nodes = 0;
    for (auto* r : P) nodes += node_count(r->sides[r->level]);
    const int prec = sizeof(T) == 8 ? W1_FP64 : W1_FP32;
    int arm = -1;
    long entry = -1;
    if ((int)pair_open_.size() <= group) {
      pair_open_.resize(group + 1, 0);
      pair_tc_.resize(group + 1);
    }
    const bool second = pair == 1 && pair_open_[group];
    pair_open_[group] = 0;
    TileChoice tc;
    if (second) {
      tc = pair_tc_[group];   // the first block's shape (never a tuner trial)
    } else {
      tc = g_tuner().pick(prec, nodes, ce, P[0]->prm.block_steps, &arm, &entry);
      if (spec) arm = -1;
    }
    const int nl = ce / tc.steps;   // the tuner only offers divisors of ce
    bool first = false;
    if (pair == 0 && pairs_ && fpr && nl == 1) {
      first = true;
      for (auto* r : P) {
        const int n = r->sides[r->level];
        if (2 * tiled_ti(n, tc.rh, tc.steps) * tiled_tj(n, tc.rw, tc.steps) > part_tiles(r->prm.n)) first = false;
      }
      if (first) {
        pair_open_[group] = 1;
        pair_tc_[group] = tc;
      }
    }
    auto lv = at_level(P);
    const std::string key = "P" + std::to_string(group) + "_" + std::to_string(tc.rh) + "x" + std::to_string(tc.rw) +
                            "_" + std::to_string(tc.steps);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (arm >= 0) {
      t0 = tune_event();
      t1 = tune_event();
    }
    // tiled work, slot ids, per-slot tile counts of the stop-test partials
    // (and the node tiles of the KKT evaluation)
    std::vector<size_t> off, cnt;
    char* base = cached_packed(key, [&] {
      Packed p;
      p.add(tiled_work(lv, tc.rh, tc.rw, tc.steps));
      std::vector<int> ids, nt;
      for (auto* r : P) {
        const int n = r->sides[r->level];
        ids.push_back(dx(r, r->level));
        nt.push_back(fpr ? tiled_ti(n, tc.rh, tc.steps) * tiled_tj(n, tc.rw, tc.steps) : simple_tiles(n));
      }
      p.add(ids);
      p.add(nt);
      if (!fpr) {
        p.add(simple_work(lv));
        p.add(gemm_work(lv));
      }
      return p;
    }, &off, &cnt, &st);
    if (st) return st;
    Work* w = (Work*)(base + off[0]);
    const int nw = (int)cnt[0];
    int* di = (int*)(base + off[1]);
    int* dn = (int*)(base + off[2]);
    const int ns = (int)cnt[1];
    const double wb = 7.0 * sizeof(T);  // read m1 m2 phi rho, write m1 m2 phi
    // node updates the launch computes, the overlapping halo included
    // (reported in the profile's fifth field for this family)
    double computed = 0;
    for (auto* r : P) computed += tiled_computed(r->sides[r->level], tc.rh, tc.rw, tc.steps);
    if (t0 && t1) HIPCHK(hipEventRecord(t0, st_));
    for (int li = 0; li < nl; ++li) {
      const bool chk = fpr && li == nl - 1;
      hipEvent_t e0, e1;
      const int pi = prof_.begin_ext(W1_FAM_PLAIN_TILED, &e0, &e1);
      // the second of a pair reads the set the first wrote (the stop test
      // that would flip the slot's current set has not run in between)
      K<T>::plain_tiled(st_, w, nw, ddesc_, dsc_, second ? 1 : li, tc.steps, tc.rh, tc.rw, chk, P[0]->prm.metric,
                        tc.nwv, second ? 1 : 0, e0, e1);
      prof_.end(pi, W1_FAM_PLAIN_TILED, nodes * tc.steps, nodes * tc.steps * wb, computed * tc.steps);
    }
    if (t0 && t1) {
      HIPCHK(hipEventRecord(t1, st_));
      tune_pending_.push_back(TunePend{t0, t1, entry, arm, nodes * ce});
    }
    if (!fpr) {
      // KKT: the minimum-norm correction potential (A A*)^{-1}(A m - rho)
      // into plane 6, then the partials
      Work* ksw = (Work*)(base + off[3]);
      const int nksw = (int)cnt[3];
      K<T>::div_pre(st_, ksw, nksw, ddesc_, dsc_, 2, K_PLAIN, 1, nl & 1);
      poisson((Work*)(base + off[4]), (int)cnt[4], 6, 1, lv);
      K<T>::kkt(st_, ksw, nksw, ddesc_, dsc_, K_PLAIN, nl & 1, 1);
    }
    if (!first) K<T>::check(st_, di, dn, ns, ddesc_, dsc_, K_PLAIN, ce, nl, second ? 2 : 1);
    HIPCHK(hipGetLastError());
    return W1_OK;
  }

  // -- Poisson solve through four DCT passes ------------------------------
  void poisson(Work* gw, int ng, int dst, int gate, const std::vector<std::pair<Request*, int>>& lv) {
    if constexpr (sizeof(T) == 4) {
      // each slot takes the FFT path or the folded matrix passes by its
      // transform length; the kernels of the other path return at once
      unsigned sizes = 0;
      bool fold = false;
      for (auto& e : lv) {
        const int N = e.first->sides[e.second] + 1;
        if (uses_fft(N, 4)) sizes |= 1u << __builtin_ctz((unsigned)(2 * (N - 1)));
        else fold = true;
      }
      if (fold) K<T>::poisson_fold(st_, gw, ng, ddesc_, dsc_, dst, gate);
      if (sizes) poisson_fft(st_, gw, ng, (const SlotDesc<float>*)ddesc_, dsc_, dst, gate, sizes);
      return;
    }
    K<T>::gemm(st_, gw, ng, ddesc_, dsc_, 0, 6, 7, 1, false, gate);   // rows:    X C^T
    K<T>::gemm(st_, gw, ng, ddesc_, dsc_, 1, 7, 6, 0, true, gate);    // columns: C X, / lambda
    K<T>::gemm(st_, gw, ng, ddesc_, dsc_, 1, 6, 7, 1, false, gate);   // columns: C^T X
    K<T>::gemm(st_, gw, ng, ddesc_, dsc_, 0, 7, dst, 0, false, gate); // rows:    X C
  }

  // -- prox: one block of check_every iterations ---------------------------
  int launch_prox_block(std::vector<Request*>& X, int group) {
    int st = W1_OK;
    const int ce = X[0]->prm.check_every;
    const bool fpr = X[0]->prm.stop_rule == W1_STOP_FPR;
    auto lv = at_level(X);
    const std::string key = "X" + std::to_string(group);
    std::vector<size_t> off, cnt;
    char* base = cached_packed(key, [&] {
      Packed p;
      p.add(simple_work(lv));
      p.add(gemm_work(lv));
      std::vector<int> ids, nt;
      for (auto* r : X) {
        ids.push_back(dx(r, r->level));
        nt.push_back(simple_tiles(r->sides[r->level]));
      }
      p.add(ids);
      p.add(nt);
      return p;
    }, &off, &cnt, &st);
    if (st) return st;
    Work* dsw = (Work*)(base + off[0]);
    Work* dgw = (Work*)(base + off[1]);
    int* di = (int*)(base + off[2]);
    int* dn = (int*)(base + off[3]);
    const int nsw = (int)cnt[0], ngw = (int)cnt[1], ns = (int)cnt[2];
    double nodes = 0, flops = 0, dbytes = 0;
    for (auto* r : X) {
      const int n1 = r->sides[r->level] + 1;
      const double N = n1;
      nodes += N * N;
      if (uses_fft(n1, (int)sizeof(T))) {
        // five passes over the plane (three transforms of line pairs, two
        // transposes); flops of the line transforms, conventionally counted
        flops += fft_poisson_flops(n1);
        dbytes += N * N * 10.0 * sizeof(T);
      } else {
        // the FP32 passes fold each length-N product into two of about
        // half the length
        flops += (sizeof(T) == 4 ? 4.0 : 8.0) * N * N * N;
        dbytes += N * N * 8.0 * sizeof(T);
      }
    }
    for (int it = 0; it < ce; ++it) {
      int pi = prof_.begin(W1_FAM_PROX_ELEM);
      K<T>::div_pre(st_, dsw, nsw, ddesc_, dsc_, 0, K_PROX, 1);
      prof_.end(pi, W1_FAM_PROX_ELEM, nodes, nodes * 6.0 * sizeof(T), 0);
      pi = prof_.begin(W1_FAM_DCT);
      poisson(dgw, ngw, 6, 1, lv);
      prof_.end(pi, W1_FAM_DCT, nodes, dbytes, flops);
      pi = prof_.begin(W1_FAM_PROX_ELEM);
      K<T>::prox_post(st_, dsw, nsw, ddesc_, dsc_, fpr && it == ce - 1);
      prof_.end(pi, W1_FAM_PROX_ELEM, 0, nodes * 13.0 * sizeof(T), 0);
    }
    if (!fpr) {
      // KKT: psi (Appendix B) into plane 8, the correction potential into 6
      K<T>::div_pre(st_, dsw, nsw, ddesc_, dsc_, 1, K_PROX, 1);
      poisson(dgw, ngw, 8, 1, lv);
      K<T>::div_pre(st_, dsw, nsw, ddesc_, dsc_, 2, K_PROX, 1);
      poisson(dgw, ngw, 6, 1, lv);
      K<T>::kkt(st_, dsw, nsw, ddesc_, dsc_, K_PROX, 0, 1);
    }
    K<T>::check(st_, di, dn, ns, ddesc_, dsc_, K_PROX, ce, 0);
    HIPCHK(hipGetLastError());
    return W1_OK;
  }

  // -- next level: prolongation (Sec. 3.3) ---------------------------------
  int advance_levels(std::vector<Request*>& up) {
    int st = W1_OK;
    std::vector<Request*> plain, prox;
    for (auto* r : up) (r->kind == K_PLAIN ? plain : prox).push_back(r);
    st = level_costs(up);
    if (st) return st;
    for (auto* r : up) start_level(r, r->level + 1);
    st = flush_desc();
    if (st) return st;
    for (int pass = 0; pass < 2; ++pass) {
      auto& grp = pass == 0 ? plain : prox;
      if (grp.empty()) continue;
      auto w = simple_work(at_level(grp));
      Work* dw = arena_.put(w, &st);
      if (st) return st;
      K<T>::prolong(st_, dw, (int)w.size(), ddesc_, dsc_, pass == 0 ? K_PLAIN : K_PROX);
      // after the prolongation, which reads the coarse plane set
      K<T>::reset_scalars(st_, dw, (int)w.size(), dsc_);
    }
    HIPCHK(hipGetLastError());
    return W1_OK;
  }

  // f(m^{K_l}) of the level just finished, for requests that ask for it:
  // the certificate's sums without the Poisson correction, read back at
  // once (the slot's partial-sum area and eval scalars are free between
  // levels; prox slots' potential plane is stale here, only P is kept)
  int level_costs(const std::vector<Request*>& up) {
    int st = W1_OK;
    bool any = false;
    for (int kind : {K_PLAIN, K_PROX}) {
      std::vector<Request*> grp;
      for (auto* r : up)
        if (r->kind == kind && (r->prm.flags & W1_FLAG_LEVEL_COST)) grp.push_back(r);
      if (grp.empty()) continue;
      any = true;
      auto lv = at_level(grp);
      auto sw = simple_work(lv);
      Work* dsw = arena_.put(sw, &st);
      if (st) return st;
      K<T>::eval_sums(st_, dsw, (int)sw.size(), ddesc_, dsc_, kind, 0);
      int *di, *dn;
      st = reduce_lists(lv, simple_tiles_f, &di, &dn);
      if (st) return st;
      K<T>::eval_final(st_, di, dn, (int)grp.size(), ddesc_, dsc_, kind, 0);
      HIPCHK(hipGetLastError());
    }
    if (!any) return W1_OK;
    HIPCHK(hipMemcpyAsync(hsc_, dsc_, sizeof(SlotScalars) * cap_, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    for (auto* r : up)
      if (r->prm.flags & W1_FLAG_LEVEL_COST)
        r->res.level_w1[r->level] = domain_scale(r->prm) * hsc_[r->slot].eval[0];
    return W1_OK;
  }

  // -- FP64 certificate and field export on the finest level ---------------
  int finalize(std::vector<Request*>& fin) {
    int st = W1_OK;
    // passes: (plain, prox) x (with, without the certificate)
    for (int pass = 0; pass < 4; ++pass) {
      const int kind = (pass & 1) == 0 ? K_PLAIN : K_PROX;
      const int cert = pass < 2 ? 1 : 0;
      std::vector<Request*> grp;
      for (auto* r : fin)
        if (r->kind == kind && (cert == 0) == ((r->prm.flags & W1_FLAG_NO_CERT) != 0)) grp.push_back(r);
      if (grp.empty()) continue;
      auto lv = at_finest(grp);
      auto sw = simple_work(lv);
      auto gw = gemm_work(lv);
      Work* dsw = arena_.put(sw, &st);
      if (st) return st;
      Work* dgw = arena_.put(gw, &st);
      if (st) return st;
      if (kind == K_PROX) {
        K<T>::div_pre(st_, dsw, (int)sw.size(), ddesc_, dsc_, 1, kind, 0);
        poisson(dgw, (int)gw.size(), 8, 0, lv);
      }
      // Algorithm 2 with the certificate: the returned flux is the FP64
      // re-projection of m^K onto {A m = rho} (m^K is feasible by
      // construction; the FP32 rounding of its last Poisson solve is
      // removed), and the certificate's correction is that flux's own
      const int polish = kind == K_PROX && cert ? 1 : 0;
      if (cert) {
        K<T>::div_pre(st_, dsw, (int)sw.size(), ddesc_, dsc_, 2, kind, 0);
        poisson(dgw, (int)gw.size(), polish ? POLISH_PLANE : 6, 0, lv);
      }
      if (polish) {
        K<T>::div_pre(st_, dsw, (int)sw.size(), ddesc_, dsc_, 3, kind, 0);
        poisson(dgw, (int)gw.size(), 6, 0, lv);
      }
      K<T>::eval_sums(st_, dsw, (int)sw.size(), ddesc_, dsc_, kind, cert, polish);
      int *di, *dn;
      st = reduce_lists(lv, simple_tiles_f, &di, &dn);
      if (st) return st;
      K<T>::eval_final(st_, di, dn, (int)grp.size(), ddesc_, dsc_, kind, cert);
      K<T>::export_fields(st_, dsw, (int)sw.size(), ddesc_, dsc_, kind, polish);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(hsc_, dsc_, sizeof(SlotScalars) * cap_, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    const double t = now_seconds();
    for (auto* r : fin) {
      const SlotScalars& s = hsc_[r->slot];
      const double c = domain_scale(r->prm);
      r->res.w1 = c * s.eval[0];
      r->res.level_w1[r->level] = c * s.eval[0];
      r->res.dual = c * s.eval[1];
      r->res.lo = c * s.eval[2];
      r->res.hi = c * s.eval[3];
      r->res.kkt = s.eval[4];
      r->res.seconds = t - r->t_submit;
      r->res.queue_seconds = r->t_admit - r->t_submit;
      r->state = Request::DONE;
      r->fields_ready = false;
    }
    ++gen_;
    return W1_OK;
  }

  // -- captured block sequences (W1_GRAPH=1) -------------------------------
  // One graph per (first block, end, speculative) of the current
  // generation: the launches of a block sequence depend only on the work
  // lists (fixed within a generation), the autotuner's settled shapes and
  // the pairing of blocks, so a replay issues the same kernels with the
  // same arguments; the gated kernels read the slots' state on the device.
  // A new generation drops every graph.
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t gen = ~0ull;
  };
  template <typename F>
  int graph_blocks(int from, int to, bool spec, F& blocks) {
    if (graphs_gen_ != gen_) {
      drop_graphs();
      graphs_gen_ = gen_;
    }
    GraphEntry& g = graphs_[std::make_tuple(from, to, spec)];
    if (!g.exec) {
      HIPCHK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
      capturing_ = true;
      const int st = blocks(from, to, spec);
      capturing_ = false;
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(st_, &graph);
      if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        graphs_.erase(std::make_tuple(from, to, spec));
        return st == kNotCaptured ? blocks(from, to, spec) : st;
      }
      if (e != hipSuccess) return hip_status(e, "hipStreamEndCapture(blocks)");
      const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        g.exec = nullptr;
        return hip_status(ei, "hipGraphInstantiate(blocks)");
      }
      g.gen = gen_;
      ++n_graphs_;
    }
    HIPCHK(hipGraphLaunch(g.exec, st_));
    return W1_OK;
  }
  void drop_graphs() {
    if (graphs_.empty()) return;
    // a replay of the previous step (its speculative blocks) may still run
    (void)hipStreamSynchronize(st_);
    for (auto& kv : graphs_)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    graphs_.clear();
  }
  static constexpr int kNotCaptured = -1000;   // internal: capture abandoned
  bool graph_ = false;
  bool capturing_ = false;
  uint64_t graphs_gen_ = ~0ull;
  uint64_t lists_gen_ = ~0ull;   // generation of the last block sequence issued
  int64_t n_graphs_ = 0;
  std::map<std::tuple<int, int, bool>, GraphEntry> graphs_;

  // timing events of the autotuner's exploration blocks
  struct TunePend {
    hipEvent_t a, b;
    long entry;
    int arm;
    double units;
  };
  hipEvent_t tune_event() {
    if (!tune_pool_.empty()) {
      hipEvent_t e = tune_pool_.back();
      tune_pool_.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  std::vector<TunePend> tune_pending_;
  std::vector<hipEvent_t> tune_pool_;
  std::vector<std::pair<size_t, char*>> retire_;
  int64_t n_steps_ = 0, n_levels_ = 0, n_uploads_ = 0, n_blocks_ = 0;

  int cap_;
  hipStream_t st_;
  hipStream_t rs_ = nullptr;        // side stream of the resident levels
  hipEvent_t ev_up_ = nullptr;      // this step's uploads, for the side stream
  hipEvent_t ev_res_ = nullptr;     // the side stream's launches of this step
  hipEvent_t ev_sc_ = nullptr;      // the slot scalars' copy of this step
  hipEvent_t ev_arena_ = nullptr;   // after the last upload of the previous step
  bool arena_pending_ = false;
  bool speculate_ = true;
  bool side_stream_ = true;
  bool pairs_ = true;                  // W1_PAIRED_CHECK=0: a stop test after every block
  double step_budget_us_ = kServedStepUs;   // device work queued per host synchronisation
  int nb_cap_ = kServedStepBlocks;          // and the most iteration blocks in it
  std::vector<char> pair_open_;        // per plain group: a pair's first block is queued
  std::vector<TileChoice> pair_tc_;    // its launch shape
  bool res_side_ = false;
  int64_t fail_at_ = 0;              // W1_FAIL_AT_STEP (tests only)
  Arena arena_;
  bool ok_ = false;
  std::vector<Request*> slots_;
  std::vector<SlotDesc<T>> hdesc_;
  SlotDesc<T>* ddesc_ = nullptr;
  SlotScalars* dsc_ = nullptr;
  SlotScalars* hsc_ = nullptr;
  std::vector<int> dirty_;
  uint64_t gen_ = 0;
  std::map<std::string, DevList> lists_;
  mutable Prof prof_;
  std::vector<std::pair<int, std::vector<Request*>>> resident_pending_;
};

std::unique_ptr<BatchBase> make_batch(bool fp64, int capacity, hipStream_t stream) {
  if (fp64) return std::unique_ptr<BatchBase>(new Batch<double>(capacity, stream));
  return std::unique_ptr<BatchBase>(new Batch<float>(capacity, stream));
}

}  // namespace w1
