// The Neumann Poisson solve u = (A A*)^{-1} r of the eq. (pdhg) projection
// and of Appendix B (the same kernels as w1_op_poisson) without any device
// allocation, for callers that cannot allocate: its working memory (the
// orthonormal DCT-II tables of length N = n+1, two node planes, the slot
// descriptor and the work list) lives in a file-scope device array,
// `scratch`, of NOALLOC_BYTES per GPU, held until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy is taken once per device with
// hipGetSymbolAddress (with that device current) and kept; every kernel
// argument and copy below uses that address.  Every call on one GPU shares
// that GPU's array and rewrites all of it, so calls that overlap on one GPU
// (other streams or host threads) race and must be serialised by the caller.
#include <cmath>
#include <mutex>

#include "engine.hpp"

namespace w1 {
namespace {

constexpr int NOALLOC_MAX_N = 512;                     // largest side n
constexpr size_t NOALLOC_BYTES = (size_t)12 << 20;     // 12 MiB per GPU
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_scratch_mu;
char* g_scratch[MAX_DEVICES] = {};

// the device address of the current device's array (taken on first use)
int scratch_base(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return W1_EDEVICE;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = (char*)p;
  }
  *out = g_scratch[dev];
  return W1_OK;
}

inline size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }
inline int cdiv_(int a, int b) { return (a + b - 1) / b; }

// byte offsets of the pieces inside the array for side n
template <typename T>
struct Layout {
  size_t desc, scal, work, p6, p7, C, Ct, Cp, Ctp, s, total;
  int tiles;   // work items (tiles x tiles per slot)
  explicit Layout(int n) {
    const int N = n + 1;
    tiles = sizeof(T) == 4 ? fold_tiles(N) : cdiv_(N, GEMM_T);
    const size_t plane = up256((size_t)N * N * sizeof(T));
    const size_t mat = up256((size_t)N * N * sizeof(T));
    size_t o = 0;
    desc = o;  o += up256(sizeof(SlotDesc<T>));
    scal = o;  o += up256(sizeof(SlotScalars));
    work = o;  o += up256((size_t)tiles * tiles * sizeof(Work));
    p6 = o;    o += plane;
    p7 = o;    o += plane;
    C = o;     o += mat;
    Ct = o;    o += mat;
    Cp = o;    o += sizeof(T) == 4 ? mat : 0;
    Ctp = o;   o += sizeof(T) == 4 ? mat : 0;
    s = o;     o += up256((size_t)N * sizeof(double));
    total = o;
  }
};

// The orthonormal DCT-II matrix of length N, C[k][j] = s_k cos(pi k (2j+1) /
// 2N) (s_0 = sqrt(1/N), else sqrt(2/N)), its transpose, for FP32 the rows
// in even-then-odd frequency order and that transpose, and the eigenvalue
// table 4 sin^2(pi k / 2N) of the Neumann Laplacian (the closed forms the
// engine's host-built tables use).
template <typename T>
__global__ __launch_bounds__(256) void k_na_tables(int N, T* __restrict__ C, T* __restrict__ Ct,
                                                   T* __restrict__ Cp, T* __restrict__ Ctp, double* __restrict__ s) {
  const double pi = 3.14159265358979323846;
  const int ne = N - N / 2;
  const long long NN = (long long)N * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < NN; e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / N), j = (int)(e - (long long)k * N);
    const double sk = k == 0 ? sqrt(1.0 / N) : sqrt(2.0 / N);
    const double v = sk * cos(pi * k * (2.0 * j + 1.0) / (2.0 * N));
    C[(size_t)k * N + j] = (T)v;
    Ct[(size_t)j * N + k] = (T)v;
    if (Cp) {
      const int src = k < ne ? 2 * k : 2 * (k - ne) + 1;   // row k of the folded order
      const double sp = src == 0 ? sqrt(1.0 / N) : sqrt(2.0 / N);
      const double vp = sp * cos(pi * src * (2.0 * j + 1.0) / (2.0 * N));
      Cp[(size_t)k * N + j] = (T)vp;
      Ctp[(size_t)j * N + k] = (T)vp;
    }
    if (e < N) {
      const double sn = sin(pi * (double)e / (2.0 * N));
      s[e] = 4.0 * sn * sn;
    }
  }
}

// the work list (descriptor 0, every tile of a tiles x tiles grid), the
// descriptor and cleared slot scalars
template <typename T>
__global__ __launch_bounds__(256) void k_na_setup(SlotDesc<T> d, SlotDesc<T>* __restrict__ dd,
                                                  SlotScalars* __restrict__ sc, Work* __restrict__ work, int tiles) {
  const int nw = tiles * tiles;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nw; e += gridDim.x * blockDim.x) {
    const int a = e / tiles, b = e - a * tiles;
    work[e] = make_int4(0, a, b, e);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *dd = d;
    SlotScalars z{};
    *sc = z;
  }
}

template <typename T>
int poisson_noalloc(int n, const void* r, void* u, hipStream_t s) {
  const Layout<T> L(n);
  if (L.total > NOALLOC_BYTES) return W1_EINVAL;   // not reached for n <= NOALLOC_MAX_N
  char* base = nullptr;
  int st = scratch_base(&base);
  if (st) return st;
  const int N = n + 1;
  SlotDesc<T> d{};
  d.n = n;
  d.pitch = N;
  d.h = 1.0 / n;
  d.ih = (T)(double)n;
  d.mud = d.taud = 0.5;
  d.mu = d.tau = (T)0.5;
  d.metric = 1;
  d.rule = RULE_FPR;
  d.tol = -1.0;
  d.cap = 1 << 30;
  d.p[6] = (T*)(base + L.p6);
  d.p[7] = (T*)(base + L.p7);
  d.p[8] = (T*)u;
  d.dctC = (const T*)(base + L.C);
  d.dctCt = (const T*)(base + L.Ct);
  d.dctCp = sizeof(T) == 4 ? (const T*)(base + L.Cp) : nullptr;
  d.dctCtp = sizeof(T) == 4 ? (const T*)(base + L.Ctp) : nullptr;
  d.dcts = (const double*)(base + L.s);
  auto* dd = (SlotDesc<T>*)(base + L.desc);
  auto* dsc = (SlotScalars*)(base + L.scal);
  auto* work = (Work*)(base + L.work);
  const int nw = L.tiles * L.tiles;
  hipLaunchKernelGGL(k_na_setup<T>, dim3(cdiv_(nw, 256)), dim3(256), 0, s, d, dd, dsc, work, L.tiles);
  const int tb = std::min(cdiv_(N * N, 256), 2048);
  hipLaunchKernelGGL(k_na_tables<T>, dim3(tb), dim3(256), 0, s, N, (T*)(base + L.C), (T*)(base + L.Ct),
                     sizeof(T) == 4 ? (T*)(base + L.Cp) : nullptr, sizeof(T) == 4 ? (T*)(base + L.Ctp) : nullptr,
                     (double*)(base + L.s));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "noalloc setup launch");
  // r (dense, pitch n+1) into plane 6; r and u may alias
  e = hipMemcpyAsync(d.p[6], r, (size_t)N * N * sizeof(T), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_status(e, "noalloc copy");
  if constexpr (sizeof(T) == 4) {
    K<T>::poisson_fold(s, work, nw, dd, dsc, 8, 0);
  } else {
    K<T>::gemm(s, work, nw, dd, dsc, 0, 6, 7, 1, false, 0);   // rows:    X C^T
    K<T>::gemm(s, work, nw, dd, dsc, 1, 7, 6, 0, true, 0);    // columns: C X, / lambda
    K<T>::gemm(s, work, nw, dd, dsc, 1, 6, 7, 1, false, 0);   // columns: C^T X
    K<T>::gemm(s, work, nw, dd, dsc, 0, 7, 8, 0, false, 0);   // rows:    X C
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "noalloc poisson launch");
  return W1_OK;
}

}  // namespace
}  // namespace w1

using namespace w1;

extern "C" int w1_op_poisson_noalloc(int32_t n, int32_t precision, const void* r, void* u, void* hip_stream) {
  if (n < 1 || n > NOALLOC_MAX_N || !r || !u) return W1_EINVAL;
  if (precision != W1_FP32 && precision != W1_FP64) return W1_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  return precision == W1_FP32 ? poisson_noalloc<float>(n, r, u, s) : poisson_noalloc<double>(n, r, u, s);
}

extern "C" size_t w1_noalloc_bytes(void) { return NOALLOC_BYTES; }
