// Algorithms 1 / 3 and 2 / 4 in d = 3 (the paper states the method for any d: the
// divergence of Sec. 2.2 summed over three axes, the interpolations of
// Sec. 3.3 as products of 1-D factors).  One pair per call (or a list of
// pairs over concurrent streams), levels run one after the other.
//
// Layout: a level of side n holds (n+1)^3 nodes, index
// e = (i1 (n+1) + i2) (n+1) + i3 with i3 contiguous; flux components m1, m2,
// m3 (m_a on the last node of axis a is not a variable and stays 0), the
// extrapolated flux b = 2 m+ - m (Algorithm 1) or v (Algorithm 2), vphi and
// vphibar, the potential phi, rho and the Poisson residual and scratch, all
// in the iterate precision T, plus two FP64 planes for the density pyramid
// and the DCT tables.
//
// An Algorithm 1 iteration is two node-parallel kernels: the flux half (reads
// phi at the node and its three forward neighbours, writes m+ and b) and the
// potential half (reads b at the node and its three backward neighbours,
// updates phi in place).  An Algorithm 2 iteration is a pre kernel
// (v = m - mu vphibar and r = A v - rho), the Neumann Poisson solve as six
// one-axis DCT passes (products with the orthonormal DCT matrix, on the
// matrix cores in FP32, the eigenvalue division fused into the third), and
// a post kernel (m+, vphi+, vphibar+).  The stop test's sums (R^k of eq.
// (pd_stop), G^k of eq. (pdhg_stop), or the normalised KKT residual) are
// block partials in FP64, finished by a one-block kernel that decides the
// stop on the device every `check_every` iterations; the iteration kernels
// skip their work once the level has stopped, so the host queues many
// blocks between its reads of the stop state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <thread>
#include <type_traits>
#include <vector>

#include "engine.hpp"
#include "mfma_tile.hpp"
#include "w1.h"

namespace w1 {
namespace cube {

constexpr int NT = 256;     // threads per block of every kernel here
constexpr int NQ3 = 8;      // FP64 partial sums per block
constexpr int MAXB = 2048;  // blocks of the node-parallel kernels (grid-stride)

// stop-test state of the running level in device memory: the iteration
// kernels of a block skip all work once `status` leaves G_RUN, so the host
// queues several blocks of `check_every` iterations between reads
enum { G_RUN = 0, G_CONV = 1, G_CAP = 2, G_DIVERGED = 3 };
struct Gate {
  int status;
  int iters;
  double measure;
  int rises;   // stop tests in a row whose measure rose
  int pad;
};

#define CHK(x)                                      \
  do {                                              \
    hipError_t _e = (x);                            \
    if (_e != hipSuccess) return hip_status(_e, #x); \
  } while (0)

template <typename T> __device__ __forceinline__ T abs3_(T a) { return a < T(0) ? -a : a; }
template <typename T> __device__ __forceinline__ T max3_(T a, T b) { return a > b ? a : b; }
template <typename T> __device__ __forceinline__ T min3_(T a, T b) { return a < b ? a : b; }
__device__ __forceinline__ float fma3_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma3_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float sqrt3_(float a) { return sqrtf(a); }
__device__ __forceinline__ double sqrt3_(double a) { return sqrt(a); }

// prox of mu ||.||_p at a node with three components.  p = 1: soft threshold
// per component; p = 2: isotropic shrink; p = inf: v minus its projection
// onto the l_1 ball of radius mu (Moreau, Sec. 4.2), the projection by the
// sort-and-threshold rule of Duchi et al.: with the magnitudes sorted
// decreasingly into u and partial sums c_j, k counts the j with
// u_j > (c_j - mu)/j and theta = (c_k - mu)/k; then each component keeps its
// sign and min(|v_i|, theta), and a vector inside the ball maps to 0.
template <typename T, int METRIC>
__device__ __forceinline__ void shrink3_(const T v[3], T mu, T o[3]) {
  if constexpr (METRIC == 1) {
    for (int a = 0; a < 3; ++a) {
      const T r = max3_(abs3_(v[a]) - mu, T(0));
      o[a] = v[a] < T(0) ? -r : r;
    }
  } else if constexpr (METRIC == 2) {
    const T s2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const T s = s2 > mu * mu ? T(1) - mu / sqrt3_(s2) : T(0);
    for (int a = 0; a < 3; ++a) o[a] = v[a] * s;
  } else {
    const T x = abs3_(v[0]), y = abs3_(v[1]), z = abs3_(v[2]);
    const T u0 = max3_(max3_(x, y), z), u2 = min3_(min3_(x, y), z);
    const T u1 = max3_(min3_(x, y), min3_(max3_(x, y), z));
    const T c2 = u0 + u1, c3 = c2 + u2;
    if (x + y + z <= mu) {
      o[0] = o[1] = o[2] = T(0);
      return;
    }
    const int k = 1 + (u1 > (c2 - mu) / T(2) ? 1 : 0) + (u2 > (c3 - mu) / T(3) ? 1 : 0);
    const T theta = k == 1 ? u0 - mu : (k == 2 ? (c2 - mu) / T(2) : (c3 - mu) / T(3));
    for (int a = 0; a < 3; ++a) {
      const T r = min3_(abs3_(v[a]), theta);
      o[a] = v[a] < T(0) ? -r : r;
    }
  }
}

template <typename T, int METRIC>
__device__ __forceinline__ T norm_p3_(T a, T b, T c) {
  const T x = abs3_(a), y = abs3_(b), z = abs3_(c);
  if constexpr (METRIC == 1) return x + y + z;
  else if constexpr (METRIC == 2) return sqrt3_(a * a + b * b + c * c);
  else return max3_(max3_(x, y), z);
}
// dual norm q of a gradient (inf, 2, 1 for p = 1, 2, inf)
template <typename T, int METRIC>
__device__ __forceinline__ T norm_q3_(T a, T b, T c) {
  const T x = abs3_(a), y = abs3_(b), z = abs3_(c);
  if constexpr (METRIC == 1) return max3_(max3_(x, y), z);
  else if constexpr (METRIC == 2) return sqrt3_(a * a + b * b + c * c);
  else return x + y + z;
}

struct Idx {
  int i1, i2, i3;
};
__device__ __forceinline__ Idx split_(long long e, int N1) {
  Idx r;
  r.i3 = (int)(e % N1);
  const long long q = e / N1;
  r.i2 = (int)(q % N1);
  r.i1 = (int)(q / N1);
  return r;
}

// block sum of NQ3 doubles into part[blockIdx.x * NQ3 + q]; q = 5 is a max
__device__ __forceinline__ void block_out_(double v[NQ3], double* part) {
  __shared__ double sh[NQ3][NT];
  for (int q = 0; q < NQ3; ++q) sh[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < NQ3; ++q) {
        const double a = sh[q][threadIdx.x], b = sh[q][threadIdx.x + w];
        sh[q][threadIdx.x] = q == 5 ? (a > b ? a : b) : a + b;
      }
    __syncthreads();
  }
  if (threadIdx.x < NQ3) part[(size_t)blockIdx.x * NQ3 + threadIdx.x] = sh[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// flux half: m+ = shrink(m + mu grad+ phi), b = 2 m+ - m
// ---------------------------------------------------------------------------
template <typename T, int METRIC>
__global__ __launch_bounds__(NT) void k3_flux(int n, T* __restrict__ m0, T* __restrict__ m1, T* __restrict__ m2,
                                              T* __restrict__ b0, T* __restrict__ b1, T* __restrict__ b2,
                                              const T* __restrict__ phi, T ih, T mu,
                                              const int* __restrict__ gate) {
  if (gate && *gate != G_RUN) return;
  const int N1 = n + 1;
  const long long S1 = (long long)N1 * N1, N = S1 * N1;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, N1);
    const T pc = phi[e];
    const T g0 = x.i1 < n ? (phi[e + S1] - pc) * ih : T(0);
    const T g1 = x.i2 < n ? (phi[e + N1] - pc) * ih : T(0);
    const T g2 = x.i3 < n ? (phi[e + 1] - pc) * ih : T(0);
    const T m[3] = {m0[e], m1[e], m2[e]};
    const T v[3] = {fma3_(mu, g0, m[0]), fma3_(mu, g1, m[1]), fma3_(mu, g2, m[2])};
    T o[3];
    shrink3_<T, METRIC>(v, mu, o);
    m0[e] = o[0];
    m1[e] = o[1];
    m2[e] = o[2];
    b0[e] = fma3_(T(2), o[0], -m[0]);
    b1[e] = fma3_(T(2), o[1], -m[1]);
    b2[e] = fma3_(T(2), o[2], -m[2]);
  }
}

// divergence of a flux at node e (Sec. 2.2 summed over the three axes),
// without the 1/h factor
template <typename T>
__device__ __forceinline__ T div3_(const T* f0, const T* f1, const T* f2, long long e, Idx x, int n, int N1,
                                   long long S1) {
  T s = (x.i1 < n ? f0[e] : T(0)) - (x.i1 > 0 ? f0[e - S1] : T(0));
  s += (x.i2 < n ? f1[e] : T(0)) - (x.i2 > 0 ? f1[e - N1] : T(0));
  s += (x.i3 < n ? f2[e] : T(0)) - (x.i3 > 0 ? f2[e - 1] : T(0));
  return s;
}

// ---------------------------------------------------------------------------
// potential half: phi+ = phi + tau (A b - rho); CHECK adds the sums of
// R^k: sum |dm|^2, sum dphi^2, sum dphi A dm (dm = b - m+)
// ---------------------------------------------------------------------------
template <typename T, bool CHECK>
__global__ __launch_bounds__(NT) void k3_pot(int n, const T* __restrict__ b0, const T* __restrict__ b1,
                                             const T* __restrict__ b2, const T* __restrict__ m0,
                                             const T* __restrict__ m1, const T* __restrict__ m2,
                                             T* __restrict__ phi, const T* __restrict__ rho, T ih, T tau,
                                             double* __restrict__ part, const int* __restrict__ gate) {
  if (gate && *gate != G_RUN) return;   // the same value for every thread of the launch
  const int N1 = n + 1;
  const long long S1 = (long long)N1 * N1, N = S1 * N1;
  double v[NQ3] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, N1);
    const T db = div3_(b0, b1, b2, e, x, n, N1, S1);
    const T pc = phi[e];
    const T pn = fma3_(tau, db * ih - rho[e], pc);
    phi[e] = pn;
    if constexpr (CHECK) {
      // dm at the node and at the backward neighbours: b - m+ there
      const T d0 = b0[e] - m0[e], d1 = b1[e] - m1[e], d2 = b2[e] - m2[e];
      T adm = (x.i1 < n ? d0 : T(0)) - (x.i1 > 0 ? b0[e - S1] - m0[e - S1] : T(0));
      adm += (x.i2 < n ? d1 : T(0)) - (x.i2 > 0 ? b1[e - N1] - m1[e - N1] : T(0));
      adm += (x.i3 < n ? d2 : T(0)) - (x.i3 > 0 ? b2[e - 1] - m2[e - 1] : T(0));
      const T dp = pn - pc;
      v[0] += (double)(d0 * d0) + (double)(d1 * d1) + (double)(d2 * d2);
      v[1] += (double)(dp * dp);
      v[2] += (double)(dp * (adm * ih));
    }
  }
  if constexpr (CHECK) block_out_(v, part);
}

// ---------------------------------------------------------------------------
// evaluation sums for a flux m and a potential pot taken with sign sgn
// (psi = sgn pot: -phi for Algorithm 1, the Appendix B potential for
// Algorithm 2): q0 sum ||m||_p, q1 sum psi rho, q4 sum
// (||grad psi||_q - 1)_+^2, q5 max ||grad psi||_q, q6 sum pot, and with the
// correction potential c = (A A*)^{-1}(A m - rho) (may be NULL) q2 sum
// |grad+ c|^2 (the squared norm of the least-norm flux correction A* c,
// over h^3) and q7 sum ||m - A* c||_p (the flux made feasible); q3 is 0
// ---------------------------------------------------------------------------
template <typename T, int METRIC>
__global__ __launch_bounds__(NT) void k3_eval(int n, const T* __restrict__ m0, const T* __restrict__ m1,
                                              const T* __restrict__ m2, const T* __restrict__ pot, double sgn,
                                              const T* __restrict__ rho, const T* __restrict__ corr,
                                              double* __restrict__ part, const int* __restrict__ gate) {
  if (gate && *gate != G_RUN) return;
  const int N1 = n + 1;
  const long long S1 = (long long)N1 * N1, N = S1 * N1;
  const double ih = (double)n;
  double v[NQ3] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, N1);
    const double a = (double)m0[e], b = (double)m1[e], c = (double)m2[e];
    const double pr = (double)pot[e], pc = sgn * pr, rr = (double)rho[e];
    const double g0 = x.i1 < n ? (sgn * (double)pot[e + S1] - pc) * ih : 0.0;
    const double g1 = x.i2 < n ? (sgn * (double)pot[e + N1] - pc) * ih : 0.0;
    const double g2 = x.i3 < n ? (sgn * (double)pot[e + 1] - pc) * ih : 0.0;
    const double gq = norm_q3_<double, METRIC>(g0, g1, g2);
    const double ex = gq > 1.0 ? gq - 1.0 : 0.0;
    v[0] += norm_p3_<double, METRIC>(a, b, c);
    v[1] += pc * rr;
    v[4] += ex * ex;
    v[5] = gq > v[5] ? gq : v[5];
    v[6] += pr;
    if (corr) {
      const double cc = (double)corr[e];
      const double c0 = x.i1 < n ? ((double)corr[e + S1] - cc) * ih : 0.0;
      const double c1 = x.i2 < n ? ((double)corr[e + N1] - cc) * ih : 0.0;
      const double c2 = x.i3 < n ? ((double)corr[e + 1] - cc) * ih : 0.0;
      v[2] += c0 * c0 + c1 * c1 + c2 * c2;
      v[7] += norm_p3_<double, METRIC>(a + c0, b + c1, c + c2);
    }
  }
  block_out_(v, part);
}

// sums the nb block partials (compensated; q5 a max) into out[0..NQ3)
// (thread 0 also receives them in q0)
__device__ __forceinline__ void final_sums_(const double* __restrict__ part, int nb, double* __restrict__ out,
                                            double q0[NQ3]);
__global__ __launch_bounds__(NT) void k3_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  double q[NQ3];
  final_sums_(part, nb, out, q);
}

// the stop test of a block of `steps` iterations (one block of threads):
// rule 2 R^k of eq. (pd_stop) (Algorithm 1, from the potential half's sums)
// or G^k of eq. (pdhg_stop) (Algorithm 2, from the post kernel's sums),
// rule 1 the normalised KKT residual from the evaluation sums (as the
// oracle defines it); the level stops at meas <= tol, on a non-finite
// measure, or at the cap
__global__ __launch_bounds__(NT) void k3_check(const double* __restrict__ part, int nb, double* __restrict__ sums,
                                               Gate* __restrict__ gate, int kind, int rule, double mu, double tau,
                                               int n, double tol, int steps, int cap, int divwin) {
  if (gate->status != G_RUN) return;   // read by every thread before any write below
  double q[NQ3];
  final_sums_(part, nb, sums, q);
  if (threadIdx.x == 0) {
    const double h3 = 1.0 / ((double)n * n * n);
    double meas;
    if (rule == W1_STOP_FPR) {
      // R^k (eq. (pd_stop)) or G^k (eq. (pdhg_stop))
      meas = kind == W1_ALGO_PLAIN ? (q[0] / mu + q[1] / tau - 2.0 * q[2]) * h3
                                   : (q[0] / mu + q[1] / tau + 2.0 * q[2]) * h3;
    } else {
      const double P = q[0] * h3, D = q[1] * h3;
      const double rp = sqrt(q[2] * h3) / fmax(P, 1e-300);
      const double rd = sqrt(q[4] * h3);
      const double gap = fabs(P - D) / fmax(fmax(fabs(P), fabs(D)), 1e-300);
      meas = fmax(rp, fmax(rd, gap));
    }
    const int it = gate->iters + steps;
    // the FPR rule's guard: a measure that rises at divwin tests in a row
    const int rises = gate->iters > 0 && meas > gate->measure ? gate->rises + 1 : 0;
    gate->iters = it;
    gate->measure = meas;
    gate->rises = rises;
    // (a negative R^k / G^k: the step metric is no longer positive definite)
    const bool guard = rule == W1_STOP_FPR && divwin > 0;
    gate->status = !isfinite(meas) || (guard && meas < 0.0) ? G_DIVERGED
                   : meas <= tol ? G_CONV
                   : (guard && rises >= divwin) ? G_DIVERGED
                   : it >= cap ? G_CAP : G_RUN;
  }
}

__device__ __forceinline__ void final_sums_(const double* __restrict__ part, int nb, double* __restrict__ out,
                                            double q0[NQ3]) {
  __shared__ double sh[NQ3][NT];
  for (int q = 0; q < NQ3; ++q) {
    double s = 0.0, comp = 0.0, mx = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += NT) {
      const double x = part[(size_t)i * NQ3 + q];
      const double t = s + x;
      comp += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
      s = t;
      mx = x > mx ? x : mx;
    }
    sh[q][threadIdx.x] = q == 5 ? mx : s + comp;
  }
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < NQ3; ++q) {
        const double a = sh[q][threadIdx.x], b = sh[q][threadIdx.x + w];
        sh[q][threadIdx.x] = q == 5 ? (a > b ? a : b) : a + b;
      }
    __syncthreads();
  }
  if (threadIdx.x < NQ3) out[threadIdx.x] = sh[threadIdx.x][0];
  if (threadIdx.x == 0)
    for (int q = 0; q < NQ3; ++q) q0[q] = sh[q][0];
}

// ---------------------------------------------------------------------------
// Algorithm 2 (eq. (pdhg)): v = m - mu vphibar and r = A v - rho (pre), the
// Neumann Poisson solve u = (A A*)^{-1} r by DCT (R3), then m+ = v - A* u,
// vphi+ = Proj(vphi + tau m+), vphibar+ = 2 vphi+ - vphi (post)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k3_prox_pre(int n, const T* __restrict__ m0, const T* __restrict__ m1,
                                                  const T* __restrict__ m2, const T* __restrict__ wb0,
                                                  const T* __restrict__ wb1, const T* __restrict__ wb2,
                                                  const T* __restrict__ rho, T* __restrict__ v0, T* __restrict__ v1,
                                                  T* __restrict__ v2, T* __restrict__ r, T ih, T mu,
                                                  const int* __restrict__ gate) {
  if (gate && *gate != G_RUN) return;
  const int N1 = n + 1;
  const long long S1 = (long long)N1 * N1, N = S1 * N1;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, N1);
    const T a0 = fma3_(-mu, wb0[e], m0[e]), a1 = fma3_(-mu, wb1[e], m1[e]), a2 = fma3_(-mu, wb2[e], m2[e]);
    T d = (x.i1 < n ? a0 : T(0)) - (x.i1 > 0 ? fma3_(-mu, wb0[e - S1], m0[e - S1]) : T(0));
    d += (x.i2 < n ? a1 : T(0)) - (x.i2 > 0 ? fma3_(-mu, wb1[e - N1], m1[e - N1]) : T(0));
    d += (x.i3 < n ? a2 : T(0)) - (x.i3 > 0 ? fma3_(-mu, wb2[e - 1], m2[e - 1]) : T(0));
    v0[e] = a0;
    v1[e] = a1;
    v2[e] = a2;
    r[e] = d * ih - rho[e];
  }
}

// projection onto the unit ball of the dual norm q (inf, 2, 1 for
// p = 1, 2, inf; the l_1 ball by the same sort-and-threshold rule)
template <typename T, int METRIC>
__device__ __forceinline__ void proj3_(const T w[3], T o[3]) {
  if constexpr (METRIC == 1) {
    for (int a = 0; a < 3; ++a) o[a] = w[a] > T(1) ? T(1) : (w[a] < T(-1) ? T(-1) : w[a]);
  } else if constexpr (METRIC == 2) {
    const T nw = sqrt3_(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (int a = 0; a < 3; ++a) o[a] = nw > T(1) ? w[a] / nw : w[a];
  } else {
    const T x = abs3_(w[0]), y = abs3_(w[1]), z = abs3_(w[2]);
    if (x + y + z <= T(1)) {
      for (int a = 0; a < 3; ++a) o[a] = w[a];
      return;
    }
    const T u0 = max3_(max3_(x, y), z), u2 = min3_(min3_(x, y), z);
    const T u1 = max3_(min3_(x, y), min3_(max3_(x, y), z));
    const T c2 = u0 + u1, c3 = c2 + u2;
    const int k = 1 + (u1 > (c2 - T(1)) / T(2) ? 1 : 0) + (u2 > (c3 - T(1)) / T(3) ? 1 : 0);
    const T theta = k == 1 ? u0 - T(1) : (k == 2 ? (c2 - T(1)) / T(2) : (c3 - T(1)) / T(3));
    for (int a = 0; a < 3; ++a) {
      const T r = max3_(abs3_(w[a]) - theta, T(0));
      o[a] = w[a] < T(0) ? -r : r;
    }
  }
}

template <typename T, int METRIC, bool CHECK>
__global__ __launch_bounds__(NT) void k3_prox_post(int n, const T* __restrict__ v0, const T* __restrict__ v1,
                                                   const T* __restrict__ v2, const T* __restrict__ u,
                                                   T* __restrict__ m0, T* __restrict__ m1, T* __restrict__ m2,
                                                   T* __restrict__ w0, T* __restrict__ w1, T* __restrict__ w2,
                                                   T* __restrict__ wb0, T* __restrict__ wb1, T* __restrict__ wb2,
                                                   T ih, T tau, double* __restrict__ part,
                                                   const int* __restrict__ gate) {
  if (gate && *gate != G_RUN) return;
  const int N1 = n + 1;
  const long long S1 = (long long)N1 * N1, N = S1 * N1;
  double acc[NQ3] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, N1);
    const T uc = u[e];
    // A* u: (u(x) - u(x + h e_a)) / h, 0 on the last node of axis a
    const T n0 = v0[e] - (x.i1 < n ? (uc - u[e + S1]) * ih : T(0));
    const T n1 = v1[e] - (x.i2 < n ? (uc - u[e + N1]) * ih : T(0));
    const T n2 = v2[e] - (x.i3 < n ? (uc - u[e + 1]) * ih : T(0));
    const T wo[3] = {w0[e], w1[e], w2[e]};
    const T q[3] = {fma3_(tau, n0, wo[0]), fma3_(tau, n1, wo[1]), fma3_(tau, n2, wo[2])};
    T pw[3];
    proj3_<T, METRIC>(q, pw);
    if constexpr (CHECK) {
      const T d0 = n0 - m0[e], d1 = n1 - m1[e], d2 = n2 - m2[e];
      const T e0 = pw[0] - wo[0], e1 = pw[1] - wo[1], e2 = pw[2] - wo[2];
      acc[0] += (double)(d0 * d0) + (double)(d1 * d1) + (double)(d2 * d2);
      acc[1] += (double)(e0 * e0) + (double)(e1 * e1) + (double)(e2 * e2);
      acc[2] += (double)(e0 * d0) + (double)(e1 * d1) + (double)(e2 * d2);
    }
    m0[e] = n0;
    m1[e] = n1;
    m2[e] = n2;
    w0[e] = pw[0];
    w1[e] = pw[1];
    w2[e] = pw[2];
    wb0[e] = fma3_(T(2), pw[0], -wo[0]);
    wb1[e] = fma3_(T(2), pw[1], -wo[1]);
    wb2[e] = fma3_(T(2), pw[2], -wo[2]);
  }
  if constexpr (CHECK) block_out_(acc, part);
}

// r = A f - rho (rho may be NULL: r = A f)
template <typename T>
__global__ __launch_bounds__(NT) void k3_div(int n, const T* __restrict__ f0, const T* __restrict__ f1,
                                             const T* __restrict__ f2, const T* __restrict__ rho,
                                             T* __restrict__ r, const int* __restrict__ gate) {
  if (gate && *gate != G_RUN) return;
  const int N1 = n + 1;
  const long long S1 = (long long)N1 * N1, N = S1 * N1;
  const T ih = (T)n;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, N1);
    const T d = div3_(f0, f1, f2, e, x, n, N1, S1) * ih;
    r[e] = rho ? d - rho[e] : d;
  }
}

// One axis of the orthonormal DCT of length N = n+1 on every line along
// AXIS (0: i1, 1: i2, 2: i3): MODE 0 forward (C), MODE 1 forward and then
// the spectral division by the FP64 eigenvalues of A A*
// (4/h^2) sum_a sin^2(pi k_a / 2N), the constant mode set to 0, MODE 2
// inverse (C^T).  Both read the matrix by columns of the output index k
// (forward from Ct = C^T, inverse from C), so the lanes of a wavefront that
// hold consecutive k along i3 read consecutive entries; N x N row-major,
// s[k] = sin^2(pi k / 2N).
template <typename T, int AXIS, int MODE>
__global__ __launch_bounds__(NT) void k3_dct(int n, const T* __restrict__ in, T* __restrict__ out,
                                             const T* __restrict__ C, const T* __restrict__ Ct,
                                             const double* __restrict__ s, const int* __restrict__ gate) {
  if (gate && *gate != G_RUN) return;
  const int N1 = n + 1;
  const long long S1 = (long long)N1 * N1, N = S1 * N1;
  const long long stride = AXIS == 0 ? S1 : (AXIS == 1 ? N1 : 1);
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, N1);
    const int k = AXIS == 0 ? x.i1 : (AXIS == 1 ? x.i2 : x.i3);
    const long long base = e - (long long)k * stride;
    const T* M = (MODE == 2 ? C : Ct) + k;
    T acc = T(0);
    for (int j = 0; j < N1; ++j) acc = fma3_(M[(size_t)j * N1], in[base + j * stride], acc);
    if constexpr (MODE == 1) {
      const double lam = 4.0 * (double)n * (double)n * (s[x.i1] + s[x.i2] + s[x.i3]);
      acc = (x.i1 | x.i2 | x.i3) == 0 ? T(0) : (T)((double)acc / lam);
    }
    out[e] = acc;
  }
}

// The same one-axis DCT pass in FP32 on the matrix cores: a product with the
// DCT matrix in 64 x 64 output tiles (K = N).  Along i1 and i2 the tile is
// (frequency k) x (the contiguous index), Out = M In, batched over i1 for
// the i2 pass; along the contiguous axis i3 it is (line) x (frequency k),
// Out = In M^T, so every operand load runs along contiguous memory.
template <int AXIS, int MODE>
__global__ __launch_bounds__(NT) void k3_dct_mfma(int n, const float* __restrict__ in, float* __restrict__ out,
                                                  const float* __restrict__ C, const double* __restrict__ s,
                                                  int tiles_r, int tiles_c, const int* __restrict__ gate) {
  __shared__ float As[2][64][33];
  __shared__ float Bs[2][32][68];
  if (gate && *gate != G_RUN) return;
  const int N1 = n + 1;
  const long long S1 = (long long)N1 * N1;
  const int tr = blockIdx.x % tiles_r, tc = (blockIdx.x / tiles_r) % tiles_c, bt = blockIdx.x / (tiles_r * tiles_c);
  const int r0 = tr * 64, c0 = tc * 64;
  // M(k, j): C[k][j] forward, C[j][k] inverse
  auto Mkj = [&](int k, int j) { return MODE == 2 ? C[(size_t)j * N1 + k] : C[(size_t)k * N1 + j]; };
  const long long rows = AXIS == 2 ? S1 : N1, cols = AXIS == 0 ? S1 : N1;
  float acc[16];
  if constexpr (AXIS == 0) {
    auto la = [&](int i, int kk) { return Mkj(min(r0 + i, N1 - 1), kk); };
    auto lb = [&](int kk, int j) {
      const long long c = c0 + j < S1 ? c0 + j : S1 - 1;
      return in[(long long)kk * S1 + c];
    };
    mfma_tile64_(la, lb, N1, As, Bs, acc);
  } else if constexpr (AXIS == 1) {
    const long long base = (long long)bt * S1;
    auto la = [&](int i, int kk) { return Mkj(min(r0 + i, N1 - 1), kk); };
    auto lb = [&](int kk, int j) { return in[base + (long long)kk * N1 + min(c0 + j, N1 - 1)]; };
    mfma_tile64_(la, lb, N1, As, Bs, acc);
  } else {
    auto la = [&](int i, int kk) {
      const long long r = r0 + i < S1 ? r0 + i : S1 - 1;
      return in[r * N1 + kk];
    };
    auto lb = [&](int kk, int j) { return Mkj(min(c0 + j, N1 - 1), kk); };
    mfma_tile64_(la, lb, N1, As, Bs, acc);
  }
  const int col = c0 + mfma_col_();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const long long row = r0 + mfma_row_(r);
    if (row >= rows || col >= cols) continue;
    const long long e = AXIS == 0 ? row * S1 + col : (AXIS == 1 ? (long long)bt * S1 + row * N1 + col : row * N1 + col);
    float v = acc[r];
    if constexpr (MODE == 1) {
      const Idx x = split_(e, N1);
      const double lam = 4.0 * (double)n * (double)n * (s[x.i1] + s[x.i2] + s[x.i3]);
      v = (x.i1 | x.i2 | x.i3) == 0 ? 0.f : (float)((double)v / lam);
    }
    out[e] = v;
  }
}

// ---------------------------------------------------------------------------
// density pyramid (FP64): input checks, scaling, restriction, rho
// ---------------------------------------------------------------------------
// q0 sum p0, q1 sum p1, q2 count of negative or non-finite masses
__global__ __launch_bounds__(NT) void k3_mass(long long N, const double* __restrict__ p0,
                                              const double* __restrict__ p1, double* __restrict__ part) {
  double v[NQ3] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const double a = p0[e], b = p1[e];
    v[0] += a;
    v[1] += b;
    v[2] += (isfinite(a) && isfinite(b) && a >= 0.0 && b >= 0.0) ? 0.0 : 1.0;
  }
  block_out_(v, part);
}

__global__ __launch_bounds__(NT) void k3_scale2(long long N, double* __restrict__ x, double sx,
                                                double* __restrict__ y, double sy) {
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    x[e] *= sx;
    y[e] *= sy;
  }
}

// coarse = D^-1 P^T fine per axis (the potential interpolation's weights
// 1 at the coinciding fine node and 1/2 at its two neighbours, divided by
// their sum), for both densities
__global__ __launch_bounds__(NT) void k3_restrict(int nc, const double* __restrict__ f0,
                                                  const double* __restrict__ f1, double* __restrict__ c0,
                                                  double* __restrict__ c1) {
  const int C1 = nc + 1, nf = 2 * nc, F1 = nf + 1;
  const long long N = (long long)C1 * C1 * C1;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, C1);
    const int c[3] = {x.i1, x.i2, x.i3};
    double wsum[3];
    for (int a = 0; a < 3; ++a) wsum[a] = 1.0 + (c[a] > 0 ? 0.5 : 0.0) + (c[a] < nc ? 0.5 : 0.0);
    double s0 = 0.0, s1 = 0.0;
    for (int d1 = -1; d1 <= 1; ++d1) {
      const int I1 = 2 * c[0] + d1;
      if (I1 < 0 || I1 > nf) continue;
      const double w1 = d1 == 0 ? 1.0 : 0.5;
      for (int d2 = -1; d2 <= 1; ++d2) {
        const int I2 = 2 * c[1] + d2;
        if (I2 < 0 || I2 > nf) continue;
        const double w2 = w1 * (d2 == 0 ? 1.0 : 0.5);
        for (int d3 = -1; d3 <= 1; ++d3) {
          const int I3 = 2 * c[2] + d3;
          if (I3 < 0 || I3 > nf) continue;
          const double w = w2 * (d3 == 0 ? 1.0 : 0.5);
          const long long f = ((long long)I1 * F1 + I2) * F1 + I3;
          s0 += w * f0[f];
          s1 += w * f1[f];
        }
      }
    }
    const double dn = wsum[0] * wsum[1] * wsum[2];
    c0[e] = s0 / dn;
    c1[e] = s1 / dn;
  }
}

// q0 sum (r0 - r1)
__global__ __launch_bounds__(NT) void k3_diffsum(long long N, const double* __restrict__ r0,
                                                 const double* __restrict__ r1, double* __restrict__ part) {
  double v[NQ3] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT)
    v[0] += r0[e] - r1[e];
  block_out_(v, part);
}

template <typename T>
__global__ __launch_bounds__(NT) void k3_rho(long long N, const double* __restrict__ r0,
                                             const double* __restrict__ r1, double mean, T* __restrict__ rho) {
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT)
    rho[e] = (T)((r0[e] - r1[e]) - mean);
}

// ---------------------------------------------------------------------------
// prolongation (Sec. 3.3): potential linear along every axis; flux
// component a nearest-neighbour along axis a (coarse index floor(I/2), the
// coarse edge containing the fine one) and linear across, 0 on the last
// fine node of axis a
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k3_prolong(int nc, int comp, const T* __restrict__ c, T* __restrict__ f) {
  const int C1 = nc + 1, nf = 2 * nc, F1 = nf + 1;
  const long long N = (long long)F1 * F1 * F1;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    const Idx x = split_(e, F1);
    const int I[3] = {x.i1, x.i2, x.i3};
    if (comp >= 0 && I[comp] == nf) {
      f[e] = T(0);
      continue;
    }
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      if (a == comp || (I[a] & 1) == 0) {
        lo[a] = hi[a] = I[a] >> 1;
      } else {
        lo[a] = (I[a] - 1) >> 1;
        hi[a] = (I[a] + 1) >> 1;
      }
    }
    // mean over the (at most 8) coarse nodes of the product neighbourhood
    double s = 0.0;
    int cnt = 0;
    for (int j1 = lo[0]; j1 <= hi[0]; ++j1)
      for (int j2 = lo[1]; j2 <= hi[1]; ++j2)
        for (int j3 = lo[2]; j3 <= hi[2]; ++j3) {
          s += (double)c[((long long)j1 * C1 + j2) * C1 + j3];
          ++cnt;
        }
    f[e] = (T)(s / cnt);
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k3_export(long long N, const T* __restrict__ m0, const T* __restrict__ m1,
                                                const T* __restrict__ m2, const T* __restrict__ pot, double mean,
                                                double sgn, double* __restrict__ om, double* __restrict__ opsi) {
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < N; e += (long long)gridDim.x * NT) {
    if (om) {
      om[e] = (double)m0[e];
      om[N + e] = (double)m1[e];
      om[2 * N + e] = (double)m2[e];
    }
    if (opsi) opsi[e] = sgn * ((double)pot[e] - mean);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
inline int blocks_for(long long N) {
  const long long b = (N + NT - 1) / NT;
  return (int)(b < MAXB ? (b > 0 ? b : 1) : MAXB);
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// a solve's device block from the library's exact-size cache; returned
// after the stream has drained (also on an error path)
struct Staged {
  char* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  ~Staged() {
    if (!p) return;
    (void)hipStreamSynchronize(s);
    stage_free(bytes, p);
  }
};

// planes of one level: Algorithm 1 uses m, b (= 2 m+ - m), phi; Algorithm 2
// uses m, w (vphi), wb (vphibar), b (= v), r (residual, then u) and t (DCT
// scratch); rho, the FP64 density pair and the DCT tables always
constexpr int NPL3 = 16;
template <typename T>
struct Level {
  int n = 0;
  long long N = 0;
  T *m[3] = {}, *b[3] = {}, *w[3] = {}, *wb[3] = {}, *phi = nullptr, *rho = nullptr, *r = nullptr, *t = nullptr;
  double *r0 = nullptr, *r1 = nullptr;
  T* C = nullptr;        // orthonormal DCT-II matrix, N x N
  T* Ct = nullptr;       // its transpose
  double* s = nullptr;   // sin^2(pi k / 2N)
};

template <typename T>
size_t level_bytes(int n) {
  const size_t N = (size_t)(n + 1) * (n + 1) * (n + 1), L = (size_t)(n + 1);
  return N * (NPL3 * sizeof(T) + 2 * sizeof(double)) + 2 * L * L * sizeof(T) + L * sizeof(double) + 21 * 256;
}

// orthonormal DCT-II of length N: C[k][j] = sqrt((k ? 2 : 1)/N) cos(pi k (2j+1) / 2N)
template <typename T>
int upload_dct(hipStream_t st, Level<T>& V) {
  const int N = V.n + 1;
  std::vector<T> C((size_t)N * N), Ct((size_t)N * N);
  std::vector<double> sv(N);
  const double pi = std::acos(-1.0);
  for (int k = 0; k < N; ++k) {
    const double a = std::sqrt((k ? 2.0 : 1.0) / N);
    for (int j = 0; j < N; ++j) {
      const T c = (T)(a * std::cos(pi * k * (2.0 * j + 1.0) / (2.0 * N)));
      C[(size_t)k * N + j] = c;
      Ct[(size_t)j * N + k] = c;
    }
    const double sn = std::sin(pi * k / (2.0 * N));
    sv[k] = sn * sn;
  }
  CHK(hipMemcpyAsync(V.C, C.data(), C.size() * sizeof(T), hipMemcpyHostToDevice, st));
  CHK(hipMemcpyAsync(V.Ct, Ct.data(), Ct.size() * sizeof(T), hipMemcpyHostToDevice, st));
  CHK(hipMemcpyAsync(V.s, sv.data(), sv.size() * sizeof(double), hipMemcpyHostToDevice, st));
  CHK(hipStreamSynchronize(st));   // the host vectors end with this scope
  return W1_OK;
}

// u = (A A*)^{-1} x in place of x (R3), t scratch: three forward passes (the
// last divides by the eigenvalues), three inverse passes
template <typename T>
int poisson3(hipStream_t s, const Level<T>& V, T* x, T* t, const int* gate) {
  if constexpr (std::is_same<T, float>::value) {
    const int N1 = V.n + 1, tn = (N1 + 63) / 64;
    const long long S1 = (long long)N1 * N1;
    const int ts = (int)((S1 + 63) / 64);
    k3_dct_mfma<2, 0><<<ts * tn, NT, 0, s>>>(V.n, x, t, V.C, V.s, ts, tn, gate);
    k3_dct_mfma<1, 0><<<tn * tn * N1, NT, 0, s>>>(V.n, t, x, V.C, V.s, tn, tn, gate);
    k3_dct_mfma<0, 1><<<tn * ts, NT, 0, s>>>(V.n, x, t, V.C, V.s, tn, ts, gate);
    k3_dct_mfma<0, 2><<<tn * ts, NT, 0, s>>>(V.n, t, x, V.C, V.s, tn, ts, gate);
    k3_dct_mfma<1, 2><<<tn * tn * N1, NT, 0, s>>>(V.n, x, t, V.C, V.s, tn, tn, gate);
    k3_dct_mfma<2, 2><<<ts * tn, NT, 0, s>>>(V.n, t, x, V.C, V.s, ts, tn, gate);
    CHK(hipGetLastError());
    return W1_OK;
  }
  const int nb = blocks_for(V.N);
  k3_dct<T, 2, 0><<<nb, NT, 0, s>>>(V.n, x, t, V.C, V.Ct, V.s, gate);
  k3_dct<T, 1, 0><<<nb, NT, 0, s>>>(V.n, t, x, V.C, V.Ct, V.s, gate);
  k3_dct<T, 0, 1><<<nb, NT, 0, s>>>(V.n, x, t, V.C, V.Ct, V.s, gate);
  k3_dct<T, 0, 2><<<nb, NT, 0, s>>>(V.n, t, x, V.C, V.Ct, V.s, gate);
  k3_dct<T, 1, 2><<<nb, NT, 0, s>>>(V.n, x, t, V.C, V.Ct, V.s, gate);
  k3_dct<T, 2, 2><<<nb, NT, 0, s>>>(V.n, t, x, V.C, V.Ct, V.s, gate);
  CHK(hipGetLastError());
  return W1_OK;
}

template <typename T>
int launch_steps(hipStream_t s, const Level<T>& L, int metric, T mu, T tau, int steps, bool check_last,
                 double* part, const int* gate) {
  const int nb = blocks_for(L.N);
  const T ih = (T)L.n;
  for (int k = 0; k < steps; ++k) {
    switch (metric) {
      case 1:
        k3_flux<T, 1><<<nb, NT, 0, s>>>(L.n, L.m[0], L.m[1], L.m[2], L.b[0], L.b[1], L.b[2], L.phi, ih, mu, gate);
        break;
      case 2:
        k3_flux<T, 2><<<nb, NT, 0, s>>>(L.n, L.m[0], L.m[1], L.m[2], L.b[0], L.b[1], L.b[2], L.phi, ih, mu, gate);
        break;
      default:
        k3_flux<T, 3><<<nb, NT, 0, s>>>(L.n, L.m[0], L.m[1], L.m[2], L.b[0], L.b[1], L.b[2], L.phi, ih, mu, gate);
    }
    if (check_last && k == steps - 1)
      k3_pot<T, true><<<nb, NT, 0, s>>>(L.n, L.b[0], L.b[1], L.b[2], L.m[0], L.m[1], L.m[2], L.phi, L.rho, ih, tau,
                                        part, gate);
    else
      k3_pot<T, false><<<nb, NT, 0, s>>>(L.n, L.b[0], L.b[1], L.b[2], L.m[0], L.m[1], L.m[2], L.phi, L.rho, ih,
                                         tau, part, gate);
  }
  CHK(hipGetLastError());
  return W1_OK;
}

template <typename T, int METRIC>
void prox_post_(hipStream_t s, const Level<T>& L, int nb, T ih, T tau, bool chk, double* part, const int* gate) {
  if (chk)
    k3_prox_post<T, METRIC, true><<<nb, NT, 0, s>>>(L.n, L.b[0], L.b[1], L.b[2], L.r, L.m[0], L.m[1], L.m[2],
                                                    L.w[0], L.w[1], L.w[2], L.wb[0], L.wb[1], L.wb[2], ih, tau,
                                                    part, gate);
  else
    k3_prox_post<T, METRIC, false><<<nb, NT, 0, s>>>(L.n, L.b[0], L.b[1], L.b[2], L.r, L.m[0], L.m[1], L.m[2],
                                                     L.w[0], L.w[1], L.w[2], L.wb[0], L.wb[1], L.wb[2], ih, tau,
                                                     part, gate);
}

template <typename T>
int launch_prox_steps(hipStream_t s, const Level<T>& L, int metric, T mu, T tau, int steps, bool check_last,
                      double* part, const int* gate) {
  const int nb = blocks_for(L.N);
  const T ih = (T)L.n;
  for (int k = 0; k < steps; ++k) {
    k3_prox_pre<T><<<nb, NT, 0, s>>>(L.n, L.m[0], L.m[1], L.m[2], L.wb[0], L.wb[1], L.wb[2], L.rho, L.b[0],
                                     L.b[1], L.b[2], L.r, ih, mu, gate);
    int st = poisson3<T>(s, L, L.r, L.t, gate);
    if (st) return st;
    const bool chk = check_last && k == steps - 1;
    switch (metric) {
      case 1: prox_post_<T, 1>(s, L, nb, ih, tau, chk, part, gate); break;
      case 2: prox_post_<T, 2>(s, L, nb, ih, tau, chk, part, gate); break;
      default: prox_post_<T, 3>(s, L, nb, ih, tau, chk, part, gate);
    }
  }
  CHK(hipGetLastError());
  return W1_OK;
}

// final sums of `nb` partials, copied to host `out`
inline int finish_sums(hipStream_t s, const double* part, int nb, double* dout, double* out) {
  k3_final<<<1, NT, 0, s>>>(part, nb, dout);
  CHK(hipGetLastError());
  CHK(hipMemcpyAsync(out, dout, NQ3 * sizeof(double), hipMemcpyDeviceToHost, s));
  CHK(hipStreamSynchronize(s));
  return W1_OK;
}

template <typename T>
int eval_sums(hipStream_t s, const Level<T>& L, int metric, const T* pot, double sgn, const T* corr, double* part,
              const int* gate) {
  const int nb = blocks_for(L.N);
  switch (metric) {
    case 1: k3_eval<T, 1><<<nb, NT, 0, s>>>(L.n, L.m[0], L.m[1], L.m[2], pot, sgn, L.rho, corr, part, gate); break;
    case 2: k3_eval<T, 2><<<nb, NT, 0, s>>>(L.n, L.m[0], L.m[1], L.m[2], pot, sgn, L.rho, corr, part, gate); break;
    default: k3_eval<T, 3><<<nb, NT, 0, s>>>(L.n, L.m[0], L.m[1], L.m[2], pot, sgn, L.rho, corr, part, gate);
  }
  CHK(hipGetLastError());
  return W1_OK;
}

// P, D, lo, hi, kkt from the evaluation sums of a level of side n
struct Eval {
  double P, D, lo, hi, kkt, mean;
};
inline Eval eval_of(const double* q, int n, bool cert) {
  const double h3 = 1.0 / ((double)n * n * n);
  const double N = (double)(n + 1) * (n + 1) * (n + 1);
  Eval e;
  e.P = q[0] * h3;
  e.D = q[1] * h3;
  const double rp = std::sqrt(q[2] * h3) / std::fmax(e.P, 1e-300);
  const double rd = std::sqrt(q[4] * h3);
  const double gap = std::fabs(e.P - e.D) / std::fmax(std::fmax(std::fabs(e.P), std::fabs(e.D)), 1e-300);
  e.kkt = std::fmax(rp, std::fmax(rd, gap));
  e.lo = e.D / (q[5] > 1.0 ? q[5] : 1.0);
  e.hi = cert ? q[7] * h3 : std::numeric_limits<double>::quiet_NaN();
  e.mean = q[6] / N;
  return e;
}

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// the potential of a finished level: phi (Algorithm 1, psi = -phi) or
// psi = (A A*)^{-1} A vphi in plane r (Algorithm 2, Appendix B)
template <typename T>
int level_potential(hipStream_t s, const Level<T>& V, bool prox, const T** pot, double* sgn) {
  if (!prox) {
    *pot = V.phi;
    *sgn = -1.0;
    return W1_OK;
  }
  k3_div<T><<<blocks_for(V.N), NT, 0, s>>>(V.n, V.w[0], V.w[1], V.w[2], nullptr, V.r, nullptr);
  CHK(hipGetLastError());
  int st = poisson3<T>(s, V, V.r, V.t, nullptr);
  if (st) return st;
  *pot = V.r;
  *sgn = 1.0;
  return W1_OK;
}

template <typename T>
size_t solve_bytes(const w1_params& prm) {
  size_t bytes = 0;
  for (int l = 0; l < prm.levels; ++l) bytes += level_bytes<T>(prm.n >> (prm.levels - 1 - l));
  return bytes + (size_t)MAXB * NQ3 * sizeof(double) + 256 + NQ3 * sizeof(double) + 256 + sizeof(Gate) + 256;
}

// one solve in the caller's device block `mem` of solve_bytes<T>(prm) bytes
template <typename T>
int solve_in(const w1_params& prm, const double* p0, const double* p1, int on_device, w1_result* out, double* m_out,
             double* psi_out, hipStream_t s, void* mem) {
  const double t0 = now_s();
  const int L = prm.levels;
  const bool prox = prm.algo == W1_ALGO_PROX;
  std::vector<Level<T>> lv(L);
  for (int l = 0; l < L; ++l) {
    lv[l].n = prm.n >> (L - 1 - l);
    lv[l].N = (long long)(lv[l].n + 1) * (lv[l].n + 1) * (lv[l].n + 1);
  }
  const size_t bytes = solve_bytes<T>(prm);
  char* p = (char*)mem;
  auto take = [&](size_t b) {
    char* r = p;
    p += (b + 255) / 256 * 256;
    return r;
  };
  for (int l = 0; l < L; ++l) {
    Level<T>& V = lv[l];
    const size_t pe = (size_t)V.N * sizeof(T);
    for (int a = 0; a < 3; ++a) V.m[a] = (T*)take(pe);
    for (int a = 0; a < 3; ++a) V.b[a] = (T*)take(pe);
    for (int a = 0; a < 3; ++a) V.w[a] = (T*)take(pe);
    for (int a = 0; a < 3; ++a) V.wb[a] = (T*)take(pe);
    V.phi = (T*)take(pe);
    V.rho = (T*)take(pe);
    V.r = (T*)take(pe);
    V.r0 = (double*)take((size_t)V.N * 8);
    V.r1 = (double*)take((size_t)V.N * 8);
    V.C = (T*)take((size_t)(V.n + 1) * (V.n + 1) * sizeof(T));
    V.Ct = (T*)take((size_t)(V.n + 1) * (V.n + 1) * sizeof(T));
    V.s = (double*)take((size_t)(V.n + 1) * sizeof(double));
    V.t = (T*)take(pe);
  }
  double* part = (double*)take((size_t)MAXB * NQ3 * sizeof(double));
  double* dout = (double*)take(NQ3 * sizeof(double));
  Gate* gate = (Gate*)take(sizeof(Gate));
  if ((size_t)(p - (char*)mem) > bytes) return W1_EINVAL;   // layout and size disagree (not expected)
  for (int l = 0; l < L; ++l) {
    int st = upload_dct<T>(s, lv[l]);
    if (st) return st;
  }
  double q[NQ3];

  // input masses -> finest r0, r1; checks (Sec. 2.2 samples the densities on
  // the nodes; both renormalised to unit mass)
  Level<T>& F = lv[L - 1];
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  CHK(hipMemcpyAsync(F.r0, p0, (size_t)F.N * 8, kind, s));
  CHK(hipMemcpyAsync(F.r1, p1, (size_t)F.N * 8, kind, s));
  {
    const int nb = blocks_for(F.N);
    k3_mass<<<nb, NT, 0, s>>>(F.N, F.r0, F.r1, part);
    CHK(hipGetLastError());
    int st = finish_sums(s, part, nb, dout, q);
    if (st) return st;
    if (q[2] > 0 || !(q[0] > 0) || !(std::fabs(q[0] - q[1]) <= 1e-9 * q[0])) return W1_EINVAL;
    const double h3 = 1.0 / ((double)F.n * F.n * F.n);
    k3_scale2<<<nb, NT, 0, s>>>(F.N, F.r0, 1.0 / (q[0] * h3), F.r1, 1.0 / (q[1] * h3));
    CHK(hipGetLastError());
  }
  // coarse densities: D^-1 P^T per axis, each renormalised to unit mass (R6)
  for (int l = L - 2; l >= 0; --l) {
    const int nb = blocks_for(lv[l].N);
    k3_restrict<<<nb, NT, 0, s>>>(lv[l].n, lv[l + 1].r0, lv[l + 1].r1, lv[l].r0, lv[l].r1);
    k3_mass<<<nb, NT, 0, s>>>(lv[l].N, lv[l].r0, lv[l].r1, part);
    CHK(hipGetLastError());
    int st = finish_sums(s, part, nb, dout, q);
    if (st) return st;
    const double h3 = 1.0 / ((double)lv[l].n * lv[l].n * lv[l].n);
    k3_scale2<<<nb, NT, 0, s>>>(lv[l].N, lv[l].r0, 1.0 / (q[0] * h3), lv[l].r1, 1.0 / (q[1] * h3));
    CHK(hipGetLastError());
  }
  for (int l = 0; l < L; ++l) {
    const int nb = blocks_for(lv[l].N);
    k3_diffsum<<<nb, NT, 0, s>>>(lv[l].N, lv[l].r0, lv[l].r1, part);
    CHK(hipGetLastError());
    int st = finish_sums(s, part, nb, dout, q);
    if (st) return st;
    k3_rho<T><<<nb, NT, 0, s>>>(lv[l].N, lv[l].r0, lv[l].r1, q[0] / (double)lv[l].N, lv[l].rho);
    CHK(hipGetLastError());
  }

  *out = w1_result{};
  for (int l = 0; l < W1_MAX_LEVELS; ++l) out->level_w1[l] = std::numeric_limits<double>::quiet_NaN();
  out->status = W1_SOLVE_OK;
  const double sc = prm.step_scale > 0 ? prm.step_scale : 0.5;
  const int ce = prm.check_every;
  for (int l = 0; l < L; ++l) {
    Level<T>& V = lv[l];
    const int nb = blocks_for(V.N);
    const size_t pe = (size_t)V.N * sizeof(T);
    if (l == 0) {
      for (int a = 0; a < 3; ++a) {
        CHK(hipMemsetAsync(V.m[a], 0, pe, s));
        if (prox) CHK(hipMemsetAsync(V.w[a], 0, pe, s));
      }
      if (!prox) CHK(hipMemsetAsync(V.phi, 0, pe, s));
    } else {
      const Level<T>& C = lv[l - 1];
      for (int a = 0; a < 3; ++a) {
        k3_prolong<T><<<nb, NT, 0, s>>>(C.n, a, C.m[a], V.m[a]);
        if (prox) k3_prolong<T><<<nb, NT, 0, s>>>(C.n, a, C.w[a], V.w[a]);
      }
      if (!prox) k3_prolong<T><<<nb, NT, 0, s>>>(C.n, -1, C.phi, V.phi);
      CHK(hipGetLastError());
    }
    // vphibar = vphi at every level start (R5)
    if (prox)
      for (int a = 0; a < 3; ++a) CHK(hipMemcpyAsync(V.wb[a], V.w[a], pe, hipMemcpyDeviceToDevice, s));
    // R4 with d = 3: Algorithm 1 mu = tau = scale / ||A||, ||A|| <= 2 sqrt(3) / h;
    // Algorithm 2 mu = tau = scale
    const double mu = prox ? sc : sc / (2.0 * std::sqrt(3.0) * V.n);
    const double tol = prm.tol * std::pow(2.0, (double)(L - 1 - l) * prm.alpha);
    // blocks of check_every iterations, each ending in the stop test on the
    // device; the host reads the gate after 4, 8, ... 64 queued blocks (the
    // blocks queued past the stop skip their work)
    CHK(hipMemsetAsync(gate, 0, sizeof(Gate), s));
    const bool fpr = prm.stop_rule == W1_STOP_FPR;
    const int cap = prm.level_caps[l] > 0 ? prm.level_caps[l] : prm.max_iters;
    const int total = cap / ce;
    int queued = 0, burst = 4;
    Gate g{G_RUN, 0, 0.0, 0, 0};
    while (g.status == G_RUN && queued < total) {
      const int B = std::min(burst, total - queued);
      for (int b = 0; b < B; ++b) {
        int st = prox ? launch_prox_steps<T>(s, V, prm.metric, (T)mu, (T)mu, ce, fpr, part, &gate->status)
                      : launch_steps<T>(s, V, prm.metric, (T)mu, (T)mu, ce, fpr, part, &gate->status);
        if (st) return st;
        if (!fpr) {
          const T* pot = V.phi;
          double sgn = -1.0;
          if (prox) {
            k3_div<T><<<nb, NT, 0, s>>>(V.n, V.w[0], V.w[1], V.w[2], nullptr, V.r, &gate->status);
            st = poisson3<T>(s, V, V.r, V.t, &gate->status);
            if (st) return st;
            pot = V.r;
            sgn = 1.0;
          }
          // the correction potential (A A*)^{-1}(A m - rho) in b[0] (b is
          // free between iterations), b[1] scratch
          k3_div<T><<<nb, NT, 0, s>>>(V.n, V.m[0], V.m[1], V.m[2], V.rho, V.b[0], &gate->status);
          CHK(hipGetLastError());
          st = poisson3<T>(s, V, V.b[0], V.b[1], &gate->status);
          if (st) return st;
          st = eval_sums<T>(s, V, prm.metric, pot, sgn, V.b[0], part, &gate->status);
          if (st) return st;
        }
        k3_check<<<1, NT, 0, s>>>(part, nb, dout, gate, prm.algo, prm.stop_rule, mu, mu, V.n, tol, ce, cap,
                                  prm.diverge_window);
        CHK(hipGetLastError());
      }
      queued += B;
      burst = std::min(2 * burst, 64);
      CHK(hipMemcpyAsync(&g, gate, sizeof(Gate), hipMemcpyDeviceToHost, s));
      CHK(hipStreamSynchronize(s));
    }
    if (g.status == G_DIVERGED) out->status = W1_SOLVE_DIVERGED;
    if (g.status == G_CAP) out->status = W1_SOLVE_MAXITER;
    out->iters[l] = g.iters;
    out->measure[l] = g.measure;
    out->levels_run = l + 1;
    int st = eval_sums<T>(s, V, prm.metric, prox ? V.w[0] : V.phi, -1.0, nullptr, part, nullptr);
    if (st) return st;
    st = finish_sums(s, part, nb, dout, q);
    if (st) return st;
    out->level_w1[l] = eval_of(q, V.n, false).P;
    out->level_seconds[l] = now_s() - t0;
    if (out->status == W1_SOLVE_DIVERGED) break;
  }
  // certificate of the last level run: its potential, and the minimum-norm
  // correction c = (A A*)^{-1}(A m - rho) (planes b, free now) for hi
  const Level<T>& V = lv[out->levels_run - 1];
  const T* pot = nullptr;
  double sgn = 0;
  int st = level_potential<T>(s, V, prox, &pot, &sgn);
  if (st) return st;
  k3_div<T><<<blocks_for(V.N), NT, 0, s>>>(V.n, V.m[0], V.m[1], V.m[2], V.rho, V.b[0], nullptr);
  CHK(hipGetLastError());
  st = poisson3<T>(s, V, V.b[0], V.b[1], nullptr);
  if (st) return st;
  st = eval_sums<T>(s, V, prm.metric, pot, sgn, V.b[0], part, nullptr);
  if (st) return st;
  st = finish_sums(s, part, blocks_for(V.N), dout, q);
  if (st) return st;
  const Eval ev = eval_of(q, V.n, true);
  // outputs on [0, c]^3 (w1_params.h): W1 by c, flux by 1/c^2, potential by c
  const double c = domain_scale(prm);
  out->w1 = c * ev.P;
  out->dual = c * ev.D;
  out->lo = c * ev.lo;
  out->hi = c * ev.hi;
  out->kkt = ev.kkt;
  for (int l = 0; l < out->levels_run; ++l) out->level_w1[l] *= c;
  if ((m_out || psi_out) && out->levels_run == L) {
    DevBuf ex;
    const size_t need = (m_out ? 3 : 0) * (size_t)V.N * 8 + (psi_out ? (size_t)V.N * 8 : 0);
    CHK(dev_malloc(&ex.p, need));
    double* om = m_out ? (double*)ex.p : nullptr;
    double* op = psi_out ? (double*)ex.p + (m_out ? 3 * V.N : 0) : nullptr;
    // psi: -(phi - mean) for Algorithm 1, Appendix B's psi as is for Algorithm 2
    k3_export<T><<<blocks_for(V.N), NT, 0, s>>>(V.N, V.m[0], V.m[1], V.m[2], pot, prox ? 0.0 : ev.mean, sgn, om,
                                                op);
    CHK(hipGetLastError());
    if (m_out) CHK(hipMemcpyAsync(m_out, om, 3 * (size_t)V.N * 8, hipMemcpyDeviceToHost, s));
    if (psi_out) CHK(hipMemcpyAsync(psi_out, op, (size_t)V.N * 8, hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    if (c != 1.0) {
      if (m_out)
        for (long long e = 0; e < 3 * V.N; ++e) m_out[e] /= c * c;
      if (psi_out)
        for (long long e = 0; e < V.N; ++e) psi_out[e] *= c;
    }
  }
  out->seconds = now_s() - t0;
  return W1_OK;
}

template <typename T>
int solve(const w1_params& prm, const double* p0, const double* p1, int on_device, w1_result* out, double* m_out,
          double* psi_out, hipStream_t s) {
  Staged mem;
  mem.bytes = solve_bytes<T>(prm);
  mem.s = s;
  int st = stage_alloc(mem.bytes, &mem.p);
  if (st) return st;
  return solve_in<T>(prm, p0, p1, on_device, out, m_out, psi_out, s, mem.p);
}

// `count` pairs over `workers` host threads, each with its own stream and
// device block, taking pairs in turn: the launch-bound small levels of
// different pairs overlap on the device
template <typename T>
int solve_batch(const w1_params& prm, int count, const double* const* p0, const double* const* p1, int on_device,
                w1_result* out, int workers) {
  int dev = 0;
  CHK(hipGetDevice(&dev));
  std::atomic<int> next{0}, err{W1_OK};
  auto run = [&]() {
    int st = hip_status(hipSetDevice(dev), "hipSetDevice");
    hipStream_t s = nullptr;
    if (!st) st = hip_status(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    {
      Staged mem;
      mem.bytes = solve_bytes<T>(prm);
      mem.s = s;
      if (!st) st = stage_alloc(mem.bytes, &mem.p);
      while (!st && err.load() == W1_OK) {
        const int i = next.fetch_add(1);
        if (i >= count) break;
        st = solve_in<T>(prm, p0[i], p1[i], on_device, &out[i], nullptr, nullptr, s, mem.p);
      }
    }   // the block goes back to the cache once the stream has drained
    if (s) (void)hipStreamDestroy(s);
    if (st) {
      int expected = W1_OK;
      err.compare_exchange_strong(expected, st);
    }
  };
  std::vector<std::thread> th;
  for (int k = 0; k < workers; ++k) th.emplace_back(run);
  for (auto& t : th) t.join();
  return err.load();
}

// single-step entry points: steps iterations in place on caller arrays
template <typename T>
int steps3(int n, int metric, bool prox, double scale, int steps, void* const* f, const void* rho, double* fpr_out,
           hipStream_t s) {
  Level<T> V;
  V.n = n;
  V.N = (long long)(n + 1) * (n + 1) * (n + 1);
  for (int a = 0; a < 3; ++a) V.m[a] = (T*)f[a];
  if (prox) {
    for (int a = 0; a < 3; ++a) {
      V.w[a] = (T*)f[3 + a];
      V.wb[a] = (T*)f[6 + a];
    }
  } else {
    V.phi = (T*)f[3];
  }
  V.rho = (T*)rho;
  DevBuf mem;
  const size_t pe = ((size_t)V.N * sizeof(T) + 255) / 256 * 256;
  const size_t mat = ((size_t)(n + 1) * (n + 1) * sizeof(T) + 255) / 256 * 256;
  const size_t tab = 2 * mat + ((size_t)(n + 1) * 8 + 255) / 256 * 256;
  CHK(dev_malloc(&mem.p, 5 * pe + tab + (size_t)MAXB * NQ3 * 8 + 256 + NQ3 * 8));
  char* p = (char*)mem.p;
  for (int a = 0; a < 3; ++a) V.b[a] = (T*)(p + a * pe);
  V.r = (T*)(p + 3 * pe);
  V.t = (T*)(p + 4 * pe);
  V.C = (T*)(p + 5 * pe);
  V.Ct = (T*)(p + 5 * pe + mat);
  V.s = (double*)(p + 5 * pe + 2 * mat);
  double* part = (double*)(p + 5 * pe + tab);
  double* dout = part + (size_t)MAXB * NQ3 + 32;
  int st = W1_OK;
  if (prox) {
    st = upload_dct<T>(s, V);
    if (st) return st;
  }
  const double sc = scale > 0 ? scale : 0.5;
  const double mu = prox ? sc : sc / (2.0 * std::sqrt(3.0) * n);
  st = prox ? launch_prox_steps<T>(s, V, metric, (T)mu, (T)mu, steps, fpr_out != nullptr, part, nullptr)
            : launch_steps<T>(s, V, metric, (T)mu, (T)mu, steps, fpr_out != nullptr, part, nullptr);
  if (st) return st;
  if (fpr_out) {
    double q[NQ3];
    st = finish_sums(s, part, blocks_for(V.N), dout, q);
    if (st) return st;
    const double h3 = 1.0 / ((double)n * n * n);
    *fpr_out = prox ? (q[0] / mu + q[1] / mu + 2.0 * q[2]) * h3 : (q[0] / mu + q[1] / mu - 2.0 * q[2]) * h3;
  } else {
    CHK(hipStreamSynchronize(s));
  }
  return W1_OK;
}

// parameter checks of the d = 3 entry points (no masses needed for them)
bool params_ok(const w1_params* p) {
  if (p->n < 2 || p->n > 1024 || p->levels < 1 || p->levels > W1_MAX_LEVELS) return false;
  if (p->n % (1 << (p->levels - 1)) != 0 || (p->n >> (p->levels - 1)) < 2) return false;
  if (p->metric < W1_METRIC_L1 || p->metric > W1_METRIC_LINF) return false;
  if (p->algo != W1_ALGO_PLAIN && p->algo != W1_ALGO_PROX) return false;
  if (p->precision != W1_FP32 && p->precision != W1_FP64) return false;
  if (p->stop_rule != W1_STOP_KKT && p->stop_rule != W1_STOP_FPR) return false;
  if (!(p->tol > 0) || !std::isfinite(p->tol) || !std::isfinite(p->alpha) || !std::isfinite(p->h)) return false;
  if (p->max_iters < 1 || p->check_every < 1 || p->max_iters % p->check_every != 0) return false;
  for (int l = 0; l < W1_MAX_LEVELS; ++l) {
    const int c = p->level_caps[l];
    if (c < 0 || (c > 0 && (l >= p->levels || c % p->check_every != 0))) return false;
  }
  if (p->diverge_window < 0 || p->reserved != 0) return false;
  // steps above the practical choice only under the FPR rule's rise guard
  if (!std::isfinite(p->step_scale) || p->step_scale > 2.0) return false;
  if (p->step_scale > 1.0 && (p->diverge_window < 1 || p->stop_rule != W1_STOP_FPR)) return false;
  return true;
}

}  // namespace cube
}  // namespace w1

using namespace w1;

extern "C" int w1_solve3d(const w1_params* p, const double* p0, const double* p1, int32_t on_device,
                          w1_result* out, double* m_out, double* psi_out, void* hip_stream) {
  if (!p || !p0 || !p1 || !out || !cube::params_ok(p)) return W1_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  return p->precision == W1_FP32 ? cube::solve<float>(*p, p0, p1, on_device, out, m_out, psi_out, s)
                                 : cube::solve<double>(*p, p0, p1, on_device, out, m_out, psi_out, s);
}

extern "C" int w1_solve3d_batch(const w1_params* p, int32_t count, const double* const* p0,
                                const double* const* p1, int32_t on_device, w1_result* out, int32_t workers) {
  if (!p || count < 0 || (count > 0 && (!p0 || !p1 || !out)) || workers < 0 || workers > 16) return W1_EINVAL;
  if (count == 0) return W1_OK;
  for (int i = 0; i < count; ++i)
    if (!p0[i] || !p1[i]) return W1_EINVAL;
  // the same parameter checks as w1_solve3d (no masses needed for them)
  if (!cube::params_ok(p)) return W1_EINVAL;
  const int w = std::min(workers > 0 ? workers : 4, count);
  return p->precision == W1_FP32 ? cube::solve_batch<float>(*p, count, p0, p1, on_device, out, w)
                                 : cube::solve_batch<double>(*p, count, p0, p1, on_device, out, w);
}

extern "C" int w1_op_plain_steps3d(int32_t n, int32_t metric, int32_t precision, double step_scale, int32_t steps,
                                   void* m1, void* m2, void* m3, void* phi, const void* rho, double* fpr_out,
                                   void* hip_stream) {
  if (n < 1 || n > 1024 || steps < 1 || metric < W1_METRIC_L1 || metric > W1_METRIC_LINF) return W1_EINVAL;
  if (!m1 || !m2 || !m3 || !phi || !rho || !(step_scale <= 1.0)) return W1_EINVAL;
  void* f[4] = {m1, m2, m3, phi};
  hipStream_t s = (hipStream_t)hip_stream;
  if (precision == W1_FP32) return cube::steps3<float>(n, metric, false, step_scale, steps, f, rho, fpr_out, s);
  if (precision == W1_FP64) return cube::steps3<double>(n, metric, false, step_scale, steps, f, rho, fpr_out, s);
  return W1_EINVAL;
}

extern "C" int w1_op_prox_steps3d(int32_t n, int32_t metric, int32_t precision, double step_scale, int32_t steps,
                                  void* m1, void* m2, void* m3, void* w1, void* w2, void* w3, void* wb1, void* wb2,
                                  void* wb3, const void* rho, double* fpr_out, void* hip_stream) {
  if (n < 1 || n > 1024 || steps < 1 || metric < W1_METRIC_L1 || metric > W1_METRIC_LINF) return W1_EINVAL;
  if (!m1 || !m2 || !m3 || !w1 || !w2 || !w3 || !wb1 || !wb2 || !wb3 || !rho || !(step_scale <= 1.0))
    return W1_EINVAL;
  void* f[9] = {m1, m2, m3, w1, w2, w3, wb1, wb2, wb3};
  hipStream_t s = (hipStream_t)hip_stream;
  if (precision == W1_FP32) return cube::steps3<float>(n, metric, true, step_scale, steps, f, rho, fpr_out, s);
  if (precision == W1_FP64) return cube::steps3<double>(n, metric, true, step_scale, steps, f, rho, fpr_out, s);
  return W1_EINVAL;
}
