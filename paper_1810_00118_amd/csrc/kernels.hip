// HIP kernels of the multilevel W1 solver for gfx950 (CDNA4).
//
// Every kernel is batched over a device work list: one workgroup per work
// item (descriptor index, tile row, tile column, tile index), so one launch
// covers any mix of pairs, grid sides and ground metrics.  Padding items
// (descriptor index -1) return at once.
//
// All per-node arithmetic lives in the __device__ helpers below and is
// compiled without floating-point contraction (-ffp-contract=off); the few
// fused multiply-adds are explicit.  The tiled, resident and single-step
// kernels therefore produce bitwise identical iterates for a node whatever
// tiling, temporal-block depth or batch it runs in.
//
// Plain-PDHG iterate at node x (eq. (primaldual), A* = minus forward
// difference, so m - mu A* phi = m + mu grad phi):
//   m+    = shrink_p(m + mu grad+ phi, mu)
//   mbar  = 2 m+ - m
//   phi+  = phi + tau (div mbar - rho)
// Prox-PDHG iterate (eq. (pdhg)):
//   v = m - mu vphibar;  u = (A A*)^{-1}(A v - rho);  m+ = v + grad+ u;
//   vphi+ = Proj_{||.||_q <= 1}(vphi + tau m+);  vphibar+ = 2 vphi+ - vphi.
#include "w1_internal.hpp"
#include "mfma_tile.hpp"
#include <hip/hip_ext.h>
#include <cmath>
#include <cstdio>
#include <type_traits>

namespace w1 {

// ---------------------------------------------------------------------------
// per-node helpers
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T fma_(T a, T b, T c);
template <> __device__ __forceinline__ float fma_(float a, float b, float c) { return __fmaf_rn(a, b, c); }
template <> __device__ __forceinline__ double fma_(double a, double b, double c) { return __fma_rn(a, b, c); }

template <typename T> __device__ __forceinline__ T sqrt_(T a);
template <> __device__ __forceinline__ float sqrt_(float a) { return sqrtf(a); }
template <> __device__ __forceinline__ double sqrt_(double a) { return sqrt(a); }

template <typename T> __device__ __forceinline__ T abs_(T a) { return a < T(0) ? -a : a; }

// Plane and table pointers come from the slot descriptors in memory, so the
// compiler sees generic pointers and emits flat loads, which also count
// against the LDS wait counter: every wait for an LDS read then waits for
// the global prefetches in flight too.  The planes and tables are device
// global memory; through these views the loads and stores are global ones.
#define W1_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ const W1_GLOBAL T* gld_(const T* p) { return (const W1_GLOBAL T*)p; }
template <typename T> __device__ __forceinline__ W1_GLOBAL T* gst_(T* p) { return (W1_GLOBAL T*)p; }

// Ground metric codes: 1 = l_1, 2 = l_2, 3 = l_inf (dual norms inf, 2, 1).
//
// prox of mu ||.||_inf at one node (Sec. 4.2, the p = inf case): v minus
// the projection of v onto the l_1 ball of radius mu (Moreau).  With two
// components that projection has a closed form: when one magnitude exceeds
// the other by mu or more only the larger one moves, by mu; otherwise both
// become (|v1| + |v2| - mu)/2 (0 when |v|_1 <= mu).  Signs are kept.
template <typename T>
__device__ __forceinline__ void shrink_inf_(T v1, T v2, T mu, T& o1, T& o2) {
  const T a = abs_(v1), b = abs_(v2);
  T x1, x2;
  if (a - b >= mu) {
    x1 = a - mu;
    x2 = b;
  } else if (b - a >= mu) {
    x1 = a;
    x2 = b - mu;
  } else {
    const T t = (a + b - mu) * T(0.5);
    x1 = t > T(0) ? t : T(0);
    x2 = x1;
  }
  o1 = v1 < T(0) ? -x1 : x1;
  o2 = v2 < T(0) ? -x2 : x2;
}

// prox of mu ||.||_p at one node: p = 1 soft-threshold per component,
// p = 2 isotropic shrink (0 when ||v|| <= mu), p = inf as above.  The FP32
// isotropic factor 1 - mu/||v|| uses the hardware reciprocal square root
// (about 1 ulp); FP64 keeps the correctly rounded square root and division.
template <typename T>
__device__ __forceinline__ void shrink_(T v1, T v2, T mu, int metric, T& o1, T& o2);
template <>
__device__ __forceinline__ void shrink_(float v1, float v2, float mu, int metric, float& o1, float& o2) {
  if (metric == 3) {
    shrink_inf_(v1, v2, mu, o1, o2);
  } else if (metric == 1) {
    float a1 = fabsf(v1) - mu, a2 = fabsf(v2) - mu;
    a1 = a1 > 0.f ? a1 : 0.f;
    a2 = a2 > 0.f ? a2 : 0.f;
    o1 = v1 < 0.f ? -a1 : a1;
    o2 = v2 < 0.f ? -a2 : a2;
  } else {
    const float s2 = v1 * v1 + v2 * v2;
    const float s = s2 > mu * mu ? 1.f - mu * __builtin_amdgcn_rsqf(s2) : 0.f;
    o1 = v1 * s;
    o2 = v2 * s;
  }
}
template <>
__device__ __forceinline__ void shrink_(double v1, double v2, double mu, int metric, double& o1, double& o2) {
  if (metric == 3) {
    shrink_inf_(v1, v2, mu, o1, o2);
  } else if (metric == 1) {
    double a1 = fabs(v1) - mu, a2 = fabs(v2) - mu;
    a1 = a1 > 0.0 ? a1 : 0.0;
    a2 = a2 > 0.0 ? a2 : 0.0;
    o1 = v1 < 0.0 ? -a1 : a1;
    o2 = v2 < 0.0 ? -a2 : a2;
  } else {
    const double s2 = v1 * v1 + v2 * v2;
    const double nv = sqrt(s2);
    const double s = nv > mu ? 1.0 - mu / nv : 0.0;
    o1 = v1 * s;
    o2 = v2 * s;
  }
}

// projection onto the unit ball of the dual norm q (q = inf for p = 1,
// q = 2 for p = 2, q = 1 for p = inf: the l_1 ball, a vector outside it
// loses (|w1| + |w2| - 1)/2 from both magnitudes, or keeps only its larger
// component, as sign 1, when that exceeds the other by 1 or more)
template <typename T>
__device__ __forceinline__ void proj_ball_(T w1, T w2, int metric, T& o1, T& o2) {
  if (metric == 3) {
    const T a = abs_(w1), b = abs_(w2);
    T x1 = a, x2 = b;
    if (a + b > T(1)) {
      if (a - b >= T(1)) {
        x1 = T(1);
        x2 = T(0);
      } else if (b - a >= T(1)) {
        x1 = T(0);
        x2 = T(1);
      } else {
        x1 = (a - b + T(1)) * T(0.5);
        x2 = (b - a + T(1)) * T(0.5);
      }
    }
    o1 = w1 < T(0) ? -x1 : x1;
    o2 = w2 < T(0) ? -x2 : x2;
  } else if (metric == 1) {
    o1 = w1 > T(1) ? T(1) : (w1 < T(-1) ? T(-1) : w1);
    o2 = w2 > T(1) ? T(1) : (w2 < T(-1) ? T(-1) : w2);
  } else {
    T s2 = w1 * w1 + w2 * w2;
    T nw = sqrt_(s2);
    if (nw > T(1)) {
      o1 = w1 / nw;
      o2 = w2 / nw;
    } else {
      o1 = w1;
      o2 = w2;
    }
  }
}

template <typename T>
__device__ __forceinline__ T norm_p_(T a, T b, int metric) {
  const T x = abs_(a), y = abs_(b);
  return metric == 1 ? x + y : (metric == 3 ? (x > y ? x : y) : sqrt_(a * a + b * b));
}
// dual norm q of a gradient
template <typename T>
__device__ __forceinline__ T norm_q_(T a, T b, int metric) {
  const T x = abs_(a), y = abs_(b);
  return metric == 1 ? (x > y ? x : y) : (metric == 3 ? x + y : sqrt_(a * a + b * b));
}

// flux half of the plain iterate; hd / hr say whether the node has a
// neighbour along x1 / x2 (false on the last row / column)
template <typename T>
__device__ __forceinline__ void plain_flux_(T m1, T m2, T pc, T pd, T pr, bool hd, bool hr, T ih, T mu,
                                            int metric, T& n1, T& n2) {
  T g1 = hd ? (pd - pc) * ih : T(0);
  T g2 = hr ? (pr - pc) * ih : T(0);
  T v1 = fma_(mu, g1, m1);
  T v2 = fma_(mu, g2, m2);
  shrink_(v1, v2, mu, metric, n1, n2);
}

// potential half: b1c, b2c extrapolated flux at the node, b1u at (i-1, j),
// b2l at (i, j-1) (zero outside the grid)
template <typename T>
__device__ __forceinline__ T plain_potential_(T pc, T b1c, T b1u, T b2c, T b2l, T rho, T ih, T tau) {
  T dv = ((b1c - b1u) + (b2c - b2l)) * ih;
  return fma_(tau, dv - rho, pc);
}

template <typename T> __device__ __forceinline__ bool finite_(T v) { return isfinite(v); }

// Neumaier-compensated FP64 accumulation
struct Acc {
  double s, c;
  __device__ void add(double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  __device__ double get() const { return s + c; }
};

// Block reduction of NQ doubles per thread into out[0..NQ): wave shuffles,
// then waves in order through LDS.  `maxmask` marks quantities reduced with
// max instead of sum.  Deterministic for a fixed block size.
template <int NT, int NUSED = NQ>
__device__ void block_reduce_(double (&v)[NQ], double* out, double* lds, unsigned maxmask) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = NUSED; q < NQ; ++q) v[q] = 0.0;
#pragma unroll
  for (int q = 0; q < NUSED; ++q) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_xor(v[q], off, 64);
      v[q] = ((maxmask >> q) & 1) ? (o > v[q] ? o : v[q]) : v[q] + o;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[wv * NQ + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    const int q = threadIdx.x;
    double s = lds[q];
    for (int k = 1; k < NT / 64; ++k) {
      double o = lds[k * NQ + q];
      s = ((maxmask >> q) & 1) ? (o > s ? o : s) : s + o;
    }
    out[q] = s;
  }
}

// simple tile: 16 rows x 64 columns, 256 threads, 4 rows per thread
#define SIMPLE_TILE_LOOP(d, w, ...)                                         \
  {                                                                         \
    const int _c = threadIdx.x & 63, _r0 = threadIdx.x >> 6;                \
    _Pragma("unroll") for (int _k = 0; _k < 4; ++_k) {                      \
      const int i = (w).y * ST_H + _r0 + 4 * _k;                            \
      const int j = (w).z * ST_W + _c;                                      \
      if (i <= (d).n && j <= (d).n) {                                       \
        const size_t off = (size_t)i * (d).pitch + j;                       \
        (void)off;                                                          \
        __VA_ARGS__                                                         \
      }                                                                     \
    }                                                                       \
  }

// ---------------------------------------------------------------------------
// utility kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_zero(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                              unsigned mask) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  SIMPLE_TILE_LOOP(d, w, {
    for (int k = 0; k < NPLANES; ++k)
      if ((mask >> k) & 1) d.p[k][off] = T(0);
  })
}

// a slot's scalars at a level start: status RUN, iteration 0, iterate in
// plane set A (the list's item with tile index 0 writes them)
__global__ __launch_bounds__(64) void k_reset_scalars(const Work* __restrict__ work, SlotScalars* __restrict__ scal) {
  const Work w = work[blockIdx.x];
  if (w.x < 0 || w.w != 0 || threadIdx.x != 0) return;
  SlotScalars z{};
  z.status = ST_RUN;
  scal[w.x / MAXL] = z;
}

// copy a dense (pitch n+1) array into / out of a plane
template <typename T>
__global__ __launch_bounds__(256) void k_import(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                                int plane, const T* __restrict__ src) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  T* dst = plane < NPLANES ? d.p[plane] : d.rho;
  SIMPLE_TILE_LOOP(d, w, { dst[off] = src[(size_t)i * (d.n + 1) + j]; })
}

template <typename T>
__global__ __launch_bounds__(256) void k_export(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                                int plane, T* __restrict__ dst) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  const T* src = plane < NPLANES ? d.p[plane] : d.rho;
  SIMPLE_TILE_LOOP(d, w, { dst[(size_t)i * (d.n + 1) + j] = src[off]; })
}

// per-slot reduction of tile partials: one workgroup per listed descriptor
template <typename T>
__global__ __launch_bounds__(256) void k_reduce(const int* __restrict__ idx, const int* __restrict__ ntiles,
                                                const SlotDesc<T>* __restrict__ desc, SlotScalars* __restrict__ sc,
                                                int nq, int out_base, unsigned maxmask) {
  __shared__ double lds[4 * NQ];
  __shared__ double res[NQ];
  const int x = idx[blockIdx.x];
  const int nt = ntiles[blockIdx.x];
  const SlotDesc<T>& d = desc[x];
  double v[NQ];
  for (int q = 0; q < NQ; ++q) {
    Acc a{0.0, 0.0};
    double mx = -INFINITY;
    if (q < nq) {
      for (int t = threadIdx.x; t < nt; t += 256) {
        double p = d.part[(size_t)t * NQ + q];
        a.add(p);
        mx = p > mx ? p : mx;
      }
    }
    v[q] = ((maxmask >> q) & 1) ? mx : a.get();
  }
  block_reduce_<256>(v, res, lds, maxmask);
  __syncthreads();
  if (threadIdx.x < nq && out_base + (int)threadIdx.x < 8) sc[x / MAXL].sums[out_base + threadIdx.x] = res[threadIdx.x];
}

// ---------------------------------------------------------------------------
// input preparation and the density pyramid (Sec. 2.2; restriction by
// normalised full weighting, the transpose of eq. (inter_phi))
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_prep_stats(const Work* __restrict__ work,
                                                    const SlotDesc<T>* __restrict__ desc) {
  __shared__ double lds[4 * NQ];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  double v[NQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  SIMPLE_TILE_LOOP(d, w, {
    const size_t o = (size_t)i * (d.n + 1) + j;
    double a = d.in0[o], b = d.in1[o];
    if (!(isfinite(a) && isfinite(b)) || a < 0.0 || b < 0.0) v[2] += 1.0;
    else { v[0] += a; v[1] += b; }
  })
  block_reduce_<256>(v, d.part + (size_t)w.w * NQ, lds, 0u);
}

// rho^k = p^k / (S^k h^2) on the finest level (FP64 staging planes)
template <typename T>
__global__ __launch_bounds__(256) void k_prep_scale(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                                    const SlotScalars* __restrict__ sc) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  const SlotScalars& s = sc[w.x / MAXL];
  const double h2 = d.h * d.h;
  const double a0 = s.sums[0] * h2, a1 = s.sums[1] * h2;
  SIMPLE_TILE_LOOP(d, w, {
    const size_t o = (size_t)i * (d.n + 1) + j;
    d.r0[off] = d.in0[o] / a0;
    d.r1[off] = d.in1[o] / a1;
  })
}

// 1-D factor of the restriction: weights of fine index I for coarse a
__device__ __forceinline__ double rw1d_(int I, int a, int nf) {
  int dI = I - 2 * a;
  if (I < 0 || I > nf) return 0.0;
  return dI == 0 ? 1.0 : ((dI == 1 || dI == -1) ? 0.5 : 0.0);
}

// coarse level x from fine level x+1: c = D^{-1} P^T f, both staging planes;
// partial sums of the result (for the unit-mass renormalisation)
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc) {
  __shared__ double lds[4 * NQ];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  const SlotDesc<T>& f = desc[w.x + 1];
  const int nf = f.n;
  double v[NQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  SIMPLE_TILE_LOOP(d, w, {
    double s0 = 0.0, s1 = 0.0, wi_sum = 0.0, wj_sum = 0.0;
    for (int di = -1; di <= 1; ++di) wi_sum += rw1d_(2 * i + di, i, nf);
    for (int dj = -1; dj <= 1; ++dj) wj_sum += rw1d_(2 * j + dj, j, nf);
    for (int di = -1; di <= 1; ++di) {
      const int I = 2 * i + di;
      const double wi = rw1d_(I, i, nf);
      if (wi == 0.0) continue;
      for (int dj = -1; dj <= 1; ++dj) {
        const int J = 2 * j + dj;
        const double wj = rw1d_(J, j, nf);
        if (wj == 0.0) continue;
        const size_t fo = (size_t)I * f.pitch + J;
        s0 += wi * wj * f.r0[fo];
        s1 += wi * wj * f.r1[fo];
      }
    }
    const double dw = wi_sum * wj_sum;
    const double c0 = s0 / dw, c1 = s1 / dw;
    d.r0[off] = c0;
    d.r1[off] = c1;
    v[0] += c0;
    v[1] += c1;
  })
  block_reduce_<256>(v, d.part + (size_t)w.w * NQ, lds, 0u);
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale_level(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                                     const SlotScalars* __restrict__ sc) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  const SlotScalars& s = sc[w.x / MAXL];
  const double h2 = d.h * d.h;
  const double a0 = s.sums[0] * h2, a1 = s.sums[1] * h2;
  SIMPLE_TILE_LOOP(d, w, {
    d.r0[off] = d.r0[off] / a0;
    d.r1[off] = d.r1[off] / a1;
  })
}

template <typename T>
__global__ __launch_bounds__(256) void k_rho_diff(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc) {
  __shared__ double lds[4 * NQ];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  double v[NQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  SIMPLE_TILE_LOOP(d, w, { v[0] += d.r0[off] - d.r1[off]; })
  block_reduce_<256>(v, d.part + (size_t)w.w * NQ, lds, 0u);
}

// rho_l = rho0_l - rho1_l - mean, cast to the iterate precision
template <typename T>
__global__ __launch_bounds__(256) void k_rho_write(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                                   const SlotScalars* __restrict__ sc) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  const double N = (double)(d.n + 1);
  const double mean = sc[w.x / MAXL].sums[0] / (N * N);
  SIMPLE_TILE_LOOP(d, w, { d.rho[off] = (T)((d.r0[off] - d.r1[off]) - mean); })
}

// ---------------------------------------------------------------------------
// prolongation, Sec. 3.3: eq. (inter_phi) (bilinear) for the potential and
// eq. (inter_m) for the flux and the edge dual (nearest along the edge's own
// axis with the tie to x_i - h_l, average across).  Work items tile the fine
// level x; the coarse level is x - 1, read from its current plane set.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T pro_node_(const T* c, int pc, int I, int J) {
  const int a0 = I >> 1, a1 = (I + 1) >> 1, b0 = J >> 1, b1 = (J + 1) >> 1;
  if (!(I & 1) && !(J & 1)) return c[(size_t)a0 * pc + b0];
  if ((I & 1) && !(J & 1)) return (c[(size_t)a0 * pc + b0] + c[(size_t)a1 * pc + b0]) / T(2);
  if (!(I & 1) && (J & 1)) return (c[(size_t)a0 * pc + b0] + c[(size_t)a0 * pc + b1]) / T(2);
  return (((c[(size_t)a0 * pc + b0] + c[(size_t)a0 * pc + b1]) + c[(size_t)a1 * pc + b0]) + c[(size_t)a1 * pc + b1]) /
         T(4);
}
// flux along x1: coarse row floor(I/2), average across J
template <typename T>
__device__ __forceinline__ T pro_e1_(const T* c, int pc, int I, int J) {
  const int a = I >> 1, b0 = J >> 1, b1 = (J + 1) >> 1;
  if (!(J & 1)) return c[(size_t)a * pc + b0];
  return (c[(size_t)a * pc + b0] + c[(size_t)a * pc + b1]) / T(2);
}
template <typename T>
__device__ __forceinline__ T pro_e2_(const T* c, int pc, int I, int J) {
  const int b = J >> 1, a0 = I >> 1, a1 = (I + 1) >> 1;
  if (!(I & 1)) return c[(size_t)a0 * pc + b];
  return (c[(size_t)a0 * pc + b] + c[(size_t)a1 * pc + b]) / T(2);
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                                 const SlotScalars* __restrict__ scal, int kind) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  const SlotDesc<T>& c = desc[w.x - 1];
  const int pc = c.pitch, nf = d.n;
  if (kind == K_PLAIN) {
    const int cs = scal[w.x / MAXL].cur & 1;
    const T* c1 = c.p[3 * cs];
    const T* c2 = c.p[3 * cs + 1];
    const T* cp = c.p[3 * cs + 2];
    SIMPLE_TILE_LOOP(d, w, {
      d.p[0][off] = i < nf ? pro_e1_(c1, pc, i, j) : T(0);
      d.p[1][off] = j < nf ? pro_e2_(c2, pc, i, j) : T(0);
      d.p[2][off] = pro_node_(cp, pc, i, j);
    })
  } else {
    SIMPLE_TILE_LOOP(d, w, {
      d.p[0][off] = i < nf ? pro_e1_(c.p[0], pc, i, j) : T(0);
      d.p[1][off] = j < nf ? pro_e2_(c.p[1], pc, i, j) : T(0);
      const T q1 = i < nf ? pro_e1_(c.p[2], pc, i, j) : T(0);
      const T q2 = j < nf ? pro_e2_(c.p[3], pc, i, j) : T(0);
      d.p[2][off] = q1;
      d.p[3][off] = q2;
      d.p[4][off] = q1;   // vphibar starts equal to vphi at a level start
      d.p[5][off] = q2;
    })
  }
}

// ---------------------------------------------------------------------------
// cross-lane moves inside a 64-wide wavefront (DPP wave shifts, readlane)
// ---------------------------------------------------------------------------
// lane i receives lane i-1 (lane 0 receives 0)
__device__ __forceinline__ int lane_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
// lane i receives lane i+1 (lane 63 receives 0)
__device__ __forceinline__ int lane_next_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }

// rotations: lane i receives lane i+1 (lane 63 receives lane 0) / lane i-1
// (lane 0 receives lane 63)
__device__ __forceinline__ int lane_rot_next_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x134, 0xf, 0xf, true); }
__device__ __forceinline__ int lane_rot_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x13c, 0xf, 0xf, true); }
__device__ __forceinline__ float lane_rot_next(float v) { return __int_as_float(lane_rot_next_i(__float_as_int(v))); }
__device__ __forceinline__ float lane_rot_prev(float v) { return __int_as_float(lane_rot_prev_i(__float_as_int(v))); }
__device__ __forceinline__ double lane_rot_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_rot_next_i((int)(b & 0xffffffffll)), hi = lane_rot_next_i((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_rot_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_rot_prev_i((int)(b & 0xffffffffll)), hi = lane_rot_prev_i((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(lane_prev_i(__float_as_int(v))); }
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(lane_next_i(__float_as_int(v))); }
__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_prev_i((int)(b & 0xffffffffll)), hi = lane_prev_i((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_next_i((int)(b & 0xffffffffll)), hi = lane_next_i((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_read(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ---------------------------------------------------------------------------
// Algorithm 1, tiled with temporal blocking, iterate held in registers.
// A workgroup of 8 wavefronts covers a 64 x 128 region: wavefront w owns
// rows [8w, 8w+8), lane l owns columns l and l+64 (16 wavefronts: rows
// [4w, 4w+4)).  The 64 x 64 region (RWID = 64, lane l owns column l) spreads
// a grid over twice as many workgroups at a larger halo share, for launches
// that leave most of the device idle; the 32 x 64 region over 8 wavefronts
// (4 rows each) halves the work of a workgroup again, for the launches of a
// few slots late in a batch.  The region is the
// output tile plus a halo of `steps` nodes on every side; after s steps the
// flux is valid on rows [s-1, 63-s] and the potential on [s, 63-s] (same for
// columns), so `steps` iterations run without leaving the workgroup and the
// (64 - 2 steps) x (128 - 2 steps) interior is exact.
// Every node's neighbours come from registers: the next / previous row of
// the thread's own column strip, the next / previous column through DPP
// wave shifts (readlane across the two column halves).  Only the first
// potential row and the last extrapolated-flux row of each strip cross
// wavefronts, through 8 KB of LDS, so a step costs two barriers.
// The launch with index li inside a block reads plane set cur ^ (li & 1)
// and writes the other one.  The last step is peeled off the loop; with
// CHECK it also produces the FPR partials of eq. (pd_stop) over the
// interior: sum |dm|^2, sum dphi^2, sum dphi * A dm, without extra
// per-node state (the checked step needs no more registers
// than a plain one, so both variants run at the same occupancy).
// ---------------------------------------------------------------------------
#ifndef W1_TILED_WPE
#define W1_TILED_WPE 2
#endif
#ifndef W1_TILED_WPE_CHECK
#define W1_TILED_WPE_CHECK 4
#endif
template <typename T, bool CHECK, int METRIC, int NWV = 8, int RWID = TILED_RW, int RHT = TILED_RH,
          int WAVES_PER_EU = (NWV == 16 ? (sizeof(T) == 4 ? 8 : 4)
                                        : (sizeof(T) == 4 ? (CHECK ? W1_TILED_WPE_CHECK : W1_TILED_WPE) : 2))>
__global__ __launch_bounds__(NWV * 64) __attribute__((amdgpu_waves_per_eu(WAVES_PER_EU, 8))) void k_plain_tiled(
    const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc, const SlotScalars* __restrict__ scal,
    int li, int steps, int second) {
  constexpr int RH = RHT, RW = RWID, NR = RH / NWV, NC = RW / 64;
  static_assert(NC == 1 || NC == 2, "regions are 64 or 128 columns wide");
  static_assert(NR * NWV == RH, "wavefronts split the region's rows evenly");
  __shared__ T Bp[NWV][RW];   // first potential row of each strip
  __shared__ T Bb[NWV][RW];   // last extrapolated-flux row (axis 1) of each strip
  __shared__ double lds[NWV * NQ];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotScalars& sc = scal[w.x / MAXL];
  if (sc.status != ST_RUN) return;
  const SlotDesc<T>& d = desc[w.x];
  if (d.metric != METRIC) return;
  const int n = d.n, pitch = d.pitch, S = steps;
  const int OH = RH - 2 * S, OW = RW - 2 * S;
  const int gi0 = w.y * OH - S, gj0 = w.z * OW - S;
  const int rs = (sc.cur ^ li) & 1, ws = rs ^ 1;
  const W1_GLOBAL T* __restrict__ sm1 = gld_(d.p[3 * rs]);
  const W1_GLOBAL T* __restrict__ sm2 = gld_(d.p[3 * rs + 1]);
  const W1_GLOBAL T* __restrict__ sph = gld_(d.p[3 * rs + 2]);
  const W1_GLOBAL T* __restrict__ srho = gld_(d.rho);
  const T ih = d.ih, mu = d.mu, tau = d.tau;
  constexpr int metric = METRIC;   // one launch per ground metric
  // the wavefront index is uniform across the wavefront: held in a scalar
  // register, every row test below is a scalar branch
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = wv * NR;

  // per-node geometry: row / column inside the grid, has-next flags
  bool rin[NR], rhd[NR];
  bool cin[NC], chr[NC];
#pragma unroll
  for (int a = 0; a < NR; ++a) {
    const int gi = gi0 + r0 + a;
    rin[a] = (unsigned)gi <= (unsigned)n;
    rhd[a] = gi < n && r0 + a + 1 < RH;
  }
#pragma unroll
  for (int b = 0; b < NC; ++b) {
    const int c = lane + 64 * b, gj = gj0 + c;
    cin[b] = (unsigned)gj <= (unsigned)n;
    // no neighbour to the right outside the grid either (gj < 0): every
    // node outside the grid then keeps zero iterates without masking (its
    // gradient, flux, extrapolated flux and divergence are all zero)
    chr[b] = gj >= 0 && gj < n && c + 1 < RW;
  }

  // a row of the strip, or a column half, that lies wholly outside the grid
  // keeps zero iterates: its arithmetic is skipped (wave-uniform test)
  bool hact[NC];
#pragma unroll
  for (int b = 0; b < NC; ++b) hact[b] = gj0 + 64 * b <= n;

  T m1[NR][NC], m2[NR][NC], ph[NR][NC], rh[NR][NC], b1[NR][NC], b2[NR][NC];
#pragma unroll
  for (int a = 0; a < NR; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      const bool in = rin[a] && cin[b];
      const size_t off = in ? (size_t)(gi0 + r0 + a) * pitch + (gj0 + lane + 64 * b) : 0;
      m1[a][b] = in ? sm1[off] : T(0);
      m2[a][b] = in ? sm2[off] : T(0);
      ph[a][b] = in ? sph[off] : T(0);
      rh[a][b] = in ? srho[off] : T(0);
      b1[a][b] = T(0);
      b2[a][b] = T(0);
    }

  // Stop-test partials of the last step (CHECK), summed over the interior.
  // The flux change is not stored: after the flux half, m holds m+ and b
  // holds 2 m+ - m, so b - m is the change, and A dm is read from the same
  // neighbours as the divergence of b (the last new-flux row of each strip
  // crosses wavefronts through Bm).
  __shared__ T Bm[CHECK ? NWV : 1][RW];
  // per-thread partials in the iterate precision (16 nodes per thread),
  // summed in FP64 across the workgroup
  // (a non-finite iterate makes q0 or q1 non-finite, and with them the
  // measure, which the stop test reports as divergence)
  T q0 = T(0), q1 = T(0), q2 = T(0);

  // one step; KEEP marks the checked last step
  auto step = [&](auto keep) {
    constexpr bool KEEP = decltype(keep)::value;
#pragma unroll
    for (int b = 0; b < NC; ++b) Bp[wv][lane + 64 * b] = ph[0][b];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NR; ++a) {
      // potential at the next column: lane + 1, crossing into the second
      // column half at lane 63 (lane 0 offers that half's first column to
      // the rotation); the region's last column has no neighbour
      T x0, x1 = T(0);
      if constexpr (NC == 2) {
        x0 = lane_rot_next(lane == 0 ? ph[a][NC - 1] : ph[a][0]);
        x1 = lane_next(ph[a][NC - 1]);
      } else {
        x0 = lane_next(ph[a][0]);
      }
#pragma unroll
      for (int b = 0; b < NC; ++b) {
        if (!(rin[a] && hact[b])) continue;
        const T pc = ph[a][b];
        const T pd = a + 1 < NR ? ph[a + 1 < NR ? a + 1 : a][b] : (wv + 1 < NWV ? Bp[wv + 1 < NWV ? wv + 1 : wv][lane + 64 * b] : pc);
        const T pr = b == 0 ? x0 : x1;
        T n1, n2;
        plain_flux_(m1[a][b], m2[a][b], pc, pd, pr, rhd[a], chr[b], ih, mu, metric, n1, n2);
        b1[a][b] = fma_(T(2), n1, -m1[a][b]);   // 2 n1 is exact: the same rounding as (n1 + n1) - m1
        b2[a][b] = fma_(T(2), n2, -m2[a][b]);
        if constexpr (KEEP) {
          const int r = r0 + a, c = lane + 64 * b;
          const T e1 = n1 - m1[a][b], e2 = n2 - m2[a][b];
          if (rin[a] && cin[b] && r >= S && r < RH - S && c >= S && c < RW - S)
            q0 = fma_(e1, e1, fma_(e2, e2, q0));
        }
        m1[a][b] = n1;
        m2[a][b] = n2;
      }
    }
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      Bb[wv][lane + 64 * b] = b1[NR - 1][b];
      if constexpr (KEEP) Bm[wv][lane + 64 * b] = m1[NR - 1][b];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NR; ++a) {
      // extrapolated flux (axis 2) at the previous column: lane - 1,
      // crossing back from the second column half at lane 0 (lane 63
      // offers the first half's last column to the rotation)
      const T y0 = lane_prev(b2[a][0]);
      T y1 = T(0);
      if constexpr (NC == 2) y1 = lane_rot_prev(lane == 63 ? b2[a][0] : b2[a][NC - 1]);
      // the same shifts of the new flux (axis 2) for the checked step; the
      // cross-lane reads run with every lane active, outside any per-lane
      // condition, so no lane reads a masked-off neighbour
      T z0 = T(0), z1 = T(0);
      if constexpr (KEEP) {
        z0 = lane_prev(m2[a][0]);
        if constexpr (NC == 2) z1 = lane_rot_prev(lane == 63 ? m2[a][0] : m2[a][NC - 1]);
      }
#pragma unroll
      for (int b = 0; b < NC; ++b) {
        if (!(rin[a] && hact[b])) continue;
        const T b1u = a > 0 ? b1[a > 0 ? a - 1 : 0][b] : (wv > 0 ? Bb[wv > 0 ? wv - 1 : 0][lane + 64 * b] : T(0));
        const T b2l = b == 0 ? y0 : y1;
        const T pn = plain_potential_(ph[a][b], b1[a][b], b1u, b2[a][b], b2l, rh[a][b], ih, tau);
        if constexpr (KEEP) {
          const int r = r0 + a, c = lane + 64 * b;
          // flux change at the node, at (i-1, j) and at (i, j-1); interior
          // nodes have r, c >= S >= 1, so both neighbours are in the region
          const T m1u = a > 0 ? m1[a > 0 ? a - 1 : 0][b] : (wv > 0 ? Bm[wv > 0 ? wv - 1 : 0][lane + 64 * b] : T(0));
          const T m2l = b == 0 ? z0 : z1;
          if (rin[a] && cin[b] && r >= S && r < RH - S && c >= S && c < RW - S) {
            const T e1c = b1[a][b] - m1[a][b], e1u = b1u - m1u;
            const T e2c = b2[a][b] - m2[a][b], e2l = b2l - m2l;
            const T adm = ((e1c - e1u) + (e2c - e2l)) * ih;
            const T pe = pn - ph[a][b];
            q1 = fma_(pe, pe, q1);
            q2 = fma_(pe, adm, q2);
          }
        }
        ph[a][b] = pn;
      }
    }
  };

  // two steps per trip: the new flux lands in the registers the old one
  // frees, with no copies between steps
  int s = 0;
  for (; s + 2 <= S - 1; s += 2) {
    step(std::false_type{});
    step(std::false_type{});
  }
  if (s < S - 1) step(std::false_type{});
  if constexpr (CHECK) {
    step(std::true_type{});
    double v[NQ] = {(double)q0, (double)q1, (double)q2, 0, 0, 0, 0, 0};
    // the second block of a pair writes after the first block's partials
    const size_t off =
        second ? (size_t)((n + RH - 2 * S) / (RH - 2 * S)) * ((n + RW - 2 * S) / (RW - 2 * S)) : 0;
    block_reduce_<NWV * 64, 4>(v, d.part + (off + (size_t)w.w) * NQ, lds, 0u);
  } else {
    step(std::false_type{});
  }

  W1_GLOBAL T* __restrict__ om1 = gst_(d.p[3 * ws]);
  W1_GLOBAL T* __restrict__ om2 = gst_(d.p[3 * ws + 1]);
  W1_GLOBAL T* __restrict__ oph = gst_(d.p[3 * ws + 2]);
#pragma unroll
  for (int a = 0; a < NR; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      const int r = r0 + a, c = lane + 64 * b;
      if (rin[a] && cin[b] && r >= S && r < RH - S && c >= S && c < RW - S) {
        const size_t off = (size_t)(gi0 + r) * pitch + (gj0 + c);
        // streaming stores: the next launch reads these planes from other
        // compute units, so they need not stay in this XCD's L2 (fewer dirty
        // lines to write back when the launch ends; ~1% per launch)
        __builtin_nontemporal_store(m1[a][b], &om1[off]);
        __builtin_nontemporal_store(m2[a][b], &om2[off]);
        __builtin_nontemporal_store(ph[a][b], &oph[off]);
      }
    }
}

// ---------------------------------------------------------------------------
// Algorithm 1, whole level resident in one workgroup.
// For grids whose potential and both extrapolated-flux planes fit in LDS
// (3 (n+1)^2 sizeof(T) bytes), one workgroup per pair runs the level to its
// stop test or cap without touching HBM in between.  Node e (row-major,
// dense) belongs to thread e mod the workgroup size; the flux, rho and the
// node's own potential and extrapolated flux stay in registers, the planes
// in LDS carry the neighbours: an iteration is two phases with one barrier
// each (flux half writing 2 m+ - m, potential half reading it at (i-1, j)
// and (i, j-1)).  Stop tests (both rules) run every `check_every`
// iterations and at the cap, with the flux change (FPR) or the new flux
// (KKT) exchanged through the same planes.  Reads and writes plane set A.
// A launch runs at most `chunk` iterations (0: no limit) and resumes from
// the slot's iteration count, so long levels can run in bounded pieces.
// ---------------------------------------------------------------------------
// workgroup size and nodes per thread of the resident Algorithm 1 kernel:
// 16 wavefronts for FP32, 8 for FP64 (its iterate needs twice the registers)
template <typename T> struct ResCfg;
template <> struct ResCfg<float> { static constexpr int NT = 1024, NPT = 5, MAXN = 65; };
template <> struct ResCfg<double> { static constexpr int NT = 512, NPT = 9, MAXN = 65; };

template <typename T, int NPT, int METRIC>
__global__ __launch_bounds__(ResCfg<T>::NT) void k_plain_resident(const int* __restrict__ idx,
                                                                const SlotDesc<T>* __restrict__ desc,
                                                                SlotScalars* __restrict__ scal, int check_every,
                                                                int chunk) {
  extern __shared__ double smem_d[];
  constexpr int NT = ResCfg<T>::NT;
  static_assert(NPT <= 32, "column masks hold 32 nodes");
  const int x = idx[blockIdx.x];
  const SlotDesc<T>& d = desc[x];
  if (d.metric != METRIC) return;
  SlotScalars& sc = scal[x / MAXL];
  const int n = d.n, N = n + 1, NN = N * N, pitch = d.pitch;
  const int last_row = NN - N;          // e >= last_row  <=>  row n
  double* red = smem_d;                 // [16 * NQ]
  double* res = smem_d + 16 * NQ;       // [NQ]
  int* flag = (int*)(smem_d + 17 * NQ);
  T* Lp = (T*)(smem_d + 18 * NQ);       // potential
  T* Lb = Lp + NN;                      // extrapolated flux, axis 1
  T* Lc = Lb + NN;                      // extrapolated flux, axis 2
  const T ih = d.ih, mu = d.mu, tau = d.tau;
  constexpr int metric = METRIC;   // one launch per ground metric
  const int cap = d.cap;
  const double h2 = d.h * d.h;

  T m1[NPT], m2[NPT], rh[NPT], pv[NPT], b1[NPT], b2[NPT];
  unsigned first_col = 0u, last_col = 0u;   // bit s: node s is on column 0 / column n
#pragma unroll
  for (int s = 0; s < NPT; ++s) {
    const int e = threadIdx.x + NT * s;
    m1[s] = m2[s] = rh[s] = pv[s] = b1[s] = b2[s] = T(0);
    if (e < NN) {
      const int r = e / N, c = e - r * N;
      if (c == 0) first_col |= 1u << s;
      if (c == n) last_col |= 1u << s;
      const size_t off = (size_t)r * pitch + c;
      m1[s] = d.p[0][off];
      m2[s] = d.p[1][off];
      rh[s] = d.rho[off];
      pv[s] = d.p[2][off];
      Lp[e] = pv[s];
    }
  }
  __syncthreads();

  // resume where the previous chunk of this level stopped
  int k = sc.iters;
  const int kend = chunk > 0 ? k + chunk : cap;
  int status = ST_RUN;
  double measure = sc.measure;
  int rises = sc.rises;
  bool tested = k > 0;   // a stop test of this level has run
  const bool fpr = d.rule == RULE_FPR;
  // one iteration; CHK keeps the flux change and the potential change of
  // every node for the stop test that follows it (the other iterations
  // carry no such state)
  T e1[NPT], e2[NPT], dp[NPT];
#pragma unroll
  for (int s = 0; s < NPT; ++s) e1[s] = e2[s] = dp[s] = T(0);
  auto iter = [&](auto chk_tag) __attribute__((always_inline)) {
    constexpr bool CHK = decltype(chk_tag)::value;
    // flux half: potential neighbours from LDS; 2 m+ - m to Lb, Lc
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
      const int e = threadIdx.x + NT * s;
      if (e < NN) {
        const bool hd = e < last_row, hr = !((last_col >> s) & 1u);
        const T pc = pv[s];
        const T pd = hd ? Lp[e + N] : pc;
        const T pr = hr ? Lp[e + 1] : pc;
        T n1, n2;
        plain_flux_(m1[s], m2[s], pc, pd, pr, hd, hr, ih, mu, metric, n1, n2);
        b1[s] = fma_(T(2), n1, -m1[s]);
        b2[s] = fma_(T(2), n2, -m2[s]);
        Lb[e] = b1[s];
        Lc[e] = b2[s];
        if constexpr (CHK) {
          e1[s] = n1 - m1[s];
          e2[s] = n2 - m2[s];
        }
        m1[s] = n1;
        m2[s] = n2;
      }
    }
    __syncthreads();
    // potential half: extrapolated flux at (i-1, j) and (i, j-1)
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
      const int e = threadIdx.x + NT * s;
      if (e < NN) {
        const T b1u = e >= N ? Lb[e - N] : T(0);
        const T b2l = ((first_col >> s) & 1u) ? T(0) : Lc[e - 1];
        const T pn = plain_potential_(pv[s], b1[s], b1u, b2[s], b2l, rh[s], ih, tau);
        if constexpr (CHK) dp[s] = pn - pv[s];
        pv[s] = pn;
        Lp[e] = pn;
      }
    }
    __syncthreads();
  };
  while (k < kend) {
    // the iterations up to the next stop test (a multiple of check_every,
    // or the cap) or to the end of this launch's chunk; the tested one last
    int next = (k / check_every + 1) * check_every;
    if (next > cap) next = cap;
    if (next > kend) next = kend;
    const bool tested_here = next % check_every == 0 || next >= cap;
    for (int plain = next - k - (tested_here ? 1 : 0); plain > 0; --plain) iter(std::false_type{});
    k = next;
    if (!tested_here) continue;   // a chunk that ends between stop tests
    iter(std::true_type{});

    // ---- stop test ----
    // exchange the flux change (FPR) or the new flux (KKT) through Lb, Lc;
    // every read of those planes in this iteration is behind the barrier
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
      const int e = threadIdx.x + NT * s;
      if (e < NN) {
        Lb[e] = fpr ? e1[s] : m1[s];
        Lc[e] = fpr ? e2[s] : m2[s];
      }
    }
    __syncthreads();
    double v[NQ] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
      const int e = threadIdx.x + NT * s;
      if (e < NN) {
        const T u1 = e >= N ? Lb[e - N] : T(0);
        const T l2 = ((first_col >> s) & 1u) ? T(0) : Lc[e - 1];
        if (fpr) {
          const double adm = (double)(((e1[s] - u1) + (e2[s] - l2)) * ih);
          const double ep = (double)dp[s];
          v[0] += (double)e1[s] * (double)e1[s] + (double)e2[s] * (double)e2[s];
          v[1] += ep * ep;
          v[2] += ep * adm;
          if (!(finite_(m1[s]) && finite_(m2[s]) && finite_(pv[s]))) v[3] += 1.0;
        } else {
          // KKT: Lipschitz excess of grad phi, cost, <phi, rho>
          const bool hd = e < last_row, hr = !((last_col >> s) & 1u);
          const double rr = (double)rh[s];
          const T pc = pv[s];
          const T g1 = hd ? (Lp[e + N] - pc) * ih : T(0);
          const T g2 = hr ? (Lp[e + 1] - pc) * ih : T(0);
          const double gq = (double)norm_q_(g1, g2, metric);
          const double ex = gq > 1.0 ? gq - 1.0 : 0.0;
          v[2] += ex * ex;
          v[3] += (double)norm_p_(m1[s], m2[s], metric);
          v[4] += (double)pc * rr;
          v[6] += (double)pc;
          v[7] += rr;
        }
      }
    }
    if (!fpr) {
      // primal part of the KKT residual: ||A* c||_h^2 with c = (A A*)^{-1} r,
      // r = A m - rho, is h^2 sum_x c r = h^4 sum_{(k,l) != 0} rhat_kl^2 /
      // (s_k + s_l) in the orthonormal DCT-II basis (rhat = C r C^T,
      // s_k = 4 sin^2(pi k / 2N)): the forward transform alone, C read from
      // global memory.  r goes to Lp (the potential is restored from the
      // registers afterwards), the row transform to Lb.
      __syncthreads();
#pragma unroll
      for (int s = 0; s < NPT; ++s) {
        const int e = threadIdx.x + NT * s;
        if (e < NN) {
          const T u1 = e >= N ? Lb[e - N] : T(0);
          const T l2 = ((first_col >> s) & 1u) ? T(0) : Lc[e - 1];
          Lp[e] = ((m1[s] - u1) + (m2[s] - l2)) * ih - rh[s];
        }
      }
      __syncthreads();
      const W1_GLOBAL T* C = gld_(d.dctC);
#pragma unroll 1
      for (int e = threadIdx.x; e < NN; e += NT) {
        const int kr = e / N, j = e - kr * N;
        T acc = T(0);
        for (int i = 0; i < N; ++i) acc = fma_(C[kr * N + i], Lp[i * N + j], acc);
        Lb[e] = acc;
      }
      __syncthreads();
      double sp = 0.0;
#pragma unroll 1
      for (int e = threadIdx.x; e < NN; e += NT) {
        const int kr = e / N, l = e - kr * N;
        T acc = T(0);
        for (int j = 0; j < N; ++j) acc = fma_(Lb[kr * N + j], C[l * N + j], acc);
        if (e != 0) sp += (double)acc * (double)acc / (d.dcts[kr] + d.dcts[l]);
      }
#pragma unroll
      for (int s = 0; s < NPT; ++s) {
        const int e = threadIdx.x + NT * s;
        if (e < NN) Lp[e] = pv[s];
      }
      v[0] = sp * h2;
    }
    // the FPR test uses the first four sums only
    if (fpr)
      block_reduce_<NT, 4>(v, res, red, 0u);
    else
      block_reduce_<NT>(v, res, red, 0u);
    __syncthreads();
    if (threadIdx.x == 0) {
      double m;
      if (fpr) {
        m = h2 * (res[0] / d.mud + res[1] / d.taud - 2.0 * res[2]);
        if (res[3] > 0.0) m = NAN;
      } else {
        const double P = res[3] * h2;
        const double rp = sqrt(res[0] * h2) / fmax(P, 1e-300);
        const double rdl = sqrt(res[2] * h2);
        const double D = -(res[4] - res[6] / (double)NN * res[7]) * h2;
        const double den = fmax(fmax(fabs(P), fabs(D)), 1e-300);
        const double gap = fabs(P - D) / den;
        m = fmax(rp, fmax(rdl, gap));
      }
      rises = tested && m > measure ? rises + 1 : 0;
      int st = ST_RUN;
      if (!isfinite(m) || (d.divwin > 0 && m < 0.0)) st = ST_DIVERGED;
      else if (m <= d.tol) st = ST_CONV;
      else if (d.divwin > 0 && rises >= d.divwin) st = ST_DIVERGED;
      else if (k >= cap) st = ST_CAP;
      flag[0] = st;
      res[0] = m;
    }
    tested = true;
    __syncthreads();
    status = flag[0];
    measure = res[0];
    __syncthreads();
    if (status != ST_RUN) break;
  }

#pragma unroll
  for (int s = 0; s < NPT; ++s) {
    const int e = threadIdx.x + NT * s;
    if (e < NN) {
      const int r = e / N, c = e - r * N;
      const size_t off = (size_t)r * pitch + c;
      d.p[0][off] = m1[s];
      d.p[1][off] = m2[s];
      d.p[2][off] = pv[s];
    }
  }
  if (threadIdx.x == 0) {
    sc.iters = k;
    sc.status = status;
    sc.measure = measure;
    sc.rises = rises;
    sc.cur = 0;
  }
}

// The guard of steps beyond the convergence condition (divwin > 0, FPR
// rule): R^k and G^k are squared norms of the iterate change in a metric
// that is positive definite only while mu tau ||A||^2 < 1 (Sec. 3.1), so a
// negative measure, or one that rises at divwin tests in a row, ends the
// level as diverged.
//
// Stop measure from the reduced partials r[0..NQ): R^k (plain) or G^k (prox)
// of eq. (pd_stop) / eq. (pdhg_stop) for RULE_FPR, else the normalised KKT
// residual max(||A* c||_h / P, RMS Lipschitz excess, relative gap), where
// A* c is the least-norm flux correction that makes m feasible (r[0] holds
// ||A* c||_h^2 / h^2).
__device__ double measure_from_(const double* r, int kind, int rule, double h2, double mud, double taud, int NN) {
  if (rule == RULE_FPR) {
    if (r[3] > 0.0) return NAN;
    if (kind == K_PLAIN) return h2 * (r[0] / mud + r[1] / taud - 2.0 * r[2]);
    return h2 * (r[0] / mud + r[1] / taud + 2.0 * r[2]);
  }
  const double P = r[3] * h2;
  const double rp = sqrt(r[0] * h2) / fmax(P, 1e-300);
  const double rdl = sqrt(r[2] * h2);
  const double sgn = kind == K_PLAIN ? -1.0 : 1.0;
  const double D = sgn * (r[4] - r[6] / (double)NN * r[7]) * h2;
  const double den = fmax(fmax(fabs(P), fabs(D)), 1e-300);
  return fmax(rp, fmax(rdl, fabs(P - D) / den));
}

// ---------------------------------------------------------------------------
// Algorithm 2, whole level resident in one workgroup (sides up to 65).
// The iterate (m, vphi, vphibar) and rho stay in registers (node e of the
// dense (n+1)^2 grid belongs to thread e mod 1024); LDS holds the even and
// odd DCT-II blocks, the FP64 factors h^2 / lambda, three node planes for
// the divergence, the Poisson solve and the gradient, and two folded planes.
// One iteration: v = m - mu vphibar, r = A v - rho, u = (A A*)^{-1} r by the
// folded transform below, m+ = v + grad+ u, vphi+ = Proj(vphi + tau m+),
// vphibar+ = 2 vphi+ - vphi -- the same node arithmetic as the batched
// kernels.  Stop tests every `check_every` iterations and at the cap: G^k of
// eq. (pdhg_stop) (pointwise sums) or the normalised KKT residual with
// psi = (A A*)^{-1} A vphi.  Reads and writes planes 0..5; runs at most
// `chunk` iterations (0: no limit), resuming from the slot's count.
// ---------------------------------------------------------------------------
// The Poisson solve in LDS uses the even/odd symmetry of the DCT-II basis
// (C[k][N-1-j] = (-1)^k C[k][j], and C[k][(N-1)/2] = 0 for odd k when N is
// odd) along both axes.  With h = N/2, ne = N - h even and no = h odd
// frequencies, a butterfly over the node quads (p, q), (p, N-1-q),
// (N-1-p, q), (N-1-p, N-1-q) (p, q < ne) gives four folded blocks
// XF_ab (a, b in {even, odd}); the 2D transform is then block diagonal:
// Y_ab = C_a XF_ab C_b^T with C_e[k][p] = C[2k][p] (ne x ne) and
// C_o[k][p] = C[2k+1][p] (no x no).  The eigenvalue division runs on the
// blocks with the frequencies 2k / 2k+1, the inverse is U_ab = C_a^T Z_ab C_b
// and an inverse butterfly restores the nodes.  Four times fewer products
// per block, half the flops of the dense passes, and every pass a plain
// matrix product on the matrix cores (v_mfma_f32_16x16x4f32: A[i][k] at lane
// i + 16 k, B[k][j] at lane j + 16 k, accumulator register r of lane l holds
// row 4 (l / 16) + r, column l % 16).
//
// LDS layout of the folded planes: rows and columns in the folded index
// (even block [0, ne), odd block [ne, N)), stride fs, zero beyond N.  C_e and
// C_o are stored zero padded to 16-row multiples, so that the contraction
// runs in steps of 4 with no bounds tests: the padded terms multiply a zero
// coefficient by a finite plane entry.
// ---------------------------------------------------------------------------
typedef float w1_f32x4 __attribute__((ext_vector_type(4)));

struct FoldLay {
  int N, h, ne, no, re, ro, fs, fr, sde, sdo;
  __host__ __device__ explicit FoldLay(int n1) : N(n1) {
    h = N / 2;
    ne = N - h;
    no = h;
    re = (ne + 15) & ~15;   // C_e rows (16-padded)
    ro = (no + 15) & ~15;   // C_o rows
    fs = (N + 16) | 1;      // folded plane stride (odd: no bank aliasing down a column)
    fr = N + 16;            // folded plane rows
    sde = re + 1;
    sdo = ro + 1;
  }
};

// node planes (dense N x N) <-> folded planes (stride fs); end with a barrier
__device__ void res_fold_in_(const float* __restrict__ X, float* __restrict__ F, const FoldLay& L) {
  const int N = L.N, ne = L.ne, fs = L.fs;
  const float rne = 1.f / (float)ne;
  for (int Q = threadIdx.x; Q < ne * ne; Q += PRES_THREADS) {
    // Q / ne by a float reciprocal: Q < ne^2 <= 33^2, so (Q + 0.5) / ne stays
    // at least 0.5 / ne from an integer, far beyond the rounding error
    const int p = (int)(((float)Q + 0.5f) * rne), q = Q - p * ne;
    const bool pr = p < L.h, qr = q < L.h;   // the mirrored row / column is a different node
    const int pm = N - 1 - p, qm = N - 1 - q;
    const float x00 = X[p * N + q];
    const float x01 = qr ? X[p * N + qm] : 0.f;
    const float x10 = pr ? X[pm * N + q] : 0.f;
    const float x11 = (pr && qr) ? X[pm * N + qm] : 0.f;
    const float se = x00 + x01, so = x00 - x01, te = x10 + x11, to = x10 - x11;
    F[p * fs + q] = se + te;
    if (qr) F[p * fs + ne + q] = so + to;
    if (pr) F[(ne + p) * fs + q] = se - te;
    if (pr && qr) F[(ne + p) * fs + ne + q] = so - to;
  }
  __syncthreads();
}
__device__ void res_fold_out_(const float* __restrict__ F, float* __restrict__ U, const FoldLay& L) {
  const int N = L.N, ne = L.ne, fs = L.fs;
  const float rne = 1.f / (float)ne;
  for (int Q = threadIdx.x; Q < ne * ne; Q += PRES_THREADS) {
    // Q / ne by a float reciprocal: Q < ne^2 <= 33^2, so (Q + 0.5) / ne stays
    // at least 0.5 / ne from an integer, far beyond the rounding error
    const int p = (int)(((float)Q + 0.5f) * rne), q = Q - p * ne;
    const bool pr = p < L.h, qr = q < L.h;
    const int pm = N - 1 - p, qm = N - 1 - q;
    const float ee = F[p * fs + q];
    const float eo = qr ? F[p * fs + ne + q] : 0.f;
    const float oe = pr ? F[(ne + p) * fs + q] : 0.f;
    const float oo = (pr && qr) ? F[(ne + p) * fs + ne + q] : 0.f;
    const float a = ee + oe, b = eo + oo, c = ee - oe, e = eo - oo;
    U[p * N + q] = a + b;
    if (qr) U[p * N + qm] = a - b;
    if (pr) U[pm * N + q] = c + e;
    if (pr && qr) U[pm * N + qm] = c - e;
  }
  __syncthreads();
}

// one pass over the four blocks, 16 x 16 output tiles, one per wavefront at
// a time; ends with a barrier.
//   PASS 1: out_ab = in_ab C_b^T    PASS 2: out_ab = C_a in_ab, scaled by h^2 / lambda
//   PASS 3: out_ab = C_a^T in_ab    PASS 4: out_ab = in_ab C_b
template <int PASS>
__device__ void res_fold_pass_(const float* __restrict__ CE, const float* __restrict__ CO,
                               const float* __restrict__ in, float* __restrict__ out,
                               const double* __restrict__ lam, const FoldLay& L) {
  constexpr int MAXS = 9;   // contraction steps of 4 for ne <= 33 (N <= 65)
  constexpr bool colk = PASS == 1 || PASS == 4;   // contraction over the column block
  // the wavefront index through a scalar register: every tile quantity below
  // is then wave-uniform and the contraction runs without lane masking
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int rte = L.re >> 4, RT = rte + (L.ro >> 4);
  for (int tile = wv; tile < RT * RT; tile += PRES_THREADS / 64) {
    const int rt = tile / RT, ct = tile - rt * RT;
    const bool ao = rt >= rte, bo = ct >= rte;            // odd row / column block
    const int ra = ao ? L.ne : 0, rb = bo ? L.ne : 0;     // block origin in the folded index
    const int na = ao ? L.no : L.ne, nb = bo ? L.no : L.ne;
    const int i0 = (ao ? rt - rte : rt) * 16, j0 = (bo ? ct - rte : ct) * 16;   // in-block tile origin
    const bool kodd = colk ? bo : ao;
    const int K = colk ? nb : na, ko = kodd ? L.ne : 0;
    const float* Cb = kodd ? CO : CE;
    const int cs = kodd ? L.sdo : L.sde;
    // this lane's A row and B column: element k at p[k * stride]
    const float* pa;
    const float* pb;
    int sa, sb;
    if (colk) {
      pa = in + (ra + i0 + li) * L.fs + ko;
      sa = 1;
    } else if (PASS == 2) {
      pa = Cb + (i0 + li) * cs;
      sa = 1;
    } else {
      pa = Cb + i0 + li;
      sa = cs;
    }
    if (PASS == 1) {
      pb = Cb + (j0 + li) * cs;
      sb = 1;
    } else if (PASS == 4) {
      pb = Cb + j0 + li;
      sb = cs;
    } else {
      pb = in + ko * L.fs + rb + j0 + li;
      sb = L.fs;
    }
    const int ks = (K + 3) >> 2;
    // all operand reads first, then the matrix-core chain
    float av[MAXS], bv[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      av[s] = 0.f;
      bv[s] = 0.f;
      if (s < ks) {
        av[s] = pa[(4 * s + lk) * sa];
        bv[s] = pb[(4 * s + lk) * sb];
      }
    }
    w1_f32x4 acc = {};
#pragma unroll
    for (int s = 0; s < MAXS; ++s)
      if (s < ks) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int il = i0 + 4 * lk + r, jl = j0 + li;
      if (il < na && jl < nb) {
        float v = acc[r];
        if (PASS == 2) v = (float)((double)v * lam[(ra + il) * L.N + rb + jl]);
        out[(ra + il) * L.fs + rb + jl] = v;
      }
    }
  }
  __syncthreads();
}

// u = (A A*)^{-1} r: r in X on entry, u in X on exit; F0, F1 folded scratch;
// lam[k''][l''] = h^2 / (s_k + s_l) of the frequencies of the folded indices
// (0 at the constant mode), FP64
__device__ void res_poisson_(const float* CE, const float* CO, float* X, float* F0, float* F1,
                             const double* lam, const FoldLay& L) {
  res_fold_in_(X, F0, L);
  res_fold_pass_<1>(CE, CO, F0, F1, lam, L);
  res_fold_pass_<2>(CE, CO, F1, F0, lam, L);
  res_fold_pass_<3>(CE, CO, F0, F1, lam, L);
  res_fold_pass_<4>(CE, CO, F1, F0, lam, L);
  res_fold_out_(F0, X, L);
}

int prox_resident_lds_bytes(int side, int elem) {
  const FoldLay L(side);
  return 18 * NQ * 8 + side * side * 8 + (3 * side * side + 2 * L.fr * L.fs + L.re * L.sde + L.ro * L.sdo) * elem;
}

template <typename T, int NPT, int METRIC>
__global__ __launch_bounds__(PRES_THREADS) void k_prox_resident(const int* __restrict__ idx,
                                                               const SlotDesc<T>* __restrict__ desc,
                                                               SlotScalars* __restrict__ scal, int check_every,
                                                               int chunk) {
  extern __shared__ double smem_d[];
  constexpr int NT = PRES_THREADS;
  constexpr int metric = METRIC;
  const int x = idx[blockIdx.x];
  const SlotDesc<T>& d = desc[x];
  if (d.metric != METRIC) return;
  SlotScalars& sc = scal[x / MAXL];
  const int n = d.n, N = n + 1, NN = N * N, pitch = d.pitch;
  double* red = smem_d;                 // [16 * NQ]
  double* res = smem_d + 16 * NQ;       // [NQ]
  int* flag = (int*)(smem_d + 17 * NQ);
  static_assert(sizeof(T) == 4, "the resident Algorithm 2 kernel is FP32");
  const FoldLay L(N);
  double* lam = smem_d + 18 * NQ;       // [N x N] h^2 / lambda in the folded order
  T* P0 = (T*)(lam + NN);               // node planes, dense N x N
  T* P1 = P0 + NN;
  T* P2 = P1 + NN;
  T* F0 = P2 + NN;                      // folded planes, fr x fs
  T* F1 = F0 + L.fr * L.fs;
  T* CE = F1 + L.fr * L.fs;             // C_e, re x sde
  T* CO = CE + L.re * L.sde;            // C_o, ro x sdo
  const T ih = d.ih, mu = d.mu, tau = d.tau;
  const int cap = d.cap;
  const double h2 = d.h * d.h;
  for (int e = threadIdx.x; e < L.re * L.sde; e += NT) {
    const int k = e / L.sde, p = e - k * L.sde;
    CE[e] = (k < L.ne && p < L.ne) ? d.dctC[(2 * k) * N + p] : T(0);
  }
  for (int e = threadIdx.x; e < L.ro * L.sdo; e += NT) {
    const int k = e / L.sdo, p = e - k * L.sdo;
    CO[e] = (k < L.no && p < L.no) ? d.dctC[(2 * k + 1) * N + p] : T(0);
  }
  for (int e = threadIdx.x; e < 2 * L.fr * L.fs; e += NT) F0[e] = T(0);
  for (int e = threadIdx.x; e < NN; e += NT) {
    const int k = e / N, l = e - k * N;
    const int tk = k < L.ne ? 2 * k : 2 * (k - L.ne) + 1, tl = l < L.ne ? 2 * l : 2 * (l - L.ne) + 1;
    lam[e] = (tk == 0 && tl == 0) ? 0.0 : h2 / (d.dcts[tk] + d.dcts[tl]);
  }

  T m1[NPT], m2[NPT], w1[NPT], w2[NPT], b1[NPT], b2[NPT], rh[NPT];
  unsigned has_d = 0u, has_r = 0u, not_top = 0u, not_left = 0u;   // bit s: neighbour exists
#pragma unroll
  for (int s = 0; s < NPT; ++s) {
    const int e = threadIdx.x + NT * s;
    m1[s] = m2[s] = w1[s] = w2[s] = b1[s] = b2[s] = rh[s] = T(0);
    if (e < NN) {
      const int r = e / N, c = e - r * N;
      if (r < n) has_d |= 1u << s;
      if (c < n) has_r |= 1u << s;
      if (r > 0) not_top |= 1u << s;
      if (c > 0) not_left |= 1u << s;
      const size_t off = (size_t)r * pitch + c;
      m1[s] = d.p[0][off];
      m2[s] = d.p[1][off];
      w1[s] = d.p[2][off];
      w2[s] = d.p[3][off];
      b1[s] = d.p[4][off];
      b2[s] = d.p[5][off];
      rh[s] = d.rho[off];
    }
  }
  __syncthreads();

  int k = sc.iters;
  const int kend = chunk > 0 ? k + chunk : cap;
  int status = ST_RUN;
  double measure = sc.measure;
  int rises = sc.rises;
  bool tested = k > 0;   // a stop test of this level has run
  const bool fpr = d.rule == RULE_FPR;
  while (k < kend) {
    ++k;
    const bool chk = (k % check_every == 0) || (k >= cap);
    // v = m - mu vphibar (zero where the edge leaves the grid)
    T v1[NPT], v2[NPT];
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
      const int e = threadIdx.x + NT * s;
      v1[s] = ((has_d >> s) & 1u) ? fma_(-mu, b1[s], m1[s]) : T(0);
      v2[s] = ((has_r >> s) & 1u) ? fma_(-mu, b2[s], m2[s]) : T(0);
      if (e < NN) {
        P0[e] = v1[s];
        P1[e] = v2[s];
      }
    }
    __syncthreads();
    // r = A v - rho
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
      const int e = threadIdx.x + NT * s;
      if (e < NN) {
        const T v1u = ((not_top >> s) & 1u) ? P0[e - N] : T(0);
        const T v2l = ((not_left >> s) & 1u) ? P1[e - 1] : T(0);
        P2[e] = ((v1[s] - v1u) + (v2[s] - v2l)) * ih - rh[s];
      }
    }
    __syncthreads();
    res_poisson_(CE, CO, P2, F0, F1, lam, L);
    // m+ = v + grad+ u; vphi+ = Proj(vphi + tau m+); vphibar+ = 2 vphi+ - vphi
    double v[NQ] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
      const int e = threadIdx.x + NT * s;
      if (e < NN) {
        const T uc = P2[e];
        const T g1 = ((has_d >> s) & 1u) ? (P2[e + N] - uc) * ih : T(0);
        const T g2 = ((has_r >> s) & 1u) ? (P2[e + 1] - uc) * ih : T(0);
        const T n1 = v1[s] + g1, n2 = v2[s] + g2;
        T q1, q2;
        proj_ball_(fma_(tau, n1, w1[s]), fma_(tau, n2, w2[s]), metric, q1, q2);
        if (!((has_d >> s) & 1u)) q1 = T(0);
        if (!((has_r >> s) & 1u)) q2 = T(0);
        if (chk && fpr) {
          const double e1 = (double)(n1 - m1[s]), e2 = (double)(n2 - m2[s]);
          const double f1 = (double)(q1 - w1[s]), f2 = (double)(q2 - w2[s]);
          v[0] += e1 * e1 + e2 * e2;
          v[1] += f1 * f1 + f2 * f2;
          v[2] += f1 * e1 + f2 * e2;
          if (!(finite_(n1) && finite_(n2) && finite_(q1) && finite_(q2))) v[3] += 1.0;
        }
        m1[s] = n1;
        m2[s] = n2;
        b1[s] = fma_(T(2), q1, -w1[s]);
        b2[s] = fma_(T(2), q2, -w2[s]);
        w1[s] = q1;
        w2[s] = q2;
      }
    }
    if (!chk) continue;

    // ---- stop test ----
    if (!fpr) {
      __syncthreads();
      // psi = (A A*)^{-1} A vphi, then the KKT partials of (m, psi)
#pragma unroll
      for (int s = 0; s < NPT; ++s) {
        const int e = threadIdx.x + NT * s;
        if (e < NN) {
          P0[e] = w1[s];
          P1[e] = w2[s];
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < NPT; ++s) {
        const int e = threadIdx.x + NT * s;
        if (e < NN) {
          const T a1 = w1[s] - (((not_top >> s) & 1u) ? P0[e - N] : T(0));
          const T a2 = w2[s] - (((not_left >> s) & 1u) ? P1[e - 1] : T(0));
          P2[e] = (a1 + a2) * ih;
        }
      }
      __syncthreads();
      res_poisson_(CE, CO, P2, F0, F1, lam, L);
#pragma unroll
      for (int s = 0; s < NPT; ++s) {
        const int e = threadIdx.x + NT * s;
        if (e < NN) {
          P0[e] = m1[s];
          P1[e] = m2[s];
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < NPT; ++s) {
        const int e = threadIdx.x + NT * s;
        if (e < NN) {
          const double rr = (double)rh[s];
          const T pc = P2[e];
          const T g1 = ((has_d >> s) & 1u) ? (P2[e + N] - pc) * ih : T(0);
          const T g2 = ((has_r >> s) & 1u) ? (P2[e + 1] - pc) * ih : T(0);
          const double gq = (double)norm_q_(g1, g2, metric);
          const double ex = gq > 1.0 ? gq - 1.0 : 0.0;
          v[2] += ex * ex;
          v[3] += (double)norm_p_(m1[s], m2[s], metric);
          v[4] += (double)pc * rr;
          v[6] += (double)pc;
          v[7] += rr;
        }
      }
      // primal part: the correction potential c = (A A*)^{-1}(A m - rho)
      // (psi in P2 is no longer read after this barrier), then
      // sum |grad+ c|^2
      __syncthreads();
#pragma unroll
      for (int s = 0; s < NPT; ++s) {
        const int e = threadIdx.x + NT * s;
        if (e < NN) {
          const T a1 = m1[s] - (((not_top >> s) & 1u) ? P0[e - N] : T(0));
          const T a2 = m2[s] - (((not_left >> s) & 1u) ? P1[e - 1] : T(0));
          P2[e] = (a1 + a2) * ih - rh[s];
        }
      }
      __syncthreads();
      res_poisson_(CE, CO, P2, F0, F1, lam, L);
      const double ihd = 1.0 / d.h;
#pragma unroll
      for (int s = 0; s < NPT; ++s) {
        const int e = threadIdx.x + NT * s;
        if (e < NN) {
          const double cc = (double)P2[e];
          const double c1 = ((has_d >> s) & 1u) ? ((double)P2[e + N] - cc) * ihd : 0.0;
          const double c2 = ((has_r >> s) & 1u) ? ((double)P2[e + 1] - cc) * ihd : 0.0;
          v[0] += c1 * c1 + c2 * c2;
        }
      }
    }
    // (every LDS plane read above is behind the reduction's barrier)
    if (fpr) block_reduce_<NT, 4>(v, res, red, 0u);
    else block_reduce_<NT>(v, res, red, 0u);
    __syncthreads();
    if (threadIdx.x == 0) {
      const double m = measure_from_(res, K_PROX, d.rule, h2, d.mud, d.taud, NN);
      rises = tested && m > measure ? rises + 1 : 0;
      int st = ST_RUN;
      if (!isfinite(m) || (d.divwin > 0 && m < 0.0)) st = ST_DIVERGED;
      else if (m <= d.tol) st = ST_CONV;
      else if (d.divwin > 0 && rises >= d.divwin) st = ST_DIVERGED;
      else if (k >= cap) st = ST_CAP;
      flag[0] = st;
      res[0] = m;
    }
    tested = true;
    __syncthreads();
    status = flag[0];
    measure = res[0];
    // res and flag are next written after at least six more barriers
    if (status != ST_RUN) break;
  }

#pragma unroll
  for (int s = 0; s < NPT; ++s) {
    const int e = threadIdx.x + NT * s;
    if (e < NN) {
      const int r = e / N, c = e - r * N;
      const size_t off = (size_t)r * pitch + c;
      d.p[0][off] = m1[s];
      d.p[1][off] = m2[s];
      d.p[2][off] = w1[s];
      d.p[3][off] = w2[s];
      d.p[4][off] = b1[s];
      d.p[5][off] = b2[s];
    }
  }
  if (threadIdx.x == 0) {
    sc.iters = k;
    sc.status = status;
    sc.measure = measure;
    sc.rises = rises;
  }
}

// ---------------------------------------------------------------------------
// KKT partials of an Algorithm 1 iterate (current set) or of an Algorithm 2
// iterate with its potential psi in plane 8, given the minimum-norm
// correction potential c = (A A*)^{-1}(A m - rho) in plane 6:
// q0 sum |grad+ c|^2 (the squared norm of the flux correction A* c, over
// h^2), q2 sum excess^2, q3 sum ||m||_p, q4 sum pot*rho, q6 sum pot,
// q7 sum rho.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_kkt(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                             const SlotScalars* __restrict__ scal, int kind, int set_xor, int gate) {
  __shared__ double lds[4 * NQ];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotScalars& sc = scal[w.x / MAXL];
  if (gate && sc.status != ST_RUN) return;
  const SlotDesc<T>& d = desc[w.x];
  const int n = d.n, pitch = d.pitch;
  const T* m1;
  const T* m2;
  const T* pot;
  if (kind == K_PLAIN) {
    const int cs = (sc.cur ^ set_xor) & 1;
    m1 = d.p[3 * cs];
    m2 = d.p[3 * cs + 1];
    pot = d.p[3 * cs + 2];
  } else {
    m1 = d.p[0];
    m2 = d.p[1];
    pot = d.p[8];
  }
  const T ih = d.ih;
  const T* corr = d.p[6];
  const double ihd = 1.0 / d.h;
  double v[NQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  SIMPLE_TILE_LOOP(d, w, {
    const double rr = (double)d.rho[off];
    const double cc = (double)corr[off];
    const double c1 = i < n ? ((double)corr[off + pitch] - cc) * ihd : 0.0;
    const double c2 = j < n ? ((double)corr[off + 1] - cc) * ihd : 0.0;
    const T pc = pot[off];
    const T g1 = i < n ? (pot[off + pitch] - pc) * ih : T(0);
    const T g2 = j < n ? (pot[off + 1] - pc) * ih : T(0);
    const double gq = (double)norm_q_(g1, g2, d.metric);
    const double ex = gq > 1.0 ? gq - 1.0 : 0.0;
    v[0] += c1 * c1 + c2 * c2;
    v[2] += ex * ex;
    v[3] += (double)norm_p_(m1[off], m2[off], d.metric);
    v[4] += (double)pc * rr;
    v[6] += (double)pc;
    v[7] += rr;
  })
  block_reduce_<256>(v, d.part + (size_t)w.w * NQ, lds, 0u);
}

// ---------------------------------------------------------------------------
// node-field inputs of a Poisson solve, written to plane 6:
//   mode 0: A(m - mu vphibar) - rho   (projection step of eq. (pdhg))
//   mode 1: A vphi                    (Appendix B potential)
//   mode 2: A m - rho                 (certificate and KKT correction), m
//           from the plain set cur ^ set_xor (kind plain) or planes 0, 1
//           (prox)
//   mode 3: A (m + grad+ c) - rho     (prox: the re-projected flux, c in
//           POLISH_PLANE)
// Modes 2 and 3 form the residual in FP64 against the slot's FP64 densities.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_div_pre(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                                 const SlotScalars* __restrict__ scal, int mode, int kind,
                                                 int gate, int set_xor) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotScalars& sc = scal[w.x / MAXL];
  if (gate && sc.status != ST_RUN) return;
  const SlotDesc<T>& d = desc[w.x];
  const int n = d.n, pitch = d.pitch;
  const T ih = d.ih, mu = d.mu;
  const T *a1p, *a2p;
  if (mode == 1) {
    a1p = d.p[2];
    a2p = d.p[3];
  } else if (kind == K_PLAIN) {
    const int cs = (sc.cur ^ set_xor) & 1;
    a1p = d.p[3 * cs];
    a2p = d.p[3 * cs + 1];
  } else {
    a1p = d.p[0];
    a2p = d.p[1];
  }
  T* out = d.p[6];
  SIMPLE_TILE_LOOP(d, w, {
    T v1c, v1u, v2c, v2l;
    if (mode == 0) {
      v1c = i < n ? fma_(-mu, d.p[4][off], a1p[off]) : T(0);
      v1u = i > 0 ? fma_(-mu, d.p[4][off - pitch], a1p[off - pitch]) : T(0);
      v2c = j < n ? fma_(-mu, d.p[5][off], a2p[off]) : T(0);
      v2l = j > 0 ? fma_(-mu, d.p[5][off - 1], a2p[off - 1]) : T(0);
    } else {
      v1c = i < n ? a1p[off] : T(0);
      v1u = i > 0 ? a1p[off - pitch] : T(0);
      v2c = j < n ? a2p[off] : T(0);
      v2l = j > 0 ? a2p[off - 1] : T(0);
    }
    if (mode == 3) {
      // A (m + grad+ c) - rho of the re-projected flux (c in POLISH_PLANE),
      // in FP64 from the FP32 planes
      const T* c = d.p[POLISH_PLANE];
      const double ihd = (double)n, cc = (double)c[off];
      const double f1c = i < n ? (double)a1p[off] + ((double)c[off + pitch] - cc) * ihd : 0.0;
      const double f1u = i > 0 ? (double)a1p[off - pitch] + (cc - (double)c[off - pitch]) * ihd : 0.0;
      const double f2c = j < n ? (double)a2p[off] + ((double)c[off + 1] - cc) * ihd : 0.0;
      const double f2l = j > 0 ? (double)a2p[off - 1] + (cc - (double)c[off - 1]) * ihd : 0.0;
      const double rr = d.r0 ? d.r0[off] - d.r1[off] : (double)d.rho[off];
      out[off] = (T)(((f1c - f1u) + (f2c - f2l)) * ihd - rr);
    } else if (mode == 2) {
      // the residual of the correction in FP64 arithmetic against the FP64
      // densities where the slot keeps them (its constant part is ignored by
      // the Poisson solve): near feasibility A m - rho is far smaller than
      // A m, so an FP32 residual would be mostly its own rounding
      const double dv2 = (((double)v1c - (double)v1u) + ((double)v2c - (double)v2l)) * (double)n;
      const double rr = d.r0 ? d.r0[off] - d.r1[off] : (double)d.rho[off];
      out[off] = (T)(dv2 - rr);
    } else {
      const T dv = ((v1c - v1u) + (v2c - v2l)) * ih;
      out[off] = mode == 1 ? dv : dv - d.rho[off];
    }
  })
}

// ---------------------------------------------------------------------------
// One pass of the DCT Neumann-Poisson solve: a batched product with the
// orthonormal DCT-II matrix C of length N = n+1 (or its transpose).
//   MODE 0 (along rows):    Y = X * M   (M = C^T: forward, M = C: inverse)
//   MODE 1 (along columns): Y = M * X   (M = C: forward, M = C^T: inverse)
// With SCALE the result is divided by the eigenvalue
// lambda_kl = (4/h^2)(sin^2(pi k/2N) + sin^2(pi l/2N)) and mode (0,0) set to
// zero.  64 x 64 output tile per workgroup, 4 x 4 per thread, K in chunks of 16.
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool SCALE>
__global__ __launch_bounds__(256) void k_gemm(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                              const SlotScalars* __restrict__ scal, int src, int dst, int mat,
                                              int gate) {
  __shared__ T As[16][GEMM_T + 4];
  __shared__ T Bs[16][GEMM_T + 4];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  if (gate && scal[w.x / MAXL].status != ST_RUN) return;
  const SlotDesc<T>& d = desc[w.x];
  const int N = d.n + 1, ld = d.pitch;
  const T* M = mat ? d.dctCt : d.dctC;
  const T* X = d.p[src];
  T* Y = d.p[dst];
  const T* A = MODE == 0 ? X : M;
  const T* B = MODE == 0 ? M : X;
  const int lda = MODE == 0 ? ld : N;
  const int ldb = MODE == 0 ? N : ld;
  const int i0 = w.y * GEMM_T, j0 = w.z * GEMM_T;
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  T acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = T(0);
  for (int p0 = 0; p0 < N; p0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      const int ii = e >> 4, pp = e & 15;
      const int gi = i0 + ii, gp = p0 + pp;
      As[pp][ii] = (gi < N && gp < N) ? A[(size_t)gi * lda + gp] : T(0);
      const int pb = e >> 6, jj = e & 63;
      const int gq = p0 + pb, gj = j0 + jj;
      Bs[pb][jj] = (gq < N && gj < N) ? B[(size_t)gq * ldb + gj] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int pp = 0; pp < 16; ++pp) {
      T a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[pp][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[pp][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fma_(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
  const double h2 = d.h * d.h;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gi = i0 + ty * 4 + r, gj = j0 + tx * 4 + c;
      if (gi < N && gj < N) {
        T v = acc[r][c];
        if (SCALE) {
          const double lam = d.dcts[gi] + d.dcts[gj];
          v = (gi == 0 && gj == 0) ? T(0) : (T)((double)v * (h2 / lam));
        }
        Y[(size_t)gi * ld + gj] = v;
      }
    }
}

// v_mfma_f32_32x32x2f32 lane layout: A[i][k] at lane i + 32 k, B[k][j] at
// lane j + 32 k, and accumulator register r of lane l holds row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
// ---------------------------------------------------------------------------
// DCT passes with the even/odd fold (FP32, matrix cores).  The DCT-II basis
// satisfies C[k][N-1-j] = (-1)^k C[k][j] (and C[k][(N-1)/2] = 0 for odd k
// when N is odd), so a pass over length N splits into two products of half
// the length: the even frequencies see x_j + x_{N-1-j}, the odd ones
// x_j - x_{N-1-j} (forward); for the inverse the even and odd frequency sums
// give x_j = E + O and x_{N-1-j} = E - O.  Frequency indices are kept in a
// permuted order between the passes (ne even ones first, then no odd ones;
// ne = N - N/2, no = N/2), with Cp[k''][j] = C[perm(k'')][j] and Ctp its
// transpose.  Half the flops of the plain dense passes.
//   pass 1 (rows, forward):   Y1[i][k''] = sum_j X[i][j] C[perm k''][j]
//   pass 2 (columns, forward, divided by lambda):
//                             Y2[k''][l''] = sum_i C[perm k''][i] Y1[i][l'']
//   pass 3 (columns, inverse): Y3[i][l''] = sum_k'' C[perm k''][i] Y2[k''][l'']
//   pass 4 (rows, inverse):    U[i][j] = sum_l'' Y3[i][l''] C[perm l''][j]
// Work items: one square list per slot, T x T tiles with
// T = max(cdiv(N, 64), cdiv(ne, 64) + cdiv(no, 64)); each pass reads (y, z)
// in its own orientation and tiles outside its output return at once.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dct_perm_(int x, int ne) { return x < ne ? 2 * x : 2 * (x - ne) + 1; }

// (offsets in 32 bits: N <= 4097, so every plane and table offset fits, and
// the loads take a scalar base with an unsigned 32-bit lane offset)
template <int PASS>
__global__ __launch_bounds__(256) void k_dct_fold(const Work* __restrict__ work,
                                                  const SlotDesc<float>* __restrict__ desc,
                                                  const SlotScalars* __restrict__ scal, int src, int dst, int gate) {
  __shared__ float As[2][64][33];
  __shared__ float Bs[2][32][68];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  if (gate && scal[w.x / MAXL].status != ST_RUN) return;
  const SlotDesc<float>& d = desc[w.x];
  const int N = d.n + 1, ld = d.pitch, h = N / 2, ne = N - h, no = h;
  if (d.fft_tw) return;   // a slot with FFT tables is solved by the FFT path
  const W1_GLOBAL float* __restrict__ X = gld_(d.p[src]);
  W1_GLOBAL float* __restrict__ Y = gst_(d.p[dst]);
  const W1_GLOBAL float* __restrict__ Cp = gld_(d.dctCp);
  const W1_GLOBAL float* __restrict__ Ctp = gld_(d.dctCtp);
  const int nte = (ne + 63) / 64, nto = (no + 63) / 64;
  float out[16];
  if (PASS == 1 || PASS == 2) {
    // the tile along the parity blocks and the tile along the N side
    const int zb = PASS == 1 ? w.z : w.y, zn = PASS == 1 ? w.y : w.z;
    if (zb >= nte + nto || zn * 64 >= N) return;
    const bool odd = zb >= nte;
    const int cnt = odd ? no : ne, base = odd ? ne : 0, b0 = (odd ? zb - nte : zb) * 64, n0 = zn * 64;
    const int K = cnt;   // fold: ne terms (with the middle node when N is odd) or no terms
    if (PASS == 1) {
      // Y1[i][base + k2] = sum_j' fold_j'(X[i][.]) Ctp[j'][base + k2]
      auto la = [&](int il, int jp) -> float {
        const int i = n0 + il, ic = i < N ? i : N - 1;
        const float a = X[unsigned(ic * ld + jp)], b = X[unsigned(ic * ld + N - 1 - jp)];
        const float v = odd ? a - b : (jp < h ? a + b : a);
        return i < N ? v : 0.f;
      };
      auto lb = [&](int jp, int cl) -> float {
        const int k2 = b0 + cl, k2c = k2 < cnt ? k2 : cnt - 1;
        const float v = Ctp[unsigned(jp * N + base + k2c)];
        return k2 < cnt ? v : 0.f;
      };
      mfma_tile64_(la, lb, K, As, Bs, out);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = n0 + mfma_row_(r), k2 = b0 + mfma_col_();
        if (i < N && k2 < cnt) Y[unsigned(i * ld + base + k2)] = out[r];
      }
    } else {
      // Y2[base + k2][l] = sum_i' Cp[base + k2][i'] fold_i'(X[.][l]) / lambda
      auto la = [&](int kl, int ip) -> float {
        const int k2 = b0 + kl, k2c = k2 < cnt ? k2 : cnt - 1;
        const float v = Cp[unsigned((base + k2c) * N + ip)];
        return k2 < cnt ? v : 0.f;
      };
      auto lb = [&](int ip, int cl) -> float {
        const int l = n0 + cl, lc = l < N ? l : N - 1;
        const float a = X[unsigned(ip * ld + lc)], b = X[unsigned((N - 1 - ip) * ld + lc)];
        const float v = odd ? a - b : (ip < h ? a + b : a);
        return l < N ? v : 0.f;
      };
      mfma_tile64_(la, lb, K, As, Bs, out);
      const double h2 = d.h * d.h;
      const W1_GLOBAL double* __restrict__ dcts = gld_(d.dcts);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k2 = b0 + mfma_row_(r), l = n0 + mfma_col_();
        if (k2 < cnt && l < N) {
          const int kk = base + k2, tk = dct_perm_(kk, ne), tl = dct_perm_(l, ne);
          const float v = (tk == 0 && tl == 0) ? 0.f : (float)((double)out[r] * (h2 / (dcts[tk] + dcts[tl])));
          Y[unsigned(kk * ld + l)] = v;
        }
      }
    }
  } else {
    // inverse: the ne leading rows (pass 3) or columns (pass 4) from the even
    // and odd frequency sums, mirrored to N-1-i / N-1-j
    const int zh = PASS == 3 ? w.y : w.z, zn = PASS == 3 ? w.z : w.y;
    const int h0 = zh * 64, n0 = zn * 64;
    if (h0 >= ne || n0 >= N) return;
    float ev[16];
    for (int par = 0; par < 2; ++par) {
      const int K = par ? no : ne, base = par ? ne : 0;
      if (PASS == 3) {
        // rows i < ne: sum_k'' Ctp[i][base + k''] X[base + k''][l]
        auto la = [&](int il, int kk) -> float {
          const int i = h0 + il, ic = i < ne ? i : ne - 1;
          const float v = Ctp[unsigned(ic * N + base + kk)];
          return i < ne ? v : 0.f;
        };
        auto lb = [&](int kk, int cl) -> float {
          const int l = n0 + cl, lc = l < N ? l : N - 1;
          const float v = X[unsigned((base + kk) * ld + lc)];
          return l < N ? v : 0.f;
        };
        mfma_tile64_(la, lb, K, As, Bs, par ? out : ev);
      } else {
        // columns j < ne: sum_l'' X[i][base + l''] Cp[base + l''][j]
        auto la = [&](int il, int kk) -> float {
          const int i = n0 + il, ic = i < N ? i : N - 1;
          const float v = X[unsigned(ic * ld + base + kk)];
          return i < N ? v : 0.f;
        };
        auto lb = [&](int kk, int cl) -> float {
          const int j = h0 + cl, jc = j < ne ? j : ne - 1;
          const float v = Cp[unsigned((base + kk) * N + jc)];
          return j < ne ? v : 0.f;
        };
        mfma_tile64_(la, lb, K, As, Bs, par ? out : ev);
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int a = (PASS == 3 ? h0 : n0) + mfma_row_(r), b = (PASS == 3 ? n0 : h0) + mfma_col_();
      const int i = a, j = b;   // pass 3: i < ne mirrored; pass 4: j < ne mirrored
      const float e = ev[r], o = out[r];
      if (PASS == 3) {
        if (i < ne && j < N) {
          Y[unsigned(i * ld + j)] = e + o;
          if (N - 1 - i != i) Y[unsigned((N - 1 - i) * ld + j)] = e - o;
        }
      } else {
        if (i < N && j < ne) {
          Y[unsigned(i * ld + j)] = e + o;
          if (N - 1 - j != j) Y[unsigned(i * ld + (N - 1 - j))] = e - o;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Algorithm 2 update after the Poisson solve (u in plane 6), in place:
// m+ = v + grad+ u, vphi+ = Proj(vphi + tau m+), vphibar+ = 2 vphi+ - vphi.
// With CHECK: partials of G^k (eq. (pdhg_stop)): sum |dm|^2, sum |dvphi|^2,
// sum dvphi . dm, count of non-finite values.
// ---------------------------------------------------------------------------
template <typename T, bool CHECK>
__global__ __launch_bounds__(256) void k_prox_post(const Work* __restrict__ work,
                                                   const SlotDesc<T>* __restrict__ desc,
                                                   const SlotScalars* __restrict__ scal) {
  __shared__ double lds[4 * NQ];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  if (scal[w.x / MAXL].status != ST_RUN) return;
  const SlotDesc<T>& d = desc[w.x];
  const int n = d.n, pitch = d.pitch;
  const T ih = d.ih, mu = d.mu, tau = d.tau;
  const T* u = d.p[6];
  double v[NQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  SIMPLE_TILE_LOOP(d, w, {
    const T uc = u[off];
    const T g1 = i < n ? (u[off + pitch] - uc) * ih : T(0);
    const T g2 = j < n ? (u[off + 1] - uc) * ih : T(0);
    const T m1 = d.p[0][off], m2 = d.p[1][off];
    const T w1 = d.p[2][off], w2 = d.p[3][off];
    const T v1 = i < n ? fma_(-mu, d.p[4][off], m1) : T(0);
    const T v2 = j < n ? fma_(-mu, d.p[5][off], m2) : T(0);
    const T n1 = v1 + g1, n2 = v2 + g2;
    T q1, q2;
    proj_ball_(fma_(tau, n1, w1), fma_(tau, n2, w2), d.metric, q1, q2);
    if (i >= n) q1 = T(0);
    if (j >= n) q2 = T(0);
    d.p[0][off] = n1;
    d.p[1][off] = n2;
    d.p[2][off] = q1;
    d.p[3][off] = q2;
    d.p[4][off] = fma_(T(2), q1, -w1);
    d.p[5][off] = fma_(T(2), q2, -w2);
    if (CHECK) {
      const double e1 = (double)(n1 - m1), e2 = (double)(n2 - m2);
      const double f1 = (double)(q1 - w1), f2 = (double)(q2 - w2);
      v[0] += e1 * e1 + e2 * e2;
      v[1] += f1 * f1 + f2 * f2;
      v[2] += f1 * e1 + f2 * e2;
      if (!(finite_(n1) && finite_(n2) && finite_(q1) && finite_(q2))) v[3] += 1.0;
    }
  })
  if (CHECK) block_reduce_<256>(v, d.part + (size_t)w.w * NQ, lds, 0u);
}

// ---------------------------------------------------------------------------
// stop test after a block: reduce the slot's partials, form R^k / G^k or the
// normalised KKT residual, compare with tol_l and the cap.
// ---------------------------------------------------------------------------

template <typename T>
// blocks = 2: two one-launch blocks ran back to back (the second reading
// the first's output set) with their partials at tiles [0, nt) and
// [nt, 2 nt); the first block's test runs first, and the second's only if
// the slot still runs after it, so the decisions and the iterate a slot
// stops on are those of one test per block.
__global__ __launch_bounds__(64) void k_check(const int* __restrict__ idx, const int* __restrict__ ntiles,
                                              const SlotDesc<T>* __restrict__ desc, SlotScalars* __restrict__ scal,
                                              int kind, int block_len, int launches, int blocks) {
  // one wavefront per slot: each lane sums every 64th tile (compensated),
  // a butterfly leaves the totals in every lane, every lane forms the same
  // decision and lane 0 stores it; the slot's state stays in registers
  // between the blocks
  const int x = idx[blockIdx.x];
  const int nt = ntiles[blockIdx.x];
  const int lane = threadIdx.x;
  SlotScalars& sc = scal[x / MAXL];
  const SlotDesc<T>& d = desc[x];
  // the slot's state and its level's constants in one round of loads
  // (before the status test, so that no load waits for another)
  const int status0 = sc.status;
  int iters = sc.iters, rises = sc.rises, cur = sc.cur;
  double measure = sc.measure;
  const double* const part0 = d.part;
  const int N = d.n + 1, rule = d.rule, divwin = d.divwin, cap = d.cap;
  const double h2 = d.h * d.h, mud = d.mud, taud = d.taud, tol = d.tol;
  if (status0 != ST_RUN) return;
  for (int b = 0; b < blocks; ++b) {
    const double* part = part0 + (size_t)b * nt * NQ;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      Acc a{0.0, 0.0};
      for (int t = lane; t < nt; t += 64) a.add(part[(size_t)t * NQ + q]);
      v[q] = a.get();
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    const double m = measure_from_(v, kind, rule, h2, mud, taud, N * N);
    const int k = iters + block_len;
    rises = iters > 0 && m > measure ? rises + 1 : 0;
    int st = ST_RUN;
    if (!isfinite(m) || (divwin > 0 && m < 0.0)) st = ST_DIVERGED;
    else if (m <= tol) st = ST_CONV;
    else if (divwin > 0 && rises >= divwin) st = ST_DIVERGED;
    else if (k >= cap) st = ST_CAP;
    iters = k;
    measure = m;
    cur ^= launches & 1;
    if (lane == 0) {
      sc.iters = iters;
      sc.measure = measure;
      sc.rises = rises;
      sc.status = st;
      sc.cur = cur;
    }
    if (st != ST_RUN) return;
  }
}

// ---------------------------------------------------------------------------
// FP64 certificate (finest level): needs the Poisson correction
// corr = (A A*)^{-1}(A m - rho) in plane 6 (read only with cert) and, for
// prox, psi in plane 8.  With `polish` (prox) the flux m is first replaced
// by its FP64 re-projection m + grad+ c onto {A m = rho} (c in
// POLISH_PLANE, plane 6 then holds the re-projected flux's own
// correction): an Algorithm 2 iterate is feasible by construction, and in
// FP32 the rounding of its Poisson solve leaves A m - rho at the level of
// the noise's gradient, which this removes.
// q0 sum ||m||_p, q1 sum pot*rho, q2 sum ||m + grad+ corr||_p,
// q3 sum |grad+ corr|^2, q4 sum excess^2, q5 max ||grad pot||_q (max),
// q6 sum pot, q7 sum rho.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_eval_sums(const Work* __restrict__ work, const SlotDesc<T>* __restrict__ desc,
                                                   const SlotScalars* __restrict__ scal, int kind, int cert,
                                                   int polish) {
  __shared__ double lds[4 * NQ];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  const int n = d.n, pitch = d.pitch;
  const T *m1, *m2, *pot;
  if (kind == K_PLAIN) {
    const int cs = scal[w.x / MAXL].cur & 1;
    m1 = d.p[3 * cs];
    m2 = d.p[3 * cs + 1];
    pot = d.p[3 * cs + 2];
  } else {
    m1 = d.p[0];
    m2 = d.p[1];
    pot = d.p[8];
  }
  const T* corr = d.p[6];
  const T* pol = polish ? d.p[POLISH_PLANE] : nullptr;
  const double ih = 1.0 / d.h;
  double v[NQ] = {0, 0, 0, 0, 0, -INFINITY, 0, 0};
  SIMPLE_TILE_LOOP(d, w, {
    double a = (double)m1[off], b = (double)m2[off];
    if (pol) {
      const double pc0 = (double)pol[off];
      if (i < n) a += ((double)pol[off + pitch] - pc0) * ih;
      if (j < n) b += ((double)pol[off + 1] - pc0) * ih;
    }
    const double cc = cert ? (double)corr[off] : 0.0;
    const double c1 = cert && i < n ? ((double)corr[off + pitch] - cc) * ih : 0.0;
    const double c2 = cert && j < n ? ((double)corr[off + 1] - cc) * ih : 0.0;
    const double pc = (double)pot[off];
    const double g1 = i < n ? ((double)pot[off + pitch] - pc) * ih : 0.0;
    const double g2 = j < n ? ((double)pot[off + 1] - pc) * ih : 0.0;
    const double rr = (double)d.rho[off];
    const double gq = norm_q_(g1, g2, d.metric);
    const double ex = gq > 1.0 ? gq - 1.0 : 0.0;
    v[0] += norm_p_(a, b, d.metric);
    v[1] += pc * rr;
    const double f1 = a + c1, f2 = b + c2;
    v[2] += norm_p_(f1, f2, d.metric);
    v[3] += c1 * c1 + c2 * c2;
    v[4] += ex * ex;
    v[5] = gq > v[5] ? gq : v[5];
    v[6] += pc;
    v[7] += rr;
  })
  block_reduce_<256>(v, d.part + (size_t)w.w * NQ, lds, 1u << 5);
}

template <typename T>
__global__ __launch_bounds__(256) void k_eval_final(const int* __restrict__ idx, const int* __restrict__ ntiles,
                                                    const SlotDesc<T>* __restrict__ desc,
                                                    SlotScalars* __restrict__ scal, int kind, int cert) {
  __shared__ double lds[4 * NQ];
  __shared__ double res[NQ];
  const int x = idx[blockIdx.x];
  const int nt = ntiles[blockIdx.x];
  const SlotDesc<T>& d = desc[x];
  double v[NQ];
  for (int q = 0; q < NQ; ++q) {
    Acc a{0.0, 0.0};
    double mx = -INFINITY;
    for (int t = threadIdx.x; t < nt; t += 256) {
      const double p = d.part[(size_t)t * NQ + q];
      a.add(p);
      mx = p > mx ? p : mx;
    }
    v[q] = q == 5 ? mx : a.get();
  }
  block_reduce_<256>(v, res, lds, 1u << 5);
  __syncthreads();
  if (threadIdx.x == 0) {
    SlotScalars& sc = scal[x / MAXL];
    const double h2 = d.h * d.h;
    const int N = d.n + 1;
    const double mean = res[6] / ((double)N * (double)N);
    const double P = res[0] * h2;
    const double sgn = kind == K_PLAIN ? -1.0 : 1.0;
    const double D = sgn * (res[1] - mean * res[7]) * h2;
    const double hi = res[2] * h2;
    const double gmax = res[5];
    const double lo = D / (gmax > 1.0 ? gmax : 1.0);
    const double rp = sqrt(res[3] * h2) / fmax(P, 1e-300);
    const double rd = sqrt(res[4] * h2);
    const double gap = fabs(P - D) / fmax(fmax(fabs(P), fabs(D)), 1e-300);
    sc.eval[0] = P;
    sc.eval[1] = D;
    sc.eval[2] = cert ? lo : NAN;
    sc.eval[3] = cert ? hi : NAN;
    sc.eval[4] = cert ? fmax(rp, fmax(rd, gap)) : NAN;
    sc.eval[5] = gmax;
    sc.eval[6] = rp;
    sc.eval[7] = rd;
    sc.mean = mean;
  }
}

// finest-level fields to dense FP64 buffers (pitch n+1); the plain
// potential is reported as psi = -(phi - mean), the prox one is plane 8
template <typename T>
__global__ __launch_bounds__(256) void k_export_fields(const Work* __restrict__ work,
                                                       const SlotDesc<T>* __restrict__ desc,
                                                       const SlotScalars* __restrict__ scal, int kind, int polish) {
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  const SlotDesc<T>& d = desc[w.x];
  const double mean = scal[w.x / MAXL].mean;
  double* __restrict__ om1 = d.out_m1;
  double* __restrict__ om2 = d.out_m2;
  double* __restrict__ opsi = d.out_psi;
  const T *m1, *m2, *pot;
  if (kind == K_PLAIN) {
    const int cs = scal[w.x / MAXL].cur & 1;
    m1 = d.p[3 * cs];
    m2 = d.p[3 * cs + 1];
    pot = d.p[3 * cs + 2];
  } else {
    m1 = d.p[0];
    m2 = d.p[1];
    pot = d.p[8];
  }
  const T* pol = polish ? d.p[POLISH_PLANE] : nullptr;
  const int n = d.n, pitch = d.pitch;
  const double ih = 1.0 / d.h;
  SIMPLE_TILE_LOOP(d, w, {
    const size_t o = (size_t)i * (d.n + 1) + j;
    double a = (double)m1[off], b = (double)m2[off];
    if (pol) {
      const double pc0 = (double)pol[off];
      if (i < n) a += ((double)pol[off + pitch] - pc0) * ih;
      if (j < n) b += ((double)pol[off + 1] - pc0) * ih;
    }
    if (om1) om1[o] = a;
    if (om2) om2[o] = b;
    if (opsi) opsi[o] = kind == K_PLAIN ? -((double)pot[off] - mean) : (double)pot[off];
  })
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define LAUNCH(kern, grid, block, lds, s, ...) hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, __VA_ARGS__)
// the same, with events that take the dispatch's own start and end times
// (without events, an ordinary launch: it can be captured into a graph)
#define LAUNCH_EV(kern, grid, block, lds, s, e0, e1, ...)                                  \
  do {                                                                                     \
    if ((e0) || (e1))                                                                      \
      hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, e0, e1, 0, __VA_ARGS__); \
    else                                                                                   \
      hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, __VA_ARGS__);              \
  } while (0)

template <typename T> void K<T>::zero(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, unsigned mask) {
  if (nw) LAUNCH(k_zero<T>, nw, 256, 0, s, w, d, mask);
}
template <typename T> void K<T>::import_dense(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, int plane, const T* src) {
  if (nw) LAUNCH(k_import<T>, nw, 256, 0, s, w, d, plane, src);
}
template <typename T> void K<T>::export_dense(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, int plane, T* dst) {
  if (nw) LAUNCH(k_export<T>, nw, 256, 0, s, w, d, plane, dst);
}
template <typename T> void K<T>::reduce(hipStream_t s, const int* idx, const int* nt, int ns, const SlotDesc<T>* d,
                                        SlotScalars* sc, int nq, int out_base, unsigned maxmask) {
  if (ns) LAUNCH(k_reduce<T>, ns, 256, 0, s, idx, nt, d, sc, nq, out_base, maxmask);
}
template <typename T> void K<T>::prep_stats(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d) {
  if (nw) LAUNCH(k_prep_stats<T>, nw, 256, 0, s, w, d);
}
template <typename T> void K<T>::prep_scale(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc) {
  if (nw) LAUNCH(k_prep_scale<T>, nw, 256, 0, s, w, d, sc);
}
template <typename T> void K<T>::reset_scalars(hipStream_t s, const Work* w, int nw, SlotScalars* sc) {
  if (nw) LAUNCH(k_reset_scalars, nw, 64, 0, s, w, sc);
}
template <typename T> void K<T>::restrict_level(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d) {
  if (nw) LAUNCH(k_restrict<T>, nw, 256, 0, s, w, d);
}
template <typename T> void K<T>::scale_level(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc) {
  if (nw) LAUNCH(k_scale_level<T>, nw, 256, 0, s, w, d, sc);
}
template <typename T> void K<T>::rho_diff(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d) {
  if (nw) LAUNCH(k_rho_diff<T>, nw, 256, 0, s, w, d);
}
template <typename T> void K<T>::rho_write(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc) {
  if (nw) LAUNCH(k_rho_write<T>, nw, 256, 0, s, w, d, sc);
}
template <typename T> void K<T>::prolong(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                         const SlotScalars* sc, int kind) {
  if (nw) LAUNCH(k_prolong<T>, nw, 256, 0, s, w, d, sc, kind);
}
template <typename T> void K<T>::plain_tiled(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                             const SlotScalars* sc, int li, int steps, int rh, int rw, bool check,
                                             int metric, int nwv, int second, hipEvent_t ev0, hipEvent_t ev1) {
  if (!nw) return;
  const bool shape = (rh == TILED_RH && (rw == 64 || rw == 128) && (nwv == 8 || nwv == 16)) ||
                     (rh == TILED_RH_SHORT && rw == 64 && nwv == 8);
  if (!shape || steps < 1 || steps > TILED_MAX_STEPS || 2 * steps >= rw || 2 * steps >= rh ||
      (metric < 1 || metric > 3)) {
    fprintf(stderr, "w1: internal error: %d steps in a %d x %d region, metric %d, %d waves\n", steps, rh, rw,
            metric, nwv);
    return;
  }
#define W1_TILED_LAUNCH(C, M, NWV, RWD, RHD) \
  LAUNCH_EV((k_plain_tiled<T, C, M, NWV, RWD, RHD>), nw, NWV * 64, 0, s, ev0, ev1, w, d, sc, li, steps, second)
#define W1_TILED_METRIC(NWV, RWD, RHD)                   \
  switch (metric) {                                      \
    case 1:                                              \
      if (check) W1_TILED_LAUNCH(true, 1, NWV, RWD, RHD); \
      else W1_TILED_LAUNCH(false, 1, NWV, RWD, RHD);      \
      break;                                             \
    case 2:                                              \
      if (check) W1_TILED_LAUNCH(true, 2, NWV, RWD, RHD); \
      else W1_TILED_LAUNCH(false, 2, NWV, RWD, RHD);      \
      break;                                             \
    default:                                             \
      if (check) W1_TILED_LAUNCH(true, 3, NWV, RWD, RHD); \
      else W1_TILED_LAUNCH(false, 3, NWV, RWD, RHD);      \
  }
  if (rh == TILED_RH_SHORT) {
    W1_TILED_METRIC(8, 64, TILED_RH_SHORT)
  } else if (rw == 128) {
    if (nwv == 16) {
      W1_TILED_METRIC(16, 128, TILED_RH)
    } else {
      W1_TILED_METRIC(8, 128, TILED_RH)
    }
  } else {
    if (nwv == 16) {
      W1_TILED_METRIC(16, 64, TILED_RH)
    } else {
      W1_TILED_METRIC(8, 64, TILED_RH)
    }
  }
#undef W1_TILED_METRIC
#undef W1_TILED_LAUNCH
}

// resident kernel: sides up to 65, 9 nodes per thread of 512

int resident_lds_bytes(int side, int elem) { return 18 * NQ * 8 + 3 * side * side * elem; }

template <typename T> int K<T>::plain_resident_max_side() { return ResCfg<T>::MAXN; }

template <typename T> void K<T>::plain_resident(hipStream_t s, const int* idx, int ns, const SlotDesc<T>* d,
                                                SlotScalars* sc, int max_side, int check_every, int chunk,
                                                int metric) {
  if (!ns) return;
  if (max_side > ResCfg<T>::MAXN || metric < 1 || metric > 3) {
    fprintf(stderr, "w1: internal error: resident side %d, metric %d\n", max_side, metric);
    return;
  }
  static bool attr_set = false;
  const int bytes = resident_lds_bytes(max_side, sizeof(T));
  if (!attr_set) {
    const int full = resident_lds_bytes(ResCfg<T>::MAXN, sizeof(T));
    (void)hipFuncSetAttribute((const void*)k_plain_resident<T, ResCfg<T>::NPT, 1>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, full);
    (void)hipFuncSetAttribute((const void*)k_plain_resident<T, ResCfg<T>::NPT, 2>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, full);
    (void)hipFuncSetAttribute((const void*)k_plain_resident<T, ResCfg<T>::NPT, 3>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, full);
    attr_set = true;
  }
  if (metric == 1)
    LAUNCH((k_plain_resident<T, ResCfg<T>::NPT, 1>), ns, ResCfg<T>::NT, bytes, s, idx, d, sc, check_every, chunk);
  else if (metric == 2)
    LAUNCH((k_plain_resident<T, ResCfg<T>::NPT, 2>), ns, ResCfg<T>::NT, bytes, s, idx, d, sc, check_every, chunk);
  else
    LAUNCH((k_plain_resident<T, ResCfg<T>::NPT, 3>), ns, ResCfg<T>::NT, bytes, s, idx, d, sc, check_every, chunk);
}
template <typename T> void K<T>::kkt(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                     const SlotScalars* sc, int kind, int set_xor, int gate) {
  if (nw) LAUNCH(k_kkt<T>, nw, 256, 0, s, w, d, sc, kind, set_xor, gate);
}
template <typename T> void K<T>::div_pre(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                         const SlotScalars* sc, int mode, int kind, int gate, int set_xor) {
  if (nw) LAUNCH(k_div_pre<T>, nw, 256, 0, s, w, d, sc, mode, kind, gate, set_xor);
}
template <typename T> void K<T>::gemm(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                      const SlotScalars* sc, int mode, int src, int dst, int mat, bool scale,
                                      int gate) {
  if (!nw) return;
  if (mode == 0) {
    if (scale) LAUNCH((k_gemm<T, 0, true>), nw, 256, 0, s, w, d, sc, src, dst, mat, gate);
    else LAUNCH((k_gemm<T, 0, false>), nw, 256, 0, s, w, d, sc, src, dst, mat, gate);
  } else {
    if (scale) LAUNCH((k_gemm<T, 1, true>), nw, 256, 0, s, w, d, sc, src, dst, mat, gate);
    else LAUNCH((k_gemm<T, 1, false>), nw, 256, 0, s, w, d, sc, src, dst, mat, gate);
  }
}
template <typename T> void K<T>::poisson_fold(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                              const SlotScalars* sc, int dst, int gate) {
  if constexpr (sizeof(T) != 4) {
    fprintf(stderr, "w1: internal error: the folded DCT passes are FP32 only\n");
    return;
  } else {
    if (!nw) return;
    LAUNCH((k_dct_fold<1>), nw, 256, 0, s, w, d, sc, 6, 7, gate);
    LAUNCH((k_dct_fold<2>), nw, 256, 0, s, w, d, sc, 7, 6, gate);
    LAUNCH((k_dct_fold<3>), nw, 256, 0, s, w, d, sc, 6, 7, gate);
    LAUNCH((k_dct_fold<4>), nw, 256, 0, s, w, d, sc, 7, dst, gate);
  }
}
template <typename T> void K<T>::prox_post(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                           const SlotScalars* sc, bool check) {
  if (!nw) return;
  if (check) LAUNCH((k_prox_post<T, true>), nw, 256, 0, s, w, d, sc);
  else LAUNCH((k_prox_post<T, false>), nw, 256, 0, s, w, d, sc);
}
template <typename T> void K<T>::check(hipStream_t s, const int* idx, const int* nt, int ns, const SlotDesc<T>* d,
                                       SlotScalars* sc, int kind, int block_len, int launches, int blocks) {
  if (ns) LAUNCH(k_check<T>, ns, 64, 0, s, idx, nt, d, sc, kind, block_len, launches, blocks);
}
template <typename T> void K<T>::eval_sums(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                           const SlotScalars* sc, int kind, int cert, int polish) {
  if (nw) LAUNCH(k_eval_sums<T>, nw, 256, 0, s, w, d, sc, kind, cert, polish);
}
template <typename T> void K<T>::eval_final(hipStream_t s, const int* idx, const int* nt, int ns, const SlotDesc<T>* d,
                                            SlotScalars* sc, int kind, int cert) {
  if (ns) LAUNCH(k_eval_final<T>, ns, 256, 0, s, idx, nt, d, sc, kind, cert);
}
template <typename T> void K<T>::export_fields(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d,
                                               const SlotScalars* sc, int kind, int polish) {
  if (nw) LAUNCH(k_export_fields<T>, nw, 256, 0, s, w, d, sc, kind, polish);
}

// FP32 only: the FP64 iterate does not fit the register budget
template <typename T> int K<T>::prox_resident_max_side() { return sizeof(T) == 4 ? 65 : 0; }

template <typename T> void K<T>::prox_resident(hipStream_t s, const int* idx, int ns, const SlotDesc<T>* d,
                                               SlotScalars* sc, int max_side, int check_every, int chunk,
                                               int metric) {
  if (!ns) return;
  if constexpr (sizeof(T) != 4) {
    fprintf(stderr, "w1: internal error: no resident prox kernel for FP64\n");
    return;
  } else {
  if (max_side > 65 || metric < 1 || metric > 3) {
    fprintf(stderr, "w1: internal error: prox resident side %d, metric %d\n", max_side, metric);
    return;
  }
  static bool attr_set = false;
  if (!attr_set) {
    const int full = prox_resident_lds_bytes(65, sizeof(T));
    (void)hipFuncSetAttribute((const void*)k_prox_resident<T, 5, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              full);
    (void)hipFuncSetAttribute((const void*)k_prox_resident<T, 5, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              full);
    (void)hipFuncSetAttribute((const void*)k_prox_resident<T, 5, 3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              full);
    attr_set = true;
  }
  const int bytes = prox_resident_lds_bytes(max_side, sizeof(T));
  if (metric == 1) LAUNCH((k_prox_resident<T, 5, 1>), ns, PRES_THREADS, bytes, s, idx, d, sc, check_every, chunk);
  else if (metric == 2) LAUNCH((k_prox_resident<T, 5, 2>), ns, PRES_THREADS, bytes, s, idx, d, sc, check_every, chunk);
  else LAUNCH((k_prox_resident<T, 5, 3>), ns, PRES_THREADS, bytes, s, idx, d, sc, check_every, chunk);
  }
}

template struct K<float>;
template struct K<double>;

}  // namespace w1
