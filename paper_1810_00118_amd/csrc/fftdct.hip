// The Neumann Poisson solve of the eq. (pdhg) projection (and of Appendix B)
// for large grids: the orthonormal DCT-II / DCT-III of length N = n + 1 by
// fast Fourier transforms instead of products with the N x N matrix.
//
// N = 2^k + 1 has no power-of-two structure, so each length-N transform is
// computed as follows (FP32 data, tables built in FP64):
//  * Makhoul's reordering turns a DCT-II of a real line x into a length-N
//    DFT of v (v_j = x_{2j} for j <= (N-1)/2, v_{N-1-j} = x_{2j+1}):
//    sum_j x_j cos(pi k (2j+1) / 2N) = Re(e^{-i pi k / 2N} V_k); the inverse
//    runs the same steps backwards (V_k = e^{i pi k / 2N} (Y_k - i Y_{N-k}),
//    v = IDFT(V), then the reordering undone).
//  * Two real lines share one complex DFT (z = v + i v'); their spectra are
//    separated by the conjugate symmetry of a real line's DFT.
//  * The length-N DFT is Bluestein's chirp-z convolution: with
//    c_m = e^{-i pi m^2 / N}, V_k = c_k sum_j (v_j c_j) conj(c_{k-j}), a
//    convolution evaluated as a circular one of length M = 2N - 2 = 2^(k+1):
//    the offsets k - j span -(N-1)..N-1, and the only two that coincide
//    modulo M (+-(N-1)) carry the same chirp value, so no wrap-around term
//    is wrong.  Two power-of-two FFTs of length M per line pair, in LDS
//    (Stockham passes of radix 16, 8 or 4; the loads of the input are the
//    first pass's reads, and the product with the chirp's transform is
//    folded into the last pass's writes).
//
// A 2-D solve is five passes over the grid: rows forward, a transpose, the
// columns forward, divided by the eigenvalue lambda_kl = (s_k + s_l) / h^2
// (s_k = 4 sin^2(pi k / 2N), mode (0,0) set to 0) and inverted in the same
// kernel, a transpose back, rows inverse.  O(log N) flops per node and pass
// instead of O(N).
#include <cmath>
#include <complex>
#include <cstdio>
#include <type_traits>
#include <vector>

#include "w1_internal.hpp"

namespace w1 {

// The Stockham plan per transform length M: radix of pass q (0 past the
// last), 1024 = 4^5, 2048 = 8^3 4, 4096 = 8^4, 8192 = 16^3 2, so every pass
// has at least one butterfly per thread of the workgroup.
__host__ __device__ constexpr int fft_radix(int M, int q) {
  return M == 1024   ? (q < 5 ? 4 : 0)
         : M == 2048 ? (q < 3 ? 8 : q == 3 ? 4 : 0)
         : M == 4096 ? (q < 4 ? 8 : 0)
         : M == 8192 ? (q < 3 ? 16 : q == 3 ? 2 : 0)
                     : 0;
}
// threads per workgroup of a line transform of length M (every pass has
// a whole number of butterflies per thread)
__host__ __device__ constexpr int fft_threads(int M) { return M >= 4096 ? 512 : 256; }
__host__ __device__ constexpr int fft_passes(int M) {
  int q = 0;
  while (fft_radix(M, q)) ++q;
  return q;
}
// span Ns of the sub-transforms pass q combines (the product of the
// earlier radices)
__host__ __device__ constexpr int fft_ns(int M, int q) {
  int ns = 1;
  for (int p = 0; p < q; ++p) ns *= fft_radix(M, p);
  return ns;
}
// offset of pass q's twiddles in the table: (R - 1) Ns entries per pass
// with Ns > 1 (the first pass's are all 1); the total stays below M
__host__ __device__ constexpr int fft_twoff(int M, int q) {
  int off = 0;
  for (int p = 0; p < q; ++p)
    if (fft_ns(M, p) > 1) off += (fft_radix(M, p) - 1) * fft_ns(M, p);
  return off;
}

namespace {

constexpr int FT = 256;   // threads per workgroup of the transpose

// Tables and planes are device global memory.  Through generic pointers
// the compiler emits flat loads, which also count against the LDS wait
// counter (every wait for an LDS read would wait for the table loads in
// flight too); through these address-space-1 pointers they are global loads.
#define FG __attribute__((address_space(1)))
// a complex table entry through a global pointer
__device__ __forceinline__ float2 ld2_(const FG float2* p) {
  const FG float* q = (const FG float*)p;
  return make_float2(q[0], q[1]);
}

__device__ __forceinline__ float2 cmul_(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd_(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub_(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conj_(float2 a) { return make_float2(a.x, -a.y); }

// In-register DFTs of sizes 2, 4, 8 and 16 (natural order in and out).
__device__ __forceinline__ void dft2_(float2& a0, float2& a1) {
  const float2 t = a0;
  a0 = cadd_(t, a1);
  a1 = csub_(t, a1);
}
__device__ __forceinline__ void dft4_(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 s02 = cadd_(a0, a2), d02 = csub_(a0, a2), s13 = cadd_(a1, a3), d13 = csub_(a1, a3);
  const float2 md = make_float2(d13.y, -d13.x);   // -i (a1 - a3)
  a0 = cadd_(s02, s13);
  a2 = csub_(s02, s13);
  a1 = cadd_(d02, md);
  a3 = csub_(d02, md);
}
// x e^{-2 pi i m / 16} for a compile-time m (the trivial ones without a product)
template <int m>
__device__ __forceinline__ float2 w16_(float2 x) {
  constexpr int q = m & 15;
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f, r2 = 0.70710678118654752f;
  if constexpr (q == 0) return x;
  else if constexpr (q == 4) return make_float2(x.y, -x.x);
  else if constexpr (q == 8) return make_float2(-x.x, -x.y);
  else if constexpr (q == 12) return make_float2(-x.y, x.x);
  else {
    // cos and -sin of 2 pi q / 16
    constexpr float c = q == 1 ? c1 : q == 2 ? r2 : q == 3 ? s1 : q == 5 ? -s1 : q == 6 ? -r2 : q == 7 ? -c1
                      : q == 9 ? -c1 : q == 10 ? -r2 : q == 11 ? -s1 : q == 13 ? s1 : q == 14 ? r2 : c1;
    constexpr float sn = q == 1 ? -s1 : q == 2 ? -r2 : q == 3 ? -c1 : q == 5 ? -c1 : q == 6 ? -r2 : q == 7 ? -s1
                       : q == 9 ? s1 : q == 10 ? r2 : q == 11 ? c1 : q == 13 ? c1 : q == 14 ? r2 : s1;
    return make_float2(x.x * c - x.y * sn, x.x * sn + x.y * c);
  }
}
__device__ __forceinline__ void dft8_(float2 (&v)[8]) {
  // n = 2 n1 + n2, k = k1 + 4 k2
  dft4_(v[0], v[2], v[4], v[6]);
  dft4_(v[1], v[3], v[5], v[7]);
  const float2 y1[4] = {v[1], w16_<2>(v[3]), w16_<4>(v[5]), w16_<6>(v[7])};
  const float2 y0[4] = {v[0], v[2], v[4], v[6]};
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    v[k1] = cadd_(y0[k1], y1[k1]);
    v[k1 + 4] = csub_(y0[k1], y1[k1]);
  }
}
__device__ __forceinline__ void dft16_(float2 (&v)[16]) {
  // n = 4 n1 + n2, k = k1 + 4 k2: a DFT4 over n1 for each n2, twiddles
  // W16^(n2 k1), a DFT4 over n2 for each k1
  dft4_(v[0], v[4], v[8], v[12]);
  dft4_(v[1], v[5], v[9], v[13]);
  dft4_(v[2], v[6], v[10], v[14]);
  dft4_(v[3], v[7], v[11], v[15]);
  v[5] = w16_<1>(v[5]);
  v[9] = w16_<2>(v[9]);
  v[13] = w16_<3>(v[13]);
  v[6] = w16_<2>(v[6]);
  v[10] = w16_<4>(v[10]);
  v[14] = w16_<6>(v[14]);
  v[7] = w16_<3>(v[7]);
  v[11] = w16_<6>(v[11]);
  v[15] = w16_<9>(v[15]);
  // v[n2 + 4 k1] now holds y[n2][k1]; DFT4 over n2 -> X[k1 + 4 k2]
  float2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
    dft4_(a0, a1, a2, a3);
    o[k1] = a0;
    o[k1 + 4] = a1;
    o[k1 + 8] = a2;
    o[k1 + 12] = a3;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = o[k];
}
template <int R>
__device__ __forceinline__ void dftR_(float2 (&v)[R]) {
  if constexpr (R == 2) dft2_(v[0], v[1]);
  else if constexpr (R == 4) dft4_(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8_(v);
  else dft16_(v);
}

// LDS index swizzle: bits 0..4 of a buffer index are XORed with bits 4..8
// (a bijection on every length here).  The Stockham passes write at
// strides R and Ns R; without it the 64 lanes of a wavefront would write
// the first radix-16 pass into a single LDS bank.
__device__ __forceinline__ int sw_(int i) { return i ^ ((i >> 4) & 31); }

// Stockham pass q of the transform of length M: butterfly j < M / R (with
// k = j mod Ns) takes X[j + r M / R] e^{-2 pi i r k / (Ns R)}, r < R, and
// writes its length-R DFT to X'[(j / Ns) Ns R + k + r Ns].
//   SRC: the inputs come from load(p), the sequence at position p (first
//        pass only: nothing is read from LDS, so no barrier is needed
//        before the writes)
//   FB:  the outputs are written as conj(X'_p fb_p) (last pass only)
// The twiddles of pass q (Ns > 1) sit at tw + fft_twoff(M, q), at
// [(r - 1) Ns + k], so consecutive butterflies read consecutive entries.
// Reads, twiddle and fb loads are issued before the barrier; the pass ends
// synchronised.
template <int M, int q, bool SRC, bool FB, class L>
__device__ __forceinline__ void fft_pass_(float2* __restrict__ buf, const FG float2* __restrict__ tw,
                                          const FG float2* __restrict__ fb, const L& load) {
  constexpr int FL = fft_threads(M), R = fft_radix(M, q), Ns = fft_ns(M, q), NB = M / R, PB = NB / FL;
  static_assert(NB % FL == 0, "whole butterflies per thread");
  // the table pointers are made opaque here, so the compiler keeps each
  // pass's twiddle and fb loads in that pass instead of hoisting all of
  // them (loop invariants of the pair loop) into registers at the start
  const FG float2* t = tw + fft_twoff(M, q);
  asm volatile("" : "+s"(t));
  if constexpr (FB) asm volatile("" : "+s"(fb));
  float2 v[PB][R];
  float2 f[FB ? PB : 1][FB ? R : 1];
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int j = threadIdx.x + FL * b, k = j & (Ns - 1), o = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float2 x;
      if constexpr (SRC) {
        // a Bluestein input is 0 from position N = M/2 + 1 on: of the
        // upper half only position M/2 (butterfly 0) is loaded
        if (r < R / 2) x = load(j + r * NB);
        else if (r == R / 2) x = j == 0 ? load(M / 2) : make_float2(0.f, 0.f);
        else x = make_float2(0.f, 0.f);
      } else {
        x = buf[sw_(j + r * NB)];
      }
      if constexpr (Ns > 1) {
        if (r > 0) x = cmul_(x, ld2_(t + (r - 1) * Ns + k));
      }
      v[b][r] = x;
      if constexpr (FB) f[b][r] = ld2_(fb + o + r * Ns);
    }
  }
  if constexpr (!SRC) __syncthreads();
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int j = threadIdx.x + FL * b, k = j & (Ns - 1), o = (j - k) * R + k;
    dftR_<R>(v[b]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float2 y = v[b][r];
      if constexpr (FB) y = conj_(cmul_(y, f[b][r]));
      buf[sw_(o + r * Ns)] = y;
    }
  }
  __syncthreads();
}

// Forward FFT of length M into LDS (natural order, swizzled), from load()
// when SRC, else in place from LDS; with FB the result is stored as
// conj(X fb).  Ends synchronised.
template <int M, bool SRC, bool FB, class L>
__device__ __forceinline__ void fft_(float2* __restrict__ buf, const FG float2* __restrict__ tw,
                                     const FG float2* __restrict__ fb, const L& load) {
  constexpr int Q = fft_passes(M);
  fft_pass_<M, 0, SRC, FB && Q == 1>(buf, tw, fb, load);
  if constexpr (Q > 1) fft_pass_<M, 1, false, FB && Q == 2>(buf, tw, fb, load);
  if constexpr (Q > 2) fft_pass_<M, 2, false, FB && Q == 3>(buf, tw, fb, load);
  if constexpr (Q > 3) fft_pass_<M, 3, false, FB && Q == 4>(buf, tw, fb, load);
  if constexpr (Q > 4) fft_pass_<M, 4, false, FB && Q == 5>(buf, tw, fb, load);
}

// Bluestein: load(j) = a_j = z_j c_j (j < N), 0 up to M.  On exit buf[k]
// (swizzled) holds conj(y_k) with y = a (*) b (circular, length M), so the
// DFT of z is Z_k = c_k conj(buf[k]) for k < N.  fb = FFT(b) / M.
template <int M, class L>
__device__ void bluestein_(float2* __restrict__ buf, const FG float2* __restrict__ tw, const FG float2* __restrict__ fb,
                           const L& load) {
  fft_<M, true, true>(buf, tw, fb, load);   // conj(FFT(a) fb)
  fft_<M, false, false>(buf, tw, fb, load);   // FFT(conj(A)) = M conj(IFFT(A)): fb carries the 1 / M
}

// orthonormal DCT scale s_k
__device__ __forceinline__ float dct_s_(int k, int N) {
  return k == 0 ? sqrtf(1.f / (float)N) : sqrtf(2.f / (float)N);
}
// 1 / s_k
__device__ __forceinline__ float dct_is_(int k, int N) {
  return k == 0 ? sqrtf((float)N) : sqrtf(0.5f * (float)N);
}

// Makhoul's order: position j of v holds x_{src(j)}
__device__ __forceinline__ int mk_src_(int j, int N) { return j <= (N - 1) / 2 ? 2 * j : 2 * (N - 1 - j) + 1; }

// forward: lines x0 (real part) and x1 (imaginary part), read through
// `get(line, i)`: position j of the Bluestein input, a_j = z_j c_j (0 past N)
template <class G>
__device__ __forceinline__ float2 at_forward_(int j, const FG float2* chirp, int N, const G& get) {
  if (j >= N) return make_float2(0.f, 0.f);
  const int s = mk_src_(j, N);
  return cmul_(make_float2(get(0, s), get(1, s)), ld2_(chirp + j));
}

// after bluestein_ of a forward load: the two lines' orthonormal DCT-II
// coefficients X0_k, X1_k, k < N, handed to put(k, X0_k, X1_k)
template <int M, class P>
__device__ void unpack_forward_(const float2* buf, const FG float2* chirp, const FG float2* mk, int N, const P& put) {
  for (int k = threadIdx.x; k < N; k += fft_threads(M)) {
    const int kr = k == 0 ? 0 : N - k;
    const float2 Z = cmul_(ld2_(chirp + k), conj_(buf[sw_(k)]));
    const float2 Zr = conj_(cmul_(ld2_(chirp + kr), conj_(buf[sw_(kr)])));   // conj(Z_{N-k})
    // V0 = (Z + conj Zr) / 2, V1 = (Z - conj Zr) / 2i; X = s Re(mk V)
    const float2 V0 = make_float2(0.5f * (Z.x + Zr.x), 0.5f * (Z.y + Zr.y));
    const float2 V1 = make_float2(0.5f * (Z.y - Zr.y), -0.5f * (Z.x - Zr.x));
    const float s = dct_s_(k, N);
    const float2 e = ld2_(mk + k);
    put(k, s * (e.x * V0.x - e.y * V0.y), s * (e.x * V1.x - e.y * V1.y));
  }
}

// inverse: from two lines of orthonormal DCT coefficients (got through
// `get(line, k)`), position j of the Bluestein input, a_j = conj(W_j) c_j
// with W = spec(U0) + i spec(U1),
// spec(U)_k = e^{i pi k / 2N} (U_k / s_k - i U_{N-k} / s_{N-k})
template <class G>
__device__ __forceinline__ float2 at_inverse_(int j, const FG float2* chirp, const FG float2* mk, int N, const G& get) {
  if (j >= N) return make_float2(0.f, 0.f);
  const float isj = dct_is_(j, N);
  const float u0 = get(0, j) * isj, u1 = get(1, j) * isj;
  float r0 = 0.f, r1 = 0.f;
  if (j > 0) {
    const float isr = dct_is_(N - j, N);
    r0 = get(0, N - j) * isr;
    r1 = get(1, N - j) * isr;
  }
  // e^{i t} = conj(mk_j); spec = e^{i t} (u - i r)
  const float2 e = conj_(ld2_(mk + j));
  const float2 s0 = cmul_(e, make_float2(u0, -r0)), s1 = cmul_(e, make_float2(u1, -r1));
  const float2 W = make_float2(s0.x - s1.y, s0.y + s1.x);   // s0 + i s1
  return cmul_(conj_(W), ld2_(chirp + j));
}

// after bluestein_ of an inverse load: D = DFT(conj W) = c_k conj(buf[k]),
// v = conj(D) / N = (c_k conj(buf[k]))^* / N; the line values at position
// i come from v at the Makhoul index of i; handed to put(i, x0_i, x1_i)
template <int M, class P>
__device__ void unpack_inverse_(const float2* buf, const FG float2* chirp, int N, const P& put) {
  const float iN = 1.f / (float)N;
  for (int i = threadIdx.x; i < N; i += fft_threads(M)) {
    const int j = (i & 1) ? N - 1 - (i >> 1) : (i >> 1);
    const float2 v = conj_(cmul_(ld2_(chirp + j), conj_(buf[sw_(j)])));
    put(i, v.x * iN, v.y * iN);
  }
}

// Work item: slot x, tile (y, z) of a T x T list (T = cdiv(N, 64)); line
// pairs p = y T + z, y T + z + T^2, ... < cdiv(N, 2).
//   MODE 0: rows of src -> DCT-II rows of dst
//   MODE 1: rows of src (coefficients) -> DCT-III rows of dst
//   MODE 2: lines of src (the transposed row transform: line l is the
//           axis-2 frequency l) -> DCT-II, divided by lambda, DCT-III, to dst
template <int M, int MODE>
__global__ __launch_bounds__(fft_threads(M)) void k_fft_lines(const Work* __restrict__ work, const SlotDesc<float>* __restrict__ desc,
                                                  const SlotScalars* __restrict__ scal, int src, int dst, int gate) {
  __shared__ float2 buf[M];
  __shared__ float2 S[MODE == 2 ? M / 2 + 1 : 1];   // MODE 2: scaled spectra
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  if (gate && scal[w.x / MAXL].status != ST_RUN) return;
  const SlotDesc<float>& d = desc[w.x];
  const int N = d.n + 1;
  if (!d.fft_tw || 2 * (N - 1) != M) return;   // no FFT tables, or another length's launch
  const int ld = d.pitch, T = (N + 63) / 64, np = (N + 1) / 2;
  if (w.y >= T || w.z >= T) return;   // the list may be wider than T x T
  const FG float* __restrict__ X = (const FG float*)d.p[src];
  FG float* __restrict__ Y = (FG float*)d.p[dst];
  const FG float2* __restrict__ chirp = (const FG float2*)d.fft_chirp;
  const FG float2* __restrict__ fb = (const FG float2*)d.fft_fb;
  const FG float2* __restrict__ tw = (const FG float2*)d.fft_tw;
  const FG float2* __restrict__ mk = (const FG float2*)d.fft_mk;
  for (int p = w.y * T + w.z; p < np; p += T * T) {
    const int l0 = 2 * p, l1 = 2 * p + 1;
    const bool has1 = l1 < N;
    const FG float* __restrict__ x0 = X + (size_t)l0 * ld;
    const FG float* __restrict__ x1 = X + (size_t)(has1 ? l1 : l0) * ld;
    auto get = [&](int line, int i) -> float {
      if (line == 0) return x0[i];
      return has1 ? x1[i] : 0.f;
    };
    if (MODE == 1) {
      bluestein_<M>(buf, tw, fb, [&](int j) { return at_inverse_(j, chirp, mk, N, get); });
      unpack_inverse_<M>(buf, chirp, N, [&](int i, float a, float b) {
        Y[(size_t)l0 * ld + i] = a;
        if (has1) Y[(size_t)l1 * ld + i] = b;
      });
      __syncthreads();
      continue;
    }
    bluestein_<M>(buf, tw, fb, [&](int j) { return at_forward_(j, chirp, N, get); });
    if (MODE == 0) {
      unpack_forward_<M>(buf, chirp, mk, N, [&](int k, float a, float b) {
        Y[(size_t)l0 * ld + k] = a;
        if (has1) Y[(size_t)l1 * ld + k] = b;
      });
      __syncthreads();
      continue;
    }
    // MODE 2: spectra of lines l0, l1 along the axis-1 frequency k, divided
    // by lambda_{k l} (FP64 table of s), staged in S, then inverted
    const double h2 = d.h * d.h;
    const FG double* __restrict__ s = (const FG double*)d.dcts;
    unpack_forward_<M>(buf, chirp, mk, N, [&](int k, float a, float b) {
      const double f0 = (k == 0 && l0 == 0) ? 0.0 : h2 / (s[k] + s[l0]);
      const double f1 = has1 ? h2 / (s[k] + s[l1]) : 0.0;
      S[k] = make_float2((float)((double)a * f0), (float)((double)b * f1));
    });
    __syncthreads();
    auto getS = [&](int line, int k) -> float { return line ? S[k].y : S[k].x; };
    bluestein_<M>(buf, tw, fb, [&](int j) { return at_inverse_(j, chirp, mk, N, getS); });
    unpack_inverse_<M>(buf, chirp, N, [&](int i, float a, float b) {
      Y[(size_t)l0 * ld + i] = a;
      if (has1) Y[(size_t)l1 * ld + i] = b;
    });
    __syncthreads();
  }
}

// dst = src^T over the N x N grid (pitch ld), 64 x 64 tiles through LDS
__global__ __launch_bounds__(FT) void k_transpose(const Work* __restrict__ work, const SlotDesc<float>* __restrict__ desc,
                                                 const SlotScalars* __restrict__ scal, int src, int dst, int gate) {
  __shared__ float t[64][65];
  const Work w = work[blockIdx.x];
  if (w.x < 0) return;
  if (gate && scal[w.x / MAXL].status != ST_RUN) return;
  const SlotDesc<float>& d = desc[w.x];
  const int N = d.n + 1, ld = d.pitch;
  if (!d.fft_tw) return;   // solved by the matrix passes
  const FG float* __restrict__ X = (const FG float*)d.p[src];
  FG float* __restrict__ Y = (FG float*)d.p[dst];
  const int i0 = w.y * 64, j0 = w.z * 64;
  if (i0 >= N || j0 >= N) return;
  const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = r0 + 4 * q, i = i0 + r, j = j0 + c;
    t[r][c] = (i < N && j < N) ? X[(size_t)i * ld + j] : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = r0 + 4 * q, i = j0 + r, j = i0 + c;   // dst row = src column
    if (i < N && j < N) Y[(size_t)i * ld + j] = t[c][r];
  }
}

}  // namespace

// host: in-place radix-2 FFT in FP64 (table construction only)
static void fft_host(std::vector<std::complex<double>>& a) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  const double pi = 3.14159265358979323846;
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        const std::complex<double> w = std::polar(1.0, -2.0 * pi * (double)k / (double)len);
        const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

void fft_tables(int N, std::vector<float>* chirp, std::vector<float>* fb, std::vector<float>* tw,
                std::vector<float>* mk) {
  const int M = 2 * (N - 1);
  const double pi = 3.14159265358979323846;
  chirp->assign(2 * (size_t)N, 0.f);
  mk->assign(2 * (size_t)N, 0.f);
  fb->assign(2 * (size_t)M, 0.f);
  tw->assign(2 * (size_t)M, 0.f);
  std::vector<std::complex<double>> B(M);
  for (int m = 0; m < N; ++m) {
    // m^2 mod 2N in integers keeps the angle exact for large m
    const long long q = ((long long)m * m) % (2LL * N);
    const double a = -pi * (double)q / (double)N;
    (*chirp)[2 * m] = (float)std::cos(a);
    (*chirp)[2 * m + 1] = (float)std::sin(a);
    const std::complex<double> b = std::polar(1.0, -a);   // conj(c_m)
    B[m] = b;
    if (m > 0) B[M - m] = b;   // b_{-m} = b_m; m = N - 1 lands on the same slot
    const double t = -pi * (double)m / (2.0 * N);
    (*mk)[2 * m] = (float)std::cos(t);
    (*mk)[2 * m + 1] = (float)std::sin(t);
  }
  fft_host(B);
  for (int p = 0; p < M; ++p) {
    (*fb)[2 * p] = (float)(B[p].real() / M);
    (*fb)[2 * p + 1] = (float)(B[p].imag() / M);
  }
  // pass q's twiddles e^{-2 pi i r k / (Ns R)}, 1 <= r < R, k < Ns, at
  // fft_twoff(M, q) + (r - 1) Ns + k
  for (int q = 0; q < fft_passes(M); ++q) {
    const int R = fft_radix(M, q), Ns = fft_ns(M, q);
    if (Ns == 1) continue;
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < Ns; ++k) {
        const long long e = ((long long)r * k) % ((long long)Ns * R);
        const double t = -2.0 * pi * (double)e / (double)(Ns * R);
        const size_t at = (size_t)fft_twoff(M, q) + (size_t)(r - 1) * Ns + k;
        (*tw)[2 * at] = (float)std::cos(t);
        (*tw)[2 * at + 1] = (float)std::sin(t);
      }
  }
}

// (A A*)^{-1} of plane 6 into plane dst for every listed slot with
// N >= FFT_MIN_N (others return at once); plane 7 is scratch, plane 6 is
// overwritten.  `sizes`: bit m set when some slot has M = 2^m.
void poisson_fft(hipStream_t s, const Work* w, int nw, const SlotDesc<float>* d, const SlotScalars* sc, int dst,
                 int gate, unsigned sizes) {
  if (!nw || !sizes) return;
  auto rows = [&](auto Mc, int mode, int a, int b) {
    constexpr int M = decltype(Mc)::value;
    if (!(sizes & (1u << __builtin_ctz(M)))) return;
    if (mode == 0) hipLaunchKernelGGL((k_fft_lines<M, 0>), dim3(nw), dim3(fft_threads(M)), 0, s, w, d, sc, a, b, gate);
    if (mode == 1) hipLaunchKernelGGL((k_fft_lines<M, 1>), dim3(nw), dim3(fft_threads(M)), 0, s, w, d, sc, a, b, gate);
    if (mode == 2) hipLaunchKernelGGL((k_fft_lines<M, 2>), dim3(nw), dim3(fft_threads(M)), 0, s, w, d, sc, a, b, gate);
  };
  auto all = [&](int mode, int a, int b) {
    rows(std::integral_constant<int, 1024>{}, mode, a, b);
    rows(std::integral_constant<int, 2048>{}, mode, a, b);
    rows(std::integral_constant<int, 4096>{}, mode, a, b);
    rows(std::integral_constant<int, 8192>{}, mode, a, b);
  };
  all(0, 6, 7);                                                          // rows, forward
  hipLaunchKernelGGL(k_transpose, dim3(nw), dim3(FT), 0, s, w, d, sc, 7, 6, gate);
  all(2, 6, 6);                                                          // columns, both ways
  hipLaunchKernelGGL(k_transpose, dim3(nw), dim3(FT), 0, s, w, d, sc, 6, 7, gate);
  all(1, 7, dst);                                                        // rows, inverse
}

}  // namespace w1
