// One 64 x 64 output tile of a matrix product on the matrix cores (FP32,
// v_mfma_f32_32x32x2f32), shared by the d = 2 DCT passes and the d = 3 ones.
#pragma once
#include <hip/hip_runtime.h>

namespace w1 {

typedef float w1_f32x16 __attribute__((ext_vector_type(16)));

// one 64 x 64 output tile (this wavefront's 32 x 32 quarter into out[16],
// four wavefronts) of sum_k A(i, k) B(k, j), k < K.  The
// loaders take a tile-local row / column and a contraction index k < K, read
// only in-bounds addresses (clamping internally) and return 0 outside the
// operands; terms with k >= K are masked here, so no load is conditional
// and the slice loads compile without branches
template <class LA, class LB>
__device__ __forceinline__ void mfma_tile64_(const LA& la, const LB& lb, int K, float (*As)[64][33],
                                             float (*Bs)[32][68], float (&out)[16]) {
  constexpr int KT = 32;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  const int ak = t & 31, ai0 = t >> 5;
  const int bj = t & 63, bk0 = t >> 6;
  float ra[8], rb[8];
  auto load = [&](int p0) {
    const int ka = p0 + ak, kac = ka < K ? ka : K - 1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kb = p0 + bk0 + 4 * q, kbc = kb < K ? kb : K - 1;
      const float va = la(ai0 + 8 * q, kac), vb = lb(kbc, bj);
      ra[q] = ka < K ? va : 0.f;
      rb[q] = kb < K ? vb : 0.f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      As[buf][ai0 + 8 * q][ak] = ra[q];
      Bs[buf][bk0 + 4 * q][bj] = rb[q];
    }
  };
  w1_f32x16 tot = {}, comp = {};
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int p0 = 0; p0 < K; p0 += KT) {
    const bool more = p0 + KT < K;
    if (more) load(p0 + KT);
    w1_f32x16 acc = {};
#pragma unroll
    for (int kk = 0; kk < KT; kk += 2) {
      const float a = As[buf][wr + (lane & 31)][kk + (lane >> 5)];
      const float b = Bs[buf][kk + (lane >> 5)][wc + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float x = acc[r], s0 = tot[r], s1 = s0 + x;
      comp[r] += fabsf(s0) >= fabsf(x) ? (s0 - s1) + x : (x - s1) + s0;
      tot[r] = s1;
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) out[r] = tot[r] + comp[r];
}

// tile-local row / column of accumulator register r of this lane
__device__ __forceinline__ int mfma_row_(int r) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  return (wv >> 1) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}
__device__ __forceinline__ int mfma_col_() {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  return (wv & 1) * 32 + (lane & 31);
}

}  // namespace w1
