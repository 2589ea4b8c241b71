// Internal declarations shared by the HIP kernels and the host engine.
//
// Layout of one solve ("slot") in HBM: every level l owns NPLANES planes of
// (n_l+1) rows x pitch_l elements (pitch a multiple of 32 elements), one
// rho plane and two FP64 staging planes, plus a per-slot partial-sum area
// for per-tile FP64 reductions.  Plane roles:
//
//   plain (Algorithm 1/3): 0 m1[A] 1 m2[A] 2 phi[A] 3 m1[B] 4 m2[B] 5 phi[B]
//                          6, 7 Poisson ping-pong, 8 spare
//   prox  (Algorithm 2/4): 0 m1 1 m2 2 vphi1 3 vphi2 4 vphibar1 5 vphibar2
//                          6, 7 Poisson ping-pong, 8 potential psi
//
// Descriptors are indexed slot * MAXL + level (level 0 = coarsest), so a
// kernel that reads level l-1 and writes level l finds both.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <cmath>
#include <vector>

namespace w1 {

constexpr int MAXL = 12;
constexpr int NPLANES = 9;
constexpr int NQ = 8;                // FP64 partial sums per tile
constexpr int ST_H = 16;             // simple per-node tile: 16 rows x 64 cols
constexpr int ST_W = 64;
constexpr int GEMM_T = 64;           // DCT GEMM output tile
constexpr int TILED_RW = 128;        // plain tiled kernel region width
constexpr int TILED_RW_NARROW = 64;  // its narrow region (twice the workgroups)
constexpr int TILED_RH = 64;         // plain tiled kernel region height
constexpr int TILED_MAX_STEPS = 26;  // most PDHG steps per tiled launch
constexpr int TILED_NARROW_MAX_STEPS = 16;   // ... in the narrow region
constexpr int TILED_RH_SHORT = 32;           // the short narrow region's height
constexpr int TILED_SHORT_MAX_STEPS = 10;    // ... and its deepest block
constexpr int PRES_THREADS = 1024;   // resident kernel workgroup size (Algorithm 2)
constexpr int FFT_MIN_N = 1025;      // FP32 Poisson solves by FFT from this
                                     // transform length on (N = n + 1 with
                                     // 2 (N - 1) a power of two up to 8192)
constexpr int FFT_MAX_N = 4097;
constexpr int POLISH_PLANE = 4;      // prox, after the last iteration: the
                                     // re-projection potential (vphibar1 is
                                     // no longer read)

enum Status : int { ST_RUN = 0, ST_CONV = 1, ST_CAP = 2, ST_DIVERGED = 3, ST_REJECT = 4 };
enum Rule : int { RULE_KKT = 1, RULE_FPR = 2 };
enum Kind : int { K_PLAIN = 1, K_PROX = 2 };

// Per-slot, per-level descriptor read by every batched kernel.
template <typename T>
struct SlotDesc {
  T* p[NPLANES];
  T* rho;
  double* r0;          // FP64 staging: rho0_l, rho1_l
  double* r1;
  double* part;        // per-tile partial sums of the slot, NQ doubles per tile
  const T* dctC;       // orthonormal DCT-II matrix C[k][j], N x N row-major
  const T* dctCt;      // its transpose
  const double* dcts;  // 4 sin^2(pi k / 2N), k < N
  const T* dctCp;      // C with its rows in even-then-odd frequency order
  const T* dctCtp;     // and its transpose (folded FP32 passes)
  // FP32, N >= FFT_MIN_N: tables of the FFT-based transforms (M = 2N - 2):
  const float2* fft_chirp;   // c_m = e^{-i pi m^2 / N}, m < N
  const float2* fft_fb;      // FFT_M of the chirp filter conj(c), over M
  const float2* fft_tw;      // e^{-2 pi i t / M}, t < M
  const float2* fft_mk;      // e^{-i pi k / 2N}, k < N
  const double* in0;   // finest level only: input masses, dense pitch n+1
  const double* in1;
  double* out_m1;      // finest level only: exported fields, dense FP64
  double* out_m2;
  double* out_psi;
  int n, pitch;
  T ih, mu, tau;
  double h, mud, taud;  // FP64 copies of h, mu, tau for the measures
  double tol;          // stop tolerance of this level
  int metric;          // 1, 2 or 3 (l_1, l_2, l_inf)
  int divwin;          // FPR rule: rises of the measure in a row that end
                       // the level as diverged (0 = no such test)
  int rule;            // RULE_KKT or RULE_FPR
  int cap;             // iteration cap of this level
};

// Per-slot scalars written by the reduction epilogues (device memory).
struct SlotScalars {
  double sums[8];      // reduction outputs (prep: masses, level sums)
  double measure;      // last stop measure
  double eval[8];      // P, D, lo, hi, kkt, grad max, r_pri, r_dual
  double mean;         // mean of the plain potential (export)
  int status;          // Status; kernels of an iteration block skip a slot
                       // whose status is not ST_RUN
  int iters;           // iterations run at the current level
  int cur;             // plain: plane set (0 = A, 1 = B) holding the iterate
  int rises;           // stop tests in a row whose measure rose
};

// Work item: x = descriptor index (or -1 for padding), y = tile row,
// z = tile col, w = tile index inside the slot's partial area.
using Work = int4;

// ---------------- launchers (kernels.hip) ----------------
// Kernels that belong to an iteration block take `gate`: a slot whose
// status is not ST_RUN is skipped.  A plain slot's iterate is in plane set
// SlotScalars::cur; inside a block the i-th tiled launch reads set
// cur ^ (i & 1), and the stop test flips cur by the block's launch count.
template <typename T>
struct K {
  static void zero(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, unsigned mask);
  static void import_dense(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, int plane, const T* src);
  static void export_dense(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, int plane, T* dst);
  static void reduce(hipStream_t s, const int* idx, const int* ntiles, int ns, const SlotDesc<T>* d,
                     SlotScalars* sc, int nq, int out_base, unsigned maxmask);
  // scalars of every slot in the list (one item per slot has w == 0):
  // status RUN, iteration 0, iterate in plane set A, sums cleared
  static void reset_scalars(hipStream_t s, const Work* w, int nw, SlotScalars* sc);
  static void prep_stats(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d);
  static void prep_scale(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc);
  static void restrict_level(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d);
  static void scale_level(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc);
  static void rho_diff(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d);
  static void rho_write(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc);
  static void prolong(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc,
                      int kind);
  // the plain kernels are compiled per ground metric: every slot of one
  // launch has `metric` (others in the list are skipped); the tiled
  // kernel's rh x rw region (64 x 128 or 64 x 64 over nwv = 8 or 16
  // wavefronts, or 32 x 64 over 8)
  // second = 1: the second of two one-launch blocks checked together (its
  // stop-test partials go after the first block's); ev0 / ev1, when given,
  // receive the dispatch's start and end times
  static void plain_tiled(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc,
                          int launch_index, int steps, int rh, int rw, bool check, int metric, int nwv,
                          int second = 0, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
  static int plain_resident_max_side();
  static void plain_resident(hipStream_t s, const int* idx, int ns, const SlotDesc<T>* d, SlotScalars* sc,
                             int max_side, int check_every, int chunk, int metric);
  // Algorithm 2 levels with sides up to prox_resident_max_side(), one
  // workgroup per slot (planes 0..5), like plain_resident
  static int prox_resident_max_side();
  static void prox_resident(hipStream_t s, const int* idx, int ns, const SlotDesc<T>* d, SlotScalars* sc,
                            int max_side, int check_every, int chunk, int metric);
  static void kkt(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc, int kind,
                  int set_xor, int gate);
  // mode 2 of a plain slot reads plane set cur ^ set_xor (as kkt)
  static void div_pre(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc, int mode,
                      int kind, int gate, int set_xor = 0);
  static void gemm(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc, int mode,
                   int src, int dst, int mat, bool scale, int gate);
  // (A A*)^{-1} of plane 6 into plane dst with the folded FP32 passes
  // (plane 7 scratch); w: T x T tiles per slot, fold_tiles(N)
  static void poisson_fold(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc,
                           int dst, int gate);
  static void prox_post(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc,
                        bool check);
  static void check(hipStream_t s, const int* idx, const int* ntiles, int ns, const SlotDesc<T>* d,
                    SlotScalars* sc, int kind, int block_len, int launches, int blocks = 1);
  // cert = 0: no Poisson correction in plane 6; lo, hi and kkt are NaN.
  // polish = 1 (prox): the flux evaluated (and exported) is m + grad+ c with
  // c = (A A*)^{-1}(A m - rho) in POLISH_PLANE, its own correction in plane 6
  static void eval_sums(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc,
                        int kind, int cert, int polish = 0);
  static void eval_final(hipStream_t s, const int* idx, const int* ntiles, int ns, const SlotDesc<T>* d,
                         SlotScalars* sc, int kind, int cert);
  static void export_fields(hipStream_t s, const Work* w, int nw, const SlotDesc<T>* d, const SlotScalars* sc,
                            int kind, int polish = 0);
};

int resident_lds_bytes(int side, int elem);
// the FP32 Poisson solve by FFT (fftdct.hip) of every listed slot with
// FFT_MIN_N <= N <= FFT_MAX_N (others return at once): plane 6 in (and
// overwritten), plane 7 scratch, result in plane dst; the list holds
// T x T tiles per slot with T >= cdiv(N, 64).  `sizes`: bit m set when a
// listed slot has 2 (N - 1) = 2^m
void poisson_fft(hipStream_t s, const Work* w, int nw, const SlotDesc<float>* d, const SlotScalars* sc, int dst,
                 int gate, unsigned sizes);
__host__ __device__ inline bool uses_fft(int N, int elem) {
  return elem == 4 && N >= FFT_MIN_N && N <= FFT_MAX_N && ((N - 1) & (N - 2)) == 0;
}
// flops of one Poisson solve by the FFT path, counted conventionally: four
// line transforms (rows, columns both ways, rows) of ceil(N/2) line pairs,
// each pair a Bluestein DFT of two length-M FFTs (5 M log2 M) plus the
// pointwise filter (6 M) and the chirp, twiddle and unpacking work (~30 N)
inline double fft_poisson_flops(int N) {
  const double M = 2.0 * (N - 1), lg = std::log2(M);
  return 4.0 * ((N + 1) / 2) * (2.0 * 5.0 * M * lg + 6.0 * M + 30.0 * N);
}
// host tables of the FFT path for transform length N (FP64 computed,
// rounded to FP32): chirp (N), fb (M), tw (M), mk (N) complex pairs
void fft_tables(int N, std::vector<float>* chirp, std::vector<float>* fb, std::vector<float>* tw,
                std::vector<float>* mk);
// frequency order of the folded DCT: ne = N - N/2 even frequencies first,
// then the N/2 odd ones
inline int fold_perm(int x, int N) {
  const int ne = N - N / 2;
  return x < ne ? 2 * x : 2 * (x - ne) + 1;
}
// Cp[k''][j] = C[fold_perm(k'')][j] and Ctp = Cp^T from the row-major N x N C
template <typename T>
inline void fold_order(int N, const std::vector<T>& C, std::vector<T>* Cp, std::vector<T>* Ctp) {
  Cp->assign((size_t)N * N, T(0));
  Ctp->assign((size_t)N * N, T(0));
  for (int k = 0; k < N; ++k) {
    const int src = fold_perm(k, N);
    for (int j = 0; j < N; ++j) {
      (*Cp)[(size_t)k * N + j] = C[(size_t)src * N + j];
      (*Ctp)[(size_t)j * N + k] = C[(size_t)src * N + j];
    }
  }
}
// tiles per side of the folded DCT work list for transform length N
inline int fold_tiles(int N) {
  const int ne = N - N / 2, no = N / 2, a = (N + 63) / 64, b = (ne + 63) / 64 + (no + 63) / 64;
  return a > b ? a : b;
}
int prox_resident_lds_bytes(int side, int elem);

}  // namespace w1
