/*
 * w1.h -- C ABI of the MI355X multilevel Wasserstein-1 solver.
 *
 * Implements the cascadic multilevel primal-dual algorithms of
 * J. Liu, W. Yin, W. Li, Y. T. Chow, "Multilevel Optimal Transport: a Fast
 * Approximation of Wasserstein-1 distances" (arXiv 1810.00118):
 *   - Algorithm 1 (plain primal-dual, eq. (primaldual)) and its multilevel
 *     form Algorithm 3;
 *   - Algorithm 2 (proximal PDHG, eq. (pdhg)) and its multilevel form
 *     Algorithm 4;
 * on the Beckmann flux problem of eq. (opt_flux_dis):
 *   W1_h = min sum_x ||m(x)||_p h^2   s.t.   div_h m = rho0 - rho1
 * on the vertex grid {0, h, ..., 1}^2 of Sec. 2.2 (side n, h = 1/n,
 * (n+1)^2 nodes).
 *
 * Conventions shared by every call:
 *   - Node arrays are row-major [i*(n+1) + j], i along x1, j along x2.
 *   - A flux m is two such planes: m1[i,j] on the edge (i,j)->(i+1,j),
 *     m2[i,j] on (i,j)->(i,j+1).  m1[n,:] and m2[:,n] are zero.
 *   - Input masses are node masses (any positive scale); the library
 *     renormalises each to unit mass and forms rho = p/h^2 (Sec. 2.2).
 *   - The reported potential psi has the usual sign, W1_h = <psi, rho>_h
 *     at optimum, and zero mean (Appendix B).
 *   - Every call returns an int status (W1_OK = 0, negative = error);
 *     nothing throws across the ABI.  w1_strerror() names a status.
 *   - "Device" pointers are HIP device memory (for example a torch
 *     tensor's data_ptr on cuda:0); "host" pointers are ordinary memory.
 *   - Input buffers are owned by the caller and are fully consumed before
 *     the call returns.  The library owns every buffer it allocates.
 */
#ifndef W1_H
#define W1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    W1_OK = 0,
    W1_EAGAIN = 1,     /* w1_poll: the request is still running            */
    W1_EINVAL = -1,    /* bad argument: sizes, divisibility, masses        */
    W1_ENOMEM = -2,    /* device allocation failed / budget too small      */
    W1_EBUSY = -3,     /* admission queue full                             */
    W1_EDEVICE = -4,   /* a HIP runtime call failed                        */
    W1_ESTATE = -5,    /* call not valid in the handle's current state     */
    W1_ENOTFOUND = -6  /* unknown ticket                                   */
};

/* per-solve outcome in w1_result.status (not an error); W1_SOLVE_FAILED:
 * served mode only, the batch the request ran in stopped on a runtime
 * error (no values; w1_drain returns that error)                          */
enum { W1_SOLVE_OK = 0, W1_SOLVE_MAXITER = 1, W1_SOLVE_DIVERGED = 2,
       W1_SOLVE_REJECTED = 3, W1_SOLVE_FAILED = 4 };

/* ground metric ||.||_p of the flux cost (Sec. 2.1); the dual norm q of the
 * potential's constraint is inf, 2 and 1.  W1_METRIC_LINF: the l_inf prox is
 * the Moreau complement of an l_1-ball projection (Sec. 4.2, p = inf)     */
enum { W1_METRIC_L1 = 1, W1_METRIC_L2 = 2, W1_METRIC_LINF = 3 };
enum { W1_ALGO_PLAIN = 1,  /* Algorithm 1 / 3 (eq. (primaldual))           */
       W1_ALGO_PROX = 2 }; /* Algorithm 2 / 4 (eq. (pdhg))                 */
enum { W1_FP32 = 1,        /* FP32 iterates, FP64 reductions               */
       W1_FP64 = 2 };      /* FP64 throughout                              */
enum { W1_STOP_KKT = 1,    /* normalised KKT residual <= tol_l             */
       W1_STOP_FPR = 2 };  /* the paper's R^k (eq. (pd_stop)) or G^k
                              (eq. (pdhg_stop)) <= eps_l                   */

#define W1_MAX_LEVELS 12

typedef struct {
    int32_t n;            /* finest grid side; n % 2^(levels-1) == 0, n >= 2  */
    int32_t levels;       /* L >= 1; level l has side n / 2^(L-l) (Sec. 3.2) */
    int32_t metric;       /* W1_METRIC_*                                      */
    int32_t algo;         /* W1_ALGO_*                                        */
    int32_t precision;    /* W1_FP32 / W1_FP64                                */
    int32_t stop_rule;    /* W1_STOP_*                                        */
    double  tol;          /* finest-level tolerance (KKT tol or FPR eps_L);
                             <= 0 with W1_STOP_FPR selects eq. (stop_tol)    */
    double  alpha;        /* tol_l = tol * (h_l/h)^alpha, eq.
                             (tol_formula_propose); paper's choice -1        */
    double  step_scale;   /* plain: mu = tau = step_scale / (2 sqrt 2 / h);
                             prox: mu = tau = step_scale;  <= 0 selects the
                             paper's 1/2 for both; 1 is the practical choice
                             of the footnotes to Sec. 3.1 (mu = tau = 1/||A||
                             with the bound 2 sqrt 2 / h for ||A||, and 1 for
                             Algorithm 2); above 1 (at most 2) convergence
                             is not guaranteed and diverge_window must guard
                             the FPR rule                                   */
    int32_t max_iters;    /* per-level iteration cap (> 0)                    */
    int32_t check_every;  /* stop-test cadence in iterations (> 0)           */
    int32_t block_steps;  /* plain: PDHG steps fused per launch (temporal
                             block depth), 0..26; 0 = autotuned; otherwise
                             the deepest divisor of check_every not above it */
    int32_t flags;        /* W1_FLAG_* bit set                                */
    double  h;            /* finest grid spacing; <= 0 selects 1/n (Omega =
                             [0,1]^2).  The solve runs on the unit square and
                             the outputs are rescaled to Omega = [0, n h]^2
                             (Sec. 2.2 with the domain scaled by c = n h, unit
                             masses): W1, dual, lo, hi and level_w1 by c, the
                             flux by 1/c (1/c^2 in d = 3), the potential by c;
                             tolerances and stop measures refer to the unit
                             square                                          */
    int32_t level_caps[W1_MAX_LEVELS]; /* per-level iteration caps, coarsest
                             first; 0 takes max_iters; each a multiple of
                             check_every                                     */
    int32_t diverge_window; /* FPR rule: a level whose stop measure rises at
                             this many consecutive stop tests ends as
                             W1_SOLVE_DIVERGED (R^k of eq. (pd_stop) does not
                             increase while mu tau ||A||^2 < 1, Sec. 3.1);
                             0 = off; at least 1 when step_scale > 1        */
    int32_t reserved;     /* 0                                                */
} w1_params;

/* W1_FLAG_NO_RESIDENT: never keep a whole level in one workgroup's LDS     */
#define W1_FLAG_NO_RESIDENT 1
/* W1_FLAG_NO_CERT: skip the FP64 certificate at the end (w1 and dual are   */
/* still computed; lo, hi and kkt are returned as NaN)                       */
#define W1_FLAG_NO_CERT 2
/* W1_FLAG_LEVEL_COST: also evaluate f(m^{K_l}) = sum ||m||_p h_l^2 at the */
/* end of every coarser level (one FP64 reduction and a host wait per level */
/* transition; the quantity the tolerance study of Sec. 5.2 compares with   */
/* the level optimum); without it level_w1 holds NaN below the finest level */
#define W1_FLAG_LEVEL_COST 4
/* W1_FLAG_NO_FIELDS: served requests (w1_submit) keep no output fields:    */
/* the worker skips the three device-to-host copies of m1, m2 and psi and   */
/* its wait on them when the request ends; w1_poll then returns W1_EINVAL   */
/* (leaving the result pollable) if it is given field buffers.  Other bits  */
/* of flags are rejected by w1_params_check.                                */
#define W1_FLAG_NO_FIELDS 8

typedef struct {
    double  w1;           /* f(m^K) = sum ||m||_p h^2 on the finest level     */
    double  dual;         /* <psi, rho>_h                                     */
    double  lo, hi;       /* certified bracket: lo <= W1_h <= hi               */
    double  kkt;          /* normalised KKT residual of the returned fields   */
    int32_t status;       /* W1_SOLVE_*                                       */
    int32_t levels_run;
    int32_t iters[W1_MAX_LEVELS];
    double  measure[W1_MAX_LEVELS]; /* stop measure at each level's end      */
    double  seconds;      /* wall time from admission to completion           */
    double  queue_seconds;/* served requests: time waiting for admission     */
    double  level_w1[W1_MAX_LEVELS];      /* f(m^{K_l}) at each level's end
                             (W1_FLAG_LEVEL_COST; the finest always), or NaN */
    double  level_seconds[W1_MAX_LEVELS]; /* wall time from admission to the
                             host step that saw each level end            */
} w1_result;

typedef struct w1_ctx* w1_handle;

/* Fill *p with defaults: L1, prox, FP32, FPR rule with eq. (stop_tol),
 * alpha = -1, paper step sizes, cap 20000, check every 10, block auto.      */
void w1_params_default(w1_params* p);

/* Validate parameters; returns W1_OK or W1_EINVAL.                         */
int w1_params_check(const w1_params* p);

/* Device bytes one solve with these parameters keeps resident.            */
size_t w1_bytes_per_solve(const w1_params* p);

/*
 * w1_plan: create a solver handle for the multilevel method of Sec. 3.2
 * (Algorithm 3 or 4 on the level hierarchy h_l = 2^(L-l) h): per-level
 * state for every slot, the DCT tables of the Poisson solves of eq. (pdhg)
 * and Appendix B, and the launch plans.
 *   params          : used by w1_solve (copied).
 *   batch_capacity  : most pairs one w1_solve call may take (>= 1).
 *   hbm_budget_bytes: device bytes the handle may hold for solve state; 0
 *                     means 1/2 of the free device memory.  Buffers for
 *                     batch_capacity solves are allocated here (W1_ENOMEM
 *                     if they exceed the budget).
 *   hip_stream      : hipStream_t every kernel is queued on; NULL = the
 *                     library's own stream.
 * Threading: a handle is used by one thread at a time, except w1_submit
 * and w1_poll, which may be called from any thread.
 */
int w1_plan(const w1_params* params, int32_t batch_capacity,
            size_t hbm_budget_bytes, void* hip_stream, w1_handle* out);

/*
 * w1_solve: Algorithm 3 or 4 on `count` independent pairs as one batch.
 *   p0[k], p1[k]: node masses of pair k, (n+1)^2 doubles each, host
 *                 (on_device = 0) or device (on_device = 1) memory.
 *   out[k]      : result of pair k (host memory).
 * Masses must be finite and non-negative with equal totals (relative
 * difference <= 1e-9); a pair that violates this gets status
 * W1_SOLVE_REJECTED while the others are solved.  Non-convergence is not
 * an error: W1_SOLVE_MAXITER with the certificate.  Blocks until done.
 * Device masses are read in place (no staging copy): they must stay
 * allocated and unchanged until w1_solve returns; host masses are copied.
 */
int w1_solve(w1_handle h, int32_t count, const double* const* p0,
             const double* const* p1, int32_t on_device, w1_result* out);

/*
 * w1_fields: copy the finest-level fields of pair `index` of the last
 * w1_solve into caller buffers (each (n+1)^2 doubles; NULL skips one):
 * the flux m1, m2 and the usual-sign zero-mean potential psi.
 */
int w1_fields(w1_handle h, int32_t index, double* m1, double* m2,
              double* psi, int32_t on_device);

/*
 * Served mode (continuous batching).  w1_submit admits one request with
 * its own parameters; it is queued until its state fits the handle's HBM
 * budget, then joins the running batch between iteration blocks.  The
 * masses are copied before w1_submit returns.  W1_EBUSY when the pending
 * queue holds `queue_limit` requests (w1_serve_config).
 * w1_poll returns W1_EAGAIN until the ticket is done, then W1_OK with the
 * result and (optionally, (n+1)^2 doubles each) the fields; a finished
 * ticket is released by the poll that returns it.
 */
int w1_serve_config(w1_handle h, int32_t queue_limit);
int w1_submit(w1_handle h, const w1_params* per_request, const double* p0,
              const double* p1, int32_t on_device, uint64_t* ticket);
int w1_poll(w1_handle h, uint64_t ticket, w1_result* out, double* m1,
            double* m2, double* psi);
/* Engine counters since w1_plan, both precisions: [0] host steps (one
 * synchronisation each), [1] level starts, [2] work-list uploads,
 * [3] iteration blocks queued, [4] block sequences captured into HIP
 * graphs (W1_GRAPH=1 in the environment: plain-only steps replay their
 * block sequence from a graph while the slot set is unchanged).            */
int w1_engine_counters(w1_handle h, int64_t* out5);
/* Return to the device the idle solve-state blocks that finished solves
 * left in the process-wide cache (kept for reuse up to W1_BLOCK_CACHE_BYTES
 * in the environment, default 4 GiB).  Blocks in use are not touched, so
 * it may be called while solves run; released_bytes (host, may be NULL)
 * receives their size.  A failed device allocation anywhere in the library
 * does this by itself and tries once more.  Returns W1_OK.                 */
int w1_trim_cache(size_t* released_bytes);
/* Block until every submitted request is done.                             */
int w1_drain(w1_handle h);
/* Served-mode counters: [0] admitted, [1] finished, [2] queued now,
 * [3] running now, [4] device bytes in use, [5] peak device bytes.        */
int w1_serve_stats(w1_handle h, int64_t* out6);

int w1_destroy(w1_handle h);
const char* w1_strerror(int status);

/* ---- single-step entry points ------------------------------------------
 * These run one row of the method on caller-owned device buffers of a
 * single grid level (dense layout, pitch n+1), queued on `hip_stream`
 * (NULL = default stream) and synchronised before return.  `precision`
 * selects float (W1_FP32) or double (W1_FP64) element type for every
 * array argument typed `void*`.
 */

/* Input preparation and restriction (Sec. 2.2; coarse densities by
 * normalised full weighting D^-1 P^T, P the interpolation of eq.
 * (inter_phi), renormalised to unit mass): from finest node masses p0, p1
 * (double, device) produce rho_l = rho0_l - rho1_l (zero-sum) for every
 * level, written to rho_out[l] (element type by precision), l = 0 coarsest.
 * Returns W1_EINVAL for non-finite, negative or unbalanced masses.        */
int w1_op_prepare(int32_t n, int32_t levels, int32_t precision,
                  const double* p0, const double* p1, void* const* rho_out,
                  void* hip_stream);

/* Prolongation, eq. (inter_phi) for the potential and eq. (inter_m) for
 * the flux / edge dual, from side nc to 2 nc.  Any of the pairs may be
 * NULL to skip it.                                                         */
int w1_op_prolong(int32_t nc, int32_t precision,
                  const void* c_m1, const void* c_m2, const void* c_phi,
                  void* f_m1, void* f_m2, void* f_phi, void* hip_stream);

/* `steps` iterations of eq. (primaldual) in place on (m1, m2, phi), with
 * mu = tau = step_scale * h / (2 sqrt 2) (step_scale <= 0: 1/2; at most 1,
 * else W1_EINVAL).  fpr_out (host, may be NULL) receives R^k of the last step
 * (eq. (pd_stop)).  block_steps > 0 (at most 26) fuses that many steps per
 * tiled launch, block_steps < 0 runs the whole-level LDS kernel (n <= 64);
 * waves (0, 8 or 16) splits each tiled region over that many wavefronts,
 * region_width (0 or 128: 64 x 128 regions; 64: 64 x 64 regions, at most 16
 * steps per launch) sets the region's columns, region_height (0 or 64; 32
 * with region_width 64 and waves 8: 32 x 64 regions, at most 10 steps per
 * launch) its rows.  Every choice gives the same iterates bit for bit.     */
int w1_op_plain_steps(int32_t n, int32_t metric, int32_t precision,
                      double step_scale, int32_t steps, int32_t block_steps,
                      int32_t waves, int32_t region_width,
                      int32_t region_height, void* m1, void* m2, void* phi,
                      const void* rho, double* fpr_out, void* hip_stream);

/* `steps` iterations of eq. (pdhg) in place on (m1, m2, vphi1, vphi2,
 * vphibar1, vphibar2), mu = tau = step_scale (<= 0: 1/2; at most 1).  fpr_out
 * receives G^k of the last step (eq. (pdhg_stop)).  resident = 1 runs all
 * steps in one workgroup with the level in LDS (FP32, n <= 64; W1_EINVAL
 * otherwise), 0 the batched kernels (one launch sequence per step).       */
int w1_op_prox_steps(int32_t n, int32_t metric, int32_t precision,
                     double step_scale, int32_t steps, int32_t resident,
                     void* m1, void* m2, void* w1, void* w2,
                     void* wb1, void* wb2, const void* rho,
                     double* fpr_out, void* hip_stream);

/* Neumann Poisson solve u = (A A*)^{-1} r (zero-mean part; the projection
 * of eq. (pdhg) and Appendix B) by orthonormal DCT-II / DCT-III of length
 * n+1 per axis.  r and u may alias.                                        */
int w1_op_poisson(int32_t n, int32_t precision, const void* r, void* u,
                  void* hip_stream);

/* w1_op_poisson without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and kernels as w1_op_poisson
 * (r, u: device, dense (n+1)^2, may alias); 1 <= n <= 512, else W1_EINVAL
 * before any device call.  Its working memory (DCT tables, two planes, the
 * descriptor and work list) is a static device array of w1_noalloc_bytes()
 * bytes per GPU, held until the process ends and rewritten by every call;
 * calls that overlap on one GPU (other streams or threads) race and must
 * be serialised by the caller.  Queued on hip_stream (NULL: the default
 * stream) without a host synchronisation: u is ready when the stream
 * reaches the end of the call's work.                                     */
int w1_op_poisson_noalloc(int32_t n, int32_t precision, const void* r,
                          void* u, void* hip_stream);
size_t w1_noalloc_bytes(void);

/* Appendix B: psi = (A A*)^{-1} A vphi, zero mean.                        */
int w1_op_potential(int32_t n, int32_t precision, const void* w1,
                    const void* w2, void* psi, void* hip_stream);

/* FP64 certificate of a flux m and usual-sign potential psi against rho:
 * out[0] = P = f(m), out[1] = D = <psi, rho>_h,
 * out[2] = lo = D / max(1, max ||grad psi||_q),
 * out[3] = hi = f(m - A*(AA*)^{-1}(A m - rho)),
 * out[4] = kkt = max(||A*(AA*)^{-1}(Am - rho)||_{L2h}/P, RMS Lipschitz
 *          excess of psi, |P - D| / max(P, |D|)),
 * out[5] = max ||grad psi||_q.  out is host memory (6 doubles).           */
int w1_op_evaluate(int32_t n, int32_t metric, int32_t precision,
                   const void* m1, const void* m2, const void* psi,
                   const void* rho, double* out, void* hip_stream);

/* ---- d = 3 ---------------------------------------------------------------
 * The method is stated for any d (Sec. 2.2: the divergence sums D_{h,i} over
 * the d axes; Sec. 3.3: the interpolations are products of 1-D factors).
 * These run Algorithms 1 / 3 and 2 / 4 on the (n+1)^3 vertex grid of
 * [0,1]^3, one pair per call synchronously on `hip_stream` (NULL = default
 * stream), or a list of pairs over streams of their own
 * (w1_solve3d_batch).  Arrays are dense, index (i1 (n+1) + i2) (n+1) + i3,
 * i3 contiguous.
 */

/* Algorithm 3 (algo W1_ALGO_PLAIN) or 4 (W1_ALGO_PROX) in d = 3.  p0, p1:
 * node masses ((n+1)^3 doubles each, host or device by on_device; copied
 * before use, caller-owned).  Parameters as for w1_plan, with these limits:
 * tol > 0 (the paper's eq. (stop_tol) is fitted to its d = 2 experiments;
 * no default), n <= 1024; steps mu = tau = step_scale / (2 sqrt 3 / h)
 * (Algorithm 3) or step_scale (Algorithm 4).  out: w1 = f(m^K) =
 * sum ||m||_p h^3, dual = <psi, rho>_h with psi = -phi (Algorithm 3) or
 * (A A*)^{-1} A vphi (Appendix B), the certified bracket lo <= W1_h <= hi
 * (psi scaled to the Lipschitz constraint; m made feasible by the
 * minimum-norm correction), kkt = max(||A m - rho|| / ||rho||, RMS
 * Lipschitz excess, relative gap), per-level iterations, measures,
 * f(m^{K_l}) and times.  m_out (3 (n+1)^3 doubles: m1, m2, m3) and psi_out
 * ((n+1)^3 doubles) are optional host buffers.  W1_EINVAL also for
 * unbalanced, negative or non-finite masses; W1_ENOMEM when the
 * (n+1)^3 (16 sizeof(iterate) + 16) bytes per level do not fit.          */
int w1_solve3d(const w1_params* params, const double* p0, const double* p1,
               int32_t on_device, w1_result* out, double* m_out,
               double* psi_out, void* hip_stream);

/* w1_solve3d over `count` pairs (p0[i], p1[i], all host or all device by
 * on_device; out[i] their results, no fields) by `workers` host threads
 * (1..16, 0 = 4), each with its own stream and device block, taking the
 * pairs in turn, so the small levels of different pairs overlap on the
 * device.  Results equal those of w1_solve3d pair by pair.  Returns the
 * first error any pair met (the pairs after it are not started).         */
int w1_solve3d_batch(const w1_params* params, int32_t count,
                     const double* const* p0, const double* const* p1,
                     int32_t on_device, w1_result* out, int32_t workers);

/* `steps` iterations of eq. (primaldual) in d = 3 in place on device arrays
 * (m1, m2, m3, phi), rho read only, element type by precision, mu = tau =
 * step_scale / (2 sqrt 3 / h) (step_scale <= 0: 1/2; at most 1).  fpr_out
 * (host, may be NULL) receives R^k of the last step (eq. (pd_stop)).      */
int w1_op_plain_steps3d(int32_t n, int32_t metric, int32_t precision,
                        double step_scale, int32_t steps, void* m1, void* m2,
                        void* m3, void* phi, const void* rho, double* fpr_out,
                        void* hip_stream);

/* `steps` iterations of eq. (pdhg) in d = 3 in place on device arrays
 * (m1..m3, vphi1..vphi3, vphibar1..vphibar3), rho read only, mu = tau =
 * step_scale (<= 0: 1/2; at most 1).  fpr_out (host, may be NULL)
 * receives G^k of the last step (eq. (pdhg_stop)).                        */
int w1_op_prox_steps3d(int32_t n, int32_t metric, int32_t precision,
                       double step_scale, int32_t steps, void* m1, void* m2,
                       void* m3, void* w1, void* w2, void* w3, void* wb1,
                       void* wb2, void* wb3, const void* rho, double* fpr_out,
                       void* hip_stream);

/* ---- kernel timing ------------------------------------------------------
 * w1_profile(h, 1) resets and enables per-launch HIP-event timing on the
 * handle's stream (0 disables it; negative values are W1_EINVAL).  Plain
 * tiled launches take the events into the dispatch itself (their start and
 * end times); a timed dispatch ends with a cache flush, so w1_profile(h, k)
 * with k > 1 times only about one launch in k (a fixed pseudo-random
 * sample) of the tiled and the Algorithm 2 families; the whole-level
 * resident launches are timed every time.
 * w1_kernel_stats(h, family, out) then returns for one kernel family, summed
 * over both precisions and over the timed launches:
 *   out[0] launches timed, out[1] total milliseconds,
 *   out[2] node updates (one node of one PDHG iteration), out[3] algorithmic
 *   HBM bytes (per family: plain tiled 7 words per node update; prox
 *   elementwise 13 words per node per iteration; DCT pass 2 words per node
 *   per pass; resident 0), out[4] floating-point operations (DCT passes)
 *   or, for the plain tiled family, the node updates its launches compute
 *   (the overlapping halo of the temporal blocks included), out[5] the
 *   family's launches while timing was on, timed or not.  Node updates and
 *   bytes are those the launch was issued for: a slot that stops inside a
 *   step's queued blocks is skipped by the device but still counted.
 * Families: W1_FAM_PLAIN_TILED, W1_FAM_PLAIN_RESIDENT, W1_FAM_DCT,
 * W1_FAM_PROX_ELEM, W1_FAM_OTHER, W1_FAM_PROX_RESIDENT (whole small prox
 * levels in one workgroup; resident families count node updates only).    */
enum { W1_FAM_PLAIN_TILED = 0, W1_FAM_PLAIN_RESIDENT = 1, W1_FAM_DCT = 2,
       W1_FAM_PROX_ELEM = 3, W1_FAM_OTHER = 4, W1_FAM_PROX_RESIDENT = 5,
       W1_NFAM = 6 };
int w1_profile(w1_handle h, int32_t enable);
int w1_kernel_stats(w1_handle h, int32_t family, double* out6);

/* ---- launch-shape autotuner ---------------------------------------------
 * The plain tiled kernel's temporal depth and wavefronts per workgroup are
 * picked per (precision, check_every, requested depth, size class of the
 * active set) by timing each candidate on a few live iteration blocks and
 * keeping the fastest; all candidates give the same iterates bit for bit.
 * The table is process-wide.  w1_tuner_table writes it as JSON text into
 * buf (len bytes, NUL-terminated, truncated if short) and returns the full
 * length; w1_tuner_reset forgets every measurement.                        */
int w1_tuner_table(char* buf, size_t len);
int w1_tuner_reset(void);

/* Library version string.                                                  */
const char* w1_version(void);

#ifdef __cplusplus
}
#endif
#endif /* W1_H */
