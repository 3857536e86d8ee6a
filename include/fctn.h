/*
 * fctn.h - C ABI of libfctn.so: trace-regularized fully-connected tensor
 * network (FCTN) tensor completion solved by proximal alternating
 * minimization (PAM), on one AMD Instinct MI355X (gfx950).
 *
 * The operation (arXiv 2510.22506, Section 3):
 *   min over A_1..A_N, X of
 *     1/2 ||X - FCTN(A_1..A_N)||_F^2 + sum_k lambda_k/2 tr(A_k(k)^T L_k A_k(k))
 *   subject to P_Omega(X - Y) = 0                         (eq. model_1)
 * solved by PAM sweeps (Algorithms 1-2): for each k the factor A_k solves the
 * Sylvester equation A G + lambda_k L_k A + rho A = X_(k) M_k^T + rho A_k^t
 * with G = M_k M_k^T and M_k the sub-network of the other factors
 * (Property 1, eq. 4-9); then X = P_Omega^c((FCTN(A) + rho X)/(1 + rho))
 * + P_Omega(Y) (eq. 10).  L_k is the periodic negative Laplacian
 * (2 + delta_k) I - S - S^T (S the cyclic shift; positive definite).
 *
 * Conventions for every entry point
 *   - Dense tensors (Y, X, Z, mask) are row-major ("C order": the last mode
 *     varies fastest), prod(dims) elements, on the device.
 *   - Factor A_k is row-major with the modes (R_1k, .., R_{k-1,k}, I_k,
 *     R_{k,k+1}, .., R_kN) (Section 1, FCTN factor shapes).
 *   - The rank vector is R_12, R_13, .., R_1N, R_23, .., R_{N-1,N}
 *     (Section 1, r_FCTN).
 *   - Storage type ("elem") of Y, X and Z is double for FCTN_F64 and float
 *     for every other precision.
 *   - All device pointers are caller-owned and must stay valid while the plan
 *     uses them.  The library never allocates or frees device memory: all
 *     its state lives in the caller's workspace `ws_dev`.
 *   - Calls are asynchronous on the plan's HIP stream, except those that
 *     fill host-side results (stats, flags); those synchronize the stream.
 *   - Every call returns fctn_status; nothing throws across the boundary.
 *     After FCTN_E_DEVICE the plan is unusable (the error is sticky).  Besides
 *     failed HIP calls, FCTN_E_DEVICE reports a kernel whose bounded internal
 *     wait gave up (its result is then invalid); that is detected at the
 *     next call that synchronizes to return host-side results.
 *   - Calls on one plan are not thread-safe; distinct plans are independent.
 */
#ifndef FCTN_H
#define FCTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCTN_MAX_ORDER 8
#define FCTN_MAX_BONDS 28

typedef enum {
  FCTN_OK = 0,
  FCTN_E_INVALID = 1,      /* bad descriptor, pointer, size or index      */
  FCTN_E_NOMEM = 2,        /* workspace smaller than fctn_workspace_bytes */
  FCTN_E_DEVICE = 3,       /* a HIP runtime call failed                   */
  FCTN_E_NUMERIC = 4,      /* non-finite observed value on Omega          */
  FCTN_E_UNSUPPORTED = 5,  /* valid for the method, not supported here    */
  FCTN_E_CANCELLED = 6     /* a served request cancelled by the caller    */
} fctn_status;

typedef enum {
  FCTN_F64 = 0,    /* every product and reduction in double                 */
  FCTN_F32 = 1,    /* float contractions on MFMA, double reductions/solves  */
  FCTN_BF16 = 2,   /* bf16 operands on MFMA, float accumulation             */
  FCTN_BF16X3 = 3  /* split bf16 (hi*hi + hi*lo + lo*hi), float accumulation */
} fctn_precision;

typedef struct fctn_plan_s* fctn_plan_t;

/* Problem descriptor: the inputs of Algorithms 1-2 apart from Y and Omega. */
typedef struct {
  int32_t order;                    /* N; supported: N = 3 .. 8              */
  int64_t dims[FCTN_MAX_ORDER];     /* I_1 .. I_N, each >= 1                 */
  int32_t ranks[FCTN_MAX_BONDS];    /* r_FCTN in the order above, each >= 1  */
  double lambda[FCTN_MAX_ORDER];    /* lambda_k >= 0 (eq. model_1)           */
  double delta[FCTN_MAX_ORDER];     /* delta_k > 0 (L_k, Section 3.1)        */
  double rho;                       /* proximal weight rho > 0 (eq. 3)       */
  int32_t precision;                /* fctn_precision                        */
  int32_t reuse;                    /* 1: Algorithm 2 (Sections 3.3-3.4):
                                       for N = 4 the pair tensors A1xA2 and
                                       A3xA4, for N >= 5 the prefix groups
                                       A1..Aj and suffix groups Aj..AN (each
                                       grown by one factor from its neighbour)
                                       are cached and rebuilt only when one of
                                       their factors changed.  0: Algorithm 1's
                                       work: every mode's sub-network and the
                                       FCTN(A) of the X step are contracted
                                       from the factors, rebuilding the pair
                                       or the group chain each time.  Both run
                                       the same kernels on the same operands,
                                       so their iterates are bitwise equal;
                                       only the contraction work differs
                                       (Tables 1-2).  For N = 3 nothing is
                                       cached and the flag has no effect     */
  int32_t order_policy;             /* 0: factor order 1..N every sweep;
                                       1: for N = 4 alternate (1,2,3,4) and
                                       (3,4,1,2) so a cached pair carries over
                                       (Algorithm 2's permuted order)        */
  double extrap_alpha;              /* asymmetric extrapolation (Section 4.2,
                                       multi-temporal images): after each
                                       factor's subproblem, A_k <- A_k +
                                       alpha (A_k - beta A_k^t), A_k^t the
                                       factor the subproblem started from.
                                       0 = off; otherwise 0 < alpha < 1     */
  double extrap_beta;               /* beta in [0, 1] (the paper uses 0.5)   */
} fctn_desc;

/* Per-sweep scalars (Algorithm 1 stopping rule; Section 3.5 objective f). */
typedef struct {
  double rel_change;   /* ||X^{t+1} - X^t||_F / ||X^t||_F                    */
  double f_data;       /* 1/2 ||X^{t+1} - FCTN(A^{t+1})||_F^2                 */
  double f_trace;      /* sum_k lambda_k/2 tr(A_k(k)^T L_k A_k(k))            */
  double objective;    /* f_data + f_trace                                   */
  float ms_stage[8];   /* kernel milliseconds of the sweep per stage
                          (FCTN_STAGE_* below), filled by fctn_sweep while
                          per-kernel timing is on; 0 otherwise              */
} fctn_sweep_stats;

typedef struct {
  int32_t sweeps_done;
  double rel_change;
  double objective;
} fctn_stats;

/* Exact device workspace (bytes) a plan for `desc` needs; 0 if the
 * descriptor is invalid or unsupported. */
size_t fctn_workspace_bytes(const fctn_desc* desc);

/* Create a plan.  ws_dev: caller-owned device buffer of at least
 * fctn_workspace_bytes(desc) bytes, 256-byte aligned; hip_stream: the
 * hipStream_t all work is queued on (NULL = the null stream).  Builds the
 * Fourier eigenbases of every L_k (eq. 7) on the device and sets the initial
 * factors (Algorithm 1, initialization: standard normal entries): A0_host[k]
 * is factor k in float64 with the factor layout above (host memory, copied
 * before the call returns), or, if A0_host is NULL, the factors are drawn
 * from `seed` with a counter-based generator: SplitMix64 words
 * w_j = mix(seed + (j + 1) * 0x9E3779B97F4A7C15), pairs of words turned into
 * pairs of normals by the Box-Muller transform (u1 = (w >> 11) + 1 and
 * u2 = w >> 11 scaled by 2^-53; sqrt(-2 ln u1) cos(2 pi u2), then sin), factor
 * 1's entries first.  Synchronizes the stream.  Errors: FCTN_E_INVALID for a
 * bad descriptor, pointer or alignment (or a NULL A0_host[k]),
 * FCTN_E_UNSUPPORTED for a valid problem this library does not run,
 * FCTN_E_NOMEM if ws_bytes is too small, FCTN_E_DEVICE for a failed HIP
 * call. */
fctn_status fctn_plan(const fctn_desc* desc, void* ws_dev, size_t ws_bytes,
                      void* hip_stream, const double* const* A0_host, uint64_t seed,
                      fctn_plan_t* out);

/* Initial factors (Algorithm 1, initialization: standard normal entries).
 * A_host[k]: host pointer to factor k in float64 with the factor layout
 * above.  Copied (synchronously) to the device; the working-precision copy is
 * the round-to-nearest-even cast. */
fctn_status fctn_set_factors(fctn_plan_t plan, const double* const* A_host);

/* Initial factors from device memory: A_dev holds factor 1, factor 2, ..,
 * factor N in float64, each with the factor layout above, back to back.
 * Asynchronous on the plan's stream (A_dev must stay valid until the copy
 * has run). */
fctn_status fctn_set_factors_dev(fctn_plan_t plan, const double* A_dev);

/* Observed data (Algorithm 1: X^(1) = Y, read as P_Omega(Y)).  Y_dev: elem
 * tensor; mask_dev: uint8 tensor, nonzero = observed.  Values of Y off Omega
 * are never read into arithmetic (they may be NaN).  Y and mask are copied
 * into the workspace; the caller may free them afterwards.  Returns
 * FCTN_E_NUMERIC (after a stream sync) if any observed value is not finite. */
fctn_status fctn_set_observed(fctn_plan_t plan, const void* Y_dev,
                              const uint8_t* mask_dev);

/* Overwrite X (elem tensor on the device); for step-level checks and for
 * resuming a run. */
fctn_status fctn_set_x(fctn_plan_t plan, const void* X_dev);

/* Checkpoint and resume.  The sweep index t is the number of sweeps the run
 * has done; it selects the next sweep's factor order (the alternating order
 * of Section 3.3 for N = 4).  A run's state is X (fctn_get_x), the float64
 * factors (fctn_get_factor) and t: a plan with the same descriptor that is
 * given them (fctn_set_x, fctn_set_factors or fctn_set_factors_dev, then
 * fctn_set_sweep_index) after fctn_set_observed continues the run bit for
 * bit.  fctn_set_sweep_index also restarts the per-sweep history at t
 * (fctn_get_history then serves sweeps t and later).  t < 0 is
 * FCTN_E_INVALID. */
fctn_status fctn_get_sweep_index(fctn_plan_t plan, int64_t* t_host);
fctn_status fctn_set_sweep_index(fctn_plan_t plan, int64_t t);

/* Rank growth (Algorithms 1-2 start from rank ones and grow to the maximal
 * FCTN-rank; the growth rule is deferred to the paper's reference [Zheng2022]).
 * `to` is a plan with the same order, dims and precision as `from` and every
 * bond rank >= from's.  Copies from's X and observed mask into `to` and embeds
 * from's float64 factors: old entries are kept; an entry whose index along a
 * bond (j, k), j < k, is new is zero; every other new entry of factor k is
 * read from fill_dev (float64, the factors at to's ranks back to back, as for
 * fctn_set_factors_dev).  FCTN(A) and X are unchanged by the growth.  Waits
 * for from's stream, runs on to's stream and synchronizes it, so `from` may be
 * destroyed on return.  `to` starts at sweep 0 (its cached pairs are rebuilt). */
fctn_status fctn_regrow(fctn_plan_t to, fctn_plan_t from, const double* fill_dev);

/* Run `nsweeps` PAM sweeps (Algorithm 1 or 2 by desc.reuse).  If stats_host
 * is not NULL it receives the scalars of the last sweep and, with per-kernel
 * timing on (fctn_profile_enable), that sweep's kernel time per stage
 * (synchronizes). */
fctn_status fctn_sweep(fctn_plan_t plan, int32_t nsweeps,
                       fctn_sweep_stats* stats_host);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same `nsweeps` sweeps as fctn_sweep (results bit for bit equal), with the
 * split-K partial products of the Gram/right-hand-side pass (eq. 5) kept in
 * a static device array owned by the library (64 MiB, allocated on each
 * device when the library's code is loaded there and held until the process
 * ends) instead of the plan's workspace.  Calls nothing that allocates.
 * Returns FCTN_E_NOMEM if the plan's partial products exceed 64 MiB (e.g.
 * float64 plans of large tensors; fctn_sweep serves those).  Every plan on
 * one device shares that array: calls of this entry point that overlap in
 * time on one device (plans on different streams, or different threads)
 * race and must be serialized by the caller.  No stats: read them with
 * fctn_get_history. */
fctn_status fctn_sweep_noalloc(fctn_plan_t plan, int32_t nsweeps);

/* Run `nsweeps` sweeps on each of `count` independent plans, interleaving
 * their launches across the plans' streams so that their work overlaps on the
 * device (request batching).  Each plan's results equal those of fctn_sweep
 * on that plan alone, bit for bit. */
fctn_status fctn_sweep_many(fctn_plan_t* plans, int32_t count, int32_t nsweeps);

/* Algorithms 1-2 run to their stopping rule (Section 3.2: stop once
 * ||X^{t+1} - X^t||_F / ||X^t||_F <= epsilon, or after the iteration limit).
 * Runs up to max_sweeps sweeps, stopping after the first sweep whose relative
 * change is <= tol (tol <= 0: exactly max_sweeps sweeps).  The test reads the
 * relative change back to the host every `check_every` sweeps (>= 1), so with
 * check_every > 1 the run stops at the first multiple of check_every whose
 * sweep passes the test.  Copies X to X_out_dev if not NULL.  Fills
 * stats_host if not NULL; then the call synchronizes the stream, X_out
 * included.  Errors: FCTN_E_INVALID for a NULL plan, max_sweeps < 0 or
 * check_every < 1; FCTN_E_DEVICE (sticky) if a HIP call fails. */
fctn_status fctn_complete(fctn_plan_t plan, int32_t max_sweeps, double tol,
                          int32_t check_every, void* X_out_dev,
                          fctn_stats* stats_host);

/* Per-sweep history: the scalars of sweeps [first, first + count) counted
 * from the plan's creation (at most the last 4096 sweeps are kept). */
fctn_status fctn_get_history(fctn_plan_t plan, int32_t first, int32_t count,
                             fctn_sweep_stats* out_host);

/* Copy X (elem tensor) to dst_dev. */
fctn_status fctn_get_x(fctn_plan_t plan, void* dst_dev);

/* Copy the float64 master copy of factor k (factor layout) to dst_dev. */
fctn_status fctn_get_factor(fctn_plan_t plan, int32_t k, double* dst_dev);

/* ---- single steps of one sweep, on the plan's current state ------------
 * For step-level checks and profiling; a sweep is these steps in order.   */

/* Gram and right-hand side of eq. 5 for mode k from the current factors and
 * X: G_dev (s_k x s_k) = M_k M_k^T and B_dev (I_k x s_k) = X_(k) M_k^T +
 * rho A_k(k), both float64 row-major.  The s_k index is the bond multi-index
 * of A_k in its mode order with the last bond fastest; the columns of M_k
 * and X_(k) are the other physical indices, last fastest.  For N = 4 the
 * needed pair tensor is (re)built first; for N >= 5 the mode's operand
 * groups (contractions of consecutive factors) are, where stale. */
fctn_status fctn_step_gram_rhs(fctn_plan_t plan, int32_t k, double* G_dev,
                               double* B_dev);

/* Solve eq. 5 for mode k given G_dev, B_dev (layouts as above, float64) and
 * store the result as factor k (eq. 8-9), extrapolated against the previous
 * factor k when the descriptor's extrap_alpha > 0 (Section 4.2).  Returns
 * tr(A^T L_k A) of the stored factor in *trace_host if not NULL
 * (synchronizes). */
fctn_status fctn_step_solve(fctn_plan_t plan, int32_t k, const double* G_dev,
                            const double* B_dev, double* trace_host);

/* Z = FCTN(A_1..A_N) from the current factors, computed as
 * A_k(k) M_k with M_k regenerated from the factors (X step of Algorithm 2,
 * M'_k with k = last); written as an elem tensor to Z_dev. */
fctn_status fctn_step_reconstruct(fctn_plan_t plan, int32_t k, void* Z_dev);

/* eq. 10 on the plan's X with the given Z (elem tensor): X = Omega ? X :
 * (Z + rho X)/(1 + rho).  stats_host (nullable) gets rel_change and f_data
 * (f_trace and objective are 0; synchronizes). */
fctn_status fctn_step_x_update(fctn_plan_t plan, const void* Z_dev,
                               fctn_sweep_stats* stats_host);

/* Sizes of the plan's unfoldings for mode k: s_k and I_k. */
fctn_status fctn_mode_sizes(const fctn_desc* desc, int32_t k, int64_t* s_k,
                            int64_t* I_k);

/* ---- serving: continuous batching of independent completions -------------
 * A server keeps many completions (each one plan, as above) resident at once
 * and runs their sweeps concurrently.  It owns no memory of its own on the
 * device: every admitted request's plan is carved from the caller's arena, so
 * admission is by exact memory footprint (fctn_workspace_bytes).  Requests
 * are admitted first in first out whenever a slot (max_active) and arena
 * room are free; each admitted request's sweeps go to one of the caller's
 * streams (round robin), at most `depth` of them queued at a time, one
 * sweep per request per round, so requests that share a stream interleave
 * and requests on different streams overlap on the device.  A request's
 * result is that of fctn_plan + fctn_set_factors_dev + fctn_set_observed +
 * fctn_sweep(sweeps) on it alone, bit for bit: the plans share no state and
 * every kernel is deterministic.  The server is driven by fctn_server_step,
 * which never blocks; calls on one server are not thread-safe. */
typedef struct fctn_server_s* fctn_server_t;

typedef struct {
  fctn_desc desc;           /* the completion problem                         */
  const void* Y_dev;        /* observed tensor, elem (see conventions)        */
  const uint8_t* mask_dev;  /* uint8, nonzero = observed                      */
  const double* A0_dev;     /* initial factors, as for fctn_set_factors_dev   */
  void* X_out_dev;          /* receives the completed X (elem tensor)         */
  int32_t sweeps;           /* fixed number of PAM sweeps (>= 0)              */
  uint64_t tag;             /* caller's identifier, returned on completion    */
} fctn_request;
/* Y_dev, mask_dev, A0_dev and X_out_dev must stay valid until the request's
 * completion has been returned. */

typedef struct {
  uint64_t tag;
  int32_t status;           /* FCTN_OK; FCTN_E_NUMERIC: a non-finite
                               observed value (the sweeps still ran);
                               FCTN_E_DEVICE: a kernel's bounded wait gave
                               up, the result is invalid; FCTN_E_CANCELLED:
                               fctn_server_cancel stopped it (see there)     */
  int32_t sweeps_done;
  double rel_change;        /* of the last sweep (eq. 10 stopping quantity)   */
  double objective;         /* f after the last sweep (Section 3.5)           */
  double t_submit, t_admit, t_done;  /* host CLOCK_MONOTONIC, seconds        */
} fctn_completion;

/* arena_dev: caller-owned device buffer, 256-byte aligned, the memory budget
 * of all admitted requests together; streams: nstreams hipStream_t handles;
 * max_active >= 1 requests resident at once; depth >= 1 sweeps queued per
 * request.  Allocates pinned host memory for the completion scalars. */
fctn_status fctn_server_create(void* arena_dev, size_t arena_bytes,
                               void* const* streams, int32_t nstreams,
                               int32_t max_active, int32_t depth,
                               fctn_server_t* out);

/* Queue a request (copied).  FCTN_E_NOMEM if its footprint exceeds the
 * whole arena (it could never be admitted); FCTN_E_INVALID /
 * FCTN_E_UNSUPPORTED for a descriptor fctn_plan would reject. */
fctn_status fctn_server_submit(fctn_server_t server, const fctn_request* req);

/* Non-blocking progress: retire finished requests (their X has been copied
 * out) into done[0 .. *n_done) (at most max_done), admit queued requests,
 * and queue further sweeps of the admitted ones. */
fctn_status fctn_server_step(fctn_server_t server, fctn_completion* done,
                             int32_t max_done, int32_t* n_done);

/* Cancel the request with this tag.  A queued request is dropped: its
 * completion (FCTN_E_CANCELLED, sweeps_done 0, X_out untouched) comes with
 * the next fctn_server_step.  A resident request queues no further sweeps:
 * once the sweeps already queued have run, X_out receives X after them and
 * the completion reports FCTN_E_CANCELLED with that sweep count and its
 * scalars (unless a device error takes precedence).  FCTN_E_INVALID if no
 * queued or resident request that is still sweeping has the tag (the first
 * one found is cancelled when tags repeat). */
fctn_status fctn_server_cancel(fctn_server_t server, uint64_t tag);

/* Queue length, resident requests and arena bytes in use (any may be NULL). */
fctn_status fctn_server_query(fctn_server_t server, int32_t* queued,
                              int32_t* active, size_t* arena_used);

/* Waits for all of the server's streams, then releases its host state. */
fctn_status fctn_server_destroy(fctn_server_t server);

/* ---- per-kernel timing ---------------------------------------------------
 * Stages, one per kernel of a sweep: */
enum {
  FCTN_STAGE_PAIR = 0,        /* pair tensor (N = 4) or operand groups (N >= 5) */
  FCTN_STAGE_GRAM_RHS = 1,    /* fused M_k generation + Gram + RHS (eq. 5)   */
  FCTN_STAGE_REDUCE = 2,      /* float64 split-K reduction (+ rho A_k)        */
  FCTN_STAGE_SOLVE = 3,       /* per-class Cholesky solves (eq. 5-8)          */
  FCTN_STAGE_TRANSFORM = 4,   /* basis changes Q^T B and Q A~ (eq. 8), fold
                                 (eq. 9), casts                              */
  FCTN_STAGE_RECONSTRUCT = 5, /* Z = A_last M'_last (Algorithm 2, X step)    */
  FCTN_STAGE_XUPDATE = 6,     /* eq. 10 select + norm partials               */
  FCTN_STAGE_STATS = 7,       /* per-sweep scalars                           */
  FCTN_NSTAGES = 8
};

typedef struct {
  int64_t launches[FCTN_NSTAGES];
  double ms[FCTN_NSTAGES];      /* summed kernel time from HIP events         */
  double flops[FCTN_NSTAGES];   /* summed algorithmic flops of those launches */
  double bytes[FCTN_NSTAGES];   /* summed algorithmic HBM bytes               */
} fctn_profile;

/* Enable (1) or disable (0) per-launch HIP event pairs on the plan's stream.
 * Algorithmic flops count 2 per multiply-add of the paper's dense products
 * (sub-network generation, the full s_k x s_k Gram, the RHS, the
 * reconstruction, the pair tensors); algorithmic bytes count each tensor
 * read or written once. */
fctn_status fctn_profile_enable(fctn_plan_t plan, int32_t enable);

/* Accumulate every recorded launch into *out (synchronizes); reset != 0
 * clears the recorded launches afterwards. */
fctn_status fctn_profile_read(fctn_plan_t plan, fctn_profile* out, int32_t reset);

/* Release the plan's host state (the workspace stays the caller's). */
fctn_status fctn_destroy(fctn_plan_t plan);

const char* fctn_status_str(fctn_status status);

#ifdef __cplusplus
}
#endif

#endif /* FCTN_H */
