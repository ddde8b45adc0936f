/*
 * smol.h -- C ABI of libsmol, an MI355X (gfx950) solver for the truncated
 * aggregation-shattering Smoluchowski system with a low-rank kernel.
 *
 * Method: Matveev, Zhilin, Smirnov, "Adaptive time-stepping for
 * aggregation-shattering kinetics" (arXiv 2407.16559).
 *
 * Conventions shared by every entry point
 *   - Sizes s = 1..M are stored at index s-1.
 *   - The kernel K_{ij} = sum_{a<R} U_{i a} V_{a j} (Sec. 1, display after
 *     Eq. (2)).  Both factors are stored alpha-major as R x M row-major
 *     arrays: U[a*M + i-1] and V[a*M + j-1], FP64.
 *   - Array arguments are DEVICE pointers owned by the caller (for example
 *     torch tensors' data_ptr()).  The library never frees caller memory.
 *     It owns only cached plans and workspaces, keyed by (device, M, R,
 *     precision), which smol_release_plans() frees.
 *   - `stream` is a hipStream_t; NULL means the null stream.
 *   - Every call returns an int status (SMOL_OK or a negative code) and
 *     never throws across the ABI.  smol_strerror() names a code.
 *   - Calls that share a plan (same device, M, R, precision) reuse its
 *     workspaces.  The library orders them: work a call enqueues on one
 *     stream waits (hipStreamWaitEvent) for the plan's previous work on
 *     another stream.  Under HIP graph capture that ordering is not added;
 *     the capturing caller orders captured calls that share a plan.  Host
 *     threads are serialised by a library lock.
 */
#ifndef SMOL_H
#define SMOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SMOL_OK = 0,
    SMOL_EINVAL = -1,      /* bad size, pointer, tolerance, lambda or option */
    SMOL_ENOMEM = -2,      /* device allocation failed */
    SMOL_EDEVICE = -3,     /* a HIP call failed */
    SMOL_ESTEPSIZE = -4,   /* step fell below max(h_min, 10 ulps of t) */
    SMOL_EMAXSTEPS = -5,   /* step-attempt limit reached */
    SMOL_ENONFINITE = -6,  /* NaN/Inf in the state or a NaN error norm */
    SMOL_EUNSUPPORTED = -7 /* valid request the library does not provide */
};

/* Integration schemes.  SMOL_BS32 and SMOL_DP54 are embedded pairs
 * (first-same-as-last).  The paper's schemes (Sec. 2): SMOL_RKF45 is
 * Runge--Kutta--Fehlberg 4(5) propagating the fourth-order solution, with
 * the fifth-order one for the error estimate; SMOL_RK2_DBL is RK2 (Heun)
 * with step doubling: each attempt takes one step h and two steps h/2,
 * propagates the latter, and estimates the error by their difference;
 * SMOL_RK4_DBL is the same with the classical four-stage RK4 (eleven
 * evaluations per attempt).  Each attempt also evaluates S at its new
 * state, which is the next attempt's first stage (so a rejected attempt
 * costs one evaluation more than the scheme itself needs). */
enum { SMOL_BS32 = 0, SMOL_DP54 = 1, SMOL_RKF45 = 2, SMOL_RK2_DBL = 3, SMOL_RK4_DBL = 4 };

/* Arithmetic of the convolution part of the right-hand side. */
enum { SMOL_FP64 = 0, SMOL_FP32X2 = 1 };

/* Step-size controller.  PI and LEARNED use the weighted-RMS norm below.
 * The paper's rules (Sec. 2) use the Euclidean norm err = ||e||_2 / tol
 * with tol = rtol (atol is ignored), accept iff err <= 1, and set the next
 * step (after acceptance and rejection alike) by
 *   SMOL_CTRL_FEHLBERG:       h *= 0.9 err^(-1/(q+1))  (q = 4 for RKF45:
 *                             the fifth root of Fehlberg's rule)
 *   SMOL_CTRL_STEP_DOUBLING:  h *= s err^(-1/q), Eq. (6), q the scheme's
 *                             order, s = options.safety (default 1/4)
 *   SMOL_CTRL_HALVE_DOUBLE:   h *= 2 after acceptance, 1/2 after rejection
 * with the factor clipped to [0.2, 10] (err = 0 gives 10). */
enum {
    SMOL_CTRL_PI = 0,
    SMOL_CTRL_LEARNED = 1,
    SMOL_CTRL_FEHLBERG = 2,
    SMOL_CTRL_STEP_DOUBLING = 3,
    SMOL_CTRL_HALVE_DOUBLE = 4
};

typedef struct {
    int64_t n_rhs;     /* right-hand-side evaluations, including the two of
                          the starting-step procedure */
    int64_t n_accept;  /* accepted steps */
    int64_t n_reject;  /* rejected step attempts */
    double t;          /* time reached (== t_end on success) */
    double h;          /* next proposed step */
    double err;        /* weighted-RMS error norm of the last attempt */
    int32_t status;    /* SMOL_OK or the code that ended the run */
    int32_t n_fallback;/* learned controller: steps that fell back to PI */
} smol_stats;

/*
 * smol_rhs -- dndt = S(n), the right-hand side of the truncated
 * aggregation-shattering system (Sec. 1, Eq. (2) with the shattering terms
 * of Eq. (4); Sec. 2, Eq. (5) names the operator S):
 *
 *   S_1 = -n_1 sum_i K_{1i} n_i + (lam/2) sum_{i,j>=2} (i+j) K_{ij} n_i n_j
 *         + lam n_1 sum_{j>=2} j K_{1j} n_j
 *   S_s = (1/2) sum_{i+j=s} K_{ij} n_i n_j - (1+lam) n_s sum_i K_{si} n_i,
 *         s = 2..M.
 *
 * The monomer-j shattering gain carries the factor n_1 (mass balance).
 * Evaluated in O(M R log M): the birth sums are R linear convolutions done
 * with FFTs of length L = nextpow2(2M-2), the death and shattering sums are
 * 4R reductions.
 *
 * M >= 1; 1 <= R <= 32; lam >= 0 and finite; n, dndt: M doubles each, on
 * the device; dndt must not alias n.  precision: SMOL_FP64 or SMOL_FP32X2
 * (the convolutions in float-float arithmetic, everything else FP64).
 * Asynchronous on `stream`.  Errors: SMOL_EINVAL, SMOL_ENOMEM,
 * SMOL_EDEVICE, SMOL_EUNSUPPORTED (M so large that the transform would be
 * longer than 2^20).
 */
int smol_rhs(int64_t M, int32_t R, const double *U, const double *V,
             double lambda, const double *n, double *dndt, int32_t precision,
             void *stream);

/* smol_rhs plus constant sources (Eq. (3), the printed P_k read as P_s):
 * dndt = S(n) + source.  source: M doubles on the device, or NULL (no
 * sources); must not alias dndt.  Otherwise as smol_rhs. */
int smol_rhs_ex(int64_t M, int32_t R, const double *U, const double *V,
                double lambda, const double *n, const double *source,
                double *dndt, int32_t precision, void *stream);

/* smol_rhs_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): smol_rhs in FP64 (same kernels and launch schedule) whose
 * workspaces live in one fixed device array of the library (about 9.1 MiB
 * per GPU, held until the process ends) instead of a cached plan.  It calls
 * no hipMalloc, hipFree or other allocating routine; its first call on a
 * device also writes the array's unit-root tables (computed on the device,
 * so results agree with smol_rhs to rounding, not bitwise).
 *
 * Limits: M <= 65537 (transform length <= 2^17) and R <= 4; larger requests
 * return SMOL_EUNSUPPORTED.  Arguments, layout and the other errors as
 * smol_rhs.  Asynchronous on `stream`.  Every call on a GPU uses that GPU's
 * one array: calls that overlap in time on one GPU (different streams
 * without ordering, or different host threads' streams) race and give
 * wrong results; order them on one stream. */
int smol_rhs_noalloc(int64_t M, int32_t R, const double *U, const double *V,
                     double lambda, const double *n, double *dndt,
                     void *stream);

/* Kernels given by a formula (Sec. 3.1), for smol_lowrank. */
enum {
    SMOL_KERNEL_CONSTANT = 1,      /* K_ij = p0 */
    SMOL_KERNEL_BROWNIAN = 2,      /* K_ij = (i/j)^p0 + (j/i)^p0 + p1 */
    SMOL_KERNEL_FREE_MOLECULAR = 3 /* K_ij = (i^(1/3) + j^(1/3))^2 sqrt(1/i + 1/j) */
};

/* smol_lowrank -- low-rank factors K ~= U V (K_ij ~= sum_a U[a*M + i-1]
 * V[a*M + j-1]) of a kernel given by a formula, for kernels with no exact
 * low-rank form such as the free-molecular kernel of Sec. 3.1, so that the
 * O(M R log M) right-hand side and the integrators apply to them.  Adaptive
 * cross approximation with partial pivoting (Bebendorf 2000), on the GPU:
 * each term is one residual row and one residual column of K, evaluated on
 * demand; the rank grows until a new term's Frobenius norm is at most tol
 * times that of the approximation (that term is not kept), or reaches
 * max_rank.  The error
 * |K - U V| is not bounded entrywise by tol (it is measured in the tests).
 *
 * M >= 1; kernel: SMOL_KERNEL_*; p0, p1 its parameters (finite);
 * tol >= 0; 1 <= max_rank <= 32.  U, V: device arrays of max_rank * M
 * doubles each (alpha-major, the layout smol_rhs takes), distinct; rows
 * beyond *rank are left unspecified.  rank (HOST): the rank built; est
 * (HOST, may be NULL): the relative Frobenius norm of the last term
 * computed (the one that stopped the growth, or the last kept one when
 * max_rank or M ended it).
 * Synchronous.  Errors: SMOL_EINVAL, SMOL_ENOMEM, SMOL_EDEVICE,
 * SMOL_EUNSUPPORTED (M beyond the right-hand side's limit). */
int smol_lowrank(int64_t M, int32_t kernel, double p0, double p1, double tol,
                 int32_t max_rank, double *U, double *V, int32_t *rank,
                 double *est, void *stream);

/*
 * smol_integrate -- integrate dn/dt = S(n), n(0) = n0 (Sec. 2, Eq. (5)) to
 * t_end with an embedded explicit Runge--Kutta pair and adaptive steps
 * (the accept / retry pattern of Sec. 2): an attempt is accepted when the
 * weighted-RMS norm
 *     err = sqrt(mean_s (e_s / (atol + rtol * max(|n_s|, |n_new,s|)))^2)
 * of the embedded error estimate e is <= 1; the step is then changed by a
 * PI controller, h *= clamp(0.9 err^-alpha err_prev^beta, 0.2, 10)
 * (alpha = 0.7/k, beta = 0.4/k, k = embedded order + 1; no growth on the
 * step right after a rejection); a rejection shrinks h by
 * max(0.2, 0.9 err^(-1/k)).  The first step comes from Hairer's starting
 * procedure; the last one is clipped to land exactly on t_end.
 *
 * n0, n_out: M doubles on the device (n_out may alias n0).  method: one of
 * the schemes above.  rtol > 0, atol >= 0, t_end >= 0 (t_end == 0
 * returns n0 after 0 steps).  stats: HOST pointer, may be NULL.
 * Synchronous: returns after the run with n_out written.  On
 * SMOL_ESTEPSIZE / SMOL_EMAXSTEPS / SMOL_ENONFINITE, n_out holds the last
 * accepted state and stats->t < t_end.
 */
int smol_integrate(int64_t M, int32_t R, const double *U, const double *V,
                   double lambda, const double *n0, double t_end, double rtol,
                   double atol, int32_t method, int32_t precision,
                   double *n_out, smol_stats *stats, void *stream);

/* Checkpoint of a run (smol_options.state): what a run needs to continue
 * exactly as if it had not stopped -- the time, the next step, the
 * controller's memory, the counters and S at the state (the first stage of
 * the next attempt, first-same-as-last).  The state vector itself is the
 * run's n_out, passed back as n0 when resuming. */
typedef struct {
    double t;            /* time of the state */
    double h;            /* next step to attempt (before clipping to t_end) */
    double err;          /* norm of the last attempt */
    double err_prev;     /* PI memory: last accepted norm, floored at 1e-4 */
    double err_hist[4];  /* norms of the last four attempts, most recent
                            first (learned controller features) */
    int64_t n_rhs, n_accept, n_reject;  /* counters, carried on */
    int32_t n_hist;      /* entries of err_hist in use */
    int32_t rejected;    /* the last attempt was rejected */
    int32_t valid;       /* in: 1 = resume from this state, 0 = start at
                            t = 0; out: 1 when a resumable state was written
                            (status SMOL_OK or SMOL_EMAXSTEPS), else 0 */
    int32_t n_fallback;  /* learned controller: PI fallbacks so far */
    double *k1;          /* device, M doubles (natural layout): S(n) at
                            the state; required whenever `state` is set */
} smol_state;

/* Options of smol_integrate_ex; zero-initialise and set what you need. */
typedef struct {
    double h0;          /* > 0: first step; 0: starting procedure */
    double h_min;       /* > 0: smallest allowed step */
    int64_t max_steps;  /* > 0: limit on step attempts; 0: 10^8 */
    double alpha, beta; /* PI exponents; alpha <= 0: defaults for both;
                           alpha > 0: both as given (beta = 0 selects the
                           pure I controller) */
    int32_t controller; /* SMOL_CTRL_* */
    int32_t reserved;
    double *log;        /* device pointer or NULL: one row per attempt,
                           (t, h, err, accepted, t_after, M0, M1, M2, M3)
                           as 9 doubles */
    int64_t log_cap;    /* rows available in log */
    double safety;      /* SMOL_CTRL_STEP_DOUBLING's s; <= 0: 1/4 */
    const double *source; /* constant sources P_s of Eq. (3): M doubles on
                           the device, or NULL (the right-hand side is then
                           S(n) + source throughout the run) */
    smol_state *state;  /* HOST pointer or NULL: checkpoint in and out.
                           With state->valid == 1 the run resumes from it:
                           n0 is the state at time state->t (the n_out of
                           the run that wrote it), no starting-step
                           procedure runs, and the counters continue;
                           max_steps and the log count this call's attempts
                           only.  Resuming with the same scheme, controller,
                           tolerances, options and t_end continues the run
                           bitwise as if it had not stopped.  On return the
                           run's final checkpoint is written to *state
                           (k1 receives S at n_out). */
} smol_options;

/* smol_integrate with options.  The number of log rows written is
 * min(log_cap, attempts of this call).  EINVAL also for a state without k1,
 * or a resumed state with a non-finite or negative t, or h <= 0; a resumed
 * state at t >= t_end returns n0 after 0 attempts. */
int smol_integrate_ex(int64_t M, int32_t R, const double *U, const double *V,
                      double lambda, const double *n0, double t_end,
                      double rtol, double atol, int32_t method,
                      int32_t precision, const smol_options *opts,
                      double *n_out, smol_stats *stats, void *stream);

/* One instance of a batched run.  All pointers are device pointers; log
 * (optional) receives the instance's per-attempt rows as in smol_options. */
typedef struct {
    int64_t M;
    int32_t R;
    int32_t reserved;
    const double *U, *V;
    double lambda;
    const double *n0;
    double *n_out;
    double t_end, rtol, atol;
    double *log;
    int64_t log_cap;
    const double *source;  /* Eq. (3) sources (M doubles) or NULL */
} smol_instance;

/*
 * smol_integrate_batch -- advance n_inst independent instances (uneven M,
 * kernels, lambda, tolerances) with per-instance step sizes and
 * accept/reject.  `inst` and `stats` are HOST arrays of n_inst entries.  A
 * failing instance records its status in its own stats entry and does not
 * stop the others; the call returns SMOL_OK when every instance is launched
 * and finishes (check each stats[i].status).  Options apply to every
 * instance (opts->log must be NULL: logs are per instance; opts->state must
 * be NULL: batched runs start at t = 0).
 * Instances are grouped by transform length.  For each group, every kernel
 * of a step attempt is one launch over that group's running instances (a
 * block-to-instance table) under the group's launch schedule; each group's
 * chain of step attempts is captured as its own hipGraph and replayed on
 * one of four library streams (default priority), so the groups run side by
 * side; the starting steps run on `stream`, which is synchronised before
 * the replays, and the call returns after all of them.  When the number of
 * running instances halves, the tables are rebuilt over the live ones and
 * the graphs captured again.  Every instance runs exactly the kernels of its
 * single-instance run and reproduces its smol_integrate_ex result bitwise.
 */
int smol_integrate_batch(int32_t n_inst, const smol_instance *inst,
                         int32_t method, int32_t precision,
                         const smol_options *opts, smol_stats *stats,
                         void *stream);

/* Learned step proposer (the controller option SMOL_CTRL_LEARNED): a
 * 9-64-64-1 tanh MLP in FP32 (4865 parameters, layout W1[64][9], b1[64],
 * W2[64][64], b2[64], W3[64], b3).  Features at the decision after an
 * accepted attempt: log M0..log M3 of the new state divided by 40, log h
 * divided by 10, log err of the last four attempts (most recent first,
 * missing ones 0) divided by 10.  Output y: a correction to the PI rule,
 * log(h_next / h) = log(PI factor) + y, clamped to [log 0.2, log 10], and
 * not above log(PI factor) when the attempt's err exceeds 0.5; right
 * after a rejection, or for non-finite features or output, the PI rule alone
 * is used (counted in smol_stats.n_fallback).  The embedded error estimate
 * still accepts or rejects every step. */

/* Install the weights used by learned-mode runs on the current device
 * (device pointer, copied; n_params must be 4865).  Synchronous. */
int smol_proposer_set(const float *params, int32_t n_params, void *stream);

/* Y[n_rows] = network(X[n_rows][9]) for the given weights (device). */
int smol_proposer_forward(const float *params, const float *X, int64_t n_rows,
                          float *Y, void *stream);

/* Weighted-MSE loss (1/n) sum w (y - target)^2, w = over_weight when
 * y > target else 1, and its gradient (device float[4865]) over all rows. */
int smol_proposer_loss_grad(const float *params, const float *X,
                            const float *target, int64_t n_rows,
                            float over_weight, float *loss, float *grad,
                            void *stream);

/* Train in place with the library's forward, backward and Adam kernels
 * (lr, beta 0.9 / 0.999, eps 1e-8): `epochs` passes over a permutation of
 * the rows (SplitMix64 Fisher-Yates from `seed`) in minibatches of `batch`
 * rows.  loss_out (device float[epochs]): mean minibatch loss per epoch. */
int smol_proposer_train(const float *X, const float *target, int64_t n_rows,
                        float *params, int32_t epochs, int32_t batch,
                        float lr, float over_weight, uint64_t seed,
                        float *loss_out, void *stream);

/* Training rows from a run's per-attempt log (device, rows x 9 doubles as
 * written by smol_integrate_ex): one row per accepted attempt j that has a
 * successor and does not follow a rejection, features as above and target
 *   clamp(log(h_{j+1}/h_j) + (1/k) log(err_target / err_{j+1})) - log(PI_j)
 * (k = embedded order + 1): the log ratio that would have hit
 * err = err_target (0 < err_target <= 1; 0.8 is the default reading) on the
 * next attempt, clamped to [log 0.2, log 10], less the log factor the PI rule
 * with the default exponents (0.7/k, 0.4/k) gives at that decision.
 * X (rows x 9) and target (rows) are device buffers of capacity `rows`;
 * *n_out (host) receives the number of rows written.  Synchronous. */
int smol_proposer_dataset(const double *log, int64_t rows, int32_t method,
                          double err_target, float *X, float *target,
                          int64_t *n_out, void *stream);

/* Timing hook for benchmarks.  Same arguments as smol_rhs (FP64), plus:
 * iters >= 1 launches of each of the three kernels of one right-hand side
 * -- the column pass, the row-pair spectral pass, the inverse column pass
 * with the finish -- back to back, each kernel's batch bracketed by HIP
 * events on `stream`; then iters whole right-hand sides.  ms_out (HOST, 4
 * floats) receives the mean milliseconds per launch of each kernel and per
 * whole right-hand side.  dndt holds S(n) afterwards.  Synchronous. */
int smol_profile_rhs(int64_t M, int32_t R, const double *U, const double *V,
                     double lambda, const double *n, double *dndt,
                     int32_t iters, float *ms_out, void *stream);

/* Timing hook for the integrator's own stage kernels (the kernels a step
 * attempt replays; Sec. 2, Eq. (5), with the right-hand side of Eq. (4)).
 * Runs the starting step and one attempt's stages of `method` (SMOL_BS32 or
 * SMOL_DP54, FP64, rtol 1e-6, atol 1e-12) from the state n0 (device, M
 * doubles, natural layout) without taking that attempt's decision, then
 * launches each kernel `iters` times back to back between HIP events on
 * `stream`:
 *   ms_out[0] column pass of stage 2 as a step attempt runs it: the previous
 *             attempt's accept / reject decision, then y_2 = n + h a_21 k_1
 *             and its transforms (the decision's result goes to a second
 *             control block, so every launch repeats the same work);
 *   ms_out[1] row-pair spectral pass;
 *   ms_out[2] inverse column pass + finish of stage 3 fused with the stage
 *             4 state, its reductions and the next column pass;
 *   ms_out[3] inverse column pass + finish of the last stage with the
 *             error-norm and moment partials.
 * ms_out is HOST memory (4 floats, mean milliseconds per launch).  The
 * caller's arrays are only read.  EINVAL for bad sizes, pointers, lambda,
 * iters < 1 or another method.  Synchronous. */
int smol_profile_step(int64_t M, int32_t R, const double *U, const double *V,
                      double lambda, const double *n0, int32_t method, int32_t iters,
                      float *ms_out, void *stream);

/* Launch schedules.  Each of the three right-hand-side kernels (column
 * pass A, row-pair pass B, inverse column pass + finish C) comes in up to
 * four variants that differ in the radix of the in-register butterflies and
 * in the workgroup tile; the results agree to rounding (FFT normwise error
 * O(eps log L)) but are not bitwise equal across variants:
 *   variant & 1: 8 waves (512 threads) per workgroup instead of 4;
 *   variant & 2: 4 complex values per lane (radix-4 stages) instead of 8
 *                (16 for 1024-point transforms); only for transforms of
 *                length <= 256.
 * Variants 1..3 exist for FP64 and L = 2^logL >= 2^12 only; float-float
 * plans always use variant 0.  The schedule is process-wide per logL and
 * starts from a table tuned on MI355X.
 *
 * smol_set_schedule: variants (HOST, 3 ints: A, B, C) for transforms of
 * length 2^logL, 6 <= logL <= 20; EINVAL for a variant that does not exist
 * at that length.  Existing plans switch at their next call (captured step
 * graphs are rebuilt).  smol_get_schedule: the current variants. */
int smol_set_schedule(int32_t logL, const int32_t *variants);
int smol_get_schedule(int32_t logL, int32_t *variants);

/* Autotuner: times step attempts of the caller's instance (same arguments
 * as smol_integrate: U, V, n0 device arrays; method SMOL_BS32 or
 * SMOL_DP54; FP64) under candidate schedules of its transform length,
 * `attempts` attempts per run, best of `reps` runs after one untimed run,
 * and descends over the kernels (C, then B, then A), keeping a variant only
 * if it saves at least 2 %.  The chosen schedule is installed (as by
 * smol_set_schedule) and written to variants_out (HOST, 3 ints);
 * ms_out (HOST, 2 floats, may be null) receives the milliseconds per
 * attempt of the starting schedule and of the chosen one.
 * Allocates one M-vector of scratch for the duration of the call.
 * Synchronous. */
int smol_autotune(int64_t M, int32_t R, const double *U, const double *V,
                  double lambda, const double *n0, int32_t method,
                  int32_t attempts, int32_t reps, int32_t *variants_out,
                  float *ms_out, void *stream);

/* Free cached plans and workspaces on the current device. */
int smol_release_plans(void);

/* Static string naming a status code. */
const char *smol_strerror(int code);

/* Library version string. */
const char *smol_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMOL_H */
