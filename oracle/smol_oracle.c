/*
 * smol_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of what the
 * Smoluchowski aggregation-shattering hot path computes.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the GPU
 * library and must never be used as a fallback for it.
 *
 * Paper: Matveev, Zhilin, Smirnov, "Adaptive time-stepping for
 * aggregation-shattering kinetics" (arXiv 2407.16559).
 *
 * Contents and what each part follows:
 *   oracle_rhs / oracle_rhs_entries
 *       The right-hand side S(n) of the truncated aggregation-shattering
 *       system: Sec. 1, Eq. (2) (truncated birth/death sums) and Eq. (4)
 *       (shattering), written as the plain O(M^2) double sums with the
 *       kernel formed per pair from the low-rank factors K = U V (Sec. 1,
 *       display after Eq. (2)).  Reading of Eq. (4): the monomer gain from
 *       monomer--j shattering carries the factor n_1 (the printed
 *       equation omits it; without it total mass is not conserved).
 *       Pinned by: hand-expanded M = 2 formulas, the point state n = e_1,
 *       the mass and number balance identities, rank-splitting
 *       invariance, and the K == 1 closed-form trajectory.
 *   oracle_integrate
 *       Adaptive embedded explicit Runge--Kutta integration of
 *       dn/dt = S(n) (Sec. 2, Eq. (5)): Bogacki--Shampine 3(2) and
 *       Dormand--Prince 5(4) (published tableaux), weighted-RMS error norm,
 *       PI step-size controller, Hairer's starting-step procedure.  The
 *       paper's own accept / retry pattern (Sec. 2, last two paragraphs)
 *       is kept: a rejected attempt is repeated with a smaller step.
 *       Pinned by: with beta = 0 the controller reduces to the I
 *       controller of scipy's RK23 / RK45 and must reproduce their step
 *       sequences; fixed-step convergence orders; the closed form.
 *       The beta (PI) term: on the scale-invariant single-size problem
 *       dn/dt = -K n^2 (atol = 0) the error norm of an attempt depends only
 *       on K h n, so the controller settles where its step factor equals
 *       the observed step growth rho; the accepted norm must then equal
 *       (safety / rho)^(1 / (alpha - beta)).  A flipped sign of beta, or an
 *       err_prev that is never updated, settles elsewhere and fails.
 *   oracle_rk_fixed
 *       Fixed-step version of the same tableaux (order checks), and of
 *       RKF45 as printed in Sec. 2.
 *   oracle_rhs_kernel, oracle_kernel_entries
 *       The same direct sums with K_{ij} from a formula of Sec. 3.1
 *       (constant, generalised Brownian, free-molecular) for every pair: the
 *       reference for low-rank approximations of kernels with no exact
 *       low-rank form.  Pinned by: the Brownian formula equals the exact
 *       rank-3 factors; hand values and the degree-1/6 homogeneity of the
 *       free-molecular kernel; the mass balance with the formula kernel.
 *   oracle_rhs_source
 *       Eq. (3): the right-hand side plus constant sources P_s (also a
 *       field of both integrators' options).  Pinned by: K == 0 gives
 *       n(t) = n0 + P t; the K == 1 number density with a monomer source
 *       obeys N' = P_1 - N^2 / 2 (closed form); the mass balance
 *       sum s S_s = sum s P_s - F_trunc.
 *   oracle_integrate_paper
 *       The paper's own adaptive schemes (Sec. 2): RKF45 with Fehlberg's
 *       step rule, RK2 / RK4 with step doubling and the step update of
 *       Eq. (6) or the halve / double rule, Euclidean error norm.
 *       Pinned by: the K == 1 closed form: local errors of one attempt
 *       shrink as tau^(p+1) (RK2 p = 2, RK4 p = 4, RKF45's two solutions
 *       4 and 5) and the two half steps of a doubling attempt are 2^p times
 *       closer than the single step; whole runs against the closed form at
 *       several tolerances; the step-size rules' worked examples.
 *   oracle_moments, oracle_features, oracle_proposer_features
 *       Moments sum_s s^k n_s and the step-proposer feature vector.
 *   oracle_proposer_dataset, oracle_learned_factor, oracle_learned_steps
 *       The learned proposer's training rows from a run log (hindsight
 *       target less the PI rule's log factor), the learned controller's
 *       step factor exp(clamp(log PI + network output)), and the factors
 *       it takes along a logged run.  Pinned by: on a
 *       PI-controlled oracle run's log the PI part cancels exactly, leaving
 *       (1/k) log(err_target / err_{j+1}); with err = C h^k the target step
 *       meets err_target; a network with output b gives clamp(PI e^b), and
 *       output 0 the oracle integrator's own PI steps.
 *   oracle_mlp_forward / oracle_mlp_loss_grad / oracle_adam
 *       The 9-64-64-1 tanh MLP step proposer, its weighted-MSE loss and
 *       gradient by backpropagation, and one Adam update, in FP64.
 *       Pinned by central finite differences and by torch's CPU modules.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ESTEPSIZE (-4)
#define OR_EMAXSTEPS (-5)
#define OR_ENONFINITE (-6)

/* The coagulation kernel K_{ij} (i, j 1-based sizes), given either by
 * low-rank factors (R >= 1): K_{ij} = sum_a U_{i a} V_{a j}, stored
 * alpha-major U[a*M + i-1], V[a*M + j-1] (Sec. 1, display after Eq. (2));
 * or (R == 0) by one of the formulas of Sec. 3.1:
 *   ORACLE_K_CONSTANT        K = p0
 *   ORACLE_K_BROWNIAN        K = (i/j)^p0 + (j/i)^p0 + p1 (generalised
 *                            Brownian, exponent p0, constant term p1)
 *   ORACLE_K_FREE_MOLECULAR  K = (i^(1/3) + j^(1/3))^2 sqrt(1/i + 1/j) */
#define ORACLE_K_CONSTANT 1
#define ORACLE_K_BROWNIAN 2
#define ORACLE_K_FREE_MOLECULAR 3

typedef struct {
    int64_t M;
    int32_t R;
    const double *U, *V;
    int32_t formula;
    double p0, p1;
} kspec;

static kspec factors(int64_t M, int32_t R, const double *U, const double *V)
{
    kspec k = {M, R, U, V, 0, 0.0, 0.0};
    return k;
}

static __attribute__((noinline)) double kern_formula(const kspec *K, int64_t i, int64_t j)
{
    const double x = (double)i, y = (double)j;
    switch (K->formula) {
    case ORACLE_K_CONSTANT: return K->p0;
    case ORACLE_K_BROWNIAN: return pow(x / y, K->p0) + pow(y / x, K->p0) + K->p1;
    default: {
        const double c = cbrt(x) + cbrt(y);
        return c * c * sqrt(1.0 / x + 1.0 / y);
    }
    }
}

static inline __attribute__((always_inline)) double kern(const kspec *K, int64_t i, int64_t j)
{
    if (K->R > 0) {
        double k = 0.0;
        for (int32_t a = 0; a < K->R; ++a)
            k += K->U[(int64_t)a * K->M + (i - 1)] * K->V[(int64_t)a * K->M + (j - 1)];
        return k;
    }
    return kern_formula(K, i, j);
}

static void set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* S_s for one 1-based size s, excluding the s = 1 double sum, which the
 * callers provide (it does not depend on s). */
static double rhs_one(const kspec *K, double lam, const double *n, int64_t s,
                      double shatter_pairs)
{
    const int64_t M = K->M;
    if (s == 1) {
        /* Eq. (4), first line:
         *   -n_1 sum_{i=1}^{M} K_{1,i} n_i                (aggregation loss)
         *   + (lam/2) sum_{i>=2} sum_{j>=2} (i+j) K_{ij} n_i n_j
         *   + lam n_1 sum_{j>=2} j K_{1,j} n_j             (monomer--j shattering) */
        double death = 0.0, gain = 0.0;
        for (int64_t i = 1; i <= M; ++i) death += kern(K, 1, i) * n[i - 1];
        for (int64_t j = 2; j <= M; ++j) gain += (double)j * kern(K, 1, j) * n[j - 1];
        return -n[0] * death + 0.5 * lam * shatter_pairs + lam * n[0] * gain;
    }
    /* Eq. (2) birth and death with Eq. (4)'s extra shattering loss, s >= 2:
     *   (1/2) sum_{i+j=s} K_{ij} n_i n_j - (1 + lam) n_s sum_{i=1}^{M} K_{s,i} n_i */
    double birth = 0.0, death = 0.0;
    for (int64_t i = 1; i <= s - 1; ++i)
        birth += kern(K, i, s - i) * n[i - 1] * n[s - i - 1];
    for (int64_t i = 1; i <= M; ++i) death += kern(K, s, i) * n[i - 1];
    return 0.5 * birth - (1.0 + lam) * n[s - 1] * death;
}

/* sum_{i>=2} sum_{j>=2} (i+j) K_{ij} n_i n_j, summed row by row, rows in
 * ascending order (deterministic for any thread count). */
static double shatter_double_sum(const kspec *K, const double *n)
{
    const int64_t M = K->M;
    if (M < 2) return 0.0;
    double *row = (double *)malloc(sizeof(double) * (size_t)M);
    if (!row) return NAN;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 2; i <= M; ++i) {
        double acc = 0.0;
        for (int64_t j = 2; j <= M; ++j)
            acc += (double)(i + j) * kern(K, i, j) * n[i - 1] * n[j - 1];
        row[i - 1] = acc;
    }
    double total = 0.0;
    for (int64_t i = 2; i <= M; ++i) total += row[i - 1];
    free(row);
    return total;
}

static void rhs_all(const kspec *K, double lam, const double *n, double *out)
{
    double pairs = shatter_double_sum(K, n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 1; s <= K->M; ++s)
        out[s - 1] = rhs_one(K, lam, n, s, pairs);
}

int oracle_rhs(int64_t M, int32_t R, const double *U, const double *V,
               double lam, const double *n, double *out, int32_t nthreads)
{
    if (M < 1 || R < 1 || !U || !V || !n || !out) return OR_EINVAL;
    set_threads(nthreads);
    const kspec K = factors(M, R, U, V);
    rhs_all(&K, lam, n, out);
    return OR_OK;
}

/* The right-hand side with K_{ij} evaluated from a formula (see kspec) for
 * every pair: the reference for a low-rank approximation of a kernel that
 * has no exact low-rank form, such as the free-molecular kernel of Sec. 3.1. */
int oracle_rhs_kernel(int64_t M, int32_t formula, double p0, double p1, double lam,
                      const double *n, double *out, int32_t nthreads)
{
    if (M < 1 || !n || !out || formula < ORACLE_K_CONSTANT || formula > ORACLE_K_FREE_MOLECULAR)
        return OR_EINVAL;
    set_threads(nthreads);
    const kspec K = {M, 0, NULL, NULL, formula, p0, p1};
    rhs_all(&K, lam, n, out);
    return OR_OK;
}

/* K_{ij} of a formula kernel for the pairs (i[q], j[q]) (1-based sizes). */
int oracle_kernel_entries(int32_t formula, double p0, double p1, const int64_t *i,
                          const int64_t *j, int64_t npairs, double *out)
{
    if (formula < ORACLE_K_CONSTANT || formula > ORACLE_K_FREE_MOLECULAR) return OR_EINVAL;
    const kspec K = {1, 0, NULL, NULL, formula, p0, p1};
    for (int64_t q = 0; q < npairs; ++q) {
        if (i[q] < 1 || j[q] < 1) return OR_EINVAL;
        out[q] = kern(&K, i[q], j[q]);
    }
    return OR_OK;
}

/* S at selected 0-based indices idx[0..nidx) (index s-1 holds size s). */
/* Eq. (3): the same right-hand side plus constant sources P_s (src may be
 * NULL: no sources).  The printed P_k is read as P_s. */
static void rhs_src(int64_t M, int32_t R, const double *U, const double *V, double lam,
                    const double *src, const double *n, double *out, int32_t nth)
{
    oracle_rhs(M, R, U, V, lam, n, out, nth);
    if (src)
        for (int64_t s = 0; s < M; ++s) out[s] += src[s];
}

int oracle_rhs_source(int64_t M, int32_t R, const double *U, const double *V, double lam,
                      const double *n, const double *src, double *out, int32_t nthreads)
{
    if (M < 1 || R < 1 || !U || !V || !n || !out) return OR_EINVAL;
    rhs_src(M, R, U, V, lam, src, n, out, nthreads);
    return OR_OK;
}

int oracle_rhs_entries(int64_t M, int32_t R, const double *U, const double *V,
                       double lam, const double *n, const int64_t *idx,
                       int64_t nidx, double *out, int32_t nthreads)
{
    if (M < 1 || R < 1 || !U || !V || !n || !out || (nidx > 0 && !idx)) return OR_EINVAL;
    set_threads(nthreads);
    int need_pairs = 0;
    for (int64_t q = 0; q < nidx; ++q) {
        if (idx[q] < 0 || idx[q] >= M) return OR_EINVAL;
        if (idx[q] == 0) need_pairs = 1;
    }
    const kspec K = factors(M, R, U, V);
    double pairs = need_pairs ? shatter_double_sum(&K, n) : 0.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nidx; ++q)
        out[q] = rhs_one(&K, lam, n, idx[q] + 1, pairs);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Embedded Runge--Kutta pairs (exact rationals).                      */
/* ------------------------------------------------------------------ */

#define MAXST 7

typedef struct {
    int stages;            /* number of stages including the FSAL stage */
    int q;                 /* order of the embedded (error) solution */
    double a[MAXST][MAXST];
    double b[MAXST];       /* propagated (higher-order) weights */
    double bh[MAXST];      /* embedded (lower-order) weights */
} tableau;

/* Bogacki & Shampine (1989), "A 3(2) pair of Runge--Kutta formulas". */
static void tab_bs32(tableau *T)
{
    memset(T, 0, sizeof(*T));
    T->stages = 4;
    T->q = 2;
    T->a[1][0] = 1.0 / 2.0;
    T->a[2][0] = 0.0;        T->a[2][1] = 3.0 / 4.0;
    T->a[3][0] = 2.0 / 9.0;  T->a[3][1] = 1.0 / 3.0;  T->a[3][2] = 4.0 / 9.0;
    T->b[0] = 2.0 / 9.0;  T->b[1] = 1.0 / 3.0;  T->b[2] = 4.0 / 9.0;  T->b[3] = 0.0;
    T->bh[0] = 7.0 / 24.0; T->bh[1] = 1.0 / 4.0; T->bh[2] = 1.0 / 3.0; T->bh[3] = 1.0 / 8.0;
}

/* Dormand & Prince (1980), "A family of embedded Runge--Kutta formulae". */
static void tab_dp54(tableau *T)
{
    memset(T, 0, sizeof(*T));
    T->stages = 7;
    T->q = 4;
    T->a[1][0] = 1.0 / 5.0;
    T->a[2][0] = 3.0 / 40.0;  T->a[2][1] = 9.0 / 40.0;
    T->a[3][0] = 44.0 / 45.0; T->a[3][1] = -56.0 / 15.0; T->a[3][2] = 32.0 / 9.0;
    T->a[4][0] = 19372.0 / 6561.0; T->a[4][1] = -25360.0 / 2187.0;
    T->a[4][2] = 64448.0 / 6561.0; T->a[4][3] = -212.0 / 729.0;
    T->a[5][0] = 9017.0 / 3168.0;  T->a[5][1] = -355.0 / 33.0;
    T->a[5][2] = 46732.0 / 5247.0; T->a[5][3] = 49.0 / 176.0;
    T->a[5][4] = -5103.0 / 18656.0;
    T->a[6][0] = 35.0 / 384.0; T->a[6][1] = 0.0; T->a[6][2] = 500.0 / 1113.0;
    T->a[6][3] = 125.0 / 192.0; T->a[6][4] = -2187.0 / 6784.0; T->a[6][5] = 11.0 / 84.0;
    for (int j = 0; j < 6; ++j) T->b[j] = T->a[6][j];
    T->b[6] = 0.0;
    T->bh[0] = 5179.0 / 57600.0; T->bh[1] = 0.0; T->bh[2] = 7571.0 / 16695.0;
    T->bh[3] = 393.0 / 640.0; T->bh[4] = -92097.0 / 339200.0;
    T->bh[5] = 187.0 / 2100.0; T->bh[6] = 1.0 / 40.0;
}

/* Runge--Kutta--Fehlberg 4(5) as printed in Sec. 2 (Fehlberg 1970): six
 * stages; b = the fourth-order weights the paper propagates, bh = the
 * fifth-order weights of its error estimate. */
static void tab_rkf45(tableau *T)
{
    memset(T, 0, sizeof(*T));
    T->stages = 6;
    T->q = 4;
    T->a[1][0] = 1.0 / 4.0;
    T->a[2][0] = 3.0 / 32.0;  T->a[2][1] = 9.0 / 32.0;
    T->a[3][0] = 1932.0 / 2197.0; T->a[3][1] = -7200.0 / 2197.0; T->a[3][2] = 7296.0 / 2197.0;
    T->a[4][0] = 439.0 / 216.0; T->a[4][1] = -8.0; T->a[4][2] = 3680.0 / 513.0;
    T->a[4][3] = -845.0 / 4104.0;
    T->a[5][0] = -8.0 / 27.0; T->a[5][1] = 2.0; T->a[5][2] = -3544.0 / 2565.0;
    T->a[5][3] = 1859.0 / 4104.0; T->a[5][4] = -11.0 / 40.0;
    T->b[0] = 25.0 / 216.0; T->b[2] = 1408.0 / 2565.0; T->b[3] = 2197.0 / 4104.0;
    T->b[4] = -1.0 / 5.0;
    T->bh[0] = 16.0 / 135.0; T->bh[2] = 6656.0 / 12825.0; T->bh[3] = 28561.0 / 56430.0;
    T->bh[4] = -9.0 / 50.0; T->bh[5] = 2.0 / 55.0;
}

static int get_tableau(int32_t method, tableau *T)
{
    if (method == 0) { tab_bs32(T); return 0; }
    if (method == 1) { tab_dp54(T); return 0; }
    if (method == 2) { tab_rkf45(T); return 0; }
    return -1;
}

/* Copy of the tableau for the tests (order conditions). */
int oracle_tableau(int32_t method, double *a, double *b, double *bh,
                   int32_t *stages)
{
    tableau T;
    if (get_tableau(method, &T)) return OR_EINVAL;
    *stages = T.stages;
    for (int i = 0; i < T.stages; ++i) {
        for (int j = 0; j < T.stages; ++j) a[i * T.stages + j] = T.a[i][j];
        b[i] = T.b[i];
        bh[i] = T.bh[i];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Adaptive integration.                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t method;     /* 0 = BS3(2), 1 = DP5(4) */
    int32_t nthreads;
    double rtol, atol, t_end;
    double h0;          /* > 0: use this first step; <= 0: automatic */
    int64_t max_steps;  /* limit on step attempts; <= 0: 10^8 */
    double alpha, beta; /* PI exponents: alpha > 0 takes both as given (beta
                           of either sign); alpha <= 0: 0.7/k and 0.4/k */
    double safety, facmin, facmax; /* <= 0: 0.9, 0.2, 10 */
    double h_min;       /* smallest allowed step (besides 10 ulps of t) */
    const double *source; /* Eq. (3) sources P_s (M doubles) or NULL */
} oracle_opts;

typedef struct {
    int64_t n_rhs, n_accept, n_reject;
    double t, h, err;
    int32_t status;
} oracle_stats;

static double rms(const double *x, int64_t M)
{
    double s = 0.0;
    for (int64_t i = 0; i < M; ++i) s += x[i] * x[i];
    return sqrt(s / (double)M);
}

static int all_finite(const double *x, int64_t M)
{
    for (int64_t i = 0; i < M; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* Starting step of Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4,
 * with q the order of the embedded solution (exponent 1/(q+1)). */
static double initial_step(int64_t M, int32_t R, const double *U,
                           const double *V, double lam, const double *src, const double *y0,
                           const double *f0, double t_span, int q,
                           double rtol, double atol, double *work,
                           int64_t *n_rhs, int32_t nth)
{
    double *sc = work, *y1 = work + M, *f1 = work + 2 * M, *tmp = work + 3 * M;
    for (int64_t i = 0; i < M; ++i) sc[i] = atol + fabs(y0[i]) * rtol;
    for (int64_t i = 0; i < M; ++i) tmp[i] = y0[i] / sc[i];
    double d0 = rms(tmp, M);
    for (int64_t i = 0; i < M; ++i) tmp[i] = f0[i] / sc[i];
    double d1 = rms(tmp, M);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    if (h0 > t_span) h0 = t_span;
    for (int64_t i = 0; i < M; ++i) y1[i] = y0[i] + h0 * f0[i];
    rhs_src(M, R, U, V, lam, src, y1, f1, nth);
    *n_rhs += 1;
    for (int64_t i = 0; i < M; ++i) tmp[i] = (f1[i] - f0[i]) / sc[i];
    double d2 = rms(tmp, M) / h0;
    double h1;
    if (d1 <= 1e-15 && d2 <= 1e-15)
        h1 = fmax(1e-6, h0 * 1e-3);
    else
        h1 = pow(0.01 / fmax(d1, d2), 1.0 / (double)(q + 1));
    double h = 100.0 * h0;
    if (h1 < h) h = h1;
    if (t_span < h) h = t_span;
    return h;
}

/* log row layout: t_start, h, err, accepted (1/0), t_after  (5 doubles) */
int oracle_integrate(int64_t M, int32_t R, const double *U, const double *V,
                     double lam, const double *n0, const oracle_opts *o,
                     double *n_out, oracle_stats *st, double *log,
                     int64_t log_cap)
{
    if (M < 1 || R < 1 || !U || !V || !n0 || !o || !n_out || !st) return OR_EINVAL;
    if (!(o->rtol > 0) || !(o->atol >= 0) || !(o->t_end >= 0) || !isfinite(lam) || lam < 0)
        return OR_EINVAL;
    tableau T;
    if (get_tableau(o->method, &T)) return OR_EINVAL;
    const int S = T.stages, k = T.q + 1;
    const double alpha = o->alpha > 0 ? o->alpha : 0.7 / k;
    const double beta = o->alpha > 0 ? o->beta : 0.4 / k;
    const double safety = o->safety > 0 ? o->safety : 0.9;
    const double facmin = o->facmin > 0 ? o->facmin : 0.2;
    const double facmax = o->facmax > 0 ? o->facmax : 10.0;
    const int64_t max_steps = o->max_steps > 0 ? o->max_steps : 100000000LL;
    const int32_t nth = o->nthreads;
    const double *src = o->source;

    memset(st, 0, sizeof(*st));
    double *buf = (double *)malloc(sizeof(double) * (size_t)M * (size_t)(S + 7));
    if (!buf) return OR_ENOMEM;
    double *y = buf, *ynew = buf + M, *ytmp = buf + 2 * M, *work = buf + 3 * M;
    double *K[MAXST];
    for (int j = 0; j < S; ++j) K[j] = buf + (int64_t)(7 + j) * M;

    memcpy(y, n0, sizeof(double) * (size_t)M);
    double t = 0.0, h = 0.0, err_prev = 1.0;
    int64_t attempts = 0, nlog = 0;
    int status = OR_OK;
    if (!all_finite(y, M)) { status = OR_ENONFINITE; goto done; }
    if (o->t_end == 0.0) goto done;

    rhs_src(M, R, U, V, lam, src, y, K[0], nth);
    st->n_rhs = 1;
    h = o->h0 > 0 ? o->h0
                  : initial_step(M, R, U, V, lam, src, y, K[0], o->t_end, T.q,
                                 o->rtol, o->atol, work, &st->n_rhs, nth);
    if (h > o->t_end) h = o->t_end;

    while (t < o->t_end) {
        double min_step = 10.0 * fabs(nextafter(t, INFINITY) - t);
        if (o->h_min > min_step) min_step = o->h_min;
        if (h < min_step) h = min_step;
        int rejected = 0;
        for (;;) {
            if (attempts >= max_steps) { status = OR_EMAXSTEPS; goto done; }
            if (h < min_step) { status = OR_ESTEPSIZE; goto done; }
            double t_new = t + h;
            if (t_new > o->t_end) t_new = o->t_end;
            h = t_new - t;
            /* stages 2..S; K[0] holds S(y) */
            for (int i = 1; i < S; ++i) {
                double *dst = (i == S - 1) ? ynew : ytmp;
                for (int64_t s = 0; s < M; ++s) {
                    double acc = 0.0;
                    for (int j = 0; j < i; ++j) acc += T.a[i][j] * K[j][s];
                    dst[s] = y[s] + h * acc;
                }
                rhs_src(M, R, U, V, lam, src, dst, K[i], nth);
                st->n_rhs += 1;
            }
            /* the last stage of both pairs is the propagated solution (FSAL) */
            double sum = 0.0;
            for (int64_t s = 0; s < M; ++s) {
                double e = 0.0;
                for (int j = 0; j < S; ++j) e += (T.b[j] - T.bh[j]) * K[j][s];
                e *= h;
                double sc = o->atol + fmax(fabs(y[s]), fabs(ynew[s])) * o->rtol;
                double r = e / sc;
                sum += r * r;
            }
            double err = sqrt(sum / (double)M);
            ++attempts;
            st->err = err;
            /* a non-finite state or a NaN norm ends the run; an infinite
             * norm of a finite state is an ordinary (maximal) rejection */
            if (isnan(err) || !all_finite(ynew, M)) {
                status = OR_ENONFINITE;
                goto done;
            }
            int accept = err <= 1.0;
            if (log && nlog < log_cap) {
                double *row = log + 5 * nlog++;
                row[0] = t; row[1] = h; row[2] = err; row[3] = accept;
                row[4] = accept ? t_new : t;
            }
            if (accept) {
                double fac;
                if (err == 0.0)
                    fac = facmax;
                else
                    fac = safety * pow(err, -alpha) * pow(err_prev, beta);
                if (fac > facmax) fac = facmax;
                if (fac < facmin) fac = facmin;
                if (rejected && fac > 1.0) fac = 1.0;
                err_prev = fmax(err, 1e-4);
                t = t_new;
                h = h * fac;
                memcpy(y, ynew, sizeof(double) * (size_t)M);
                double *swap = K[0]; K[0] = K[S - 1]; K[S - 1] = swap;
                st->n_accept += 1;
                break;
            }
            double fac = safety * pow(err, -1.0 / (double)k);
            if (fac < facmin) fac = facmin;
            h = h * fac;
            rejected = 1;
            st->n_reject += 1;
        }
    }
done:
    st->t = t;
    st->h = h;
    st->status = status;
    memcpy(n_out, y, sizeof(double) * (size_t)M);
    free(buf);
    return status;
}

/* Fixed-step integration with the propagated (use_embedded = 0) or the
 * embedded (use_embedded = 1) weights, for order-of-accuracy checks. */
int oracle_rk_fixed(int64_t M, int32_t R, const double *U, const double *V,
                    double lam, const double *n0, int32_t method, double h,
                    int64_t nsteps, int32_t use_embedded, double *n_out,
                    int32_t nthreads)
{
    tableau T;
    if (get_tableau(method, &T) || M < 1 || nsteps < 0) return OR_EINVAL;
    const int S = T.stages;
    const double *src = NULL;
    double *buf = (double *)malloc(sizeof(double) * (size_t)M * (size_t)(S + 2));
    if (!buf) return OR_ENOMEM;
    double *y = buf, *ytmp = buf + M, *K[MAXST];
    for (int j = 0; j < S; ++j) K[j] = buf + (int64_t)(2 + j) * M;
    memcpy(y, n0, sizeof(double) * (size_t)M);
    const double *w = use_embedded ? T.bh : T.b;
    for (int64_t step = 0; step < nsteps; ++step) {
        rhs_src(M, R, U, V, lam, src, y, K[0], nthreads);
        for (int i = 1; i < S; ++i) {
            for (int64_t s = 0; s < M; ++s) {
                double acc = 0.0;
                for (int j = 0; j < i; ++j) acc += T.a[i][j] * K[j][s];
                ytmp[s] = y[s] + h * acc;
            }
            rhs_src(M, R, U, V, lam, src, ytmp, K[i], nthreads);
        }
        for (int64_t s = 0; s < M; ++s) {
            double acc = 0.0;
            for (int j = 0; j < S; ++j) acc += w[j] * K[j][s];
            y[s] = y[s] + h * acc;
        }
    }
    memcpy(n_out, y, sizeof(double) * (size_t)M);
    free(buf);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* The paper's adaptive schemes (Sec. 2).                              */
/* ------------------------------------------------------------------ */

/* scheme: 2 = RKF45 (propagate the fourth-order solution, error
 *             || n_RK5 - n^{k+1} ||_2), 3 = RK2 with step doubling,
 *             4 = RK4 with step doubling (one step tau giving n^{k+1}, two
 *             steps tau/2 giving nhat^{k+1}; error || nhat - n ||_2; the
 *             two half steps are propagated).
 * rule:   0 = Eq. (6), tau_new = s tau (tol / err)^(1/p), p the order of the
 *             scheme (2 for RK2, 4 for RK4 and RKF45);
 *         1 = halve tau after a rejection, double it after an acceptance;
 *         2 = Fehlberg's rule: the step scales with the fifth root of
 *             tol / err, times 0.9 (so err = 2 tol shrinks it by ~20 %,
 *             err = tol / 2 grows it by ~3 %, err = tol shrinks it by 10 %).
 * An attempt is accepted iff err <= tol, else repeated from the same state.
 * Readings where the paper is silent: the factor of rules 0 and 2 is clipped
 * to [0.2, 10] (err = 0 gives 10); the first step is Hairer's starting step
 * with the absolute weights sc = tol; the usual step-start clamp and t_end
 * clip apply.  S(n) at a state is evaluated once and shared by every attempt
 * and half step that starts there (counted once in n_rhs). */
typedef struct {
    int32_t scheme, rule, nthreads;
    double tol, t_end;
    double h0;          /* > 0: first step; <= 0: automatic */
    double s;           /* rule 0 safety factor; <= 0: 1/4 */
    int64_t max_steps;  /* limit on attempts; <= 0: 10^8 */
    double h_min;
    const double *source; /* Eq. (3) sources P_s (M doubles) or NULL */
} oracle_paper_opts;

static double norm2(const double *x, int64_t M)
{
    double s = 0.0;
    for (int64_t i = 0; i < M; ++i) s += x[i] * x[i];
    return sqrt(s);
}

/* One RK2 or RK4 step of size tau from y (Sec. 2, as printed: k_i = tau S(.)),
 * given f0 = S(y); writes y_out.  Returns the number of RHS evaluated. */
static int classic_step(int32_t scheme, int64_t M, int32_t R, const double *U, const double *V,
                        double lam, const double *src, const double *y, const double *f0, double tau,
                        double *y_out, double *w, int32_t nth)
{
    double *k1 = w, *k2 = w + M, *k3 = w + 2 * M, *k4 = w + 3 * M, *z = w + 4 * M;
    for (int64_t i = 0; i < M; ++i) k1[i] = tau * f0[i];
    if (scheme == 3) {
        for (int64_t i = 0; i < M; ++i) z[i] = y[i] + k1[i];
        rhs_src(M, R, U, V, lam, src, z, k2, nth);
        for (int64_t i = 0; i < M; ++i) k2[i] *= tau;
        for (int64_t i = 0; i < M; ++i) y_out[i] = y[i] + (k1[i] + k2[i]) / 2.0;
        return 1;
    }
    for (int64_t i = 0; i < M; ++i) z[i] = y[i] + 0.5 * k1[i];
    rhs_src(M, R, U, V, lam, src, z, k2, nth);
    for (int64_t i = 0; i < M; ++i) k2[i] *= tau;
    for (int64_t i = 0; i < M; ++i) z[i] = y[i] + 0.5 * k2[i];
    rhs_src(M, R, U, V, lam, src, z, k3, nth);
    for (int64_t i = 0; i < M; ++i) k3[i] *= tau;
    for (int64_t i = 0; i < M; ++i) z[i] = y[i] + k3[i];
    rhs_src(M, R, U, V, lam, src, z, k4, nth);
    for (int64_t i = 0; i < M; ++i) k4[i] *= tau;
    for (int64_t i = 0; i < M; ++i)
        y_out[i] = y[i] + (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]) / 6.0;
    return 3;
}

/* One attempt of step tau from y with f0 = S(y): RKF45 writes the fourth-
 * (y4) and fifth-order (y5) solutions; the doubling schemes write the single
 * step (y4 <- n^{k+1}) and the two half steps (y5 <- nhat^{k+1}).  The
 * propagated solution is y4 for RKF45 and y5 for the doubling schemes.
 * Returns the number of RHS evaluations (S(y) excluded). */
static int paper_attempt(int32_t scheme, int64_t M, int32_t R, const double *U, const double *V,
                         double lam, const double *src, const double *y, const double *f0, double tau, double *y4,
                         double *y5, double *w, int32_t nth)
{
    if (scheme == 2) {
        tableau T;
        tab_rkf45(&T);
        double *K[6], *z = w + 6 * M;
        for (int j = 0; j < 6; ++j) K[j] = w + (int64_t)j * M;
        /* k_1 = tau S(n^k), k_2 .. k_6 as printed */
        for (int64_t s = 0; s < M; ++s) K[0][s] = tau * f0[s];
        for (int i = 1; i < 6; ++i) {
            for (int64_t s = 0; s < M; ++s) {
                double acc = 0.0;
                for (int j = 0; j < i; ++j) acc += T.a[i][j] * K[j][s];
                z[s] = y[s] + acc;
            }
            rhs_src(M, R, U, V, lam, src, z, K[i], nth);
            for (int64_t s = 0; s < M; ++s) K[i][s] *= tau;
        }
        for (int64_t s = 0; s < M; ++s) {
            double n4 = y[s], n5 = y[s];
            for (int j = 0; j < 6; ++j) {
                n4 += T.b[j] * K[j][s];
                n5 += T.bh[j] * K[j][s];
            }
            y4[s] = n4;
            y5[s] = n5;
        }
        return 5;
    }
    /* one step tau, then two steps tau / 2 */
    double *yh = w + 5 * M, *fh = w + 6 * M;
    int n = classic_step(scheme, M, R, U, V, lam, src, y, f0, tau, y4, w, nth);
    n += classic_step(scheme, M, R, U, V, lam, src, y, f0, 0.5 * tau, yh, w, nth);
    rhs_src(M, R, U, V, lam, src, yh, fh, nth);
    n += 1;
    n += classic_step(scheme, M, R, U, V, lam, src, yh, fh, 0.5 * tau, y5, w, nth);
    return n;
}

int oracle_paper_attempt(int32_t scheme, int64_t M, int32_t R, const double *U,
                         const double *V, double lam, const double *y, double tau,
                         double *y4, double *y5, int32_t nthreads)
{
    if (scheme < 2 || scheme > 4 || M < 1) return OR_EINVAL;
    const double *src = NULL;
    double *w = (double *)malloc(sizeof(double) * (size_t)M * 8);
    if (!w) return OR_ENOMEM;
    rhs_src(M, R, U, V, lam, src, y, w + 7 * M, nthreads);
    paper_attempt(scheme, M, R, U, V, lam, src, y, w + 7 * M, tau, y4, y5, w, nthreads);
    free(w);
    return OR_OK;
}

int oracle_integrate_paper(int64_t M, int32_t R, const double *U, const double *V,
                           double lam, const double *n0, const oracle_paper_opts *o,
                           double *n_out, oracle_stats *st, double *log, int64_t log_cap)
{
    if (M < 1 || R < 1 || !U || !V || !n0 || !o || !n_out || !st) return OR_EINVAL;
    if (o->scheme < 2 || o->scheme > 4 || o->rule < 0 || o->rule > 2) return OR_EINVAL;
    if (!(o->tol > 0) || !(o->t_end >= 0) || !isfinite(lam) || lam < 0) return OR_EINVAL;
    const int p = o->scheme == 3 ? 2 : 4;       /* order of the scheme */
    const double s_fac = o->s > 0 ? o->s : 0.25;
    const int64_t max_steps = o->max_steps > 0 ? o->max_steps : 100000000LL;
    const int32_t nth = o->nthreads;
    const double *src = o->source;
    memset(st, 0, sizeof(*st));
    double *buf = (double *)malloc(sizeof(double) * (size_t)M * 14);
    if (!buf) return OR_ENOMEM;
    double *y = buf, *f = buf + M, *yfull = buf + 2 * M;
    double *yhat = buf + 4 * M, *e = buf + 5 * M, *work = buf + 6 * M;  /* work: 8 M */

    memcpy(y, n0, sizeof(double) * (size_t)M);
    double t = 0.0, h = 0.0;
    int64_t attempts = 0, nlog = 0;
    int status = OR_OK;
    if (!all_finite(y, M)) { status = OR_ENONFINITE; goto done; }
    if (o->t_end == 0.0) goto done;
    rhs_src(M, R, U, V, lam, src, y, f, nth);
    st->n_rhs = 1;
    h = o->h0 > 0 ? o->h0
                  : initial_step(M, R, U, V, lam, src, y, f, o->t_end, p, 0.0, o->tol, work,
                                 &st->n_rhs, nth);
    if (h > o->t_end) h = o->t_end;

    while (t < o->t_end) {
        double min_step = 10.0 * fabs(nextafter(t, INFINITY) - t);
        if (o->h_min > min_step) min_step = o->h_min;
        if (h < min_step) h = min_step;
        for (;;) {
            if (attempts >= max_steps) { status = OR_EMAXSTEPS; goto done; }
            if (h < min_step) { status = OR_ESTEPSIZE; goto done; }
            double t_new = t + h;
            if (t_new > o->t_end) t_new = o->t_end;
            h = t_new - t;
            st->n_rhs += paper_attempt(o->scheme, M, R, U, V, lam, src, y, f, h, yfull, yhat, work, nth);
            double *ynew = o->scheme == 2 ? yfull : yhat;
            for (int64_t s = 0; s < M; ++s) e[s] = yhat[s] - yfull[s];
            const double err = norm2(e, M) / o->tol;  /* in units of tol */
            ++attempts;
            st->err = err;
            if (isnan(err) || !all_finite(ynew, M)) {
                status = OR_ENONFINITE;
                goto done;
            }
            const int accept = err <= 1.0;
            if (log && nlog < log_cap) {
                double *row = log + 5 * nlog++;
                row[0] = t; row[1] = h; row[2] = err; row[3] = accept;
                row[4] = accept ? t_new : t;
            }
            double fac;
            if (o->rule == 1) {
                fac = accept ? 2.0 : 0.5;
            } else {
                const double ex = o->rule == 2 ? 1.0 / 5.0 : 1.0 / (double)p;
                const double sf = o->rule == 2 ? 0.9 : s_fac;
                fac = err == 0.0 ? 10.0 : sf * pow(err, -ex);
                if (fac > 10.0) fac = 10.0;
                if (fac < 0.2) fac = 0.2;
            }
            if (accept) {
                t = t_new;
                h = h * fac;
                memcpy(y, ynew, sizeof(double) * (size_t)M);
                st->n_accept += 1;
                if (t < o->t_end) {
                    rhs_src(M, R, U, V, lam, src, y, f, nth);
                    st->n_rhs += 1;
                }
                break;
            }
            h = h * fac;
            st->n_reject += 1;
        }
    }
done:
    st->t = t;
    st->h = h;
    st->status = status;
    memcpy(n_out, y, sizeof(double) * (size_t)M);
    free(buf);
    return status;
}

/* ------------------------------------------------------------------ */
/* Moments, proposer features, MLP.                                    */
/* ------------------------------------------------------------------ */

/* mom[k] = sum_{s=1}^{M} s^k n_s, k = 0..3 */
void oracle_moments(int64_t M, const double *n, double *mom)
{
    for (int k = 0; k < 4; ++k) mom[k] = 0.0;
    for (int64_t s = 1; s <= M; ++s) {
        double ds = (double)s, v = n[s - 1];
        mom[0] += v;
        mom[1] += ds * v;
        mom[2] += ds * ds * v;
        mom[3] += ds * ds * ds * v;
    }
}

/* Feature vector of the step proposer, scaled to O(1) by fixed constants so
 * that the tanh units start unsaturated: log M0..log M3 of the state / 40,
 * log h / 10, log of the last four weighted error norms / 10 (most recent
 * first; entries with no history are 0).  Moments are floored at 1e-300
 * before the log. */
void oracle_proposer_features(const double *mom, double h,
                              const double *err_hist, int32_t n_hist, double *x)
{
    for (int k = 0; k < 4; ++k) x[k] = log(fmax(mom[k], 1e-300)) / 40.0;
    x[4] = log(h) / 10.0;
    for (int q = 0; q < 4; ++q)
        x[5 + q] = q < n_hist ? log(fmax(err_hist[q], 1e-300)) / 10.0 : 0.0;
}

void oracle_features(int64_t M, const double *n, double h,
                     const double *err_hist, int32_t n_hist, double *x)
{
    double mom[4];
    oracle_moments(M, n, mom);
    oracle_proposer_features(mom, h, err_hist, n_hist, x);
}

#define NIN 9
#define NH 64
/* parameter layout: W1[NH][NIN], b1[NH], W2[NH][NH], b2[NH], W3[NH], b3 */
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NIN)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH)
#define NPARAM (OFF_B3 + 1)

int32_t oracle_mlp_nparams(void) { return NPARAM; }

static void mlp_one(const double *p, const double *x, double *h1, double *h2,
                    double *y)
{
    for (int u = 0; u < NH; ++u) {
        double z = p[OFF_B1 + u];
        for (int i = 0; i < NIN; ++i) z += p[OFF_W1 + u * NIN + i] * x[i];
        h1[u] = tanh(z);
    }
    for (int u = 0; u < NH; ++u) {
        double z = p[OFF_B2 + u];
        for (int i = 0; i < NH; ++i) z += p[OFF_W2 + u * NH + i] * h1[i];
        h2[u] = tanh(z);
    }
    double z = p[OFF_B3];
    for (int i = 0; i < NH; ++i) z += p[OFF_W3 + i] * h2[i];
    *y = z;
}

void oracle_mlp_forward(const double *params, int64_t B, const double *X,
                        double *Y)
{
    double h1[NH], h2[NH];
    for (int64_t b = 0; b < B; ++b) mlp_one(params, X + b * NIN, h1, h2, Y + b);
}

/* loss = (1/B) sum_b w_b (y_b - t_b)^2 with w_b = over_w if y_b > t_b
 * else 1; grad = d loss / d params (same layout as params). */
void oracle_mlp_loss_grad(const double *params, int64_t B, const double *X,
                          const double *target, double over_w, double *loss,
                          double *grad)
{
    double h1[NH], h2[NH], d1[NH], d2[NH];
    memset(grad, 0, sizeof(double) * NPARAM);
    double L = 0.0;
    for (int64_t b = 0; b < B; ++b) {
        const double *x = X + b * NIN;
        double y;
        mlp_one(params, x, h1, h2, &y);
        double r = y - target[b];
        double w = r > 0 ? over_w : 1.0;
        L += w * r * r;
        double dy = 2.0 * w * r / (double)B;
        grad[OFF_B3] += dy;
        for (int i = 0; i < NH; ++i) {
            grad[OFF_W3 + i] += dy * h2[i];
            d2[i] = dy * params[OFF_W3 + i] * (1.0 - h2[i] * h2[i]);
        }
        for (int u = 0; u < NH; ++u) {
            grad[OFF_B2 + u] += d2[u];
            for (int i = 0; i < NH; ++i) grad[OFF_W2 + u * NH + i] += d2[u] * h1[i];
        }
        for (int i = 0; i < NH; ++i) {
            double acc = 0.0;
            for (int u = 0; u < NH; ++u) acc += params[OFF_W2 + u * NH + i] * d2[u];
            d1[i] = acc * (1.0 - h1[i] * h1[i]);
        }
        for (int u = 0; u < NH; ++u) {
            grad[OFF_B1 + u] += d1[u];
            for (int i = 0; i < NIN; ++i) grad[OFF_W1 + u * NIN + i] += d1[u] * x[i];
        }
    }
    *loss = L / (double)B;
}

/* One Adam update (Kingma & Ba 2015, Algorithm 1); step is 1-based. */
void oracle_adam(double *params, const double *grad, double *m, double *v,
                 int64_t n, int64_t step, double lr, double b1, double b2,
                 double eps)
{
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------ */
/* Learned step proposer: training rows and decisions.                 */
/* ------------------------------------------------------------------ */

#define LOG_FACMIN (-1.6094379124341003) /* log 0.2 */
#define LOG_FACMAX (2.302585092994046)   /* log 10 */

static double clamp_log(double d)
{
    return d < LOG_FACMIN ? LOG_FACMIN : (d > LOG_FACMAX ? LOG_FACMAX : d);
}

/* log of the PI step factor with the default exponents alpha = 0.7/k,
 * beta = 0.4/k: log clamp(0.9 err^-alpha err_prev^beta, 0.2, 10), and
 * log 10 for err = 0 (the same rule as the PI controller of
 * oracle_integrate). */
static double pi_log(double err, double err_prev, int32_t k)
{
    if (err == 0.0) return LOG_FACMAX;
    const double a = 0.7 / k, b = 0.4 / k;
    return clamp_log(log(0.9) - a * log(err) + b * log(err_prev));
}

/* Training rows from a run log (rows x 9: t, h, err, accepted, t_after,
 * M0..M3 of the state after the attempt).  The network decides the step
 * after an accepted attempt j that did not follow a rejection; a row is
 * made for every such j that has a successor attempt j+1 with h_{j+1} > 0
 * and a finite err_{j+1} > 0.
 *   features: oracle_proposer_features(moments of row j, h_j,
 *             err_j, err_{j-1}, err_{j-2}, err_{j-3} as far as they exist)
 *   target:   the hindsight log step that would have met err_target on the
 *             next attempt if err scaled as h^k,
 *             d = clamp(log(h_{j+1}/h_j) + log(err_target/err_{j+1}) / k),
 *             less the PI rule's log factor at decision j (err_j and
 *             err_prev = the err of the last accepted attempt before j,
 *             floored at 1e-4, or 1 when there is none), so that the
 *             network learns a correction to the PI step.
 * X (capacity rows x 9) and target (capacity rows) receive the rows in log
 * order; returns their number. */
int64_t oracle_proposer_dataset(const double *log_rows, int64_t rows, int32_t k,
                                double err_target, double *X, double *target)
{
    int64_t n = 0;
    double err_prev = 1.0; /* last accepted err before the current row */
    for (int64_t j = 0; j + 1 < rows; ++j) {
        const double *r = log_rows + j * 9, *nx = r + 9;
        const int accepted = r[3] == 1.0;
        const int after_reject = j > 0 && log_rows[(j - 1) * 9 + 3] != 1.0;
        if (accepted && !after_reject && r[1] > 0.0 && nx[1] > 0.0 && nx[2] > 0.0 &&
            isfinite(nx[2])) {
            double hist[4];
            int32_t nh = 0;
            for (int64_t q = j; q >= 0 && nh < 4; --q) hist[nh++] = log_rows[q * 9 + 2];
            oracle_proposer_features(r + 5, r[1], hist, nh, X + n * 9);
            const double d = clamp_log(log(nx[1] / r[1]) + log(err_target / nx[2]) / k);
            target[n] = d - pi_log(r[2], err_prev, k);
            ++n;
        }
        if (accepted) err_prev = fmax(r[2], 1e-4);
    }
    return n;
}

/* The learned controller's step factor h_next / h at a decision after an
 * accepted attempt that did not follow a rejection: the network output y
 * for the features (moments of the new state, h, error history) corrects
 * the PI rule in log space, h_next / h = exp(clamp(log PI + y)) with PI at
 * (err = err_hist[0], err_prev) and exponents 0.7/k, 0.4/k; when err
 * exceeds 0.5 the factor is at most PI's. */
double oracle_learned_factor(const double *params, const double *mom, double h,
                             const double *err_hist, int32_t n_hist, double err_prev,
                             int32_t k)
{
    double x[NIN], h1[NH], h2[NH], y;
    oracle_proposer_features(mom, h, err_hist, n_hist, x);
    mlp_one(params, x, h1, h2, &y);
    const double pi = pi_log(err_hist[0], err_prev, k);
    double d = clamp_log(pi + y);
    if (err_hist[0] > 0.5 && d > pi) d = pi;
    return exp(d);
}

/* Replay of a learned-controller run log (rows x 9 as above): ratio[j] =
 * h_{j+1} / h_j that the learned controller takes at decision j, for every
 * accepted attempt j that did not follow a rejection (err_prev: the err of
 * the last accepted attempt before j, floored at 1e-4, or 1); NaN where
 * the PI rule decides (after a rejection) or attempt j was rejected.  The
 * last row's ratio is NaN (no successor). */
void oracle_learned_steps(const double *params, const double *log_rows, int64_t rows,
                          int32_t k, double *ratio)
{
    double err_prev = 1.0;
    for (int64_t j = 0; j < rows; ++j) {
        const double *r = log_rows + j * 9;
        const int accepted = r[3] == 1.0;
        const int after_reject = j > 0 && log_rows[(j - 1) * 9 + 3] != 1.0;
        ratio[j] = NAN;
        if (accepted && !after_reject && j + 1 < rows) {
            double hist[4];
            int32_t nh = 0;
            for (int64_t q = j; q >= 0 && nh < 4; --q) hist[nh++] = log_rows[q * 9 + 2];
            ratio[j] = oracle_learned_factor(params, r + 5, r[1], hist, nh, err_prev, k);
        }
        if (accepted) err_prev = fmax(r[2], 1e-4);
    }
}

