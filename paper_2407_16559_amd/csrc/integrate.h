// Embedded explicit Runge--Kutta integration of dn/dt = S(n) (Sec. 2,
// Eq. (5)) with adaptive steps, as kernels that read a device-resident
// control block.  One step attempt is a fixed kernel sequence
//     [A_i B_i C_i] for stages i = 2..S, then the controller,
// so it is captured once as a hipGraph and replayed; once the run is done
// every kernel returns at entry, which makes surplus replays no-ops.
//
// Stage i computes k_i = S(y_i).  The stage state y_{i+1} = n + h sum_j
// a_{i+1,j} k_j and its four reductions are produced in the epilogue of
// stage i's finish (phase C), so phase A of stage i+1 only reads y; stage 2
// forms y_2 = n + h a_21 k_1 in its phase A because h is only known after
// the controller.  The last stage state is the propagated solution (FSAL),
// written straight into the second state buffer; the last finish also
// accumulates the weighted-RMS error norm and the moments of n_new.
#pragma once
#include "rhs.h"

// Status codes, mirrored from smol.h for device code.
#define ST_OK 0
#define ST_ESTEPSIZE (-4)
#define ST_EMAXSTEPS (-5)
#define ST_ENONFINITE (-6)
// Controllers, mirrored from smol.h.
#define CTRL_LEARNED 1        // SMOL_CTRL_LEARNED
#define CTRL_FEHLBERG 2       // SMOL_CTRL_FEHLBERG
#define CTRL_EQ6 3            // SMOL_CTRL_STEP_DOUBLING
#define CTRL_HALVE_DOUBLE 4   // SMOL_CTRL_HALVE_DOUBLE

struct Tableau {
    int S;             // stages including the FSAL stage
    int q;             // order of the embedded solution
    double a[8][8];    // a[i][j], 0-based
    double d[8];       // b_j - bhat_j
    int fsal;          // stage slot paired with slot 0 (k_1 / k_S swap on accept)
    int program;       // 1: stages 3..S follow the RK4 step-doubling program
};

// Bogacki & Shampine (1989) 3(2), Dormand & Prince (1980) 5(4), and two of
// the paper's schemes (Sec. 2) written as tableaux whose last stage is
// evaluated at the propagated solution, so that they run on the same stage
// machinery:
//   RKF45 (Fehlberg 1970), propagating the fourth-order solution: stages 1-6
//   as printed, stage 7 = S(n^{k+1}) (the next step's k_1); d = b4 - b5.
//   RK2 with step doubling: stage 2 is the single step's second stage
//   (n + h k1), stages 3-5 the two half steps (n + h/2 k1; the midpoint
//   n + h/4 (k1 + k3); its half step n + h (k1/4 + k3/4 + k4/2)), stage 6 the
//   two-half-step solution nhat (propagated); d = nhat - single step.
__constant__ Tableau c_tab[5] = {
    {4, 2,
     {{0}, {1.0 / 2}, {0.0, 3.0 / 4}, {2.0 / 9, 1.0 / 3, 4.0 / 9}},
     {2.0 / 9 - 7.0 / 24, 1.0 / 3 - 1.0 / 4, 4.0 / 9 - 1.0 / 3, -1.0 / 8},
     3},
    {7, 4,
     {{0},
      {1.0 / 5},
      {3.0 / 40, 9.0 / 40},
      {44.0 / 45, -56.0 / 15, 32.0 / 9},
      {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
      {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656},
      {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}},
     {35.0 / 384 - 5179.0 / 57600, 0.0, 500.0 / 1113 - 7571.0 / 16695, 125.0 / 192 - 393.0 / 640,
      -2187.0 / 6784 + 92097.0 / 339200, 11.0 / 84 - 187.0 / 2100, -1.0 / 40},
     6},
    {7, 4,
     {{0},
      {1.0 / 4},
      {3.0 / 32, 9.0 / 32},
      {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197},
      {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104},
      {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40},
      {25.0 / 216, 0.0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0.0}},
     {25.0 / 216 - 16.0 / 135, 0.0, 1408.0 / 2565 - 6656.0 / 12825,
      2197.0 / 4104 - 28561.0 / 56430, -1.0 / 5 + 9.0 / 50, -2.0 / 55, 0.0},
     6},
    {6, 2,
     {{0},
      {1.0},
      {1.0 / 2, 0.0},
      {1.0 / 4, 0.0, 1.0 / 4},
      {1.0 / 4, 0.0, 1.0 / 4, 1.0 / 2},
      {1.0 / 4, 0.0, 1.0 / 4, 1.0 / 4, 1.0 / 4}},
     {1.0 / 4 - 1.0 / 2, -1.0 / 2, 1.0 / 4, 1.0 / 4, 1.0 / 4, 0.0},
     5},
    // RK4 with step doubling: twelve stages whose combinations do not fit a
    // tableau of this size; only a_21 (the single step's k_2 at n + h/2 k_1)
    // is read from here, the rest is the stage program of rk4d_epi.
    {12, 4, {{0}, {1.0 / 2}}, {0}, 5, 1},
};

struct IntegCtl {
    // problem, written by the host before a run
    const double *U, *V;
    double lam, t_end, rtol, atol, h_min, h0_user;
    double alpha, beta, safety, facmin, facmax;
    int64_t max_steps;
    double *log;
    int64_t log_cap;
    const float *mlp;  // proposer weights (learned mode)
    int32_t method, controller;
    // dynamic state
    double t, h, t_new, err, err_prev, min_step, h0;
    int64_t n_rhs, n_accept, n_reject, attempts;
    int32_t status, done, cur, kp, rejected, n_fallback;
    double err_hist[4];
    int32_t n_hist, use_pi;
    // the paper's controllers: Euclidean error norm (sc = tol), Eq. (6) safety
    int32_t l2;
    double paper_s;
    int32_t has_src;  // Eq. (3) sources present
    // an attempt has run whose accept / reject decision is still to be
    // taken (by the next stage-2 column pass of a captured step)
    int32_t pending;
};

// Step factor of the paper's rules (Sec. 2): Fehlberg's fifth-root rule
// with 0.9, Eq. (6) s (tol/err)^(1/p), or halving / doubling; clipped to
// [facmin, facmax], err = 0 giving facmax.
__device__ inline double paper_factor(const IntegCtl &c, int q, double err, bool accept)
{
    if (c.controller == CTRL_HALVE_DOUBLE) return accept ? 2.0 : 0.5;
    const bool fehl = c.controller == CTRL_FEHLBERG;
    const double ex = fehl ? 1.0 / (double)(q + 1) : 1.0 / (double)q;
    double fac = err == 0.0 ? c.facmax : (fehl ? 0.9 : c.paper_s) * pow(err, -ex);
    return fmin(fmax(fac, c.facmin), c.facmax);
}

struct IntegDev {
    int64_t M, Mt;
    int R, logL;
    double *Ut, *Vt;  // transposed copies of U and V
    IntegCtl *ctl;
    double *nb[2];
    double *kslot[8];
    double *ybuf;
    double *src;      // transposed sources (used when the control block says so)
    void *Z, *Qp;
    double *red_part, *red, *epart;
    Roots rt;
};

__device__ __forceinline__ RhsPlanDev plan_of(const IntegDev &I, const IntegCtl &c)
{
    RhsPlanDev P;
    P.M = I.M;
    P.R = I.R;
    P.logL = I.logL;
    P.logN1 = split_log_n1(I.logL);
    P.logN2 = split_log_n2(I.logL);
    P.tr = 1;
    P.ustride = I.Mt;
    P.lam = c.lam;
    P.U = I.Ut;
    P.V = I.Vt;
    P.Z = I.Z;
    P.Qp = I.Qp;
    P.red_part = I.red_part;
    P.red = I.red;
    P.src = c.has_src ? I.src : nullptr;
    P.rt = I.rt;
    return P;
}

// The plan fields that do not depend on the control block (transform
// shape, factors, workspaces, roots): all the row-pair pass uses, and what
// the finish loads before it reads the control block.
__device__ __forceinline__ RhsPlanDev plan_of_ws(const IntegDev &I)
{
    RhsPlanDev P{};
    P.M = I.M;
    P.R = I.R;
    P.U = I.Ut;
    P.V = I.Vt;
    P.logL = I.logL;
    P.logN1 = split_log_n1(I.logL);
    P.logN2 = split_log_n2(I.logL);
    P.tr = 1;
    P.ustride = I.Mt;
    P.Z = I.Z;
    P.Qp = I.Qp;
    P.red_part = I.red_part;
    P.red = I.red;
    P.rt = I.rt;
    return P;
}

// stage j (1-based) vector given the FSAL parity kp
__device__ __forceinline__ double *kvec(const IntegDev &I, const IntegCtl &c, const Tableau &T, int j)
{
    if (j == 1) return I.kslot[c.kp ? T.fsal : 0];
    if (j == T.S) return I.kslot[c.kp ? 0 : T.fsal];
    return I.kslot[j - 1];
}

// stage codes: 0 = S(n0) for the starting step, 1 = S(n0 + h0 f0), 2..S
__device__ __forceinline__ Pro stage_pro(const IntegDev &I, const IntegCtl &c, const Tableau &T,
                                         int stage)
{
    const int S = T.S;
    double *n = I.nb[c.cur];
    if (stage == 0) return Pro{A_COMBINE, n, nullptr, 0.0, nullptr};
    if (stage == 1) return Pro{A_COMBINE, n, kvec(I, c, T, 1), c.h0, I.ybuf};
    if (stage == 2) return Pro{A_COMBINE, n, kvec(I, c, T, 1), c.h * T.a[1][0], I.ybuf};
    return Pro{A_GIVEN, stage == S ? I.nb[c.cur ^ 1] : I.ybuf, nullptr, 0.0, nullptr};
}

// RK4 with step doubling (Sec. 2: one classical RK4 step of size h and two
// of size h/2 from the same state, the two half steps propagated, the error
// their difference) as a twelve-stage program on the stage machinery:
//   stages 2-4   the single step: k_2 = S(n + h/2 k_1), k_3 = S(n + h/2 k_2),
//                k_4 = S(n + h k_3);
//   stages 5-7   the first half step: k_5 = S(n + h/4 k_1),
//                k_6 = S(n + h/4 k_5), k_7 = S(n + h/2 k_6), ending on the
//                midpoint m = n + h/12 (k_1 + 2 k_5 + 2 k_6 + k_7);
//   stages 8-11  the second half step from m: k_8 = S(m),
//                k_9 = S(m + h/4 k_8), k_10 = S(m + h/4 k_9),
//                k_11 = S(m + h/2 k_10), nhat = m + h/12 (k_8 + 2 k_9 + 2 k_10 + k_11);
//   stage 12     k_12 = S(nhat), the next attempt's k_1, with the error
//                nhat - n_single = (nhat - n) + h D.
// Stage 4 stores D = -(k_1 + 2 k_2 + 2 k_3 + k_4) / 6 in place of k_4 (the
// single step is needed only through D), so seven slots suffice:
//   slot 0 / fsal  k_1 and k_12 (k_11 is written where k_12 will go);
//   1: k_2, k_5, k_8;  2: k_3, k_6, k_9;  3: D;  4: k_7, k_10;  6: m.
__device__ inline Epi rk4d_epi(const IntegDev &I, const IntegCtl &c, const Tableau &T, int stage)
{
    Epi ep{};
    ep.n = I.nb[c.cur];
    ep.h = c.h;
    ep.rtol = c.rtol;
    ep.atol = c.atol;
    ep.epart = I.epart;
    ep.mode = C_STAGE;
    ep.y = I.ybuf;
    ep.ynext = I.ybuf;
    double *k1 = kvec(I, c, T, 1), *k12 = kvec(I, c, T, T.S), *m = I.kslot[6];
    switch (stage) {
    case 2: ep.out = I.kslot[1]; ep.cS = 1.0 / 2; break;
    case 3: ep.out = I.kslot[2]; ep.cS = 1.0; break;
    case 4:
        ep.out = I.kslot[3];
        ep.ks[0] = k1;
        ep.ks[1] = I.kslot[1];
        ep.ks[2] = I.kslot[2];
        ep.coef[0] = 1.0 / 4;
        ep.nks = 3;
        ep.ocomb = 1;
        ep.oS = -1.0 / 6;
        ep.ocoef[0] = -1.0 / 6;
        ep.ocoef[1] = -1.0 / 3;
        ep.ocoef[2] = -1.0 / 3;
        break;
    case 5: ep.out = I.kslot[1]; ep.cS = 1.0 / 4; break;
    case 6: ep.out = I.kslot[2]; ep.cS = 1.0 / 2; break;
    case 7:
        ep.out = I.kslot[4];
        ep.ynext = m;
        ep.ks[0] = k1;
        ep.ks[1] = I.kslot[1];
        ep.ks[2] = I.kslot[2];
        ep.coef[0] = 1.0 / 12;
        ep.coef[1] = 1.0 / 6;
        ep.coef[2] = 1.0 / 6;
        ep.cS = 1.0 / 12;
        ep.nks = 3;
        break;
    case 8: ep.y = m; ep.n = m; ep.out = I.kslot[1]; ep.cS = 1.0 / 4; break;
    case 9: ep.n = m; ep.out = I.kslot[2]; ep.cS = 1.0 / 4; break;
    case 10: ep.n = m; ep.out = I.kslot[4]; ep.cS = 1.0 / 2; break;
    case 11:
        ep.n = m;
        ep.out = k12;
        ep.ynext = I.nb[c.cur ^ 1];
        ep.ks[0] = I.kslot[1];
        ep.ks[1] = I.kslot[2];
        ep.ks[2] = I.kslot[4];
        ep.coef[0] = 1.0 / 12;
        ep.coef[1] = 1.0 / 6;
        ep.coef[2] = 1.0 / 6;
        ep.cS = 1.0 / 12;
        ep.nks = 3;
        break;
    default:  // stage 12
        ep.mode = C_LAST;
        ep.y = I.nb[c.cur ^ 1];
        ep.out = k12;
        ep.ks[0] = I.kslot[3];
        ep.coef[0] = 1.0;
        ep.nks = 1;
        ep.diff = 1;
        break;
    }
    return ep;
}

__device__ inline Epi stage_epi(const IntegDev &I, const IntegCtl &c, const Tableau &T, int stage)
{
    const int S = T.S;
    if (T.program && stage >= 2) return rk4d_epi(I, c, T, stage);
    Epi ep{};
    ep.n = I.nb[c.cur];
    ep.h = c.h;
    ep.rtol = c.rtol;
    ep.atol = c.atol;
    ep.epart = I.epart;
    if (stage == 0) {
        ep.mode = C_INIT0;
        ep.y = ep.n;
        ep.out = kvec(I, c, T, 1);
    } else if (stage == 1) {
        ep.mode = C_INIT1;
        ep.y = I.ybuf;
        ep.ks[0] = kvec(I, c, T, 1);
        ep.coef[0] = 1.0;  // marks the slot as used: f0
        ep.nks = 1;
    } else if (stage < S) {
        // fixed slots j-1 for k_j (zero coefficients are skipped at use)
        ep.mode = C_STAGE;
        ep.y = I.ybuf;
        ep.out = kvec(I, c, T, stage);
        ep.ynext = (stage + 1 == S) ? I.nb[c.cur ^ 1] : I.ybuf;
#pragma unroll
        for (int j = 1; j < SMOL_MAX_STAGE; ++j) {
            ep.ks[j - 1] = kvec(I, c, T, j < S ? j : 1);
            ep.coef[j - 1] = j < stage ? T.a[stage][j - 1] : 0.0;
        }
        ep.nks = stage - 1;
        ep.cS = T.a[stage][stage - 1];
    } else {
        ep.mode = C_LAST;
        ep.y = I.nb[c.cur ^ 1];
        ep.out = kvec(I, c, T, S);
#pragma unroll
        for (int j = 1; j < SMOL_MAX_STAGE; ++j) {
            ep.ks[j - 1] = kvec(I, c, T, j < S ? j : 1);
            ep.coef[j - 1] = j < S ? T.d[j - 1] : 0.0;
        }
        ep.nks = S - 1;
        ep.cS = T.d[S - 1];
    }
    return ep;
}

// Device tables of a batched run.  Instances are grouped by transform shape;
// each kernel's workgroups over a shape's instances are contiguous, so one
// launch per shape covers blocks [base, base + count).
struct BatchDev {
    const IntegDev *inst;   // per instance
    const int *logL;        // per instance
    const int *first[3];    // first block of each instance per kernel A, B, C
    const int *owner[3];    // instance of each block per kernel
    const int *nC;          // finish units per instance
    const int *redA;        // column-pass reduction jobs per instance
    const int *active;      // instances still running (one controller workgroup each)
};

// Prepare the next attempt (one thread): step-start clamp, limits, t_end clip.
__device__ inline void prepare_attempt(IntegCtl &c, bool new_step)
{
    if (new_step) {
        double ms = 10.0 * fabs(nextafter(c.t, INFINITY) - c.t);
        if (c.h_min > ms) ms = c.h_min;
        c.min_step = ms;
        if (c.h < ms) c.h = ms;
    }
    if (c.attempts >= c.max_steps) {
        c.status = ST_EMAXSTEPS;
        c.done = 1;
        return;
    }
    if (!(c.h >= c.min_step)) {
        c.status = ST_ESTEPSIZE;
        c.done = 1;
        return;
    }
    double tn = c.t + c.h;
    if (tn > c.t_end) tn = c.t_end;
    c.t_new = tn;
    c.h = tn - c.t;
}

// Deterministic block reduction of epart rows, in two parts so that a
// kernel can request the rows before it knows whether it needs them.
// epart_partial: the first SMOL_WG threads each sum a fixed stride of rows
// (the others hold zeros).  epart_total (a workgroup of NT threads): the
// wave butterfly adds the threads of a wave, then the waves are added in
// order; waves beyond the first SMOL_WAVES add zeros, so any NT gives the
// same totals.  Every thread receives them.
__device__ inline void epart_partial(const double *ep, int njobs, double *acc)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < SMOL_EPART; ++q) acc[q] = 0.0;
    if (tid < SMOL_WG)
        for (int j = tid; j < njobs; j += SMOL_WG)
#pragma unroll
            for (int q = 0; q < SMOL_EPART; ++q) acc[q] += ep[(int64_t)j * SMOL_EPART + q];
}
template <int NT = SMOL_WG>
__device__ inline void epart_total(double *acc, double *tot)
{
    __shared__ double sh[NT / 64][SMOL_EPART];
#pragma unroll
    for (int q = 0; q < SMOL_EPART; ++q) acc[q] = wave_sum(acc[q]);
    if (lane_id() == 0)
#pragma unroll
        for (int q = 0; q < SMOL_EPART; ++q) sh[wave_id()][q] = acc[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SMOL_EPART; ++q) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) a += sh[w][q];
        tot[q] = a;
    }
    __syncthreads();
}
__device__ inline void block_sum_epart(const double *ep, int njobs, double *tot)
{
    double acc[SMOL_EPART];
    epart_partial(ep, njobs, acc);
    epart_total<SMOL_WG>(acc, tot);
}

// ---- learned step proposer ----------------------------------------------
// 9-64-64-1 tanh MLP, FP32, parameters W1[64][9], b1[64], W2[64][64], b2[64],
// W3[64], b3 (4865 floats).  Output: log(h_next / h).
#define MLP_NIN 9
#define MLP_NH 64
#define MLP_OFF_B1 (MLP_NH * MLP_NIN)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_NH)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_NH * MLP_NH)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_NH)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_NH)
#define MLP_NPARAM (MLP_OFF_B3 + 1)
#define MLP_LOG_FMIN (-1.6094379124341003)  // log 0.2
#define MLP_LOG_FMAX (2.302585092994046)    // log 10
#define MLP_CAP_ERR 0.5  // above this error norm the learned step never exceeds PI's

// log of the PI factor clamp(0.9 err^-alpha err_prev^beta, 0.2, 10)
// (err = 0: 10), the base the learned proposer corrects.
__host__ __device__ inline double pi_log_factor(double err, double err_prev, double alpha,
                                                double beta)
{
    const double fac = err == 0.0 ? 10.0 : 0.9 * pow(err, -alpha) * pow(err_prev, beta);
    return log(fmin(fmax(fac, 0.2), 10.0));
}

// Features: log-moments of the new state / 40, log h / 10, log of the last
// four error norms (most recent first, missing ones 0) / 10.
__device__ __forceinline__ void proposer_features(const double *mom, double h, const double *hist,
                                                  int nh, float *x)
{
    for (int k = 0; k < 4; ++k) x[k] = (float)(log(fmax(mom[k], 1e-300)) / 40.0);
    x[4] = (float)(log(h) / 10.0);
    for (int q = 0; q < 4; ++q) x[5 + q] = q < nh ? (float)(log(fmax(hist[q], 1e-300)) / 10.0) : 0.0f;
}

// Forward pass by a whole workgroup (fixed summation order); every thread
// receives the output.
__device__ inline float mlp_forward_block(const float *p, const float *x)
{
    __shared__ float h1[MLP_NH], h2[MLP_NH], y;
    const int tid = threadIdx.x;
    if (tid < MLP_NH) {
        float z = p[MLP_OFF_B1 + tid];
        for (int i = 0; i < MLP_NIN; ++i) z = fmaf(p[tid * MLP_NIN + i], x[i], z);
        h1[tid] = tanhf(z);
    }
    __syncthreads();
    if (tid < MLP_NH) {
        float z = p[MLP_OFF_B2 + tid];
        for (int i = 0; i < MLP_NH; ++i) z = fmaf(p[MLP_OFF_W2 + tid * MLP_NH + i], h1[i], z);
        h2[tid] = tanhf(z);
    }
    __syncthreads();
    if (tid == 0) {
        float z = p[MLP_OFF_B3];
        for (int i = 0; i < MLP_NH; ++i) z = fmaf(p[MLP_OFF_W3 + i], h2[i], z);
        y = z;
    }
    __syncthreads();
    const float out = y;
    __syncthreads();
    return out;
}

__device__ __forceinline__ double rms_of(double sumsq, int64_t M) { return sqrt(sumsq / (double)M); }

// Starting step, first half: d0, d1 from S(n0); h0.  With a user h0 the
// first attempt is prepared right away.  Whole workgroup.
__device__ inline void init_h0_step(const IntegDev &I, int njobs)
{
    IntegCtl &c = *I.ctl;
    if (c.done) return;
    double tot[SMOL_EPART];
    block_sum_epart(I.epart, njobs, tot);
    if (threadIdx.x) return;
    c.n_rhs = 1;
    if (tot[5] > 0.0) {
        c.status = ST_ENONFINITE;
        c.done = 1;
        c.n_rhs = 0;
        return;
    }
    const double d0 = rms_of(tot[0], I.M), d1 = rms_of(tot[1], I.M);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    if (h0 > c.t_end) h0 = c.t_end;
    c.h0 = h0;
    c.err = d1;  // kept for the second half
    if (c.h0_user > 0.0) {
        c.h = c.h0_user > c.t_end ? c.t_end : c.h0_user;
        prepare_attempt(c, true);
    }
}

// Starting step, second half (Hairer, Norsett & Wanner I, Sec. II.4).
// Whole workgroup.
__device__ inline void init_h_step(const IntegDev &I, int njobs)
{
    IntegCtl &c = *I.ctl;
    if (c.done) return;
    double tot[SMOL_EPART];
    block_sum_epart(I.epart, njobs, tot);
    if (threadIdx.x) return;
    const Tableau &T = c_tab[c.method];
    c.n_rhs = 2;
    const double d1 = c.err, h0 = c.h0;
    const double d2 = rms_of(tot[0], I.M) / h0;
    double h1;
    if (d1 <= 1e-15 && d2 <= 1e-15)
        h1 = fmax(1e-6, h0 * 1e-3);
    else
        h1 = pow(0.01 / fmax(d1, d2), 1.0 / (double)(T.q + 1));
    double h = 100.0 * h0;
    if (h1 < h) h = h1;
    if (c.t_end < h) h = c.t_end;
    c.h = h;
    c.err = 0.0;
    prepare_attempt(c, true);
}

// Accept / reject and the next step size after the last stage, from the
// attempt's reduced error partials tot.  PI control, or (learned mode) the
// proposer's log(h_next/h) after an accepted step that did not follow a
// rejection, with PI as the fallback after a rejection or for non-finite
// features.  Called by every thread of a workgroup (the proposer's forward
// pass uses them all, and a barrier separates their reads of c from the
// update); thread 0 updates c, which may be the control block itself or a
// workgroup's shared copy of it, and writes the attempt's log row when
// log_row is set.
__device__ inline void controller_decide(IntegCtl &c, const double *tot, int64_t M, bool log_row)
{
    const Tableau &T = c_tab[c.method];
    const int k = T.q + 1;
    const double err = c.l2 ? sqrt(tot[0]) : rms_of(tot[0], M);
    const bool accept = err <= 1.0;
    const bool bad = isnan(err) || tot[5] > 0.0;
    // error history including this attempt (most recent first)
    double hist[4] = {err, c.err_hist[0], c.err_hist[1], c.err_hist[2]};
    const int nh = c.n_hist < 3 ? c.n_hist + 1 : 4;
    bool learned = false;
    double dlog = 0.0;
    if (c.controller == CTRL_LEARNED && c.mlp && accept && !bad && !c.rejected) {
        float x[MLP_NIN];
        proposer_features(tot + 1, c.h, hist, nh, x);
        bool finite = true;
        for (int q = 0; q < MLP_NIN; ++q) finite = finite && isfinite(x[q]);
        if (finite) {
            const float y = mlp_forward_block(c.mlp, x);
            if (isfinite(y)) {
                learned = true;
                const double base = pi_log_factor(err, c.err_prev, c.alpha, c.beta);
                dlog = fmin(fmax(base + (double)y, MLP_LOG_FMIN), MLP_LOG_FMAX);
                // near the acceptance limit err grows much faster than h^k
                // (stability), so there the network may only shrink the step
                if (err > MLP_CAP_ERR && dlog > base) dlog = base;
            }
        }
    }
    // every thread has read c (its branches above depend on it) before
    // thread 0 updates it
    __syncthreads();
    if (threadIdx.x) return;
    c.err = err;
    c.attempts += 1;
    c.n_rhs += T.S - 1;
    for (int q = 0; q < 4; ++q) c.err_hist[q] = hist[q];
    c.n_hist = nh;
    if (c.log && log_row && c.attempts <= c.log_cap) {
        double *row = c.log + (c.attempts - 1) * 9;
        row[0] = c.t;
        row[1] = c.h;
        row[2] = err;
        row[3] = accept ? 1.0 : 0.0;
        row[4] = accept ? c.t_new : c.t;
        row[5] = tot[1];
        row[6] = tot[2];
        row[7] = tot[3];
        row[8] = tot[4];
    }
    // a NaN norm or a non-finite new state ends the run (state kept)
    if (bad) {
        c.status = ST_ENONFINITE;
        c.done = 1;
        return;
    }
    const bool paper = c.controller >= CTRL_FEHLBERG;
    if (accept) {
        double fac;
        if (paper) {
            fac = paper_factor(c, T.q, err, true);
        } else if (learned) {
            fac = exp(dlog);
        } else {
            if (c.controller == CTRL_LEARNED) c.n_fallback += 1;
            if (err == 0.0)
                fac = c.facmax;
            else
                fac = c.safety * pow(err, -c.alpha) * pow(c.err_prev, c.beta);
            if (c.rejected && fac > 1.0) fac = 1.0;
        }
        if (fac > c.facmax) fac = c.facmax;
        if (fac < c.facmin) fac = c.facmin;
        c.err_prev = fmax(err, 1e-4);
        c.t = c.t_new;
        c.h = c.h * fac;
        c.cur ^= 1;
        c.kp ^= 1;
        c.n_accept += 1;
        c.rejected = 0;
        if (c.t >= c.t_end) {
            c.status = ST_OK;
            c.done = 1;
            return;
        }
        prepare_attempt(c, true);
    } else {
        double fac;
        if (paper) {
            fac = paper_factor(c, T.q, err, false);
        } else {
            fac = c.safety * pow(err, -1.0 / (double)k);
            if (fac < c.facmin) fac = c.facmin;
        }
        c.h = c.h * fac;
        c.rejected = 1;
        c.n_reject += 1;
        prepare_attempt(c, false);
    }
}

// The decision by its own one-workgroup kernel (batched runs): the error
// rows reduced here, the control block updated in place.
__device__ inline void controller_step(const IntegDev &I, int njobs)
{
    IntegCtl &c = *I.ctl;
    if (c.done) return;
    double tot[SMOL_EPART];
    block_sum_epart(I.epart, njobs, tot);
    controller_decide(c, tot, I.M, true);
}
