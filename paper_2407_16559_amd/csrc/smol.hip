// libsmol: C ABI, plans and kernel launches (gfx950).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "sched.h"
#include "schedule_table.h"

SMOL_HIDDEN std::mutex g_mu;

#define SMOL_VERSION "0.1.0"

// --------------------------------------------------------------------------
// Kernels of this unit: layout conversion, starting step, controller, resume.
// The right-hand-side phase kernels live in phases_a/b/c.hip (see sched.h).
// --------------------------------------------------------------------------

// Layout conversion of `rows` vectors of M sizes: natural <-> transposed.
__global__ void k_to_tr(const double *src, double *dst, int64_t M, int rows, int64_t sstride,
                        int64_t dstride, int logL)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M * rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / M, idx = i % M;
        dst[r * dstride + pos_tr(idx, logL)] = src[r * sstride + idx];
    }
}
__global__ void k_from_tr(const double *src, double *dst, int64_t M, int logL)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[pos_tr(i, logL)];
}


__global__ __launch_bounds__(SMOL_WG) void k_init_h0(IntegDev I, int njobs) { init_h0_step(I, njobs); }
__global__ __launch_bounds__(SMOL_WG) void k_init_h(IntegDev I, int njobs) { init_h_step(I, njobs); }

// Resume from a checkpoint: the smallest step at the state's time, then the
// next attempt prepared as the interrupted run would have prepared it (after
// a rejection the step is not raised to the minimum).  One thread.
__global__ void k_resume(IntegDev I)
{
    if (threadIdx.x) return;
    IntegCtl &c = *I.ctl;
    double ms = 10.0 * fabs(nextafter(c.t, INFINITY) - c.t);
    if (c.h_min > ms) ms = c.h_min;
    c.min_step = ms;
    prepare_attempt(c, !c.rejected);
}

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------

namespace {



struct Plan {
    int dev = -1;
    int64_t M = 0;
    int R = 0, precision = 0;
    int logL = 0, logN1 = 0, logN2 = 0;
    cd *Z = nullptr, *Qp = nullptr;  // cd or cff storage (16 B per complex either way)
    double *red_part = nullptr, *red = nullptr, *epart = nullptr;
    // integration state (allocated on first use)
    int64_t Mt = 0;                // vector length in the transposed layout
    double *ibuf = nullptr;        // nb[2], kslot[7], ybuf, sources: 11 Mt doubles
    double *uvt = nullptr;         // transposed U and V: 2 R Mt doubles
    IntegCtl *ctl = nullptr;       // device control block
    IntegCtl *host = nullptr;      // pinned mirror
    hipStream_t cap = nullptr;     // capture stream
    hipGraphExec_t graph[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // per scheme
    // launch schedule: variant of kernels A, B, C and their grids
    int var[3] = {0, 0, 0};
    PhaseDims dA{}, dB{}, dC{}, dCf{};
    // stream order of the workspaces: the last call that enqueued work using
    // them without waiting for it recorded used_ev on used_s
    hipEvent_t used_ev = nullptr;
    hipStream_t used_s = nullptr;
    bool busy = false;
};

// Schedule variants per transform length for FP64 plans (float-float plans
// use variant 0), initialised from the tuned table and changed by
// smol_set_schedule / smol_autotune.
int g_sched[SMOL_LOG_LMAX + 1][3];
bool g_sched_init = false;

void sched_init()
{
    if (g_sched_init) return;
    memset(g_sched, 0, sizeof(g_sched));
    for (const auto &row : k_sched_table)
        if (row[0] >= 0 && row[0] <= SMOL_LOG_LMAX)
            for (int k = 0; k < 3; ++k) g_sched[row[0]][k] = row[1 + k];
    g_sched_init = true;
}

std::map<int, DevRoots> g_roots;
std::map<std::tuple<int, int64_t, int, int>, Plan *> g_plans;


}  // namespace

SMOL_HIDDEN int get_roots(int dev, DevRoots **out)
{
    auto it = g_roots.find(dev);
    if (it != g_roots.end()) {
        *out = &it->second;
        return SMOL_OK;
    }
    std::vector<cd> host(2 * SMOL_TW);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int e = 0; e < SMOL_TW; ++e) {
        long double a = two_pi * (long double)e / (long double)SMOL_TW;
        host[e] = cd{(double)cosl(a), (double)-sinl(a)};
        long double b = two_pi * (long double)e / (long double)(1 << SMOL_LOG_LMAX);
        host[SMOL_TW + e] = cd{(double)cosl(b), (double)-sinl(b)};
    }
    DevRoots r;
    HIP_TRY(hipMalloc(&r.tw, sizeof(cd) * 2 * SMOL_TW));
    r.fine = r.tw + SMOL_TW;
    HIP_TRY(hipMemcpy(r.tw, host.data(), sizeof(cd) * 2 * SMOL_TW, hipMemcpyHostToDevice));
    g_roots[dev] = r;
    *out = &g_roots[dev];
    return SMOL_OK;
}

namespace {

// Point plan p at schedule v[3] (grids, LDS); drops captured graphs.
int set_plan_sched(Plan *p, const int *v)
{
    PhaseDims a, b, c, cf;
    int rc;
    if ((rc = phase_dims(p->logL, p->precision, PH_A, v[0], p->R, false, &a))) return rc;
    if ((rc = phase_dims(p->logL, p->precision, PH_B, v[1], p->R, false, &b))) return rc;
    if ((rc = phase_dims(p->logL, p->precision, PH_C, v[2], p->R, false, &c))) return rc;
    if ((rc = phase_dims(p->logL, p->precision, PH_C, v[2], p->R, true, &cf))) return rc;
    for (auto &g : p->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (int k = 0; k < 3; ++k) p->var[k] = v[k];
    p->dA = a;
    p->dB = b;
    p->dC = c;
    p->dCf = cf;
    return SMOL_OK;
}

void free_plan(Plan *p)
{
    if (!p) return;
    if (p->used_ev) (void)hipEventDestroy(p->used_ev);
    (void)hipFree(p->Z);  // Qp lives in the same allocation
    (void)hipFree(p->red_part);
    for (auto &g : p->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    (void)hipFree(p->ibuf);
    (void)hipFree(p->uvt);
    (void)hipFree(p->ctl);
    if (p->host) (void)hipHostFree(p->host);
    delete p;
}

int get_plan(int64_t M, int R, int precision, Plan **out)
{
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    auto key = std::make_tuple(dev, M, R, precision);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second;
        return SMOL_OK;
    }
    Plan *p = new Plan();
    p->dev = dev;
    p->M = M;
    p->R = R;
    p->precision = precision;
    int logL = ilog2_ceil(2 * M - 2);
    if (logL < 6) logL = 6;
    p->logL = logL;
    p->logN1 = split_log_n1(logL);
    p->logN2 = split_log_n2(logL);
    const int64_t L = 1LL << logL;
    const int64_t N2 = 1LL << p->logN2;
    hipError_t e = hipMalloc(&p->Z, sizeof(cd) * (size_t)(R * L + L / 2));
    if (e != hipSuccess) {
        delete p;
        return SMOL_ENOMEM;
    }
    p->Qp = p->Z + R * L;
    const size_t nred = (size_t)N2 * R * 4 + (size_t)R * 4 + (size_t)N2 * SMOL_EPART;
    e = hipMalloc(&p->red_part, sizeof(double) * nred);
    if (e != hipSuccess) {
        (void)hipFree(p->Z);
        delete p;
        return SMOL_ENOMEM;
    }
    p->red = p->red_part + (size_t)N2 * R * 4;
    p->epart = p->red + (size_t)R * 4;
    sched_init();
    int vff[3];
    ff_schedule(logL, vff);
    int rc = set_plan_sched(p, precision == SMOL_FP64 ? g_sched[logL] : vff);
    if (rc) {
        free_plan(p);
        return rc;
    }
    g_plans[key] = p;
    *out = p;
    return SMOL_OK;
}

// A plan's workspaces are reused by every call with its (device, M, R,
// precision).  Work enqueued on stream s waits for the previous call's work
// when that call used another stream and may still be running.
int plan_enter(Plan *p, hipStream_t s)
{
    if (p->busy && p->used_s != s) HIP_TRY(hipStreamWaitEvent(s, p->used_ev, 0));
    return SMOL_OK;
}
// After enqueueing work on s that the caller does not wait for.
int plan_leave_async(Plan *p, hipStream_t s)
{
    if (!p->used_ev) HIP_TRY(hipEventCreateWithFlags(&p->used_ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(p->used_ev, s));
    p->used_s = s;
    p->busy = true;
    return SMOL_OK;
}
// After the call has synchronised s: nothing of the plan's is in flight.
void plan_leave_sync(Plan *p) { p->busy = false; }

RhsPlanDev dev_plan(const Plan *p, const DevRoots *r, const double *U, const double *V, double lam)
{
    RhsPlanDev d;
    d.M = p->M;
    d.R = p->R;
    d.logL = p->logL;
    d.logN1 = p->logN1;
    d.logN2 = p->logN2;
    d.tr = 0;
    d.ustride = p->M;
    d.lam = lam;
    d.U = U;
    d.V = V;
    d.Z = p->Z;
    d.Qp = p->Qp;
    d.red_part = p->red_part;
    d.red = p->red;
    d.src = nullptr;
    d.rt.tw = r->tw;
    d.rt.fine = r->fine;
    return d;
}

// Launch phases A, B, C for one right-hand side.
int launch_rhs(const Plan *p, const RhsPlanDev &P, const Pro &in, const Epi &ep, hipStream_t s)
{
    int rc;
    if ((rc = launch_rhs_A(p->logL, p->precision, p->var[0], P, in, s))) return rc;
    const int redj = (in.mode == A_COMBINE) ? p->dA.jobs : 0;
    if ((rc = launch_rhs_B(p->logL, p->precision, p->var[1], P, redj, s))) return rc;
    if ((rc = launch_rhs_C(p->logL, p->precision, p->var[2], P, ep, s))) return rc;
    HIP_TRY(hipGetLastError());
    return SMOL_OK;
}

// One stage (or starting-step evaluation) of the integrator.  Stages 0..2
// run A, B, C; from stage 3 on the column pass was done by the previous
// stage's fused finish, so only B and C run; the finish of stages
// 2..S-1 is fused with the next column pass.  decide_from (stage 2 of a
// captured attempt): the control block holding the previous attempt, whose
// decision the column pass takes before it, storing the result to I.ctl.
int launch_stage(const Plan *p, const IntegDev &I, int method, int stage, int S, hipStream_t s,
                 IntegCtl *decide_from = nullptr)
{
    int rc;
    if (stage <= 2) {
        if (decide_from) {
            IntegDev Ii = I;
            Ii.ctl = decide_from;
            rc = launch_int_A(p->logL, p->precision, p->var[0], Ii, stage, method, I.ctl,
                              p->dC.jobs, s);
        } else {
            rc = launch_int_A(p->logL, p->precision, p->var[0], I, stage, method, nullptr, 0, s);
        }
        if (rc) return rc;
    }
    if ((rc = launch_int_B(p->logL, p->precision, p->var[1], I, stage, p->dA.jobs, p->dC.jobs, s)))
        return rc;
    const bool fuse = stage >= 2 && stage < S;
    if ((rc = launch_int_C(p->logL, p->precision, p->var[2], fuse, I, stage, method, s))) return rc;
    HIP_TRY(hipGetLastError());
    return SMOL_OK;
}

int alloc_integ(Plan *p)
{
    if (p->ibuf) return SMOL_OK;
    const int64_t half = 1LL << (p->logL - 1);
    p->Mt = p->M > half + 1 ? p->M : half + 1;
    if (hipMalloc(&p->ibuf, sizeof(double) * (size_t)p->Mt * 11) != hipSuccess) return SMOL_ENOMEM;
    if (hipMalloc(&p->uvt, sizeof(double) * (size_t)p->Mt * 2 * p->R) != hipSuccess) return SMOL_ENOMEM;
    // two control blocks: captured attempts alternate between them
    if (hipMalloc(&p->ctl, 2 * sizeof(IntegCtl)) != hipSuccess) return SMOL_ENOMEM;
    HIP_TRY(hipHostMalloc(&p->host, sizeof(IntegCtl), hipHostMallocDefault));
    HIP_TRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    return SMOL_OK;
}

IntegDev integ_dev(const Plan *p, const DevRoots *r)
{
    IntegDev I{};
    I.M = p->M;
    I.R = p->R;
    I.logL = p->logL;
    I.ctl = p->ctl;
    I.Mt = p->Mt;
    I.Ut = p->uvt;
    I.Vt = p->uvt + (size_t)p->R * p->Mt;
    I.nb[0] = p->ibuf;
    I.nb[1] = p->ibuf + p->Mt;
    for (int j = 0; j < 7; ++j) I.kslot[j] = p->ibuf + (2 + j) * p->Mt;
    I.kslot[7] = nullptr;
    I.ybuf = p->ibuf + 9 * p->Mt;
    I.src = p->ibuf + 10 * p->Mt;
    I.Z = p->Z;
    I.Qp = p->Qp;
    I.red_part = p->red_part;
    I.red = p->red;
    I.epart = p->epart;
    I.rt.tw = r->tw;
    I.rt.fine = r->fine;
    return I;
}

// Capture SMOL_GRAPH_ATTEMPTS step attempts (stages 2..S) as one graph.
// Each attempt's stage-2 column pass first takes the previous attempt's
// decision: attempt a reads control block a % 2 and writes block
// (a + 1) % 2, which its later kernels read.  With an even number of
// attempts per graph, block 0 holds the latest state between replays.
int get_step_graph(Plan *p, const IntegDev &I, int method, hipGraphExec_t *out)
{
    if (p->graph[method]) {
        *out = p->graph[method];
        return SMOL_OK;
    }
    const int S = k_scheme_stages[method];
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    int rc = SMOL_OK;
    static_assert(SMOL_GRAPH_ATTEMPTS % 2 == 0, "control blocks alternate per attempt");
    for (int a = 0; a < SMOL_GRAPH_ATTEMPTS; ++a) {
        IntegDev Ia = I;
        Ia.ctl = p->ctl + ((a + 1) & 1);
        for (int st = 2; st <= S && rc == SMOL_OK; ++st)
            rc = launch_stage(p, Ia, method, st, S, p->cap, st == 2 ? p->ctl + (a & 1) : nullptr);
    }
    hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->graph[method], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *out = p->graph[method];
    return SMOL_OK;
}

}  // namespace

SMOL_HIDDEN void stats_from(const IntegCtl &c, smol_stats *st)
{
    if (!st) return;
    st->n_rhs = c.n_rhs;
    st->n_accept = c.n_accept;
    st->n_reject = c.n_reject;
    st->t = c.t;
    st->h = c.h;
    st->err = c.err;
    st->status = c.status;
    st->n_fallback = c.n_fallback;
}

SMOL_HIDDEN int check_common(int64_t M, int32_t R, const double *U, const double *V, double lambda)
{
    if (M < 1 || R < 1 || R > SMOL_MAX_R || !U || !V) return SMOL_EINVAL;
    if (!std::isfinite(lambda) || lambda < 0) return SMOL_EINVAL;
    if (2 * M - 2 > (1LL << SMOL_LOG_LMAX)) return SMOL_EUNSUPPORTED;
    return SMOL_OK;
}


// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------

extern "C" int smol_rhs_ex(int64_t M, int32_t R, const double *U, const double *V, double lambda,
                           const double *n, const double *source, double *dndt, int32_t precision,
                           void *stream)
{
    int rc = check_common(M, R, U, V, lambda);
    if (rc) return rc;
    if (!n || !dndt || n == dndt || source == dndt) return SMOL_EINVAL;
    if (precision != SMOL_FP64 && precision != SMOL_FP32X2) return SMOL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p;
    DevRoots *r;
    if ((rc = get_plan(M, R, precision, &p))) return rc;
    if ((rc = get_roots(p->dev, &r))) return rc;
    RhsPlanDev P = dev_plan(p, r, U, V, lambda);
    P.src = source;
    Pro in{A_COMBINE, n, nullptr, 0.0, nullptr};
    Epi ep{};
    ep.mode = C_RHS;
    ep.y = n;
    ep.out = dndt;
    hipStream_t s = (hipStream_t)stream;
    // under graph capture the caller orders the captured work itself
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    const bool track = cs == hipStreamCaptureStatusNone;
    if (track && (rc = plan_enter(p, s))) return rc;
    if ((rc = launch_rhs(p, P, in, ep, s))) return rc;
    return track ? plan_leave_async(p, s) : SMOL_OK;
}

extern "C" int smol_rhs(int64_t M, int32_t R, const double *U, const double *V, double lambda,
                        const double *n, double *dndt, int32_t precision, void *stream)
{
    return smol_rhs_ex(M, R, U, V, lambda, n, nullptr, dndt, precision, stream);
}

extern "C" int smol_release_plans(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceSynchronize());
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::get<0>(it->first) == dev) {
            free_plan(it->second);
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
    return SMOL_OK;
}

extern "C" const char *smol_strerror(int code)
{
    switch (code) {
    case SMOL_OK: return "ok";
    case SMOL_EINVAL: return "invalid argument";
    case SMOL_ENOMEM: return "device allocation failed";
    case SMOL_EDEVICE: return "HIP runtime error";
    case SMOL_ESTEPSIZE: return "step size fell below the minimum";
    case SMOL_EMAXSTEPS: return "step-attempt limit reached";
    case SMOL_ENONFINITE: return "non-finite state or error norm";
    case SMOL_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status code";
    }
}

extern "C" const char *smol_version(void) { return SMOL_VERSION; }


extern "C" int smol_integrate_ex(int64_t M, int32_t R, const double *U, const double *V,
                                 double lambda, const double *n0, double t_end, double rtol,
                                 double atol, int32_t method, int32_t precision,
                                 const smol_options *opts, double *n_out, smol_stats *stats,
                                 void *stream)
{
    int rc = check_common(M, R, U, V, lambda);
    if (rc) return rc;
    if (!n0 || !n_out) return SMOL_EINVAL;
    if ((rc = check_method(method))) return rc;
    if (precision != SMOL_FP64 && precision != SMOL_FP32X2) return SMOL_EINVAL;
    if (!(rtol > 0) || !(atol >= 0) || !(t_end >= 0) || !std::isfinite(t_end)) return SMOL_EINVAL;
    smol_options o{};
    if (opts) o = *opts;
    if (o.h0 < 0 || o.h_min < 0 || o.max_steps < 0 || (o.log && o.log_cap < 0)) return SMOL_EINVAL;
    if (!controller_valid(o.controller)) return SMOL_EINVAL;
    smol_state *cp = o.state;
    if (cp && !cp->k1) return SMOL_EINVAL;
    const bool resume = cp && cp->valid;
    if (resume && (!std::isfinite(cp->t) || cp->t < 0 || !std::isfinite(cp->h) || !(cp->h > 0) ||
                   cp->n_hist < 0 || cp->n_hist > 4))
        return SMOL_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (t_end == 0.0 || (resume && cp->t >= t_end)) {
        if (n_out != n0) HIP_TRY(hipMemcpyAsync(n_out, n0, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (resume && stats) {
            stats->n_rhs = cp->n_rhs;
            stats->n_accept = cp->n_accept;
            stats->n_reject = cp->n_reject;
            stats->t = cp->t;
            stats->h = cp->h;
            stats->err = cp->err;
            stats->n_fallback = cp->n_fallback;
        }
        if (cp && !resume) cp->valid = 0;  // no step taken: no checkpoint
        return SMOL_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p;
    DevRoots *r;
    if ((rc = get_plan(M, R, precision, &p))) return rc;
    if ((rc = get_roots(p->dev, &r))) return rc;
    if ((rc = alloc_integ(p))) return rc;
    if ((rc = plan_enter(p, s))) return rc;
    const IntegDev I = integ_dev(p, r);
    IntegCtl &c = *p->host;
    memset(&c, 0, sizeof(c));
    c.U = I.Ut;
    c.V = I.Vt;
    c.lam = lambda;
    c.t_end = t_end;
    c.h_min = o.h_min;
    c.h0_user = o.h0;
    c.max_steps = o.max_steps > 0 ? o.max_steps : 100000000LL;
    c.log = o.log;
    c.log_cap = o.log ? o.log_cap : 0;
    ctl_setup(c, method, o, rtol, atol);
    c.has_src = o.source != nullptr;
    if (o.controller == SMOL_CTRL_LEARNED) {
        c.mlp = proposer_weights(p->dev);
        if (!c.mlp) return SMOL_EINVAL;  // smol_proposer_set first
    }
    if (resume) {
        c.t = cp->t;
        c.h = cp->h;
        c.err = cp->err;
        c.err_prev = cp->err_prev;
        for (int q = 0; q < 4; ++q) c.err_hist[q] = cp->err_hist[q];
        c.n_hist = cp->n_hist;
        c.rejected = cp->rejected ? 1 : 0;
        c.n_rhs = cp->n_rhs;
        c.n_accept = cp->n_accept;
        c.n_reject = cp->n_reject;
        c.n_fallback = cp->n_fallback;
    }
    HIP_TRY(hipMemcpyAsync(p->ctl, &c, sizeof(c), hipMemcpyHostToDevice, s));
    // the integrator keeps every vector in the transposed layout
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, U, I.Ut, M, R, M, I.Mt, p->logL);
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, V, I.Vt, M, R, M, I.Mt, p->logL);
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, n0, I.nb[0], M, 1, M, I.Mt, p->logL);
    if (o.source)
        hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, o.source, I.src, M, 1, M, I.Mt,
                           p->logL);
    const int nC = p->dC.jobs;
    if (resume) {
        // the checkpoint's S(n) is the first stage (slot 0 at parity 0)
        hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, cp->k1, I.kslot[0], M, 1, M, I.Mt,
                           p->logL);
        hipLaunchKernelGGL(k_resume, dim3(1), dim3(64), 0, s, I);
    } else {
        // starting step: S(n0), h0, S(n0 + h0 f0), h
        if ((rc = launch_stage(p, I, method, 0, 0, s))) return rc;
        hipLaunchKernelGGL(k_init_h0, dim3(1), dim3(SMOL_WG), 0, s, I, nC);
        if (!(o.h0 > 0)) {
            if ((rc = launch_stage(p, I, method, 1, 0, s))) return rc;
            hipLaunchKernelGGL(k_init_h, dim3(1), dim3(SMOL_WG), 0, s, I, nC);
        }
    }
    HIP_TRY(hipGetLastError());
    hipGraphExec_t ge;
    if ((rc = get_step_graph(p, I, method, &ge))) return rc;
    // replay step attempts; poll the control block between chunks
    int64_t chunk = 1;
    for (;;) {
        for (int64_t i = 0; i < chunk; ++i) HIP_TRY(hipGraphLaunch(ge, s));
        HIP_TRY(hipMemcpyAsync(p->host, p->ctl, sizeof(IntegCtl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (c.done) break;
        double est = (c.h > 0) ? (c.t_end - c.t) / c.h : 1e9;
        if (!(est < 1e9)) est = 1e9;
        // nor far beyond the attempt limit (surplus attempts return at entry,
        // but each still costs its launches)
        const double left = (double)(c.max_steps - c.attempts);
        if (left < est) est = left;
        chunk = (int64_t)(0.8 * est / SMOL_GRAPH_ATTEMPTS) + 1;
        // at most 256 attempts between polls: early in a run h is small and
        // the estimate far too high, and every surplus attempt launches
        if (chunk > 256 / SMOL_GRAPH_ATTEMPTS) chunk = 256 / SMOL_GRAPH_ATTEMPTS;
        if (chunk < 1) chunk = 1;
    }
    const IntegCtl &cf = c;
    hipLaunchKernelGGL(k_from_tr, dim3(256), dim3(256), 0, s, I.nb[cf.cur], n_out, M, p->logL);
    if (cp)  // S at n_out: the first stage of the next attempt
        hipLaunchKernelGGL(k_from_tr, dim3(256), dim3(256), 0, s,
                           I.kslot[cf.kp ? k_scheme_fsal[method] : 0], cp->k1, M, p->logL);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    plan_leave_sync(p);
    stats_from(cf, stats);
    if (cp) {
        cp->t = cf.t;
        cp->h = cf.h;
        cp->err = cf.err;
        cp->err_prev = cf.err_prev;
        for (int q = 0; q < 4; ++q) cp->err_hist[q] = cf.err_hist[q];
        cp->n_hist = cf.n_hist;
        cp->rejected = cf.rejected;
        cp->n_rhs = cf.n_rhs;
        cp->n_accept = cf.n_accept;
        cp->n_reject = cf.n_reject;
        cp->n_fallback = cf.n_fallback;
        cp->valid = (cf.status == SMOL_OK || cf.status == SMOL_EMAXSTEPS) ? 1 : 0;
    }
    return cf.status;
}

extern "C" int smol_integrate(int64_t M, int32_t R, const double *U, const double *V,
                              double lambda, const double *n0, double t_end, double rtol,
                              double atol, int32_t method, int32_t precision, double *n_out,
                              smol_stats *stats, void *stream)
{
    return smol_integrate_ex(M, R, U, V, lambda, n0, t_end, rtol, atol, method, precision,
                             nullptr, n_out, stats, stream);
}


namespace {
// Mean milliseconds per launch of each phase (iters back-to-back launches)
// and per whole right-hand side, with HIP events on stream s.
int profile_phases(const Plan *p, const RhsPlanDev &P, const Pro &in, const Epi &ep, int iters,
                   float *ms, hipStream_t s)
{
    hipEvent_t ev[5];
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    int rc = SMOL_OK;
    HIP_TRY(hipEventRecord(ev[0], s));
    for (int i = 0; i < iters && !rc; ++i) rc = launch_rhs_A(p->logL, p->precision, p->var[0], P, in, s);
    HIP_TRY(hipEventRecord(ev[1], s));
    for (int i = 0; i < iters && !rc; ++i)
        rc = launch_rhs_B(p->logL, p->precision, p->var[1], P, p->dA.jobs, s);
    HIP_TRY(hipEventRecord(ev[2], s));
    for (int i = 0; i < iters && !rc; ++i) rc = launch_rhs_C(p->logL, p->precision, p->var[2], P, ep, s);
    HIP_TRY(hipEventRecord(ev[3], s));
    for (int i = 0; i < iters && !rc; ++i) rc = launch_rhs(p, P, in, ep, s);
    HIP_TRY(hipEventRecord(ev[4], s));
    HIP_TRY(hipEventSynchronize(ev[4]));
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    for (int k = 0; k < 4; ++k) {
        float t;
        HIP_TRY(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
        ms[k] = t / (float)iters;
    }
    for (auto &e : ev) HIP_TRY(hipEventDestroy(e));
    return SMOL_OK;
}
}  // namespace

// Times the kernels the integrator runs: vectors in the transposed layout.
extern "C" int smol_profile_rhs(int64_t M, int32_t R, const double *U, const double *V,
                                double lambda, const double *n, double *dndt, int32_t iters,
                                float *ms_out, void *stream)
{
    int rc = check_common(M, R, U, V, lambda);
    if (rc) return rc;
    if (!n || !dndt || n == dndt || iters < 1 || !ms_out) return SMOL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p;
    DevRoots *r;
    if ((rc = get_plan(M, R, SMOL_FP64, &p))) return rc;
    if ((rc = get_roots(p->dev, &r))) return rc;
    if ((rc = alloc_integ(p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = plan_enter(p, s))) return rc;
    const IntegDev I = integ_dev(p, r);
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, U, I.Ut, M, R, M, I.Mt, p->logL);
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, V, I.Vt, M, R, M, I.Mt, p->logL);
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, n, I.nb[0], M, 1, M, I.Mt, p->logL);
    RhsPlanDev P = dev_plan(p, r, I.Ut, I.Vt, lambda);
    P.tr = 1;
    P.ustride = I.Mt;
    Pro in{A_COMBINE, I.nb[0], nullptr, 0.0, nullptr};
    Epi ep{};
    ep.mode = C_RHS;
    ep.y = I.nb[0];
    ep.out = I.kslot[0];
    rc = profile_phases(p, P, in, ep, iters, ms_out, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_from_tr, dim3(256), dim3(256), 0, s, I.kslot[0], dndt, M, p->logL);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    plan_leave_sync(p);
    return SMOL_OK;
}

// Times the integrator's own stage kernels at the state n0: the starting
// step and one full attempt's stages run first (so every stage vector,
// spectrum and reduction row holds real data), then each kernel is launched
// iters times back to back between HIP events.  Relaunching a stage kernel
// recomputes the same workspaces from the same inputs, except that the fused
// finish of stage 3 reads and rewrites the stage state, which stays finite
// for a stable step.  The stage-2 pass is timed as a captured attempt runs
// it, taking the previous attempt's decision, with its result stored to the
// second control block: the run's block is never advanced, so every launch
// does the same full work.
extern "C" int smol_profile_step(int64_t M, int32_t R, const double *U, const double *V,
                                 double lambda, const double *n0, int32_t method, int32_t iters,
                                 float *ms_out, void *stream)
{
    int rc = check_common(M, R, U, V, lambda);
    if (rc) return rc;
    if (!n0 || iters < 1 || !ms_out) return SMOL_EINVAL;
    if (method != SMOL_BS32 && method != SMOL_DP54) return SMOL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p;
    DevRoots *r;
    if ((rc = get_plan(M, R, SMOL_FP64, &p))) return rc;
    if ((rc = get_roots(p->dev, &r))) return rc;
    if ((rc = alloc_integ(p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = plan_enter(p, s))) return rc;
    const IntegDev I = integ_dev(p, r);
    IntegCtl &c = *p->host;
    memset(&c, 0, sizeof(c));
    c.U = I.Ut;
    c.V = I.Vt;
    c.lam = lambda;
    c.t_end = 1e300;
    c.max_steps = 100000000LL;
    smol_options o{};
    ctl_setup(c, method, o, 1e-6, 1e-12);
    HIP_TRY(hipMemcpyAsync(p->ctl, &c, sizeof(c), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, U, I.Ut, M, R, M, I.Mt, p->logL);
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, V, I.Vt, M, R, M, I.Mt, p->logL);
    hipLaunchKernelGGL(k_to_tr, dim3(256), dim3(256), 0, s, n0, I.nb[0], M, 1, M, I.Mt, p->logL);
    const int S = k_scheme_stages[method];
    const int nC = p->dC.jobs;
    if ((rc = launch_stage(p, I, method, 0, 0, s))) return rc;
    hipLaunchKernelGGL(k_init_h0, dim3(1), dim3(SMOL_WG), 0, s, I, nC);
    if ((rc = launch_stage(p, I, method, 1, 0, s))) return rc;
    hipLaunchKernelGGL(k_init_h, dim3(1), dim3(SMOL_WG), 0, s, I, nC);
    for (int st = 2; st <= S && !rc; ++st) rc = launch_stage(p, I, method, st, S, s);
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    hipEvent_t ev[5];
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventRecord(ev[0], s));
    // the stage-2 pass as a captured attempt runs it: taking the decision of
    // the attempt just evaluated (block 0, marked pending) and storing the
    // result to block 1, so that every launch repeats the same work
    c.pending = 1;
    HIP_TRY(hipMemcpyAsync((char *)p->ctl + offsetof(IntegCtl, pending), &c.pending,
                           sizeof(c.pending), hipMemcpyHostToDevice, s));
    for (int i = 0; i < iters && !rc; ++i)
        rc = launch_int_A(p->logL, SMOL_FP64, p->var[0], I, 2, method, p->ctl + 1, nC, s);
    HIP_TRY(hipEventRecord(ev[1], s));
    for (int i = 0; i < iters && !rc; ++i)
        rc = launch_int_B(p->logL, SMOL_FP64, p->var[1], I, 3, p->dA.jobs, nC, s);
    HIP_TRY(hipEventRecord(ev[2], s));
    for (int i = 0; i < iters && !rc; ++i)
        rc = launch_int_C(p->logL, SMOL_FP64, p->var[2], true, I, 3, method, s);
    HIP_TRY(hipEventRecord(ev[3], s));
    for (int i = 0; i < iters && !rc; ++i)
        rc = launch_int_C(p->logL, SMOL_FP64, p->var[2], false, I, S, method, s);
    HIP_TRY(hipEventRecord(ev[4], s));
    HIP_TRY(hipEventSynchronize(ev[4]));
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    for (int k = 0; k < 4; ++k) {
        float t;
        HIP_TRY(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
        ms_out[k] = t / (float)iters;
    }
    for (auto &e : ev) HIP_TRY(hipEventDestroy(e));
    plan_leave_sync(p);
    return SMOL_OK;
}


// --------------------------------------------------------------------------
// Launch schedules and the autotuner
// --------------------------------------------------------------------------

namespace {
bool sched_valid(int logL, const int32_t *v)
{
    PhaseDims d;
    for (int ph = 0; ph < 3; ++ph)
        if (v[ph] < 0 || v[ph] >= SMOL_NVAR || phase_dims(logL, SMOL_FP64, ph, v[ph], 1, false, &d))
            return false;
    return true;
}

int set_schedule_locked(int logL, const int32_t *v)
{
    sched_init();
    if (logL < 6 || logL > SMOL_LOG_LMAX || !v || !sched_valid(logL, v)) return SMOL_EINVAL;
    int w[3] = {v[0], v[1], v[2]};
    for (auto &kv : g_plans) {
        Plan *p = kv.second;
        if (p->precision != SMOL_FP64 || p->logL != logL) continue;
        if (p->var[0] == w[0] && p->var[1] == w[1] && p->var[2] == w[2]) continue;
        int rc = set_plan_sched(p, w);
        if (rc) return rc;
    }
    for (int k = 0; k < 3; ++k) g_sched[logL][k] = w[k];
    return SMOL_OK;
}
}  // namespace

SMOL_HIDDEN void schedule_of(int logL, int precision, int *v)
{
    sched_init();
    if (precision != SMOL_FP64) {
        ff_schedule(logL, v);
        return;
    }
    for (int k = 0; k < 3; ++k) v[k] = (logL >= 6 && logL <= SMOL_LOG_LMAX) ? g_sched[logL][k] : 0;
}

extern "C" int smol_set_schedule(int32_t logL, const int32_t *variants)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return set_schedule_locked(logL, variants);
}

extern "C" int smol_get_schedule(int32_t logL, int32_t *variants)
{
    if (logL < 6 || logL > SMOL_LOG_LMAX || !variants) return SMOL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    sched_init();
    for (int k = 0; k < 3; ++k) variants[k] = g_sched[logL][k];
    return SMOL_OK;
}

extern "C" int smol_autotune(int64_t M, int32_t R, const double *U, const double *V, double lambda,
                             const double *n0, int32_t method, int32_t attempts, int32_t reps,
                             int32_t *variants_out, float *ms_out, void *stream)
{
    int rc = check_common(M, R, U, V, lambda);
    if (rc) return rc;
    if (!n0 || !variants_out || attempts < 1 || reps < 1) return SMOL_EINVAL;
    if ((rc = check_method(method))) return rc;
    const int logL = fft_log2(M);
    double *scratch = nullptr;
    HIP_TRY(hipMalloc(&scratch, sizeof(double) * (size_t)M));
    smol_options o{};
    o.max_steps = attempts;
    // seconds per step attempt of schedule v: one untimed run (captures the
    // step graph), then the best of `reps` timed runs of `attempts` attempts
    auto time_of = [&](const int32_t *v, double *sec) -> int {
        int r = smol_set_schedule(logL, v);
        if (r) return r;
        double best = 1e30;
        for (int k = 0; k <= reps; ++k) {
            smol_stats st;
            auto t0 = std::chrono::steady_clock::now();
            r = smol_integrate_ex(M, R, U, V, lambda, n0, 1e300, 1e-6, 1e-12, method, SMOL_FP64, &o,
                                  scratch, &st, stream);
            auto t1 = std::chrono::steady_clock::now();
            if (r != SMOL_OK && r != SMOL_EMAXSTEPS) return r;
            const double dt = std::chrono::duration<double>(t1 - t0).count();
            if (k > 0 && dt < best) best = dt;
        }
        *sec = best / attempts;
        return SMOL_OK;
    };
    int32_t cur[3];
    smol_get_schedule(logL, cur);
    double best = 0.0;
    rc = time_of(cur, &best);
    const double start = best;
    // coordinate descent over the kernels, largest first; a change must gain 2 %
    for (int ph : {PH_C, PH_B, PH_A}) {
        if (rc || logL < SMOL_TUNE_MIN_LOGL) break;
        for (int v = 0; v < SMOL_NVAR && !rc; ++v) {
            int32_t cand[3] = {cur[0], cur[1], cur[2]};
            if (v == cur[ph]) continue;
            cand[ph] = v;
            {
                std::lock_guard<std::mutex> lk(g_mu);
                if (!sched_valid(logL, cand)) continue;
            }
            double t;
            rc = time_of(cand, &t);
            if (!rc && t < 0.98 * best) {
                best = t;
                for (int k = 0; k < 3; ++k) cur[k] = cand[k];
            }
        }
    }
    int rc2 = smol_set_schedule(logL, cur);
    (void)hipFree(scratch);
    if (rc) return rc;
    if (rc2) return rc2;
    for (int k = 0; k < 3; ++k) variants_out[k] = cur[k];
    if (ms_out) {
        ms_out[0] = (float)(start * 1e3);
        ms_out[1] = (float)(best * 1e3);
    }
    return SMOL_OK;
}
