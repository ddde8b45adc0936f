// Batched integration of many independent instances (uneven M, kernels,
// lambda and tolerances), each with its own step size, accept / reject and
// status.  Every kernel of a step attempt is ONE launch over all instances:
// a block-to-instance table gives each workgroup its instance and unit, a
// switch selects the instance's transform shape, and per-instance control
// blocks carry the state, so the attempt is captured once as a hipGraph and
// replayed until every instance is done (finished instances' workgroups
// return at entry).  With hundreds of instances each launch holds tens of
// thousands of workgroups, which fills the chip and hides memory latency
// that a single small instance cannot.
#include <cstring>
#include <vector>

#include "host.h"

struct BatchDev {
    const IntegDev *inst;   // per instance
    const int *logL;        // per instance
    const int *first[3];    // first block of each instance per kernel A, B, C
    const int *owner[3];    // instance of each block per kernel
    const int *nC;          // finish units per instance
    const int *redA;        // column-pass reduction jobs per instance
    const int *active;      // instances still running (one controller workgroup each)
};

#define SMOL_SHAPES(X) \
    X(6, 3, 3) X(7, 4, 3) X(8, 4, 4) X(9, 5, 4) X(10, 5, 5) X(11, 6, 5) X(12, 6, 6) X(13, 7, 6) \
    X(14, 7, 7) X(15, 8, 7) X(16, 8, 8) X(17, 9, 8) X(18, 9, 9) X(19, 10, 9) X(20, 10, 10)

template <class T>
__global__ __launch_bounds__(SMOL_WG) void kb_A(BatchDev B, int stage)
{
    extern __shared__ cd lds[];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);  // neighbours share an XCD's L2
    const int b = B.owner[0][blk];
    const IntegDev &I = B.inst[b];
    const IntegCtl c = *I.ctl;  // one snapshot: all fields load together
    if (c.done) return;
    const RhsPlanDev P = plan_of(I, c);
    const Pro in = stage_pro(I, c, c_tab[c.method], stage);
    const int unit = blk - B.first[0][b];
    switch (B.logL[b]) {
#define X(LL, A, Bb) \
    case LL: PhaseA<(1 << A), (1 << Bb), T>::run(P, in, unit, (T *)lds); break;
        SMOL_SHAPES(X)
#undef X
    }
}

template <class T>
__global__ __launch_bounds__(SMOL_WG) void kb_B(BatchDev B, int stage)
{
    extern __shared__ cd lds[];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);  // neighbours share an XCD's L2
    const int b = B.owner[1][blk];
    const IntegDev &I = B.inst[b];
    const IntegCtl c = *I.ctl;  // one snapshot: all fields load together
    if (c.done) return;
    const RhsPlanDev P = plan_of(I, c);
    const int unit = blk - B.first[1][b];
    const int logL = B.logL[b];
    if (unit == (1 << ((logL + 1) / 2 - 1)) + 1) {  // N1/2 + 1: the finaliser
        finalize_reductions(P, stage <= 2 ? B.redA[b] : B.nC[b]);
        return;
    }
    switch (logL) {
#define X(LL, A, Bb) \
    case LL: PhaseB<(1 << A), (1 << Bb), T>::run(P, unit, (T *)lds); break;
        SMOL_SHAPES(X)
#undef X
    }
}

template <class T, bool FUSE>
__global__ __launch_bounds__(SMOL_WG) void kb_C(BatchDev B, int stage)
{
    extern __shared__ cd lds[];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);  // neighbours share an XCD's L2
    const int b = B.owner[2][blk];
    const IntegDev &I = B.inst[b];
    const IntegCtl c = *I.ctl;  // one snapshot: all fields load together
    if (c.done) return;
    const RhsPlanDev P = plan_of(I, c);
    const Epi ep = stage_epi(I, c, c_tab[c.method], stage);
    const int unit = blk - B.first[2][b];
    switch (B.logL[b]) {
#define X(LL, A, Bb) \
    case LL: PhaseC<(1 << A), (1 << Bb), T>::template run<FUSE>(P, ep, unit, (T *)lds); break;
        SMOL_SHAPES(X)
#undef X
    }
}

// one workgroup per listed instance
__global__ __launch_bounds__(SMOL_WG) void kb_init_h0(BatchDev B)
{
    const int b = B.active[blockIdx.x];
    init_h0_step(B.inst[b], B.nC[b]);
}
__global__ __launch_bounds__(SMOL_WG) void kb_init_h(BatchDev B)
{
    const int b = B.active[blockIdx.x];
    init_h_step(B.inst[b], B.nC[b]);
}
__global__ __launch_bounds__(SMOL_WG) void kb_ctrl(BatchDev B)
{
    const int b = B.active[blockIdx.x];
    controller_step(B.inst[b], B.nC[b]);
}

namespace {

struct BatchRun {
    int n = 0;
    std::vector<int> logL, units[3], ldsn[4];  // ldsn[3]: fused finish
    std::vector<size_t> off;     // arena offset of each instance
    int total[3] = {0, 0, 0};    // blocks of each kernel over the listed instances
    int nact = 0;                // listed instances
    size_t lds[4] = {0, 0, 0, 0};
};

// Block-to-instance tables over the instances in `ids` (device buffers
// sized for all instances are reused).
int build_tables(BatchRun &br, const std::vector<int> &ids, int *dfirst[3], int *downer[3],
                 int *dactive, hipStream_t s)
{
    std::vector<int> first[3], owner[3];
    for (int k = 0; k < 3; ++k) {
        first[k].assign(br.n + 1, 0);
        br.total[k] = 0;
        br.lds[k] = 0;
    }
    br.lds[3] = 0;
    for (int i : ids) {
        const size_t lf = sizeof(cd) * (size_t)br.ldsn[3][i];
        if (lf > br.lds[3]) br.lds[3] = lf;
        for (int k = 0; k < 3; ++k) {
            first[k][i] = br.total[k];
            for (int j = 0; j < br.units[k][i]; ++j) owner[k].push_back(i);
            br.total[k] += br.units[k][i];
            const size_t lb = sizeof(cd) * (size_t)br.ldsn[k][i];
            if (lb > br.lds[k]) br.lds[k] = lb;
        }
    }
    br.nact = (int)ids.size();
    for (int k = 0; k < 3; ++k) {
        HIP_TRY(hipMemcpyAsync(dfirst[k], first[k].data(), sizeof(int) * (br.n + 1),
                               hipMemcpyHostToDevice, s));
        if (br.total[k])
            HIP_TRY(hipMemcpyAsync(downer[k], owner[k].data(), sizeof(int) * br.total[k],
                                   hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(dactive, ids.data(), sizeof(int) * ids.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // host vectors die here
    return SMOL_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Same kernel sequence as a single instance: A only up to stage 2, the
// finish of stages 2..S-1 fused with the next column pass.
template <class T>
void launch_stage(const BatchDev &B, const BatchRun &br, int stage, int S, hipStream_t s)
{
    if (stage <= 2)
        hipLaunchKernelGGL(kb_A<T>, dim3(br.total[0]), dim3(SMOL_WG), br.lds[0], s, B, stage);
    hipLaunchKernelGGL(kb_B<T>, dim3(br.total[1]), dim3(SMOL_WG), br.lds[1], s, B, stage);
    if (stage >= 2 && stage < S)
        hipLaunchKernelGGL((kb_C<T, true>), dim3(br.total[2]), dim3(SMOL_WG), br.lds[3], s, B, stage);
    else
        hipLaunchKernelGGL((kb_C<T, false>), dim3(br.total[2]), dim3(SMOL_WG), br.lds[2], s, B, stage);
}

void launch_stage_p(int precision, const BatchDev &B, const BatchRun &br, int stage, int S,
                    hipStream_t s)
{
    if (precision == SMOL_FP32X2)
        launch_stage<cff>(B, br, stage, S, s);
    else
        launch_stage<cd>(B, br, stage, S, s);
}

}  // namespace

extern "C" int smol_integrate_batch(int32_t n_inst, const smol_instance *inst, int32_t method,
                                    int32_t precision, const smol_options *opts,
                                    smol_stats *stats, void *stream)
{
    if (n_inst < 1 || !inst || !stats) return SMOL_EINVAL;
    if (method != SMOL_BS32 && method != SMOL_DP54) return SMOL_EINVAL;
    if (precision != SMOL_FP64 && precision != SMOL_FP32X2) return SMOL_EINVAL;
    smol_options o{};
    if (opts) o = *opts;
    if (o.h0 < 0 || o.h_min < 0 || o.max_steps < 0 || o.log) return SMOL_EINVAL;
    if (o.controller != SMOL_CTRL_PI && o.controller != SMOL_CTRL_LEARNED) return SMOL_EINVAL;
    for (int i = 0; i < n_inst; ++i) {
        const smol_instance &q = inst[i];
        int rc = check_common(q.M, q.R, q.U, q.V, q.lambda);
        if (rc) return rc;
        if (!q.n0 || !q.n_out || (q.log && q.log_cap < 0)) return SMOL_EINVAL;
        if (!(q.rtol > 0) || !(q.atol >= 0) || !(q.t_end >= 0) || !std::isfinite(q.t_end))
            return SMOL_EINVAL;
    }
    memset(stats, 0, sizeof(smol_stats) * n_inst);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_mu);
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    DevRoots *roots;
    int rc = get_roots(dev, &roots);
    if (rc) return rc;
    const float *mlp = proposer_weights(dev);
    if (o.controller == SMOL_CTRL_LEARNED && !mlp) return SMOL_EINVAL;  // smol_proposer_set first

    // ---- sizes and arena layout
    BatchRun br;
    br.n = n_inst;
    std::vector<int> nC(n_inst), redA(n_inst);
    br.logL.resize(n_inst);
    br.off.resize(n_inst);
    for (int k = 0; k < 3; ++k) br.units[k].resize(n_inst);
    for (int k = 0; k < 4; ++k) br.ldsn[k].resize(n_inst);
    size_t at = align256(sizeof(IntegCtl) * n_inst);
    int64_t blocks[3] = {0, 0, 0};
    for (int i = 0; i < n_inst; ++i) {
        const smol_instance &q = inst[i];
        const int logL = fft_log2(q.M);
        br.logL[i] = logL;
        int u[8];
        if ((rc = with_shape<ShapeUnits>(logL, precision, (int)q.R, u))) return rc;
        for (int k = 0; k < 3; ++k) {
            br.units[k][i] = u[k];
            br.ldsn[k][i] = u[4 + k];
            blocks[k] += u[k];
        }
        br.ldsn[3][i] = u[7];
        nC[i] = u[2];
        redA[i] = u[3];
        const int64_t L = 1LL << logL, half = L / 2, N2 = 1LL << (logL / 2);
        const int64_t Mt = q.M > half + 1 ? q.M : half + 1;
        br.off[i] = at;
        at += align256(sizeof(double) * (size_t)Mt * 10);                 // state, stages
        at += align256(sizeof(double) * (size_t)Mt * 2 * q.R);            // U, V copies
        at += align256(sizeof(cd) * (size_t)(q.R * L + L / 2));           // spectra
        at += align256(sizeof(double) * (size_t)(N2 * q.R * 4 + 4 * q.R + N2 * SMOL_EPART));
    }
    for (int k = 0; k < 3; ++k)
        if (blocks[k] > (1LL << 30)) return SMOL_EUNSUPPORTED;
    const size_t tab_off = at;
    size_t tab_bytes = 0;
    tab_bytes += align256(sizeof(IntegDev) * n_inst);
    tab_bytes += align256(sizeof(int) * n_inst) * 4;  // logL, nC, redA, active list
    for (int k = 0; k < 3; ++k)
        tab_bytes += align256(sizeof(int) * (n_inst + 1)) + align256(sizeof(int) * blocks[k]);
    const size_t arena_bytes = at + tab_bytes;

    char *arena = nullptr;
    if (hipMalloc(&arena, arena_bytes) != hipSuccess) return SMOL_ENOMEM;
    IntegCtl *hctl = nullptr;
    hipStream_t cap = nullptr;
    hipGraphExec_t ge = nullptr;
    rc = SMOL_OK;
    do {
        if (hipHostMalloc(&hctl, sizeof(IntegCtl) * n_inst, hipHostMallocDefault) != hipSuccess) {
            rc = SMOL_ENOMEM;
            break;
        }
        // ---- per-instance device views and control blocks
        IntegCtl *dctl = (IntegCtl *)arena;
        std::vector<IntegDev> hdev(n_inst);
        const int kq = (method == SMOL_DP54 ? 4 : 2) + 1;
        for (int i = 0; i < n_inst; ++i) {
            const smol_instance &q = inst[i];
            const int logL = br.logL[i];
            const int64_t L = 1LL << logL, half = L / 2, N2 = 1LL << (logL / 2);
            const int64_t Mt = q.M > half + 1 ? q.M : half + 1;
            char *p = arena + br.off[i];
            double *ibuf = (double *)p;
            p += align256(sizeof(double) * (size_t)Mt * 10);
            double *uvt = (double *)p;
            p += align256(sizeof(double) * (size_t)Mt * 2 * q.R);
            cd *Z = (cd *)p;
            p += align256(sizeof(cd) * (size_t)(q.R * L + L / 2));
            double *red_part = (double *)p;
            IntegDev &I = hdev[i];
            memset(&I, 0, sizeof(I));
            I.M = q.M;
            I.Mt = Mt;
            I.R = q.R;
            I.logL = logL;
            I.Ut = uvt;
            I.Vt = uvt + (size_t)q.R * Mt;
            I.ctl = dctl + i;
            I.nb[0] = ibuf;
            I.nb[1] = ibuf + Mt;
            for (int j = 0; j < 7; ++j) I.kslot[j] = ibuf + (2 + j) * Mt;
            I.ybuf = ibuf + 9 * Mt;
            I.Z = Z;
            I.Qp = Z + q.R * L;
            I.red_part = red_part;
            I.red = red_part + (size_t)N2 * q.R * 4;
            I.epart = I.red + (size_t)q.R * 4;
            I.rt.tw = roots->tw;
            I.rt.fine = roots->fine;
            IntegCtl &c = hctl[i];
            memset(&c, 0, sizeof(c));
            c.U = I.Ut;
            c.V = I.Vt;
            c.lam = q.lambda;
            c.t_end = q.t_end;
            c.rtol = q.rtol;
            c.atol = q.atol;
            c.h_min = o.h_min;
            c.h0_user = o.h0;
            c.alpha = o.alpha > 0 ? o.alpha : 0.7 / kq;
            c.beta = o.alpha > 0 ? o.beta : 0.4 / kq;
            c.safety = 0.9;
            c.facmin = 0.2;
            c.facmax = 10.0;
            c.max_steps = o.max_steps > 0 ? o.max_steps : 100000000LL;
            c.method = method;
            c.controller = o.controller;
            c.mlp = o.controller == SMOL_CTRL_LEARNED ? mlp : nullptr;
            c.log = q.log;
            c.log_cap = q.log ? q.log_cap : 0;
            c.err_prev = 1.0;
            c.done = q.t_end == 0.0;  // nothing to do: n_out = n0
        }
        // ---- tables
        char *tp = arena + tab_off;
        auto take = [&](size_t bytes) -> char * {
            char *d = tp;
            tp += align256(bytes);
            return d;
        };
        BatchDev B;
        IntegDev *dinst = (IntegDev *)take(sizeof(IntegDev) * n_inst);
        int *dlogL = (int *)take(sizeof(int) * n_inst);
        int *dnC = (int *)take(sizeof(int) * n_inst);
        int *dredA = (int *)take(sizeof(int) * n_inst);
        int *dactive = (int *)take(sizeof(int) * n_inst);
        int *dfirst[3], *downer[3];
        for (int k = 0; k < 3; ++k) {
            dfirst[k] = (int *)take(sizeof(int) * (n_inst + 1));
            downer[k] = (int *)take(sizeof(int) * blocks[k]);
        }
        if (hipMemcpyAsync(dinst, hdev.data(), sizeof(IntegDev) * n_inst, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(dlogL, br.logL.data(), sizeof(int) * n_inst, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(dnC, nC.data(), sizeof(int) * n_inst, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(dredA, redA.data(), sizeof(int) * n_inst, hipMemcpyHostToDevice, s)) {
            rc = SMOL_EDEVICE;
            break;
        }
        B.inst = dinst;
        B.logL = dlogL;
        B.nC = dnC;
        B.redA = dredA;
        B.active = dactive;
        for (int k = 0; k < 3; ++k) {
            B.first[k] = dfirst[k];
            B.owner[k] = downer[k];
        }
        std::vector<int> ids;
        for (int i = 0; i < n_inst; ++i)
            if (!hctl[i].done) ids.push_back(i);
        if (hipMemcpyAsync(dctl, hctl, sizeof(IntegCtl) * n_inst, hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = SMOL_EDEVICE;
            break;
        }
        // ---- inputs into the transposed layout
        for (int i = 0; i < n_inst; ++i) {
            const smol_instance &q = inst[i];
            const IntegDev &I = hdev[i];
            hipLaunchKernelGGL(k_to_tr, dim3(128), dim3(256), 0, s, q.U, I.Ut, q.M, q.R, q.M, I.Mt, I.logL);
            hipLaunchKernelGGL(k_to_tr, dim3(128), dim3(256), 0, s, q.V, I.Vt, q.M, q.R, q.M, I.Mt, I.logL);
            hipLaunchKernelGGL(k_to_tr, dim3(128), dim3(256), 0, s, q.n0, I.nb[0], q.M, 1, q.M, I.Mt, I.logL);
        }
        // ---- starting step for every instance
        if (ids.empty()) {
            for (int i = 0; i < n_inst; ++i) stats_from(hctl[i], &stats[i]);
        }
        if (!ids.empty() && (rc = build_tables(br, ids, dfirst, downer, dactive, s))) break;
        if (!ids.empty()) {
            launch_stage_p(precision, B, br, 0, 0, s);
            hipLaunchKernelGGL(kb_init_h0, dim3(br.nact), dim3(SMOL_WG), 0, s, B);
            if (!(o.h0 > 0)) {
                launch_stage_p(precision, B, br, 1, 0, s);
                hipLaunchKernelGGL(kb_init_h, dim3(br.nact), dim3(SMOL_WG), 0, s, B);
            }
        }
        if (hipGetLastError() != hipSuccess) {
            rc = SMOL_EDEVICE;
            break;
        }
        // ---- graph of SMOL_GRAPH_ATTEMPTS attempts over the listed instances
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
            rc = SMOL_EDEVICE;
            break;
        }
        const int S = method == SMOL_DP54 ? 7 : 4;
        auto capture = [&]() -> int {
            if (ge) (void)hipGraphExecDestroy(ge);
            ge = nullptr;
            hipGraph_t g;
            HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            for (int a = 0; a < SMOL_GRAPH_ATTEMPTS; ++a) {
                for (int st = 2; st <= S; ++st) launch_stage_p(precision, B, br, st, S, cap);
                hipLaunchKernelGGL(kb_ctrl, dim3(br.nact), dim3(SMOL_WG), 0, cap, B);
            }
            HIP_TRY(hipStreamEndCapture(cap, &g));
            hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(e);
            return SMOL_OK;
        };
        // ---- replay until every instance is done; when the running set
        // halves, rebuild the tables over it and capture again, so finished
        // instances stop costing workgroups
        int64_t chunk = 1;
        bool need_capture = !ids.empty();
        while (!ids.empty()) {
            if (need_capture) {
                if ((rc = capture())) break;
                need_capture = false;
            }
            for (int64_t k = 0; k < chunk && rc == SMOL_OK; ++k)
                if (hipGraphLaunch(ge, s) != hipSuccess) rc = SMOL_EDEVICE;
            if (rc) break;
            if (hipMemcpyAsync(hctl, dctl, sizeof(IntegCtl) * n_inst, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = SMOL_EDEVICE;
                break;
            }
            std::vector<int> live;
            double most = 0.0;
            for (int i : ids) {
                if (hctl[i].done) continue;
                live.push_back(i);
                double est = hctl[i].h > 0 ? (hctl[i].t_end - hctl[i].t) / hctl[i].h : 1e9;
                if (!(est < 1e9)) est = 1e9;
                if (est > most) most = est;
            }
            if (live.empty()) break;
            if (2 * live.size() <= ids.size()) {
                ids = live;
                if ((rc = build_tables(br, ids, dfirst, downer, dactive, s))) break;
                need_capture = true;
            }
            chunk = (int64_t)(0.5 * most / SMOL_GRAPH_ATTEMPTS) + 1;
            if (chunk > 16) chunk = 16;
        }
        if (rc) break;
        if (hipMemcpyAsync(hctl, dctl, sizeof(IntegCtl) * n_inst, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = SMOL_EDEVICE;
            break;
        }
        // ---- outputs
        for (int i = 0; i < n_inst; ++i) {
            const IntegDev &I = hdev[i];
            hipLaunchKernelGGL(k_from_tr, dim3(128), dim3(256), 0, s, I.nb[hctl[i].cur], inst[i].n_out,
                               inst[i].M, I.logL);
            stats_from(hctl[i], &stats[i]);
        }
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = SMOL_EDEVICE;
    } while (0);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (cap) (void)hipStreamDestroy(cap);
    (void)hipStreamSynchronize(s);
    (void)hipFree(arena);
    if (hctl) (void)hipHostFree(hctl);
    return rc;
}
