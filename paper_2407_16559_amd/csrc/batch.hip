// Batched integration of many independent instances (uneven M, kernels,
// lambda and tolerances), each with its own step size, accept / reject and
// status, carried in per-instance control blocks.  Instances are grouped by
// transform length (shape).  Every kernel of a step attempt is one launch
// per shape over that shape's instances: block-to-instance tables give each
// workgroup its instance and unit, and the shape's tuned launch schedule
// applies.  Each shape's chain of step attempts is captured once as its own
// hipGraph and replayed on one of four streams, so the shapes run side by
// side; finished instances' workgroups return at entry, and when the
// running set halves the tables are rebuilt over the live instances and the
// graphs captured again.
#include <algorithm>
#include <cstring>
#include <vector>

#include "sched.h"

#define SMOL_BATCH_STREAMS 4  // one per hardware queue (the runtime's default count)

// The batched phase kernels (one launch per transform shape and phase over
// that shape's instances, under the shape's launch schedule) live with the
// single-instance ones in phases_a/b/c.hip.

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
__global__ __launch_bounds__(SMOL_WG) void kb_ctrl(BatchDev B, int base)
{
    const int b = B.active[base + blockIdx.x];
    controller_step(B.inst[b], B.nC[b]);
}

namespace {

struct BatchRun {
    int n = 0, precision = 0;
    std::vector<int> logL, units[3];  // per instance
    std::vector<size_t> off;          // arena offset of each instance
    int nact = 0;                     // listed instances
    // shapes of the listed instances: schedule, grids, LDS
    struct Shape {
        int logL;
        int var[3];
        int base[3], count[3];  // block range of each kernel
        int abase, acount;      // range in the list of running instances
        size_t lds[3], lds_fused;
    };
    std::vector<Shape> shapes;
};

// Block-to-instance tables over the instances in `ids`, grouped by shape
// (device buffers sized for all instances are reused).
int build_tables(BatchRun &br, std::vector<int> ids, int *dfirst[3], int *downer[3],
                 int *dactive, hipStream_t s)
{
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int x, int y) { return br.logL[x] < br.logL[y]; });
    std::vector<int> first[3], owner[3];
    for (int k = 0; k < 3; ++k) first[k].assign(br.n + 1, 0);
    br.shapes.clear();
    int total[3] = {0, 0, 0};
    for (size_t pos = 0; pos < ids.size(); ++pos) {
        const int i = ids[pos];
        if (br.shapes.empty() || br.shapes.back().logL != br.logL[i]) {
            BatchRun::Shape sh{};
            sh.logL = br.logL[i];
            schedule_of(sh.logL, br.precision, sh.var);
            PhaseDims d;
            for (int k = 0; k < 3; ++k) {
                sh.base[k] = total[k];
                int rc = phase_dims(sh.logL, br.precision, k, sh.var[k], 1, false, &d);
                if (rc) return rc;
                sh.lds[k] = d.lds_bytes;
            }
            int rc = phase_dims(sh.logL, br.precision, PH_C, sh.var[2], 1, true, &d);
            if (rc) return rc;
            sh.lds_fused = d.lds_bytes;
            sh.abase = (int)pos;
            br.shapes.push_back(sh);
        }
        br.shapes.back().acount += 1;
        for (int k = 0; k < 3; ++k) {
            first[k][i] = total[k];
            for (int j = 0; j < br.units[k][i]; ++j) owner[k].push_back(i);
            total[k] += br.units[k][i];
            br.shapes.back().count[k] = total[k] - br.shapes.back().base[k];
        }
    }
    br.nact = (int)ids.size();
    for (int k = 0; k < 3; ++k) {
        HIP_TRY(hipMemcpyAsync(dfirst[k], first[k].data(), sizeof(int) * (br.n + 1),
                               hipMemcpyHostToDevice, s));
        if (total[k])
            HIP_TRY(hipMemcpyAsync(downer[k], owner[k].data(), sizeof(int) * total[k],
                                   hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(dactive, ids.data(), sizeof(int) * ids.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // host vectors die here
    return SMOL_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Same kernel sequence as a single instance (A only up to stage 2, the
// finish of stages 2..S-1 fused with the next column pass), each kernel as
// one launch over the instances of one shape, under that shape's schedule.
int launch_stage(const BatchDev &B, const BatchRun &br, const BatchRun::Shape &sh, int method,
                 int stage, int S, hipStream_t s)
{
    int rc;
    const int p = br.precision;
    if (stage <= 2 && sh.count[0] &&
        (rc = launch_bat_A(sh.logL, p, sh.var[0], B, sh.base[0], sh.count[0], stage, method, s)))
        return rc;
    if (sh.count[1] && (rc = launch_bat_B(sh.logL, p, sh.var[1], B, sh.base[1], sh.count[1], stage, s)))
        return rc;
    const bool fuse = stage >= 2 && stage < S;
    if (sh.count[2] &&
        (rc = launch_bat_C(sh.logL, p, sh.var[2], B, sh.base[2], sh.count[2], stage, fuse, method, s)))
        return rc;
    return SMOL_OK;
}

int launch_stage_all(const BatchDev &B, const BatchRun &br, int method, int stage, int S,
                     hipStream_t s)
{
    for (const auto &sh : br.shapes) {
        int rc = launch_stage(B, br, sh, method, stage, S, s);
        if (rc) return rc;
    }
    return SMOL_OK;
}

}  // namespace

extern "C" int smol_integrate_batch(int32_t n_inst, const smol_instance *inst, int32_t method,
                                    int32_t precision, const smol_options *opts,
                                    smol_stats *stats, void *stream)
{
    if (n_inst < 1 || !inst || !stats) return SMOL_EINVAL;
    {
        const int mrc = check_method(method);
        if (mrc) return mrc;
    }
    if (precision != SMOL_FP64 && precision != SMOL_FP32X2) return SMOL_EINVAL;
    smol_options o{};
    if (opts) o = *opts;
    if (o.h0 < 0 || o.h_min < 0 || o.max_steps < 0 || o.log || o.state) return SMOL_EINVAL;
    if (!controller_valid(o.controller)) return SMOL_EINVAL;
    for (int i = 0; i < n_inst; ++i) {
        const smol_instance &q = inst[i];
        int rc = check_common(q.M, q.R, q.U, q.V, q.lambda);
        if (rc) return rc;
        if (!q.n0 || !q.n_out || (q.log && q.log_cap < 0)) return SMOL_EINVAL;
        if (q.source && q.source == q.n_out) return SMOL_EINVAL;
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
    br.precision = precision;
    std::vector<int> nC(n_inst), redA(n_inst);
    br.logL.resize(n_inst);
    br.off.resize(n_inst);
    for (int k = 0; k < 3; ++k) br.units[k].resize(n_inst);
    size_t at = align256(sizeof(IntegCtl) * n_inst);
    int64_t blocks[3] = {0, 0, 0};
    for (int i = 0; i < n_inst; ++i) {
        const smol_instance &q = inst[i];
        const int logL = fft_log2(q.M);
        br.logL[i] = logL;
        int var[3];
        schedule_of(logL, precision, var);
        PhaseDims d[3];
        for (int k = 0; k < 3; ++k) {
            if ((rc = phase_dims(logL, precision, k, var[k], (int)q.R, false, &d[k]))) return rc;
            br.units[k][i] = d[k].units;
            blocks[k] += d[k].units;
        }
        nC[i] = d[PH_C].jobs;
        redA[i] = d[PH_A].jobs;
        const int64_t L = 1LL << logL, half = L / 2, N2 = 1LL << split_log_n2(logL);
        const int64_t Mt = q.M > half + 1 ? q.M : half + 1;
        br.off[i] = at;
        at += align256(sizeof(double) * (size_t)Mt * 11);                 // state, stages, sources
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
    hipStream_t streams[SMOL_BATCH_STREAMS] = {};
    std::vector<hipGraphExec_t> ge;
    rc = SMOL_OK;
    do {
        if (hipHostMalloc(&hctl, sizeof(IntegCtl) * n_inst, hipHostMallocDefault) != hipSuccess) {
            rc = SMOL_ENOMEM;
            break;
        }
        // ---- per-instance device views and control blocks
        IntegCtl *dctl = (IntegCtl *)arena;
        std::vector<IntegDev> hdev(n_inst);
        for (int i = 0; i < n_inst; ++i) {
            const smol_instance &q = inst[i];
            const int logL = br.logL[i];
            const int64_t L = 1LL << logL, half = L / 2, N2 = 1LL << split_log_n2(logL);
            const int64_t Mt = q.M > half + 1 ? q.M : half + 1;
            char *p = arena + br.off[i];
            double *ibuf = (double *)p;
            p += align256(sizeof(double) * (size_t)Mt * 11);
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
            I.src = ibuf + 10 * Mt;
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
            c.h_min = o.h_min;
            c.h0_user = o.h0;
            c.max_steps = o.max_steps > 0 ? o.max_steps : 100000000LL;
            c.mlp = o.controller == SMOL_CTRL_LEARNED ? mlp : nullptr;
            c.log = q.log;
            c.log_cap = q.log ? q.log_cap : 0;
            ctl_setup(c, method, o, q.rtol, q.atol);
            c.has_src = q.source != nullptr;
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
            if (q.source)
                hipLaunchKernelGGL(k_to_tr, dim3(128), dim3(256), 0, s, q.source, I.src, q.M, 1, q.M,
                                   I.Mt, I.logL);
        }
        // ---- starting step for every instance
        if (ids.empty()) {
            for (int i = 0; i < n_inst; ++i) stats_from(hctl[i], &stats[i]);
        }
        if (!ids.empty() && (rc = build_tables(br, ids, dfirst, downer, dactive, s))) break;
        if (!ids.empty()) {
            if ((rc = launch_stage_all(B, br, method, 0, 0, s))) break;
            hipLaunchKernelGGL(kb_init_h0, dim3(br.nact), dim3(SMOL_WG), 0, s, B);
            if (!(o.h0 > 0)) {
                if ((rc = launch_stage_all(B, br, method, 1, 0, s))) break;
                hipLaunchKernelGGL(kb_init_h, dim3(br.nact), dim3(SMOL_WG), 0, s, B);
            }
        }
        if (hipGetLastError() != hipSuccess) {
            rc = SMOL_EDEVICE;
            break;
        }
        // ---- one graph of SMOL_GRAPH_ATTEMPTS attempts per shape, each shape
        // on its own stream (up to SMOL_BATCH_STREAMS, default priority), so
        // the shapes' independent kernel chains run side by side
        int nstream = 0;
        for (; nstream < SMOL_BATCH_STREAMS; ++nstream)
            if (hipStreamCreateWithFlags(&streams[nstream], hipStreamNonBlocking) != hipSuccess) {
                rc = SMOL_EDEVICE;
                break;
            }
        if (rc) break;
        const int S = k_scheme_stages[method];
        auto capture = [&]() -> int {
            for (auto &g : ge)
                if (g) (void)hipGraphExecDestroy(g);
            ge.assign(br.shapes.size(), nullptr);
            for (size_t j = 0; j < br.shapes.size(); ++j) {
                const auto &sh = br.shapes[j];
                hipStream_t cs = streams[j % nstream];
                hipGraph_t g = nullptr;
                HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                int r = SMOL_OK;
                for (int a = 0; a < SMOL_GRAPH_ATTEMPTS && r == SMOL_OK; ++a) {
                    for (int st = 2; st <= S && r == SMOL_OK; ++st)
                        r = launch_stage(B, br, sh, method, st, S, cs);
                    hipLaunchKernelGGL(kb_ctrl, dim3(sh.acount), dim3(SMOL_WG), 0, cs, B, sh.abase);
                }
                hipError_t e = hipStreamEndCapture(cs, &g);
                if (r) {
                    if (g) (void)hipGraphDestroy(g);
                    return r;
                }
                HIP_TRY(e);
                e = hipGraphInstantiate(&ge[j], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                HIP_TRY(e);
            }
            return SMOL_OK;
        };
        // the starting steps were queued on s
        if (hipStreamSynchronize(s) != hipSuccess) {
            rc = SMOL_EDEVICE;
            break;
        }
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
            for (size_t j = 0; j < ge.size() && rc == SMOL_OK; ++j)
                for (int64_t k = 0; k < chunk && rc == SMOL_OK; ++k)
                    if (hipGraphLaunch(ge[j], streams[j % nstream]) != hipSuccess) rc = SMOL_EDEVICE;
            for (int j = 0; j < nstream; ++j)
                if (hipStreamSynchronize(streams[j]) != hipSuccess) rc = SMOL_EDEVICE;
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
                const double left = (double)(hctl[i].max_steps - hctl[i].attempts);
                if (left < est) est = left;
                if (est > most) most = est;
            }
            if (live.empty()) break;
            // rebuild when half the instances have finished, or when every
            // instance of some shape has: that shape's graph would only replay
            // empty launches, and on a shared stream hold up a live shape
            bool shape_done = false;
            for (const auto &sh : br.shapes) {
                bool any = false;
                for (int i : live) any = any || br.logL[i] == sh.logL;
                shape_done = shape_done || !any;
            }
            if (2 * live.size() <= ids.size() || shape_done) {
                ids = live;
                if ((rc = build_tables(br, ids, dfirst, downer, dactive, s))) break;
                need_capture = true;
            }
            chunk = (int64_t)(0.5 * most / SMOL_GRAPH_ATTEMPTS) + 1;
            // at most 64 attempts of each shape between polls
            if (chunk > 64 / SMOL_GRAPH_ATTEMPTS) chunk = 64 / SMOL_GRAPH_ATTEMPTS;
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
    for (auto &g : ge)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto &st : streams)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    (void)hipStreamSynchronize(s);
    (void)hipFree(arena);
    if (hctl) (void)hipHostFree(hctl);
    return rc;
}
