// Kernels of the three right-hand-side phases, per transform shape
// (N1 x N2), complex arithmetic T and schedule variant (E elements per
// lane, W waves per workgroup), and their launch functors.  Included only by
// the phase translation units, so each kernel is compiled once.
#pragma once
#include "sched.h"

// ---- plain right-hand side -------------------------------------------------

template <int N1, int N2, class T, int E, int W>
__global__ __launch_bounds__(64 * W) void k_phaseA(RhsPlanDev P, Pro in, int nunits)
{
    extern __shared__ cd lds[];
    const int unit = xcd_remap(blockIdx.x, gridDim.x);
    if (unit < nunits) SMOL_PHASE_CALL(T, PhaseA<N1, N2, T, E, W>::run(P, in, unit, (T *)lds));
}

template <int N1, int N2, class T, int E, int W>
__global__ __launch_bounds__(64 * W) void k_phaseB(RhsPlanDev P, int red_jobs)
{
    extern __shared__ cd lds[];
    // neighbouring row pairs share the cache lines of the column-major spectra
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    if (u == PhaseB<N1, N2, T, E, W>::units()) {
        if (red_jobs > 0) finalize_reductions<64 * W>(P, red_jobs);
        return;
    }
    SMOL_PHASE_CALL(T, PhaseB<N1, N2, T, E, W>::run(P, u, (T *)lds));
}

template <int N1, int N2, class T, int E, int W>
__global__ __launch_bounds__(64 * W) void k_phaseC(RhsPlanDev P, Epi ep, int nunits)
{
    extern __shared__ cd lds[];
    const int unit = xcd_remap(blockIdx.x, gridDim.x);
    if (unit < nunits)
        SMOL_PHASE_CALL(T, PhaseC<N1, N2, T, E, W>::template run<false>(P, ep, unit, (T *)lds));
}

// ---- integrator stages: the same phases, buffers from the control block ----

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform_d(double v)
{
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

// method: the run's tableau, passed by the host so that the coefficient
// loads do not wait for the control block.
//
// CTRL (the stage-2 column pass of a captured step attempt): the control
// block I.ctl holds the previous attempt, whose error rows are in I.epart
// (njobs of them) when its flag `pending` is set.  Every workgroup takes that
// attempt's accept / reject decision and the next step itself (the same
// arithmetic in the same order, so the same result) and goes on with the
// attempt it prepared; workgroup 0 stores the updated block to cout, which
// the attempt's later kernels read and the next stage-2 pass takes as its
// input (two blocks, alternating).  The error rows are requested before the
// control block.
template <int N1, int N2, class T, int E, int W, bool CTRL>
__global__ __launch_bounds__(64 * W) void k_int_A(IntegDev I, int stage, int nunits, int method,
                                                  IntegCtl *cout, int njobs)
{
    using PA = PhaseA<N1, N2, T, E, W>;
    extern __shared__ cd lds[];
    const int unit = xcd_remap(blockIdx.x, gridDim.x);
    typename PA::Early e;  // twiddles and factors: requested before the control block
    if (unit < nunits) PA::early(plan_of_ws(I), unit, e);
    IntegCtl c;
    if constexpr (CTRL) {
        __shared__ IntegCtl sc;
        constexpr int NW = sizeof(IntegCtl) / 4;
        double acc[SMOL_EPART];
        epart_partial(I.epart, njobs, acc);
        for (int i = threadIdx.x; i < NW; i += 64 * W)
            ((uint32_t *)&sc)[i] = ((const uint32_t *)I.ctl)[i];
        __syncthreads();
        // Every thread reads the flags before any thread writes the block:
        // the decision's writes follow the barrier inside epart_total, and
        // the flag update follows the barrier below on both paths.
        if (!sc.done && sc.pending) {
            double tot[SMOL_EPART];
            epart_total<64 * W>(acc, tot);
            controller_decide(sc, tot, I.M, blockIdx.x == 0);
        }
        __syncthreads();
        if (threadIdx.x == 0) sc.pending = sc.done ? 0 : 1;
        __syncthreads();
        if (blockIdx.x == 0)
            for (int i = threadIdx.x; i < NW; i += 64 * W)
                ((uint32_t *)cout)[i] = ((const uint32_t *)&sc)[i];
        // what this pass reads of the block, as uniform values
        c.done = uniform_i(sc.done);
        c.cur = uniform_i(sc.cur);
        c.kp = uniform_i(sc.kp);
        c.has_src = uniform_i(sc.has_src);
        c.h = uniform_d(sc.h);
        c.h0 = uniform_d(sc.h0);
        c.lam = uniform_d(sc.lam);
    } else {
        c = *I.ctl;  // one snapshot: all fields load together
    }
    if (c.done) return;
    const Tableau &tab = c_tab[method];
    const RhsPlanDev P = plan_of(I, c);
    const Pro in = stage_pro(I, c, tab, stage);
    if (unit < nunits) SMOL_PHASE_CALL(T, PA::run_with(P, in, unit, (T *)lds, e));
}

// jobs_a / jobs_c: reduction partial rows written by the column pass (stages
// 0..2) or by the previous stage's fused finish (later stages).
//
// This pass reads and writes workspaces only (spectra, packed inverse input,
// reduction rows), so it does not wait for the control block: after the run
// has ended a replayed launch recomputes workspaces that nothing reads.
template <int N1, int N2, class T, int E, int W>
__global__ __launch_bounds__(64 * W) void k_int_B(IntegDev I, int stage, int jobs_a, int jobs_c)
{
    extern __shared__ cd lds[];
    const RhsPlanDev P = plan_of_ws(I);
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    if (u == PhaseB<N1, N2, T, E, W>::units()) {
        finalize_reductions<64 * W>(P, stage <= 2 ? jobs_a : jobs_c);
        return;
    }
    SMOL_PHASE_CALL(T, PhaseB<N1, N2, T, E, W>::run(P, u, (T *)lds));
}

// The packed columns, twiddles and column-pass factors do not depend on the
// control block, so they are requested before it and their round trips
// overlap.
template <int N1, int N2, class T, int E, int W, bool FUSE>
__global__ __launch_bounds__(64 * W) void k_int_C(IntegDev I, int stage, int nunits, int method)
{
    using PC = PhaseC<N1, N2, T, E, W>;
    extern __shared__ cd lds[];
    const int unit = xcd_remap(blockIdx.x, gridDim.x);
    typename PC::Early e;
    if (unit < nunits) PC::template early<FUSE>(plan_of_ws(I), unit, e);
    const IntegCtl c = *I.ctl;  // one snapshot: all fields load together
    if (c.done) return;
    const Tableau &tab = c_tab[method];
    const RhsPlanDev P = plan_of(I, c);
    const Epi ep = stage_epi(I, c, tab, stage);
    if (unit < nunits) SMOL_PHASE_CALL(T, PC::template run_with<FUSE>(P, ep, unit, (T *)lds, e));
}

// ---- batched stage kernels: blocks [base, base + gridDim) of one shape -------

template <int N1, int N2, class T, int E, int W>
__global__ __launch_bounds__(64 * W) void kb_A(BatchDev B, int base, int stage, int method)
{
    extern __shared__ cd lds[];
    const int blk = base + xcd_remap(blockIdx.x, gridDim.x);  // neighbours share an XCD
    const int b = B.owner[0][blk];
    const IntegDev &I = B.inst[b];
    const IntegCtl c = *I.ctl;
    if (c.done) return;
    const RhsPlanDev P = plan_of(I, c);
    const Pro in = stage_pro(I, c, c_tab[method], stage);
    SMOL_PHASE_CALL(T, PhaseA<N1, N2, T, E, W>::run(P, in, blk - B.first[0][b], (T *)lds));
}

template <int N1, int N2, class T, int E, int W>
__global__ __launch_bounds__(64 * W) void kb_B(BatchDev B, int base, int stage)
{
    extern __shared__ cd lds[];
    const int blk = base + xcd_remap(blockIdx.x, gridDim.x);
    const int b = B.owner[1][blk];
    const IntegDev &I = B.inst[b];
    const IntegCtl c = *I.ctl;
    if (c.done) return;
    const RhsPlanDev P = plan_of(I, c);
    const int unit = blk - B.first[1][b];
    if (unit == PhaseB<N1, N2, T, E, W>::units()) {
        finalize_reductions<64 * W>(P, stage <= 2 ? B.redA[b] : B.nC[b]);
        return;
    }
    SMOL_PHASE_CALL(T, PhaseB<N1, N2, T, E, W>::run(P, unit, (T *)lds));
}

template <int N1, int N2, class T, int E, int W, bool FUSE>
__global__ __launch_bounds__(64 * W) void kb_C(BatchDev B, int base, int stage, int method)
{
    extern __shared__ cd lds[];
    const int blk = base + xcd_remap(blockIdx.x, gridDim.x);
    const int b = B.owner[2][blk];
    const IntegDev &I = B.inst[b];
    const IntegCtl c = *I.ctl;
    if (c.done) return;
    const RhsPlanDev P = plan_of(I, c);
    const Epi ep = stage_epi(I, c, c_tab[method], stage);
    SMOL_PHASE_CALL(T, PhaseC<N1, N2, T, E, W>::template run<FUSE>(P, ep, blk - B.first[2][b],
                                                                   (T *)lds));
}

// ---- launch functors (used through with_variant) ----------------------------

struct RhsA {
    template <int N1, int N2, class T, int E, int W>
    static int run(const RhsPlanDev &P, const Pro &in, hipStream_t s)
    {
        using A = PhaseA<N1, N2, T, E, W>;
        const int n = A::units(P.R);
        hipLaunchKernelGGL((k_phaseA<N1, N2, T, E, W>), dim3(n), dim3(A::NT), sizeof(cd) * A::LDS,
                           s, P, in, n);
        return SMOL_OK;
    }
};
struct RhsB {
    template <int N1, int N2, class T, int E, int W>
    static int run(const RhsPlanDev &P, int red_jobs, hipStream_t s)
    {
        using B = PhaseB<N1, N2, T, E, W>;
        hipLaunchKernelGGL((k_phaseB<N1, N2, T, E, W>), dim3(B::units() + 1), dim3(B::NT),
                           sizeof(cd) * B::LDS, s, P, red_jobs);
        return SMOL_OK;
    }
};
struct RhsC {
    template <int N1, int N2, class T, int E, int W>
    static int run(const RhsPlanDev &P, const Epi &ep, hipStream_t s)
    {
        using C = PhaseC<N1, N2, T, E, W>;
        const int n = C::units();
        hipLaunchKernelGGL((k_phaseC<N1, N2, T, E, W>), dim3(n), dim3(C::NT), sizeof(cd) * C::LDS,
                           s, P, ep, n);
        return SMOL_OK;
    }
};
struct IntA {
    template <int N1, int N2, class T, int E, int W>
    static int run(const IntegDev &I, int stage, int method, IntegCtl *cout, int njobs,
                   hipStream_t s)
    {
        using A = PhaseA<N1, N2, T, E, W>;
        const int n = A::units(I.R);
        if (cout)
            hipLaunchKernelGGL((k_int_A<N1, N2, T, E, W, true>), dim3(n), dim3(A::NT),
                               sizeof(cd) * A::LDS, s, I, stage, n, method, cout, njobs);
        else
            hipLaunchKernelGGL((k_int_A<N1, N2, T, E, W, false>), dim3(n), dim3(A::NT),
                               sizeof(cd) * A::LDS, s, I, stage, n, method, cout, njobs);
        return SMOL_OK;
    }
};
struct IntB {
    template <int N1, int N2, class T, int E, int W>
    static int run(const IntegDev &I, int stage, int jobs_a, int jobs_c, hipStream_t s)
    {
        using B = PhaseB<N1, N2, T, E, W>;
        hipLaunchKernelGGL((k_int_B<N1, N2, T, E, W>), dim3(B::units() + 1), dim3(B::NT),
                           sizeof(cd) * B::LDS, s, I, stage, jobs_a, jobs_c);
        return SMOL_OK;
    }
};
struct IntC {
    template <int N1, int N2, class T, int E, int W>
    static int run(const IntegDev &I, int stage, bool fuse, int method, hipStream_t s)
    {
        using C = PhaseC<N1, N2, T, E, W>;
        const int n = C::units();
        if (fuse)
            hipLaunchKernelGGL((k_int_C<N1, N2, T, E, W, true>), dim3(n), dim3(C::NT),
                               sizeof(cd) * C::LDS_FUSE, s, I, stage, n, method);
        else
            hipLaunchKernelGGL((k_int_C<N1, N2, T, E, W, false>), dim3(n), dim3(C::NT),
                               sizeof(cd) * C::LDS, s, I, stage, n, method);
        return SMOL_OK;
    }
};

struct BatA {
    template <int N1, int N2, class T, int E, int W>
    static int run(const BatchDev &B, int base, int count, int stage, int method, hipStream_t s)
    {
        using A = PhaseA<N1, N2, T, E, W>;
        hipLaunchKernelGGL((kb_A<N1, N2, T, E, W>), dim3(count), dim3(A::NT), sizeof(cd) * A::LDS,
                           s, B, base, stage, method);
        return SMOL_OK;
    }
};
struct BatB {
    template <int N1, int N2, class T, int E, int W>
    static int run(const BatchDev &B, int base, int count, int stage, hipStream_t s)
    {
        using P = PhaseB<N1, N2, T, E, W>;
        hipLaunchKernelGGL((kb_B<N1, N2, T, E, W>), dim3(count), dim3(P::NT), sizeof(cd) * P::LDS,
                           s, B, base, stage);
        return SMOL_OK;
    }
};
struct BatC {
    template <int N1, int N2, class T, int E, int W>
    static int run(const BatchDev &B, int base, int count, int stage, bool fuse, int method,
                   hipStream_t s)
    {
        using C = PhaseC<N1, N2, T, E, W>;
        if (fuse)
            hipLaunchKernelGGL((kb_C<N1, N2, T, E, W, true>), dim3(count), dim3(C::NT),
                               sizeof(cd) * C::LDS_FUSE, s, B, base, stage, method);
        else
            hipLaunchKernelGGL((kb_C<N1, N2, T, E, W, false>), dim3(count), dim3(C::NT),
                               sizeof(cd) * C::LDS, s, B, base, stage, method);
        return SMOL_OK;
    }
};
