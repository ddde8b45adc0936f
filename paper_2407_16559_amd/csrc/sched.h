// Launch schedules of the three right-hand-side kernels.
//
// For each kernel a schedule picks the radix of the in-register butterflies
// (E, elements per lane) and the workgroup tile (W, waves per workgroup,
// i.e. how many transforms a workgroup owns).  A kernel's variant v encodes
// both:
//   bit 0 set -> W = 8, else W = 4;
//   bit 1 set -> E = 4, else the default (8, or 16 for 1024-point transforms).
// Variant 0 exists for every shape and precision; the others exist for FP64
// transforms of length L >= 2^SMOL_TUNE_MIN_LOGL (E = 4 only where 64 lanes
// can hold a transform, N <= 256).  The kernels of each variant live in
// their own translation unit per phase (phases_a/b/c.hip).
#pragma once
#include <type_traits>

#include "host.h"

#define SMOL_NVAR 4
#define SMOL_TUNE_MIN_LOGL 12
// dynamic LDS a variant may ask for: gfx950 gives a workgroup up to 160 KiB,
// less a margin for the kernels' static shared arrays
#define SMOL_LDS_DYN_MAX (144 * 1024)

enum { PH_A = 0, PH_B = 1, PH_C = 2 };

struct PhaseDims {
    int units;      // workgroups (phase B: row pairs + the reduction finaliser)
    int threads;    // per workgroup
    int lds_bytes;  // dynamic LDS per workgroup
    int jobs;       // A: reduction partial rows; C: finish units (error partial rows)
};

// Call F::template run<N1, N2, T, E, W>(args...) for variant v of a kernel
// whose transforms have length N (N1 for phases A and C, N2 for phase B).
template <class F, int PH, int LOGL, int N1, int N2, class T, class... Args>
int run_variant(int v, Args &&...args)
{
    constexpr int N = PH == PH_B ? N2 : N1;
    constexpr int E0 = fft_default_e(N);
    constexpr bool tuned = std::is_same<T, cd>::value && LOGL >= SMOL_TUNE_MIN_LOGL;
    constexpr bool alt_e = tuned && fft_valid_e(N, 4) && E0 != 4;
    // float-float row-pair pass: the radix-4 form only (see ff_schedule)
    constexpr bool ff_b = std::is_same<T, cff>::value && PH == PH_B &&
                          LOGL >= SMOL_TUNE_MIN_LOGL && fft_valid_e(N, 4) && E0 != 4;
    switch (v) {
    case 0: return F::template run<N1, N2, T, E0, 4>(args...);
    case 1:
        if constexpr (tuned) return F::template run<N1, N2, T, E0, 8>(args...);
        return SMOL_EUNSUPPORTED;
    case 2:
        if constexpr (alt_e) return F::template run<N1, N2, T, 4, 4>(args...);
        return SMOL_EUNSUPPORTED;
    case 3:
        if constexpr (alt_e || ff_b) return F::template run<N1, N2, T, 4, 8>(args...);
        return SMOL_EUNSUPPORTED;
    default: return SMOL_EUNSUPPORTED;
    }
}

// Schedule of float-float plans (not tuned): the row-pair pass with radix-4
// butterflies (variant 3) where its rows allow it (N2 <= 256), which keeps
// its float-float registers from spilling; everything else variant 0.
inline void ff_schedule(int logL, int *v)
{
    v[0] = v[2] = 0;
    v[1] = (logL >= SMOL_TUNE_MIN_LOGL && (1 << split_log_n2(logL)) <= 256) ? 3 : 0;
}

template <class F, int PH, class... Args>
int with_variant(int logL, int precision, int v, Args &&...args)
{
    switch (logL) {
#define CASE(LL)                                                                        \
    case LL:                                                                            \
        return precision == SMOL_FP32X2                                                 \
                   ? run_variant<F, PH, LL, (1 << split_log_n1(LL)),                    \
                                 (1 << split_log_n2(LL)), cff>(v, args...)              \
                   : run_variant<F, PH, LL, (1 << split_log_n1(LL)),                    \
                                 (1 << split_log_n2(LL)), cd>(v, args...);
        CASE(6)
        CASE(7)
        CASE(8)
        CASE(9)
        CASE(10)
        CASE(11)
        CASE(12)
        CASE(13)
        CASE(14)
        CASE(15)
        CASE(16)
        CASE(17)
        CASE(18)
        CASE(19)
        CASE(20)
#undef CASE
    default: return SMOL_EUNSUPPORTED;
    }
}

// Grid and LDS of each phase's kernel for a variant (host only, no kernels).
struct DimsA {
    template <int N1, int N2, class T, int E, int W>
    static int run(int R, bool, PhaseDims *o)
    {
        using P = PhaseA<N1, N2, T, E, W>;
        *o = PhaseDims{P::units(R), P::NT, (int)sizeof(cd) * P::LDS, P::red_jobs()};
        return SMOL_OK;
    }
};
struct DimsB {
    template <int N1, int N2, class T, int E, int W>
    static int run(int, bool, PhaseDims *o)
    {
        using P = PhaseB<N1, N2, T, E, W>;
        *o = PhaseDims{P::units() + 1, P::NT, (int)sizeof(cd) * P::LDS, 0};
        return SMOL_OK;
    }
};
struct DimsC {
    template <int N1, int N2, class T, int E, int W>
    static int run(int, bool fuse, PhaseDims *o)
    {
        using P = PhaseC<N1, N2, T, E, W>;
        *o = PhaseDims{P::units(), P::NT, (int)sizeof(cd) * (fuse ? P::LDS_FUSE : P::LDS),
                       P::units()};
        return SMOL_OK;
    }
};

inline int phase_dims(int logL, int precision, int ph, int v, int R, bool fuse, PhaseDims *o)
{
    int rc;
    switch (ph) {
    case PH_A: rc = with_variant<DimsA, PH_A>(logL, precision, v, R, fuse, o); break;
    case PH_B: rc = with_variant<DimsB, PH_B>(logL, precision, v, R, fuse, o); break;
    case PH_C:
        // a C variant must also fit fused with the next column pass
        rc = with_variant<DimsC, PH_C>(logL, precision, v, R, true, o);
        if (!rc && o->lds_bytes > SMOL_LDS_DYN_MAX) return SMOL_EUNSUPPORTED;
        rc = with_variant<DimsC, PH_C>(logL, precision, v, R, fuse, o);
        break;
    default: return SMOL_EINVAL;
    }
    if (!rc && o->lds_bytes > SMOL_LDS_DYN_MAX) return SMOL_EUNSUPPORTED;
    return rc;
}

// Launchers (defined in phases_a.hip, phases_b.hip, phases_c.hip).  Each
// launches one kernel of the given variant on stream s; grids come from
// phase_dims.  rhs_*: the plain right-hand side; int_*: the integrator's
// stage kernels, which read their buffers from the device control block.
SMOL_HIDDEN int launch_rhs_A(int logL, int precision, int v, const RhsPlanDev &P, const Pro &in,
                             hipStream_t s);
SMOL_HIDDEN int launch_rhs_B(int logL, int precision, int v, const RhsPlanDev &P, int red_jobs,
                             hipStream_t s);
SMOL_HIDDEN int launch_rhs_C(int logL, int precision, int v, const RhsPlanDev &P, const Epi &ep,
                             hipStream_t s);
// cout non-null: the stage-2 pass that also takes the previous attempt's
// decision (njobs error rows) and stores the updated control block there.
SMOL_HIDDEN int launch_int_A(int logL, int precision, int v, const IntegDev &I, int stage,
                             int method, IntegCtl *cout, int njobs, hipStream_t s);
SMOL_HIDDEN int launch_int_B(int logL, int precision, int v, const IntegDev &I, int stage,
                             int jobs_a, int jobs_c, hipStream_t s);
SMOL_HIDDEN int launch_int_C(int logL, int precision, int v, bool fuse, const IntegDev &I,
                             int stage, int method, hipStream_t s);
// Batched stage kernels over blocks [base, base + count) of one shape.
SMOL_HIDDEN int launch_bat_A(int logL, int precision, int v, const BatchDev &B, int base,
                             int count, int stage, int method, hipStream_t s);
SMOL_HIDDEN int launch_bat_B(int logL, int precision, int v, const BatchDev &B, int base,
                             int count, int stage, hipStream_t s);
SMOL_HIDDEN int launch_bat_C(int logL, int precision, int v, const BatchDev &B, int base,
                             int count, int stage, bool fuse, int method, hipStream_t s);
// Launch schedule (variants of A, B, C) currently installed for 2^logL
// (float-float: variant 0); caller holds the library lock.
SMOL_HIDDEN void schedule_of(int logL, int precision, int *v);
