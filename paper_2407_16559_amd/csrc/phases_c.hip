// Inverse-column-pass + finish kernels (phase C) of every shape and schedule
// variant, plain and fused with the next stage's column pass.
#include "kernels.h"

SMOL_HIDDEN int launch_rhs_C(int logL, int precision, int v, const RhsPlanDev &P, const Epi &ep,
                             hipStream_t s)
{
    return with_variant<RhsC, PH_C>(logL, precision, v, P, ep, s);
}

SMOL_HIDDEN int launch_int_C(int logL, int precision, int v, bool fuse, const IntegDev &I,
                             int stage, int method, hipStream_t s)
{
    return with_variant<IntC, PH_C>(logL, precision, v, I, stage, fuse, method, s);
}

SMOL_HIDDEN int launch_bat_C(int logL, int precision, int v, const BatchDev &B, int base, int count,
                             int stage, bool fuse, int method, hipStream_t s)
{
    return with_variant<BatC, PH_C>(logL, precision, v, B, base, count, stage, fuse, method, s);
}
