// Column-pass kernels (phase A) of every shape and schedule variant.
#include "kernels.h"

SMOL_HIDDEN int launch_rhs_A(int logL, int precision, int v, const RhsPlanDev &P, const Pro &in,
                             hipStream_t s)
{
    return with_variant<RhsA, PH_A>(logL, precision, v, P, in, s);
}

SMOL_HIDDEN int launch_int_A(int logL, int precision, int v, const IntegDev &I, int stage,
                             int method, IntegCtl *cout, int njobs, hipStream_t s)
{
    return with_variant<IntA, PH_A>(logL, precision, v, I, stage, method, cout, njobs, s);
}

SMOL_HIDDEN int launch_bat_A(int logL, int precision, int v, const BatchDev &B, int base, int count,
                             int stage, int method, hipStream_t s)
{
    return with_variant<BatA, PH_A>(logL, precision, v, B, base, count, stage, method, s);
}
