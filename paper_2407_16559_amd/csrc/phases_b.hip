// Row-pair kernels (phase B) of every shape and schedule variant.
#include "kernels.h"

SMOL_HIDDEN int launch_rhs_B(int logL, int precision, int v, const RhsPlanDev &P, int red_jobs,
                             hipStream_t s)
{
    return with_variant<RhsB, PH_B>(logL, precision, v, P, red_jobs, s);
}

SMOL_HIDDEN int launch_int_B(int logL, int precision, int v, const IntegDev &I, int stage,
                             int jobs_a, int jobs_c, hipStream_t s)
{
    return with_variant<IntB, PH_B>(logL, precision, v, I, stage, jobs_a, jobs_c, s);
}

SMOL_HIDDEN int launch_bat_B(int logL, int precision, int v, const BatchDev &B, int base, int count,
                             int stage, hipStream_t s)
{
    return with_variant<BatB, PH_B>(logL, precision, v, B, base, count, stage, s);
}
