// Host-side helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "../../include/smol.h"
#include "integrate.h"

#define SMOL_HIDDEN __attribute__((visibility("hidden")))
#define SMOL_GRAPH_ATTEMPTS 4  // step attempts captured per graph

inline int hip_fail(hipError_t e, const char *what)
{
    if (getenv("SMOL_DEBUG")) fprintf(stderr, "libsmol: %s: %s\n", what, hipGetErrorString(e));
    return SMOL_EDEVICE;
}
#define HIP_TRY(x)                                     \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #x); \
    } while (0)

struct DevRoots {
    cd *tw = nullptr, *fine = nullptr;
};

inline int ilog2_ceil(int64_t x)
{
    int l = 0;
    while ((1LL << l) < x) ++l;
    return l;
}

// log2 of the convolution transform length for M sizes
inline int fft_log2(int64_t M)
{
    const int l = ilog2_ceil(2 * M - 2);
    return l < 6 ? 6 : l;
}

// serialises plan / table creation and use across host threads
extern SMOL_HIDDEN std::mutex g_mu;
SMOL_HIDDEN int get_roots(int dev, DevRoots **out);
SMOL_HIDDEN void stats_from(const IntegCtl &c, smol_stats *st);
SMOL_HIDDEN const float *proposer_weights(int dev);  // null until smol_proposer_set
SMOL_HIDDEN int check_common(int64_t M, int32_t R, const double *U, const double *V, double lambda);

// layout conversion kernels (defined in smol.hip)
__global__ void k_to_tr(const double *src, double *dst, int64_t M, int rows, int64_t sstride,
                        int64_t dstride, int logL);
__global__ void k_from_tr(const double *src, double *dst, int64_t M, int logL);
