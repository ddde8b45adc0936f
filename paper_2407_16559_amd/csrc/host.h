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

// Call F::template run<N1, N2, T>(args...) for the transform shape of logL
// and the complex arithmetic of `precision` (cd: FP64, cff: float-float).
template <class F, class... Args>
int with_shape(int logL, int precision, Args &&...args)
{
    switch (logL) {
#define CASE(LL, A, B)                                                        \
    case LL:                                                                  \
        return precision == SMOL_FP32X2                                       \
                   ? F::template run<(1 << A), (1 << B), cff>(args...)        \
                   : F::template run<(1 << A), (1 << B), cd>(args...);
        CASE(6, 3, 3)
        CASE(7, 4, 3)
        CASE(8, 4, 4)
        CASE(9, 5, 4)
        CASE(10, 5, 5)
        CASE(11, 6, 5)
        CASE(12, 6, 6)
        CASE(13, 7, 6)
        CASE(14, 7, 7)
        CASE(15, 8, 7)
        CASE(16, 8, 8)
        CASE(17, 9, 8)
        CASE(18, 9, 9)
        CASE(19, 10, 9)
        CASE(20, 10, 10)
#undef CASE
    default: return SMOL_EUNSUPPORTED;
    }
}

// Workgroups of the three kernels of one right-hand side for a shape.
struct ShapeUnits {
    template <int N1, int N2, class T>
    static int run(int R, int *out)
    {
        out[0] = PhaseA<N1, N2, T>::units(R);
        out[1] = PhaseB<N1, N2, T>::units() + 1;  // + the reduction finaliser
        out[2] = PhaseC<N1, N2, T>::units();
        out[3] = PhaseA<N1, N2, T>::red_jobs();
        out[4] = PhaseA<N1, N2, T>::LDS;  // dynamic LDS entries of each kernel
        out[5] = PhaseB<N1, N2, T>::LDS;
        out[6] = PhaseC<N1, N2, T>::LDS;
        out[7] = PhaseC<N1, N2, T>::LDS_FUSE;
        return SMOL_OK;
    }
};
