// Host-side helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "../../include/smol.h"
#include "integrate.h"

#define SMOL_HIDDEN __attribute__((visibility("hidden")))
#define SMOL_GRAPH_ATTEMPTS 16  // step attempts captured per graph
static_assert(SMOL_GRAPH_ATTEMPTS >= 1 && SMOL_GRAPH_ATTEMPTS <= 64, "graph size");

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

// Stages (with the stage evaluated at the new state) and error-estimate
// order q of each scheme, indexed by SMOL_BS32 .. SMOL_RK4_DBL.
static const int k_scheme_stages[5] = {4, 7, 7, 6, 12};
static const int k_scheme_q[5] = {2, 4, 4, 2, 4};
// Stage slot that alternates with slot 0 as the first stage (the fsal field
// of each scheme's tableau in integrate.h).
static const int k_scheme_fsal[5] = {3, 6, 6, 5, 5};

// SMOL_OK for a known scheme, SMOL_EINVAL otherwise.
inline int check_method(int32_t method)
{
    return (method >= SMOL_BS32 && method <= SMOL_RK4_DBL) ? SMOL_OK : SMOL_EINVAL;
}
inline bool controller_valid(int32_t c) { return c >= SMOL_CTRL_PI && c <= SMOL_CTRL_HALVE_DOUBLE; }

// Control-block settings shared by single and batched runs: tolerances,
// controller constants and the paper rules' Euclidean norm (sc = tol = rtol).
inline void ctl_setup(IntegCtl &c, int32_t method, const smol_options &o, double rtol, double atol)
{
    const int k = k_scheme_q[method] + 1;
    c.rtol = rtol;
    c.atol = atol;
    if (o.alpha > 0) {
        c.alpha = o.alpha;
        c.beta = o.beta;
    } else {
        c.alpha = 0.7 / k;
        c.beta = 0.4 / k;
    }
    c.safety = 0.9;
    c.facmin = 0.2;
    c.facmax = 10.0;
    c.method = method;
    c.controller = o.controller;
    c.err_prev = 1.0;
    if (o.controller >= SMOL_CTRL_FEHLBERG) {
        c.l2 = 1;
        c.rtol = 0.0;
        c.atol = rtol;
        c.paper_s = o.safety > 0 ? o.safety : 0.25;
    }
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
