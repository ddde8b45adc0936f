// smol_rhs_noalloc: the FP64 right-hand side with every workspace in one
// fixed device array of this library, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Same three phase kernels, launch
// schedule and arithmetic as smol_rhs; only the workspaces differ.
#include <hip/hip_runtime.h>

#include "sched.h"

// Largest request served: transforms up to 2^17 (M <= 2^16 + 1) and rank 4.
#define NA_LOGL_MAX 17
#define NA_RMAX 4
#define NA_MAX_DEV 64

namespace {
constexpr size_t NA_L = size_t(1) << NA_LOGL_MAX;
constexpr size_t NA_N2 = size_t(1) << split_log_n2(NA_LOGL_MAX);
// layout in 16-byte entries: unit roots | spectra Z | packed inverse input Qp
// | reduction partials and totals (doubles)
constexpr size_t NA_OFF_Z = 2 * SMOL_TW;
constexpr size_t NA_OFF_QP = NA_OFF_Z + NA_RMAX * NA_L;
constexpr size_t NA_OFF_RED = NA_OFF_QP + NA_L / 2;
constexpr size_t NA_RED_DOUBLES = NA_N2 * NA_RMAX * 4 + NA_RMAX * 4;
constexpr size_t NA_BYTES = 16 * NA_OFF_RED + 8 * NA_RED_DOUBLES;
}  // namespace

// The workspaces (about 9.1 MiB).  Host code never uses this name as an
// address: it takes the device address from hipGetSymbolAddress once per
// device and passes that to the kernels.
static __device__ __align__(256) double scratch[NA_BYTES / 8];

// Unit-root tables W_1024^e and W_{2^20}^e, e < 1024, in FP64 (sincospi takes
// the angle as a multiple of pi, so the argument e / 512 or e / 2^19 is exact).
__global__ void k_noalloc_roots(cd *tw)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= SMOL_TW) return;
    double s, c;
    sincospi((double)e / (double)(SMOL_TW / 2), &s, &c);
    tw[e] = cd{c, -s};
    sincospi((double)e / (double)(1 << (SMOL_LOG_LMAX - 1)), &s, &c);
    tw[SMOL_TW + e] = cd{c, -s};
}

namespace {
void *g_na_ptr[NA_MAX_DEV];    // device address of `scratch` per device
bool g_na_roots[NA_MAX_DEV];   // unit roots written by an eager (uncaptured) launch

// Set-up on the first call on a device (that device current): the array's
// device address, checked.
int na_setup(int dev, void **out)
{
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_na_ptr[dev] = p;
    }
    *out = g_na_ptr[dev];
    return SMOL_OK;
}
}  // namespace

extern "C" int smol_rhs_noalloc(int64_t M, int32_t R, const double *U, const double *V,
                                double lambda, const double *n, double *dndt, void *stream)
{
    int rc = check_common(M, R, U, V, lambda);
    if (rc) return rc;
    if (!n || !dndt || n == dndt) return SMOL_EINVAL;
    const int logL = fft_log2(M);
    if (logL > NA_LOGL_MAX || R > NA_RMAX) return SMOL_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NA_MAX_DEV) return SMOL_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    void *base;
    if ((rc = na_setup(dev, &base))) return rc;
    cd *ws = (cd *)base;
    if (!g_na_roots[dev]) {
        // under capture the root kernel becomes part of the caller's graph, so
        // it is launched again on the next eager call
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(s, &cs));
        hipLaunchKernelGGL(k_noalloc_roots, dim3(SMOL_TW / 256), dim3(256), 0, s, ws);
        HIP_TRY(hipGetLastError());
        if (cs == hipStreamCaptureStatusNone) g_na_roots[dev] = true;
    }
    int v[3];
    schedule_of(logL, SMOL_FP64, v);
    PhaseDims dA;
    if ((rc = phase_dims(logL, SMOL_FP64, PH_A, v[0], R, false, &dA))) return rc;
    RhsPlanDev P;
    P.M = M;
    P.R = R;
    P.logL = logL;
    P.logN1 = split_log_n1(logL);
    P.logN2 = split_log_n2(logL);
    P.tr = 0;
    P.ustride = M;
    P.lam = lambda;
    P.U = U;
    P.V = V;
    P.Z = ws + NA_OFF_Z;
    P.Qp = ws + NA_OFF_QP;
    P.red_part = (double *)(ws + NA_OFF_RED);
    P.red = P.red_part + (size_t)dA.jobs * R * 4;
    P.src = nullptr;
    P.rt.tw = ws;
    P.rt.fine = ws + SMOL_TW;
    Pro in{A_COMBINE, n, nullptr, 0.0, nullptr};
    Epi ep{};
    ep.mode = C_RHS;
    ep.y = n;
    ep.out = dndt;
    if ((rc = launch_rhs_A(logL, SMOL_FP64, v[0], P, in, s))) return rc;
    if ((rc = launch_rhs_B(logL, SMOL_FP64, v[1], P, dA.jobs, s))) return rc;
    if ((rc = launch_rhs_C(logL, SMOL_FP64, v[2], P, ep, s))) return rc;
    HIP_TRY(hipGetLastError());
    return SMOL_OK;
}
