// Shared device helpers: complex arithmetic, unit-root tables, wave sync.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SMOL_WG 256            // threads per workgroup (4 wave64)
#define SMOL_WAVES (SMOL_WG / 64)
#define SMOL_NUM_CU 256        // compute units of an MI355X (8 XCDs x 32)
#define SMOL_MAX_R 32
#define SMOL_LOG_TW 10         // unit-root tables have 2^10 entries
#define SMOL_TW (1 << SMOL_LOG_TW)
#define SMOL_LOG_LMAX 20       // longest convolution transform: 2^20

// Four-step split of a transform of length L = 2^logL into N1 x N2: log2 of
// the column length N1 (the rest, N2 = L / N1, is the row length).
__host__ __device__ constexpr int split_log_n1(int logL) { return (logL + 1) / 2; }
__host__ __device__ constexpr int split_log_n2(int logL) { return logL - split_log_n1(logL); }

struct __align__(16) cd {
    double x, y;
};

__device__ __forceinline__ cd cmk(double x, double y) { return cd{x, y}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd cmul(cd a, cd b)
{
    return cd{fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
__device__ __forceinline__ cd cmulc(cd a, cd b)
{
    return cd{fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y)};
}
__device__ __forceinline__ cd cconj(cd a) { return cd{a.x, -a.y}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ cd crot(cd a)
{
    return INV ? cd{-a.y, a.x} : cd{a.y, -a.x};
}

// Unit roots.  tw[e] = exp(-2 pi i e / 2^10) and fine[e] = exp(-2 pi i e / 2^20),
// e < 2^10, both computed on the host in extended precision and rounded.
struct Roots {
    const cd *tw;    // W_1024^e
    const cd *fine;  // W_{2^20}^e
};

// W_N^e (or its conjugate) for N = 2^logN <= 1024, 0 <= e < N.
template <bool INV>
__device__ __forceinline__ cd root_small(const Roots &rt, int logN, int e)
{
    cd w = rt.tw[e << (SMOL_LOG_TW - logN)];
    return INV ? cconj(w) : w;
}

// W_L^e (or conjugate) for L = 2^logL <= 2^20, any e >= 0, via
// W_{2^20}^E = W_1024^(E >> 10) * W_{2^20}^(E & 1023).
template <bool INV>
__device__ __forceinline__ cd root_big(const Roots &rt, int logL, uint32_t e)
{
    uint32_t E = (e << (SMOL_LOG_LMAX - logL)) & ((1u << SMOL_LOG_LMAX) - 1u);
    cd w = cmul(rt.tw[E >> SMOL_LOG_TW], rt.fine[E & (SMOL_TW - 1)]);
    return INV ? cconj(w) : w;
}

// Order LDS traffic of one wavefront: its lanes run in lockstep and its LDS
// operations complete in issue order, so a compiler-level fence suffices.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Map workgroup b to a logical index so that consecutive logical indices land
// on the same XCD (workgroups are dealt round-robin over the 8 XCDs, each with
// its own L2): the first nb - nb % 8 workgroups are remapped, the rest kept.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int full = nb & ~7;
    if (b >= full) return b;
    return (b % 8) * (full / 8) + b / 8;
}
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

// Lane exchanges of a double without LDS traffic: ds_swizzle in bit mode
// (lane i reads lane ((i & 31) ^ X) of its 32-lane half; pattern 0x1F | X << 10)
// and DPP quad permutations (CTRL = quad_perm code).
template <int PAT>
__device__ __forceinline__ double swizzle_d(double v)
{
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), PAT);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), PAT);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Deterministic wave-wide sum: the xor butterfly over lane offsets 32, 16,
// 8, 4, 2, 1 (each lane adds its partner's value to its own).  Offset 32
// goes through a lane permute, 16..4 through ds_swizzle, 2 and 1 through
// DPP quad permutations [2,3,0,1] and [1,0,3,2].
__device__ __forceinline__ double wave_sum(double v)
{
    v += __shfl_xor(v, 32, 64);
    v += swizzle_d<0x1F | (16 << 10)>(v);
    v += swizzle_d<0x1F | (8 << 10)>(v);
    v += swizzle_d<0x1F | (4 << 10)>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0xB1>(v);
    return v;
}
