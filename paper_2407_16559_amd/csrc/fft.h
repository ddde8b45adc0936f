// Wavefront-level Stockham FFT for lengths N = 2^3 .. 2^10.
//
// One transform of length N is owned by G = N/E lanes of a single wave64,
// each lane holding E complex values in registers (E = 8, or 16 for
// N = 1024); a wave runs B = 64/G transforms side by side.  The complex type
// C is cd (FP64) or cff (float-float); the code is the same for both.  Radix-E
// butterflies run in registers; the exchanges between stages go through a
// per-transform LDS region of N entries, ordered by wave_sync() only (no
// workgroup barrier).  Stockham's self-sorting form keeps both the input and
// the output in natural order with the same register layout:
//     lane g (0 <= g < G) register i holds element g + i*G.
// so the first stage reads registers loaded straight from global memory and
// the last stage leaves the spectrum in registers for a direct store.
#pragma once
#include "common.h"
#include "ff.h"

// conversions from FP64 complex values (unit roots, inputs)
template <class C>
__device__ __forceinline__ C from_cd(cd v);
template <>
__device__ __forceinline__ cd from_cd<cd>(cd v)
{
    return v;
}
template <>
__device__ __forceinline__ cff from_cd<cff>(cd v)
{
    return cff{ff_from(v.x), ff_from(v.y)};
}
template <class C>
__device__ __forceinline__ C czero()
{
    return from_cd<C>(cd{0.0, 0.0});
}
__device__ __forceinline__ double re_d(cd v) { return v.x; }
__device__ __forceinline__ double im_d(cd v) { return v.y; }
__device__ __forceinline__ double re_d(cff v) { return ff_to(v.x); }
__device__ __forceinline__ double im_d(cff v) { return ff_to(v.y); }

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// Elements per lane: the radix of the in-register butterflies.  8 by
// default (16 at N = 1024, where a transform must fit one wave); 4 and 16
// are the alternatives a schedule may pick (G = N/E lanes must fit a wave).
constexpr int fft_default_e(int N) { return N == 1024 ? 16 : 8; }
constexpr bool fft_valid_e(int N, int E)
{
    return (E == 4 || E == 8 || E == 16) && E <= N && N / E <= 64;
}

template <int N, int E_ = fft_default_e(N)>
struct FftShape {
    static_assert(N >= 8 && N <= 1024 && (N & (N - 1)) == 0, "FFT length");
    static_assert(fft_valid_e(N, E_), "elements per lane");
    static constexpr int LOGN = ilog2c(N);
    static constexpr int E = E_;                    // elements per lane
    static constexpr int G = N / E;                 // lanes per transform
    static constexpr int B = 64 / G;                // transforms per wave
    static constexpr int LOGE = ilog2c(E);
    // stage radices: E repeated, then one smaller radix for the remainder
    static constexpr int NFULL = LOGN / LOGE;
    static constexpr int REM = LOGN % LOGE;
    static constexpr int NST = NFULL + (REM ? 1 : 0);
    static constexpr int radix(int st) { return st < NFULL ? E : (1 << REM); }
    static constexpr int log_span(int st) { return st < NFULL ? st * LOGE : NFULL * LOGE; }
};

// ---------------------------------------------------------------------
// In-register DFTs of length 2, 4, 8, 16 (radix-2 decimation in time).
// ---------------------------------------------------------------------

// cos / sin of 2 pi m / 16, m = 0..7
__device__ __forceinline__ double c16(int m)
{
    switch (m) {
    case 0: return 1.0;
    case 1: return 0.92387953251128675613;
    case 2: return 0.70710678118654752440;
    case 3: return 0.38268343236508977173;
    case 4: return 0.0;
    case 5: return -0.38268343236508977173;
    case 6: return -0.70710678118654752440;
    default: return -0.92387953251128675613;
    }
}
// sin(2 pi m / 16) = cos(2 pi (m - 4) / 16)
__device__ __forceinline__ double s16(int m) { return c16(m <= 4 ? 4 - m : m - 4); }

// multiply by W_R^k (forward: exp(-2 pi i k / R)), k < R/2, R | 16
template <int R, bool INV, class C>
__device__ __forceinline__ C twiddle_const(C a, int k)
{
    const int m = k * (16 / R);  // angle 2 pi m / 16, 0 <= m < 8
    if (m == 0) return a;
    if (m == 4) return crot<INV>(a);
    const double c = c16(m);
    const double s = INV ? s16(m) : -s16(m);  // forward uses exp(-i theta)
    if constexpr (__is_same(C, cd)) {
        return cd{fma(a.x, c, -a.y * s), fma(a.x, s, a.y * c)};
    } else {
        return cmul(a, from_cd<C>(cd{c, s}));
    }
}

template <int R, bool INV, class C>
struct Dft {
    __device__ __forceinline__ static void run(C (&v)[R])
    {
        C e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<R / 2, INV, C>::run(e);
        Dft<R / 2, INV, C>::run(o);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            C t = twiddle_const<R, INV>(o[k], k);
            v[k] = cadd(e[k], t);
            v[k + R / 2] = csub(e[k], t);
        }
    }
};
template <bool INV, class C>
struct Dft<2, INV, C> {
    __device__ __forceinline__ static void run(C (&v)[2])
    {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <bool INV, class C>
struct Dft<1, INV, C> {
    __device__ __forceinline__ static void run(C (&)[1]) {}
};

// ---------------------------------------------------------------------
// Stockham stages.
// ---------------------------------------------------------------------

// w^q for q = 0..R-1 by a multiplication tree of depth <= 4 (a few ulps).
template <int R, class C>
__device__ __forceinline__ void pow_tree(C w, C (&o)[R])
{
    o[0] = from_cd<C>(cd{1.0, 0.0});
    if constexpr (R > 1) o[1] = w;
    if constexpr (R > 2) o[2] = cmul(w, w);
    if constexpr (R > 3) o[3] = cmul(o[2], w);
    if constexpr (R > 4) {
        o[4] = cmul(o[2], o[2]);
        o[5] = cmul(o[4], w);
        o[6] = cmul(o[4], o[2]);
        o[7] = cmul(o[4], o[3]);
    }
    if constexpr (R > 8) {
        o[8] = cmul(o[4], o[4]);
#pragma unroll
        for (int q = 9; q < R; ++q) o[q] = cmul(o[8], o[q - 8]);
    }
}

// Per-lane base twiddles of every stage after the first, W_{Ns r}^k with
// k = j mod Ns, loaded once before the data arrives (split into float-float
// from the FP64 table when C = cff).
template <int N, bool INV, class C, int E = fft_default_e(N)>
struct FftTw {
    using S = FftShape<N, E>;
    static constexpr int PMAX = (S::E / 2 > 0) ? S::E / 2 : 1;
    C w[S::NST > 1 ? S::NST - 1 : 1][PMAX];

    __device__ __forceinline__ void load(int g, const Roots &rt) { load_st<1>(g, rt); }
    template <int ST>
    __device__ __forceinline__ void load_st(int g, const Roots &rt)
    {
        if constexpr (ST < S::NST) {
            constexpr int r = S::radix(ST);
            constexpr int LR = ilog2c(r);
            constexpr int P = S::E / r;
            constexpr int LNS = S::log_span(ST);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int k = (g + p * S::G) & ((1 << LNS) - 1);
                w[ST - 1][p] = from_cd<C>(root_small<INV>(rt, LNS + LR, k));
            }
            load_st<ST + 1>(g, rt);
        }
    }
};

template <int N, bool INV, int ST, class C, int E = fft_default_e(N)>
struct FftStage {
    using S = FftShape<N, E>;
    __device__ __forceinline__ static void run(C (&v)[S::E], C *buf, int g,
                                               const FftTw<N, INV, C, E> &tw)
    {
        constexpr int r = S::radix(ST);
        constexpr int LR = ilog2c(r);
        constexpr int P = S::E / r;          // butterflies per lane
        constexpr int LNS = S::log_span(ST); // log2 of the span Ns
        constexpr int Ns = 1 << LNS;
        constexpr int Nr = N / r;
        if constexpr (ST > 0) {
            wave_sync();
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int q = 0; q < r; ++q) v[p + q * P] = buf[g + p * S::G + q * Nr];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            C t[r];
#pragma unroll
            for (int q = 0; q < r; ++q) t[q] = v[p + q * P];
            if constexpr (Ns > 1) {
                C wq[r];
                pow_tree<r>(tw.w[ST - 1][p], wq);
#pragma unroll
                for (int q = 1; q < r; ++q) t[q] = cmul(t[q], wq[q]);
            }
            Dft<r, INV, C>::run(t);
#pragma unroll
            for (int q = 0; q < r; ++q) v[p + q * P] = t[q];
        }
        if constexpr (ST + 1 < S::NST) {
            wave_sync();
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int j = g + p * S::G;
                const int k = j & (Ns - 1);
                const int base = ((j >> LNS) << (LNS + LR)) + k;
#pragma unroll
                for (int q = 0; q < r; ++q) buf[base + q * Ns] = v[p + q * P];
            }
            FftStage<N, INV, ST + 1, C, E>::run(v, buf, g, tw);
        }
    }
};

// Transform the N values held by lanes g = 0..G-1 (layout above) in place.
// buf: this transform's LDS region (N entries); tw: loaded base twiddles.
template <int N, bool INV, class C, int E>
__device__ __forceinline__ void wave_fft(C (&v)[E], C *buf, int g, const FftTw<N, INV, C, E> &tw)
{
    FftStage<N, INV, 0, C, E>::run(v, buf, g, tw);
}

// Lane's four-step twiddles W_L^{e (g + i G)}, i = 0..E-1, from two table
// lookups (base W_L^{e g} and step W_L^{e G}) and a power tree.
template <int E, bool INV, class C>
__device__ __forceinline__ void step_twiddles(const Roots &rt, int logL, uint32_t e, int g, int G,
                                              C (&o)[E])
{
    const C base = from_cd<C>(root_big<INV>(rt, logL, e * (uint32_t)g));
    const C step = from_cd<C>(root_big<INV>(rt, logL, e * (uint32_t)G));
    pow_tree<E>(step, o);
#pragma unroll
    for (int i = 0; i < E; ++i) o[i] = cmul(base, o[i]);
}
