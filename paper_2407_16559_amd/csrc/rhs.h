// The O(M R log M) right-hand side of the truncated aggregation-shattering
// system (Sec. 1, Eq. (2) and Eq. (4); Sec. 2, Eq. (5)).
//
// Birth: with a_al[i] = U_{i al} y_i and b_al[j] = V_{al j} y_j (sizes 1..M-1
// at indices 0..M-2), (1/2) sum_{i+j=s} K_ij y_i y_j = (1/2) sum_al c_al[s-2]
// where c_al is the linear convolution a_al * b_al.  All R convolutions are
// summed in the frequency domain: z_al = a_al + i b_al is transformed with
// one complex FFT of length L >= 2M-2 (no wrap-around for the outputs used),
// A = (Z_k + conj Z_{L-k})/2, B = (Z_k - conj Z_{L-k})/(2i), so
//     P_k = sum_al A_al B_al = sum_al (Z_al,k^2 - conj(Z_al,L-k)^2) / (4i)
// and c = sum_al c_al = IDFT_L(P), which is real.
//
// Death and shattering: four reductions per rank,
//     w_al = sum_{j>=1} V_{al j} y_j,  t_al = sum_{j>=2} j V_{al j} y_j,
//     r_al = sum_{i>=2} U_{i al} y_i,  p_al = sum_{i>=2} i U_{i al} y_i,
// give sum_i K_si y_i = sum_al U_{s al} w_al and, with q_al = w_al - V_{al 1} y_1,
//     S_1 = -y_1 sum_al U_{1 al} w_al + (lam/2) sum_al (p_al q_al + r_al t_al)
//           + lam y_1 sum_al U_{1 al} t_al,
//     S_s = (1/2) c[s-2] - (1 + lam) y_s sum_al U_{s al} w_al,  s >= 2.
//
// FFT of length L = N1 * N2 in four steps (index n = N2 n1 + n2, frequency
// k = k1 + N1 k2), run as three phases separated by grid-wide barriers:
//   A  column pass: per column n2, DFT over n1 (length N1; rows n1 >= N1/2
//      are zero padding), times W_L^{n2 k1}; stored column by column
//      (Z[n2][k1]: one contiguous run per column; phase B reads its rows
//      with stride N1, neighbouring row pairs sharing cache lines).
//   B  per row pair {k1, N1-k1}: DFT over n2 (length N2) of every rank's two
//      rows, the spectral product P (rows k1 and N1-k1 hold k and L-k), then
//      the inverse DFT over k2 times W_L^{-a k1}, with columns a and a+N2/2
//      packed into one complex value (c is real).
//   C  per packed column: inverse DFT over k1 (length N1) gives
//      L (c[a + N2 b] + i c[a + N2/2 + N2 b]); the finish computes S and the
//      caller's fused epilogue (stage state, error norm, ...), spread over
//      the whole workgroup (or over two workgroups, one per real column).
//
// Layouts of the per-size vectors (state, stages, U, V): natural (size s at
// index s-1) or transposed, where index idx = N2 n1 + n2 < L/2 lives at
// n2 (N1/2) + n1 and idx = L/2 (only when M - 1 = L/2) at L/2.  In the
// transposed layout every column pass reads, and every finish writes,
// contiguous runs; the integrator keeps its vectors that way.
#pragma once
#include "fft.h"

// A call of one of a phase's large member functions.  The float-float bodies
// are beyond the inliner's size limit, and an out-of-line call passes the
// tile state through the stack (scratch memory), so for that type the call is
// forced inline; FP64 calls are left to the inliner, which inlines them.
#define SMOL_PHASE_CALL(C, ...)                  \
    do {                                         \
        if constexpr (__is_same(C, cff)) {       \
            [[clang::always_inline]] __VA_ARGS__; \
        } else {                                 \
            __VA_ARGS__;                         \
        }                                        \
    } while (0)

enum { A_GIVEN = 0, A_COMBINE = 1 };
enum { C_RHS = 0, C_STAGE = 1, C_LAST = 2, C_INIT0 = 3, C_INIT1 = 4 };
#define SMOL_MAX_STAGE 8
#define SMOL_EPART 8   // doubles per error/moment partial row

struct RhsPlanDev {
    int64_t M;
    int R;
    int logL, logN1, logN2;
    int tr;               // 1: transposed vector layout
    int64_t ustride;      // distance between the rank rows of U and V
    double lam;
    const double *U, *V;  // alpha-major, rows of ustride
    void *Z;              // R * L complex (cd or cff)
    void *Qp;             // L / 2 complex
    double *red_part;     // [jobs][R][4]
    double *red;          // [R][4]: w, t, r, p
    const double *src;    // constant sources P_s of Eq. (3) (plan layout) or null
    Roots rt;
};

// position of size index idx (0-based) in the transposed layout
__host__ __device__ __forceinline__ int64_t pos_tr(int64_t idx, int logL)
{
    const int logN1 = split_log_n1(logL), logN2 = split_log_n2(logL);
    const int64_t half = 1LL << (logL - 1);
    if (idx >= half) return half;
    return ((idx & ((1LL << logN2) - 1)) << (logN1 - 1)) + (idx >> logN2);
}

// position of size index idx (0-based) in a vector of the plan's layout
__device__ __forceinline__ int64_t pos_of(const RhsPlanDev &P, int64_t idx)
{
    return P.tr ? pos_tr(idx, P.logL) : idx;
}

// Phase-A input: y = base + c * kc (A_COMBINE) or y given (A_GIVEN).
struct Pro {
    int mode;
    const double *y;   // A_GIVEN: y; A_COMBINE: base
    const double *kc;  // may be null when c == 0
    double c;
    double *ywrite;    // A_COMBINE: y is written here when non-null
};

// Phase-C epilogue.
struct Epi {
    int mode;
    const double *y;        // the stage's y (death term)
    double *out;            // S is written here (k_i or dndt)
    const double *n;        // current state (stage modes) or n0 (init modes)
    const double *ks[SMOL_MAX_STAGE];
    double coef[SMOL_MAX_STAGE];
    int nks;                // previous stage vectors used
    double cS;              // coefficient of this S
    double h;
    double *ynext;          // C_STAGE: next stage state
    double rtol, atol;
    double *epart;          // C_LAST / C_INIT*: [jobs][SMOL_EPART]
    // C_STAGE with ocomb: out receives oS S + sum_j ocoef[j] ks[j] instead of S
    int ocomb;
    double oS;
    double ocoef[SMOL_MAX_STAGE];
    int diff;               // C_LAST: the error estimate also adds y - n
};

// Sum per-wave values sh[w][0..nq) over the W waves in order (after a barrier).
template <int W = SMOL_WAVES>
__device__ __forceinline__ double sum_waves(const double *sh, int nq, int q)
{
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) a += sh[w * nq + q];
    return a;
}

// acc + a^2 - conj(b)^2 (one rank's term of the spectral product, times 4i)
__device__ __forceinline__ cd spec_term(cd acc, cd a, cd b)
{
    const double re = (a.x * a.x - a.y * a.y) - (b.x * b.x - b.y * b.y);
    const double im = 2.0 * (a.x * a.y + b.x * b.y);
    return cd{acc.x + re, acc.y + im};
}
__device__ __forceinline__ cff spec_term(cff acc, cff a, cff b)
{
    const cff bc = cconj(b);
    return cadd(acc, csub(cmul(a, a), cmul(bc, bc)));
}
// x / (4i) = (x.y, -x.x) / 4 (exact)
__device__ __forceinline__ cd div4i(cd x) { return cd{0.25 * x.y, -0.25 * x.x}; }
__device__ __forceinline__ cff div4i(cff x) { return cff{ff_scale2(x.y, 0.25f), ff_scale2(ff_neg(x.x), 0.25f)}; }

// --------------------------------------------------------------------------
// Phase A
// --------------------------------------------------------------------------

// E: elements per lane of the column transforms; W: waves per workgroup.
template <int N1, int N2, class C, int E = fft_default_e(N1), int W = SMOL_WAVES>
struct PhaseA {
    using F = FftShape<N1, E>;
    static constexpr int NT = 64 * W;                                // threads
    static constexpr int COLS = (F::B < N2) ? F::B : N2;             // per wave
    static constexpr int GA = (W * COLS < N2) ? W * COLS : N2;       // per unit
    static constexpr int WUSED = GA / COLS;
    static constexpr int NG = N2 / GA;                                // column groups
    static constexpr int LDS = W * 64 * F::E;                         // entries
    static __host__ __device__ int units(int R) { return R * NG; }
    static __host__ __device__ int red_jobs() { return NG; }

    static constexpr int H = F::E / 2;
    // Loads that need only the transform shape and the factors: twiddles and
    // this lane's U, V values (the integrator issues them before its
    // control-block load).
    struct Early {
        FftTw<N1, false, C, E> tw;
        C t4[F::E];
        double u0[H], x0[H];
    };
    __device__ static void early(const RhsPlanDev &P, int unit, Early &e)
    {
        const int lane = lane_id(), w = wave_id();
        const int f = lane / F::G, g = lane % F::G;
        const int al = unit / NG, grp = unit % NG;
        const int n2 = grp * GA + w * COLS + f;
        const bool active = (w < WUSED) && (f < COLS);
        const double *Ua = P.U + (int64_t)al * P.ustride, *Va = P.V + (int64_t)al * P.ustride;
        if (active) {
            e.tw.load(g, P.rt);
            step_twiddles<F::E, false>(P.rt, P.logL, (uint32_t)n2, g, F::G, e.t4);
        }
#pragma unroll
        for (int i = 0; i < H; ++i) {
            e.u0[i] = e.x0[i] = 0.0;
            const int64_t idx = (int64_t)(g + i * F::G) * N2 + n2;
            if (active && idx < P.M) {
                const int64_t q = pos_of(P, idx);
                e.u0[i] = Ua[q];
                e.x0[i] = Va[q];
            }
        }
    }

    // one unit = (rank al, group of GA columns); whole workgroup
    __device__ static void run(const RhsPlanDev &P, const Pro &in, int unit, C *lds)
    {
        Early e;
        early(P, unit, e);
        SMOL_PHASE_CALL(C, run_with(P, in, unit, lds, e));
    }

    __device__ static void run_with(const RhsPlanDev &P, const Pro &in, int unit, C *lds, Early &e)
    {
        __shared__ double sh[W * 4];
        const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
        const int f = lane / F::G, g = lane % F::G;
        const int al = unit / NG, grp = unit % NG;
        const int n2 = grp * GA + w * COLS + f;
        const bool active = (w < WUSED) && (f < COLS);
        const int64_t M = P.M;
        const double *Ua = P.U + (int64_t)al * P.ustride, *Va = P.V + (int64_t)al * P.ustride;
        const FftTw<N1, false, C, E> &tw = e.tw;
        const C(&t4)[F::E] = e.t4;
        const double(&u0)[H] = e.u0;
        const double(&x0)[H] = e.x0;
        C v[F::E];
        double sw = 0, st = 0, sr = 0, sp = 0;
        const bool comb = in.mode == A_COMBINE;
        // every load first (the y store below could alias them, which would
        // otherwise serialise one memory round trip per element)
        double y0[H], k0[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            y0[i] = k0[i] = 0.0;
            const int64_t idx = (int64_t)(g + i * F::G) * N2 + n2;
            if (active && idx < M) {
                const int64_t q = pos_of(P, idx);
                y0[i] = in.y[q];
                if (comb && in.kc) k0[i] = in.kc[q];
            }
        }
#pragma unroll
        for (int i = 0; i < F::E; ++i) {
            v[i] = czero<C>();
            if (i < H && active) {
                const int64_t idx = (int64_t)(g + i * F::G) * N2 + n2;
                if (idx < M) {
                    double yv = y0[i];
                    if (comb) {
                        if (in.kc) yv = fma(in.c, k0[i], yv);
                        if (in.ywrite && al == 0) in.ywrite[pos_of(P, idx)] = yv;
                    }
                    const double u = u0[i] * yv, x = x0[i] * yv;
                    if (idx < M - 1) v[i] = from_cd<C>(cd{u, x});
                    if (comb) {
                        const double s = (double)(idx + 1);
                        sw += x;
                        if (idx >= 1) {
                            st = fma(s, x, st);
                            sr += u;
                            sp = fma(s, u, sp);
                        }
                    }
                }
            }
        }
        // When L = 2M - 2 the largest size sits at index L/2 (row N1/2 of
        // column 0): not an FFT input, but part of y and of the reductions.
        if (comb && active && n2 == 0 && g == 0 && (int64_t)(N1 / 2) * N2 < M) {
            const int64_t idx = (int64_t)(N1 / 2) * N2;
            const int64_t q = pos_of(P, idx);
            double yv = in.y[q];
            if (in.kc) yv = fma(in.c, in.kc[q], yv);
            if (in.ywrite && al == 0) in.ywrite[q] = yv;
            const double s = (double)(idx + 1);
            const double u = Ua[q] * yv, x = Va[q] * yv;
            sw += x;
            st = fma(s, x, st);
            sr += u;
            sp = fma(s, u, sp);
        }
        C *wl = lds + w * 64 * F::E;
        if (active) {
            wave_fft<N1, false>(v, wl + f * N1, g, tw);
            // spectra are stored column by column: one contiguous run per column
            C *Za = (C *)P.Z + ((int64_t)al << P.logL) + (int64_t)n2 * N1;
#pragma unroll
            for (int i = 0; i < F::E; ++i) Za[g + i * F::G] = cmul(v[i], t4[i]);
        }
        if (comb) {
            sw = wave_sum(sw);
            st = wave_sum(st);
            sr = wave_sum(sr);
            sp = wave_sum(sp);
            if (lane == 0) {
                sh[w * 4 + 0] = sw;
                sh[w * 4 + 1] = st;
                sh[w * 4 + 2] = sr;
                sh[w * 4 + 3] = sp;
            }
            __syncthreads();
            if (tid < 4) P.red_part[((int64_t)grp * P.R + al) * 4 + tid] = sum_waves<W>(sh, 4, tid);
        }
    }
};

// --------------------------------------------------------------------------
// Phase B
// --------------------------------------------------------------------------

// E: elements per lane of the row transforms; W: waves per workgroup.
template <int N1, int N2, class C, int E = fft_default_e(N2), int W = SMOL_WAVES>
struct PhaseB {
    using F = FftShape<N2, E>;
    static constexpr int NT = 64 * W;
    static constexpr int SLOTS = W * F::B;           // row transforms per round
    static constexpr int AL_PER_ROUND = SLOTS / 2;   // ranks per round (2 rows each)
    static __host__ __device__ int units() { return N1 / 2 + 1; }
    // LDS entries: SLOTS rows + P for the two rows
    static constexpr int LDS = SLOTS * N2 + 2 * N2;

    // unit k1 in [0, N1/2]; whole workgroup
    __device__ static void run(const RhsPlanDev &P, int k1, C *lds)
    {
        const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
        const int f = lane / F::G, g = lane % F::G;
        const int slot = wave * F::B + f;
        const int k1p = (N1 - k1) & (N1 - 1);
        const bool single = (k1 == k1p);  // k1 = 0 or N1/2
        C *rows = lds;
        C *P1 = lds + SLOTS * N2, *P2 = P1 + N2;
        FftTw<N2, false, C, E> twf;
        twf.load(g, P.rt);
        // twiddles of the two inverse row transforms (slots 0 and 1), loaded
        // now so that the inverse pass does not wait on a table read
        const bool inv = slot < (single ? 1 : 2);
        FftTw<N2, true, C, E> twi;
        C t4[F::E];
        if (inv) {
            twi.load(g, P.rt);
            step_twiddles<F::E, true>(P.rt, P.logL, (uint32_t)(slot ? k1p : k1), g, F::G, t4);
        }
        for (int a0 = 0; a0 < P.R; a0 += AL_PER_ROUND) {
            const int na = min(AL_PER_ROUND, P.R - a0);
            // slot 2m holds rank a0+m row k1, slot 2m+1 its row N1-k1
            {
                const int m = slot >> 1, which = slot & 1;
                if (m < na && !(single && which)) {
                    const int krow = which ? k1p : k1;
                    // row krow of the column-major spectra: stride N1
                    const C *src = (const C *)P.Z + ((int64_t)(a0 + m) << P.logL) + krow;
                    C v[F::E];
#pragma unroll
                    for (int i = 0; i < F::E; ++i) v[i] = src[(int64_t)(g + i * F::G) * N1];
                    wave_fft<N2, false>(v, rows + slot * N2, g, twf);
                    wave_sync();
#pragma unroll
                    for (int i = 0; i < F::E; ++i) rows[slot * N2 + g + i * F::G] = v[i];
                }
            }
            __syncthreads();
            const bool last = a0 + AL_PER_ROUND >= P.R;
            for (int k2 = tid; k2 < N2; k2 += NT) {
                // partner of (k1, k2) is (k1p, k2p)
                const int k2p = (k1 == 0) ? ((N2 - k2) & (N2 - 1)) : (N2 - 1 - k2);
                C acc = a0 ? P1[k2] : czero<C>();
                for (int m = 0; m < na; ++m) {
                    const C a = rows[(2 * m) * N2 + k2];
                    const C b = rows[(2 * m + (single ? 0 : 1)) * N2 + k2p];
                    acc = spec_term(acc, a, b);
                }
                if (last) {
                    // divide by 4i: x / (4i) = (x.y, -x.x) / 4; partner row
                    // by conjugate reversal
                    const C q = div4i(acc);
                    P1[k2] = q;
                    if (!single) P2[N2 - 1 - k2] = cconj(q);
                } else {
                    P1[k2] = acc;
                }
            }
            __syncthreads();
        }
        // inverse DFT over k2 of rows k1 (slot 0) and N1-k1 (slot 1)
        if (inv) {
            const int krow = slot ? k1p : k1;
            const C *src = slot ? P2 : P1;
            C v[F::E];
#pragma unroll
            for (int i = 0; i < F::E; ++i) v[i] = src[g + i * F::G];
            wave_fft<N2, true>(v, rows + slot * N2, g, twi);
            C *dst = (C *)P.Qp + (int64_t)krow * (N2 / 2);
#pragma unroll
            for (int i = 0; i < F::E / 2; ++i) {
                const C lo = cmul(v[i], t4[i]);
                const C hi = cmul(v[i + F::E / 2], t4[i + F::E / 2]);
                dst[g + i * F::G] = cadd(lo, crot<true>(hi));  // lo + i*hi
            }
        }
    }
};

// Sum reduction partials [njobs][R][4] in a fixed order into red[R][4]
// (threads take fixed stripes of jobs, then the stripes are added in order).
template <int NT = SMOL_WG>
__device__ inline void finalize_reductions(const RhsPlanDev &P, int njobs)
{
    __shared__ double sh[NT];
    const int tid = threadIdx.x, nq = 4 * P.R, ns = NT / nq;
    const int q = tid % nq, s = tid / nq;
    double acc = 0.0;
    if (s < ns)
        for (int j = s; j < njobs; j += ns) acc += P.red_part[(int64_t)j * nq + q];
    sh[tid] = acc;
    __syncthreads();
    if (tid < nq) {
        double tot = 0.0;
        for (int k = 0; k < ns; ++k) tot += sh[k * nq + tid];
        P.red[tid] = tot;
    }
}

// --------------------------------------------------------------------------
// Phase C
// --------------------------------------------------------------------------

// E: elements per lane of the column transforms (inverse, and the fused
// next column pass); W: waves per workgroup.
template <int N1, int N2, class C, int E = fft_default_e(N1), int W = SMOL_WAVES>
struct PhaseC {
    using F = FftShape<N1, E>;
    static constexpr int NT = 64 * W;
    static constexpr int HALF = N2 / 2;
    static constexpr int COLS = (F::B < HALF) ? F::B : HALF;  // packed columns per unit
    // Workgroups per unit.  A packed column holds two real columns (real and
    // imaginary part); where a unit has one packed column and four waves and
    // the units alone would leave compute units idle (N2 / 2 < 256), its two
    // real columns go to two workgroups, each running the unit's inverse
    // transform itself: twice the workgroups (a full chip at L = 2^17) for
    // one more packed-column read each.
    static constexpr int S = (COLS == 1 && W == 4 && HALF < SMOL_NUM_CU) ? 2 : 1;
    static constexpr int NPOS = COLS * N1 / S;                 // outputs per workgroup
    static constexpr int PP = (NPOS + NT - 1) / NT;            // per thread
    static constexpr int LDS = 64 * F::E;                      // wave 0 scratch
    static constexpr int NCOL = 2 * COLS / S;                  // real columns per workgroup
    // fused with the next column pass: W waves of scratch + the next stage
    // state of the workgroup's NCOL columns (doubles)
    // (NCOL columns x N1/2 rows of doubles = NCOL N1 / 4 sixteen-byte entries)
    static constexpr int LDS_FUSE = W * 64 * F::E + NCOL * N1 / 4;
    static __host__ __device__ int units() { return HALF / COLS * S; }
    static __host__ __device__ int jobs() { return units(); }

    // Output e of workgroup `unit` (0 <= e < NPOS): row b of the unit's
    // packed column f, real (hh = 0) or imaginary part; its local column
    // (NCOL of them) orders the fused column pass.  Sizes m + 2 with
    // m = ac + hh HALF + N2 b, ac = cu COLS + f the packed column.
    __device__ static void decode(int unit, int e, int &cu, int &b, int &hh, int &f, int &lc)
    {
        cu = unit / S;
        b = e % (N1 / 2);
        if constexpr (S == 1) {
            hh = (e / (N1 / 2)) & 1;
            f = e / N1;
            lc = hh * COLS + f;
        } else {
            hh = unit % S;
            f = e / (N1 / 2);
            lc = f;
        }
    }
    // the workgroup that computes size 1: the last unit (with two workgroups
    // per unit, the one with its imaginary half)
    __device__ static bool owns_size1(int unit) { return unit == units() - 1; }

    static constexpr int KMAX = 6;  // stage vectors an epilogue combines
    static constexpr int RPRE = 4;  // ranks whose U, V are prefetched

    // FUSE (stage epilogue only): a workgroup's outputs y_{i+1} fill exactly
    // its NCOL columns ac+1 and/or ac+1+N2/2 of the next column pass (the
    // workgroup that computes size 1 also owns column 0: its imaginary half
    // wraps onto row b+1), so the workgroup runs that pass itself and writes
    // the next spectra.
    struct ColPre;
    struct Early;

    template <bool FUSE = false>
    __device__ static void run(const RhsPlanDev &P, const Epi &ep, int unit, C *lds)
    {
        Early e;
        early<FUSE>(P, unit, e);
        SMOL_PHASE_CALL(C, run_with<FUSE>(P, ep, unit, lds, e));
    }

    template <bool FUSE>
    __device__ static void run_with(const RhsPlanDev &P, const Epi &ep, int unit, C *lds, Early &e)
    {
        __shared__ double sh[W * 16];
        const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
        const int64_t M = P.M;
        const int R = P.R;
        const double lam = P.lam;
        const int mode = ep.mode;
        const bool need_n = mode != C_RHS;
        const bool need_v = mode == C_STAGE;
        const int nk = (mode == C_STAGE || mode == C_LAST || mode == C_INIT1) ? ep.nks : 0;
        const int rp = R < RPRE ? R : RPRE;
        // ---- prefetch every per-size input of this thread's outputs
        int64_t qv[PP], sz[PP];
        double yv[PP], nv[PP], sv[PP], kv[PP][KMAX], Uv[PP][RPRE], Vv[PP][RPRE];
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            const int e = tid + j * NT;
            qv[j] = -1;
            sz[j] = 0;
            yv[j] = nv[j] = sv[j] = 0.0;
            if (e < NPOS) {
                int cu, b, hh, f, lc;
                decode(unit, e, cu, b, hh, f, lc);
                const int64_t m = cu * COLS + f + hh * HALF + (int64_t)N2 * b;
                if (m <= M - 2) {
                    const int64_t q = pos_of(P, m + 1);
                    qv[j] = q;
                    sz[j] = m + 2;
                    yv[j] = ep.y[q];
                    if (P.src) sv[j] = P.src[q];
                    if (need_n) nv[j] = ep.n[q];
#pragma unroll
                    for (int k = 0; k < KMAX; ++k)
                        kv[j][k] = (k < nk && (ep.coef[k] != 0.0 || ep.ocoef[k] != 0.0))
                                       ? ep.ks[k][q]
                                       : 0.0;
#pragma unroll
                    for (int a = 0; a < RPRE; ++a) {
                        if (a < rp) {
                            Uv[j][a] = P.U[(int64_t)a * P.ustride + q];
                            if (need_v) Vv[j][a] = P.V[(int64_t)a * P.ustride + q];
                        }
                    }
                }
            }
        }
        // ---- uniform inputs, loaded before any store: the death-rate
        // factors w_alpha and, in the last unit, everything size 1 needs
        // (monomer balance with the shattering gains)
        double wred[RPRE];
#pragma unroll
        for (int a = 0; a < RPRE; ++a) wred[a] = a < rp ? P.red[4 * a] : 0.0;
        const bool last = owns_size1(unit);
        double S1 = 0.0, y1 = 0.0, n1v = 0.0, k1v[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) k1v[k] = 0.0;
        if (last) {
            y1 = ep.y[0];
            if (need_n) n1v = ep.n[0];
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < nk && (ep.coef[k] != 0.0 || ep.ocoef[k] != 0.0)) k1v[k] = ep.ks[k][0];
            double d1 = 0.0, g1 = 0.0, pairs = 0.0;
            for (int al = 0; al < R; ++al) {
                const double wv = P.red[4 * al], t = P.red[4 * al + 1];
                const double r = P.red[4 * al + 2], pp = P.red[4 * al + 3];
                const double u1 = P.U[(int64_t)al * P.ustride];
                const double q = wv - P.V[(int64_t)al * P.ustride] * y1;
                d1 = fma(u1, wv, d1);
                g1 = fma(u1, t, g1);
                pairs = fma(pp, q, fma(r, t, pairs));
            }
            S1 = -y1 * d1 + 0.5 * lam * pairs + lam * y1 * g1;
            if (P.src) S1 += P.src[0];
        }
        ColPre &pre = e.pre;
        // ---- inverse DFT over k1 of this unit's packed columns (wave 0)
        if (w == 0) {
            const int f = lane / F::G, g = lane % F::G;
            C(&v)[F::E] = e.v;
            wave_fft<N1, true>(v, lds + f * N1, g, e.tw);
            wave_sync();
            if (f < COLS) {
#pragma unroll
                for (int i = 0; i < F::E / 2; ++i) lds[f * (N1 / 2) + g + i * F::G] = v[i];
            }
        }
        __syncthreads();
        // ---- finish: S, then the fused epilogue
        const double invL = 1.0 / (double)(1LL << P.logL);
        double acc[SMOL_EPART];
#pragma unroll
        for (int q = 0; q < SMOL_EPART; ++q) acc[q] = 0.0;
        double yn[PP];
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            yn[j] = 0.0;
            if (qv[j] >= 0) {
                const int e = tid + j * NT;
                int cu, b, hh, f, lc;
                decode(unit, e, cu, b, hh, f, lc);
                const C val = lds[f * (N1 / 2) + b];
                const double c = (hh ? im_d(val) : re_d(val)) * invL;
                double dsum = 0.0;
#pragma unroll
                for (int a = 0; a < RPRE; ++a)
                    if (a < rp) dsum = fma(Uv[j][a], wred[a], dsum);
                for (int a = RPRE; a < R; ++a)
                    dsum = fma(P.U[(int64_t)a * P.ustride + qv[j]], P.red[4 * a], dsum);
                const double S = fma(-(1.0 + lam) * yv[j], dsum, 0.5 * c) + sv[j];
                yn[j] = finish(ep, qv[j], (double)sz[j], S, yv[j], nv[j], kv[j], nk, acc);
            }
        }
        // ---- size 1 (index 0): monomer balance with the shattering gains
        const bool mono = last && tid == 0;
        double yn1 = 0.0;
        if (mono) yn1 = finish(ep, 0, 1.0, S1, y1, n1v, k1v, nk, acc);
        double *ycol = (double *)(lds + W * 64 * F::E);
        if constexpr (FUSE) {
            // next stage state by (local column, row) for the column pass below
#pragma unroll
            for (int j = 0; j < PP; ++j) {
                if (qv[j] >= 0) {
                    const int e = tid + j * NT;
                    int cu, b, hh, f, lc;
                    decode(unit, e, cu, b, hh, f, lc);
                    const int wrap = (cu * COLS + f + 1 + hh * HALF) == N2;
                    const int n1 = b + wrap;
                    if (n1 < N1 / 2) ycol[lc * (N1 / 2) + n1] = yn[j];
                }
            }
            if (mono) ycol[(NCOL - 1) * (N1 / 2)] = yn1;
        }
        if constexpr (FUSE) {
            // the next column pass first: its spectra are the bulk of the
            // kernel's stores, so they drain while the reductions run
            __syncthreads();
            column_pass(P, unit, lds, ycol, pre);
        }
        if (mode == C_STAGE) {
            // reductions of the next stage state, four ranks per pass
            for (int a0 = 0; a0 < R; a0 += 4) {
                double s4[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) s4[k] = 0.0;
#pragma unroll
                for (int j = 0; j < PP; ++j) {
                    if (qv[j] >= 0) {
                        const double szd = (double)sz[j];
#pragma unroll
                        for (int a = 0; a < 4; ++a) {
                            if (a0 + a < R) {
                                double u, x;
                                if (a0 == 0) {
                                    u = Uv[j][a];
                                    x = Vv[j][a];
                                } else {
                                    u = P.U[(int64_t)(a0 + a) * P.ustride + qv[j]];
                                    x = P.V[(int64_t)(a0 + a) * P.ustride + qv[j]];
                                }
                                x *= yn[j];
                                u *= yn[j];
                                s4[4 * a] += x;
                                s4[4 * a + 1] = fma(szd, x, s4[4 * a + 1]);
                                s4[4 * a + 2] += u;
                                s4[4 * a + 3] = fma(szd, u, s4[4 * a + 3]);
                            }
                        }
                    }
                }
                if (mono)
                    for (int a = 0; a < 4 && a0 + a < R; ++a)
                        s4[4 * a] += P.V[(int64_t)(a0 + a) * P.ustride] * yn1;
                const int na = (R - a0) < 4 ? (R - a0) : 4;
                // all 16 sums unconditionally: independent butterflies
                // interleave, where guarded ones would run one after another
#pragma unroll
                for (int k = 0; k < 16; ++k) s4[k] = wave_sum(s4[k]);
                if (lane == 0)
                    for (int k = 0; k < 4 * na; ++k) sh[w * 16 + k] = s4[k];
                __syncthreads();
                if (tid < 4 * na)
                    P.red_part[((int64_t)unit * R + a0) * 4 + tid] = sum_waves<W>(sh, 16, tid);
                __syncthreads();
            }
        } else if (mode != C_RHS) {
#pragma unroll
            for (int q = 0; q < SMOL_EPART; ++q) acc[q] = wave_sum(acc[q]);
            if (lane == 0)
#pragma unroll
                for (int q = 0; q < SMOL_EPART; ++q) sh[w * SMOL_EPART + q] = acc[q];
            __syncthreads();
            if (tid < SMOL_EPART)
                ep.epart[(int64_t)unit * SMOL_EPART + tid] = sum_waves<W>(sh, SMOL_EPART, tid);
        }
    }

    // The next stage's column pass over this unit's 2 COLS columns x R ranks
    // (same arithmetic as phase A given y), one transform per wave slot.
    // Everything a slot's first transform reads besides y (factors U, V,
    // twiddles) is loaded at kernel entry, so that pass starts as soon as the
    // finish has written y.
    struct ColPre {
        FftTw<N1, false, C, E> tw;
        C t4[F::E];
        double u[F::E / 2], x[F::E / 2];
    };
    struct Early {
        FftTw<N1, true, C, E> tw;  // wave 0: inverse twiddles
        C v[F::E];                 // wave 0: the unit's packed columns
        ColPre pre;                // FUSE: this wave slot's first column-pass transform
    };

    // column-pass transform `job` of workgroup `unit`: local column jj (as
    // decode() numbers them), rank al, global column n2
    __device__ static void col_job(const RhsPlanDev &P, int unit, int job, int &jj, int &al, int &n2)
    {
        jj = job % NCOL;
        al = job / NCOL;
        const int hh = S == 1 ? jj / COLS : unit % S, fc = S == 1 ? jj % COLS : jj;
        n2 = ((unit / S) * COLS + fc + 1 + hh * HALF) & (N2 - 1);
    }

    __device__ static void col_load(const RhsPlanDev &P, int unit, int job, ColPre &pre)
    {
        const int lane = lane_id(), g = lane % F::G;
        int jj, al, n2;
        col_job(P, unit, job, jj, al, n2);
        const double *Ua = P.U + (int64_t)al * P.ustride, *Va = P.V + (int64_t)al * P.ustride;
        pre.tw.load(g, P.rt);
        step_twiddles<F::E, false>(P.rt, P.logL, (uint32_t)n2, g, F::G, pre.t4);
#pragma unroll
        for (int i = 0; i < F::E / 2; ++i) {
            const int n1 = g + i * F::G;
            const int64_t idx = (int64_t)n1 * N2 + n2;
            pre.u[i] = pre.x[i] = 0.0;
            if (idx < P.M - 1) {
                const int64_t q = pos_of(P, idx);
                pre.u[i] = Ua[q];
                pre.x[i] = Va[q];
            }
        }
    }

    // Loads that need only the transform shape and workspaces: wave 0's
    // packed columns of the inverse pass with their twiddles, and (fused)
    // the factors and twiddles of each wave slot's first column-pass
    // transform.  The integrator issues them before its control-block load.
    template <bool FUSE>
    __device__ static void early(const RhsPlanDev &P, int unit, Early &e)
    {
        const int lane = lane_id(), w = wave_id();
        if constexpr (FUSE) {
            const int job = w * F::B + lane / F::G;
            if (job < NCOL * P.R) SMOL_PHASE_CALL(C, col_load(P, unit, job, e.pre));
        }
        if (w == 0) {
            const int f = lane / F::G, g = lane % F::G;
            const int ac = (unit / S) * COLS + f;
            e.tw.load(g, P.rt);
            const C *Qp = (const C *)P.Qp;
#pragma unroll
            for (int i = 0; i < F::E; ++i)
                e.v[i] = f < COLS ? Qp[(int64_t)(g + i * F::G) * HALF + ac] : czero<C>();
        }
    }

    __device__ static void column_pass(const RhsPlanDev &P, int unit, C *lds, const double *ycol,
                                       ColPre &pre)
    {
        const int lane = lane_id(), w = wave_id();
        const int f = lane / F::G, g = lane % F::G;
        const int64_t M = P.M;
        const int nj = NCOL * P.R;
        for (int r0 = 0; r0 < nj; r0 += W * F::B) {
            const int job = r0 + w * F::B + f;
            if (job < nj) {
                int jj, al, n2;
                col_job(P, unit, job, jj, al, n2);
                if (r0 > 0) SMOL_PHASE_CALL(C, col_load(P, unit, job, pre));
                C v[F::E];
#pragma unroll
                for (int i = 0; i < F::E; ++i) {
                    v[i] = czero<C>();
                    if (i < F::E / 2) {
                        const int n1 = g + i * F::G;
                        const int64_t idx = (int64_t)n1 * N2 + n2;
                        if (idx < M - 1) {
                            const double yv = ycol[jj * (N1 / 2) + n1];
                            v[i] = from_cd<C>(cd{pre.u[i] * yv, pre.x[i] * yv});
                        }
                    }
                }
                wave_fft<N1, false>(v, lds + w * 64 * F::E + f * N1, g, pre.tw);
                C *Za = (C *)P.Z + ((int64_t)al << P.logL) + (int64_t)n2 * N1;
#pragma unroll
                for (int i = 0; i < F::E; ++i) Za[g + i * F::G] = cmul(v[i], pre.t4[i]);
            }
        }
    }

    // Store S and the mode's result at position q (size s); returns the next
    // stage state (C_STAGE) and accumulates partial sums.
    __device__ static double finish(const Epi &ep, int64_t q, double s, double S, double y,
                                    double n, const double (&k)[KMAX], int nk, double *acc)
    {
        switch (ep.mode) {
        case C_RHS:
            ep.out[q] = S;
            return 0.0;
        case C_STAGE: {
            if (ep.ocomb) {
                double o = ep.oS * S;
#pragma unroll
                for (int j = 0; j < KMAX; ++j)
                    if (j < nk) o = fma(ep.ocoef[j], k[j], o);
                ep.out[q] = o;
            } else {
                ep.out[q] = S;
            }
            double a = ep.cS * S;
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < nk) a = fma(ep.coef[j], k[j], a);  // zero coefficients: k[j] = 0
            const double yn = fma(ep.h, a, n);
            ep.ynext[q] = yn;
            return yn;
        }
        case C_LAST: {
            ep.out[q] = S;
            double e = ep.cS * S;
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < nk) e = fma(ep.coef[j], k[j], e);
            e *= ep.h;
            if (ep.diff) e += y - n;
            const double sc = fma(ep.rtol, fmax(fabs(n), fabs(y)), ep.atol);
            const double r = e / sc;
            acc[0] = fma(r, r, acc[0]);
            acc[1] += y;
            acc[2] = fma(s, y, acc[2]);
            acc[3] = fma(s * s, y, acc[3]);
            acc[4] = fma(s * s * s, y, acc[4]);
            if (!isfinite(y)) acc[5] += 1.0;
            return 0.0;
        }
        case C_INIT0: {
            ep.out[q] = S;
            const double sc = fma(ep.rtol, fabs(y), ep.atol);
            const double a = y / sc, b = S / sc;
            acc[0] = fma(a, a, acc[0]);
            acc[1] = fma(b, b, acc[1]);
            if (!isfinite(y)) acc[5] += 1.0;
            return 0.0;
        }
        default: {  // C_INIT1: y = n0 + h0 f0, n = n0, k[0] = f0
            const double sc = fma(ep.rtol, fabs(n), ep.atol);
            const double d = (S - k[0]) / sc;
            acc[0] = fma(d, d, acc[0]);
            return 0.0;
        }
        }
    }
};
