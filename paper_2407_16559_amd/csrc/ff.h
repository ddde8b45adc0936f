// Float-float ("double-word") arithmetic: a real is an unevaluated sum
// h + l of two FP32 numbers with |l| <= ulp(h)/2, giving about 48 bits of
// significand.  Error-free transformations (Knuth's TwoSum, Dekker's
// FastTwoSum, FMA-based TwoProd) and the double-word addition and
// multiplication of Joldes, Muller and Popescu, "Tight and rigorous error
// bounds for basic building blocks of double-word arithmetic" (ACM TOMS
// 2017): AccurateDWPlusDW (relative error <= 3u^2) and DWTimesDW with FMA
// (<= 5u^2), u = 2^-24.  Used for the convolution transforms of the
// float-float precision variant; everything else stays FP64.
#pragma once
#include "common.h"

struct ff {
    float h, l;
};

// complex float-float; 16 bytes, the same storage as a complex double
struct __align__(16) cff {
    ff x, y;
};

__device__ __forceinline__ ff ff_from(double d)
{
#pragma clang fp contract(off)
    const float h = (float)d;
    return ff{h, (float)(d - (double)h)};
}
__device__ __forceinline__ double ff_to(ff a) { return (double)a.h + (double)a.l; }

__device__ __forceinline__ ff two_sum(float a, float b)
{
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    return ff{s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ ff fast_two_sum(float a, float b)
{
#pragma clang fp contract(off)
    const float s = a + b;
    return ff{s, b - (s - a)};
}
__device__ __forceinline__ ff ff_add(ff x, ff y)
{
#pragma clang fp contract(off)
    const ff s = two_sum(x.h, y.h);
    const ff t = two_sum(x.l, y.l);
    const ff v = fast_two_sum(s.h, s.l + t.h);
    return fast_two_sum(v.h, t.l + v.l);
}
__device__ __forceinline__ ff ff_neg(ff x) { return ff{-x.h, -x.l}; }
__device__ __forceinline__ ff ff_sub(ff x, ff y) { return ff_add(x, ff_neg(y)); }
__device__ __forceinline__ ff ff_mul(ff x, ff y)
{
#pragma clang fp contract(off)
    const float ch = x.h * y.h;
    const float cl1 = fmaf(x.h, y.h, -ch);
    const float tl0 = x.l * y.l;
    const float tl1 = fmaf(x.h, y.l, tl0);
    const float cl2 = fmaf(x.l, y.h, tl1);
    return fast_two_sum(ch, cl1 + cl2);
}
// exact scaling by a power of two
__device__ __forceinline__ ff ff_scale2(ff x, float p2) { return ff{x.h * p2, x.l * p2}; }

// ---- complex operations with the same names as the FP64 ones -------------

__device__ __forceinline__ cff cadd(cff a, cff b) { return cff{ff_add(a.x, b.x), ff_add(a.y, b.y)}; }
__device__ __forceinline__ cff csub(cff a, cff b) { return cff{ff_sub(a.x, b.x), ff_sub(a.y, b.y)}; }
__device__ __forceinline__ cff cmul(cff a, cff b)
{
    return cff{ff_sub(ff_mul(a.x, b.x), ff_mul(a.y, b.y)), ff_add(ff_mul(a.x, b.y), ff_mul(a.y, b.x))};
}
__device__ __forceinline__ cff cconj(cff a) { return cff{a.x, ff_neg(a.y)}; }
template <bool INV>
__device__ __forceinline__ cff crot(cff a)
{
    return INV ? cff{ff_neg(a.y), a.x} : cff{a.y, ff_neg(a.x)};
}
