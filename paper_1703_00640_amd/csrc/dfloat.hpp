// Double-float ("compensated FP32") complex arithmetic for the FP32 path of
// the convolution (Section 2.1's Convolution routine at a working precision
// p below FP64's 53 bits, the fixed-word-size scenario of Section 2.3).
//
// A real is the unevaluated sum hi + lo of two floats, |lo| <= ulp(hi)/2,
// about 48 significant bits.  Sums use Knuth's two-sum and products the FMA
// two-product (error-free transformations), followed by a renormalising
// fast two-sum.  Additions take the cheaper form (two-sum of the high parts,
// low parts added in FP32): its error is at most a few units of 2^-48 of the
// larger operand, which is what the norm-wise error analysis of an FFT needs.
// Every operation here is compiled with floating-point contraction off: a
// product fused into the following two-sum would break the error-free
// transformation (measured: the relative error of a 1024-point transform
// grew from 2^-47 to 2^-24 with contraction on).
//
// Twiddle factors are generated in FP64 and split into (hi, lo) pairs, so
// the FP32 path keeps FP64 for twiddle generation, the ring maps, theta, the
// 2^b scaling and the rounding; only the FFT passes run in double-float.
#pragma once
#include <hip/hip_runtime.h>

namespace tmul {

struct df {
    float hi, lo;
};

struct __align__(16) dfc {
    df x, y;  // real and imaginary parts
};

__device__ __forceinline__ df df_two_sum(float a, float b)
{
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return df{s, e};
}

__device__ __forceinline__ df df_fast_two_sum(float a, float b)
{
#pragma clang fp contract(off)
    const float s = a + b;
    return df{s, b - (s - a)};
}

__device__ __forceinline__ df df_add(df a, df b)
{
#pragma clang fp contract(off)
    df s = df_two_sum(a.hi, b.hi);
    s.lo = s.lo + (a.lo + b.lo);
    return df_fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ df df_neg(df a) { return df{-a.hi, -a.lo}; }
__device__ __forceinline__ df df_sub(df a, df b) { return df_add(a, df_neg(b)); }

__device__ __forceinline__ df df_mul(df a, df b)
{
#pragma clang fp contract(off)
    const float p = a.hi * b.hi;
    float e = __builtin_fmaf(a.hi, b.hi, -p);
    e = __builtin_fmaf(a.hi, b.lo, e);
    e = __builtin_fmaf(a.lo, b.hi, e);
    return df_fast_two_sum(p, e);
}

// FP64 value split into a double-float (hi the nearest float, lo the nearest
// float to the remainder) and back.
__host__ __device__ constexpr df df_from(double v)
{
    return df{(float)v, (float)(v - (double)(float)v)};
}
__device__ __forceinline__ double df_to(df a) { return (double)a.hi + (double)a.lo; }

__device__ __forceinline__ dfc to_dfc(double2 v) { return dfc{df_from(v.x), df_from(v.y)}; }
__device__ __forceinline__ double2 from_dfc(dfc v) { return make_double2(df_to(v.x), df_to(v.y)); }

// ------------------------------------------------- complex operations
// (overloads of the FP64 ones in fft_tile.hpp)

__device__ __forceinline__ dfc cadd(dfc a, dfc b) { return dfc{df_add(a.x, b.x), df_add(a.y, b.y)}; }
__device__ __forceinline__ dfc csub(dfc a, dfc b) { return dfc{df_sub(a.x, b.x), df_sub(a.y, b.y)}; }
__device__ __forceinline__ dfc cconj(dfc a) { return dfc{a.x, df_neg(a.y)}; }
__device__ __forceinline__ dfc cneg(dfc a) { return dfc{df_neg(a.x), df_neg(a.y)}; }
__device__ __forceinline__ dfc cmul(dfc a, dfc b)
{
    return dfc{df_sub(df_mul(a.x, b.x), df_mul(a.y, b.y)), df_add(df_mul(a.x, b.y), df_mul(a.y, b.x))};
}
// times a real constant given in FP64
__device__ __forceinline__ dfc cscale(dfc a, double s)
{
    const df d = df_from(s);
    return dfc{df_mul(a.x, d), df_mul(a.y, d)};
}
// times -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ dfc mul_mi(dfc a)
{
    return INV ? dfc{df_neg(a.y), a.x} : dfc{a.y, df_neg(a.x)};
}

// Conversions used where FP64 values (twiddles from the FP64 tables, map
// outputs) enter a tile of element type C, and where results leave it.
template <typename C>
__device__ __forceinline__ C to_elem(double2 v);
template <>
__device__ __forceinline__ double2 to_elem<double2>(double2 v) { return v; }
template <>
__device__ __forceinline__ dfc to_elem<dfc>(double2 v) { return to_dfc(v); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(dfc v) { return from_dfc(v); }

// ---------------------------------------------------------- codelets
// The same DFTs as the FP64 codelets, written with the operations above.

template <bool INV>
__device__ __forceinline__ void dft2(dfc* v)
{
    const dfc a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(dfc* v)
{
    const double h = 0.86602540378443864676;  // sin(2 pi / 3)
    const dfc s = cadd(v[1], v[2]);
    const dfc d = csub(v[1], v[2]);
    const dfc t = csub(v[0], cscale(s, 0.5));
    const dfc u = mul_mi<INV>(cscale(d, h));
    v[0] = cadd(v[0], s);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
}

template <bool INV>
__device__ __forceinline__ void dft4(dfc* v)
{
    const dfc t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const dfc t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(dfc* v)
{
    const double c = 0.70710678118654752440;
    dfc e[4] = {v[0], v[2], v[4], v[6]};
    dfc o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    // o_k times exp(-+2 pi i k / 8)
    o[1] = cscale(INV ? dfc{df_sub(o[1].x, o[1].y), df_add(o[1].x, o[1].y)}
                      : dfc{df_add(o[1].x, o[1].y), df_sub(o[1].y, o[1].x)}, c);
    o[2] = mul_mi<INV>(o[2]);
    o[3] = cscale(INV ? dfc{df_neg(df_add(o[3].x, o[3].y)), df_sub(o[3].x, o[3].y)}
                      : dfc{df_sub(o[3].y, o[3].x), df_neg(df_add(o[3].x, o[3].y))}, c);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        v[k] = cadd(e[k], o[k]);
        v[k + 4] = csub(e[k], o[k]);
    }
}

// v * exp(-+2 pi i M / 16)
template <int M, bool INV>
__device__ __forceinline__ dfc tw16(dfc v)
{
    constexpr int m = M & 15;
    if constexpr (m == 0) return v;
    else if constexpr (m == 4) return mul_mi<INV>(v);
    else if constexpr (m == 8) return cneg(v);
    else if constexpr (m == 12) return mul_mi<!INV>(v);
    else {
        constexpr double C1 = 0.92387953251128675613, S1 = 0.38268343236508977173;
        constexpr double H = 0.70710678118654752440;
        constexpr double cs[16] = {1, C1, H, S1, 0, -S1, -H, -C1, -1, -C1, -H, -S1, 0, S1, H, C1};
        constexpr double cc = cs[m], sn = cs[(m + 12) & 15];
        const double s = INV ? sn : -sn;
        const df dc = df_from(cc), ds = df_from(s);
        return dfc{df_sub(df_mul(dc, v.x), df_mul(ds, v.y)), df_add(df_mul(dc, v.y), df_mul(ds, v.x))};
    }
}

template <bool INV>
__device__ __forceinline__ void dft16(dfc* v)
{
    dfc y[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; n1++) {
        dfc t[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
        dft4<INV>(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; k2++) y[n1][k2] = t[k2];
    }
    y[1][1] = tw16<1, INV>(y[1][1]);
    y[1][2] = tw16<2, INV>(y[1][2]);
    y[1][3] = tw16<3, INV>(y[1][3]);
    y[2][1] = tw16<2, INV>(y[2][1]);
    y[2][2] = tw16<4, INV>(y[2][2]);
    y[2][3] = tw16<6, INV>(y[2][3]);
    y[3][1] = tw16<3, INV>(y[3][1]);
    y[3][2] = tw16<6, INV>(y[3][2]);
    y[3][3] = tw16<9, INV>(y[3][3]);
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++) {
        dfc t[4] = {y[0][k2], y[1][k2], y[2][k2], y[3][k2]};
        dft4<INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; k1++) v[k2 + 4 * k1] = t[k1];
    }
}

// radix 5 and 7 have no double-float codelet (the FP32 path's lengths are
// powers of two and 3 times powers of two): instantiating one is an error
template <bool INV>
__device__ __forceinline__ void dft5(dfc*)
{
    static_assert(INV && !INV, "no double-float radix-5 codelet");
}
template <bool INV>
__device__ __forceinline__ void dft7(dfc*)
{
    static_assert(INV && !INV, "no double-float radix-7 codelet");
}

}  // namespace tmul
