// Planner: (kind, n) -> digit size b, convolution length N, series length
// lambda, FFT split and workspace layout.  Host only, deterministic.
//
// Constraints (Theorems on the full, low and high product):
//   full: N_digits b >= n, convolution length 2 N_digits;
//   low:  b >= 4, N >= 3, N b >= n;
//   high: b >= 4, N >= 3, (N + 1) b >= n + lg N + 2.
// Lengths are restricted to {2^a, 3 * 2^a, 5 * 2^a, 7 * 2^a} (smooth lengths,
// Section 2.2) and split as M = N/2 = L1 * Lm * L2.
#pragma once
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#include "tmul.h"

namespace tmul {

constexpr int B_TRUNC = 11;          // digit size of the truncated products
// Every kind accepts digit sizes 8..16: the generic (runtime-b) K1 instances
// size their staged digit windows for fields of at most 16 bits, K4 sizes
// its per-thread limb arrays for b <= 16, and its limb carry needs b >= 8
// (at most 9 coefficients start in one 64-bit limb).
constexpr int B_MIN = 8, B_MAX = 16;
constexpr int B_FULL = 16;           // digit size of the full product
constexpr uint64_t TRUNC_MIN_BITS = 1025;  // below: full product + extraction
constexpr uint32_t L2_MAX = 1024, L1_MAX = 4096, LM_MAX = 256;
#ifndef TM_NT4
#define TM_NT4 1024
#endif
#ifndef TM_DPT
#define TM_DPT 8
#endif
constexpr int DPW_HOST = TM_DPT * TM_NT4;  // coefficients per K4 workgroup

struct Plan {
    bool df = false;    // FP32 path: double-float FFT passes
    bool fused = false; // small size: K0 (whole transform in LDS) replaces K1, K2, K3
    int req_kind = 0;   // requested tm_kind
    int kind = 0;       // algorithm run (TM_FULL/TM_LO/TM_HI)
    bool via_full = false;
    uint64_t n = 0, L = 0;
    int b = 0, lam = 0;
    uint64_t N = 0;       // real convolution length
    uint64_t digits = 0;  // digits per operand
    uint64_t M = 0;
    uint32_t L1 = 0, L2 = 0, Lm = 1;  // M = L1 * Lm * L2
    uint32_t jmax = 0;
    int64_t shift = 0;
    uint64_t off = 0, out_bits = 0, out_limbs = 0;
    uint64_t ncoef = 0, ncover = 0;
    uint32_t nstatus = 0;
    size_t o_za = 0, o_zb = 0, o_status = 0, o_ticket = 0, o_guard = 0, o_theta = 0, ws_bytes = 0;
};

inline int lg_ceil(uint64_t x)
{
    int r = 0;
    while ((1ull << r) < x) r++;
    return r;
}

inline bool l1_supported(uint64_t x)
{
    if (x < 2 || x > L1_MAX) return false;
    uint64_t y = x % 3 == 0 ? x / 3 : x % 5 == 0 ? x / 5 : x % 7 == 0 ? x / 7 : x;
    return (y & (y - 1)) == 0;
}

// Row lengths with a K2 instance besides the powers of two 16..1024: the
// odd factor 3 times a power of two (the truncated products' lengths
// N = 3 2^a), so that the column pass can keep a power-of-two length.
inline bool l2_supported(uint64_t x)
{
    if (x >= 16 && x <= 1024 && (x & (x - 1)) == 0) return true;
    return x % 3 == 0 && x >= 96 && x <= 768 && ((x / 3) & (x / 3 - 1)) == 0;
}

// M = L1 * L2 with L2 = 2^lg near sqrt(M), or 2^force_lg when given.
// odd_row: the odd factor of M goes to the row length instead, L2 = odd
// 2^lg (lg: the largest that keeps L2 <= 1024, or force_lg), and L1 is a
// power of two (no effect when M is a power of two).
inline bool split_M(uint64_t M, uint32_t& L1, uint32_t& L2, int force_lg = 0, bool odd_row = false)
{
    if (M < 32) return false;
    int a = 0;
    while (((M >> a) & 1) == 0) a++;
    uint64_t odd = M >> a;
    if (odd != 1 && odd != 3 && odd != 5 && odd != 7) return false;
    if (odd_row && odd != 1) {
        int lg = 0;
        while ((odd << (lg + 1)) <= 1024 && lg + 1 <= a) lg++;
        if (force_lg) {
            if (force_lg < 4 || force_lg > lg) return false;
            lg = force_lg;
        }
        const uint64_t l2 = odd << lg;
        if (!l2_supported(l2) || M / l2 < 2) return false;
        L2 = (uint32_t)l2;
        L1 = (uint32_t)(M / l2);
        return l1_supported(L1);
    }
    int lg = (lg_ceil(M) + 1) / 2;
    if (lg < 4) lg = 4;
    if (lg > 10) lg = 10;
    if (force_lg) {
        if (force_lg < 4 || force_lg > 10) return false;
        lg = force_lg;
    }
    if (lg > a) lg = a;
    L2 = 1u << lg;
    uint64_t l1 = M / L2;
    if (!l1_supported(l1)) return false;
    L1 = (uint32_t)l1;
    return true;
}

// Forced FFT split (the autotuner's choice): low 16 bits the middle length
// Lm (0: the planner's search, >= 1: exactly that Lm), bits 16..23 log2 of
// the power-of-two part of the row length L2 (0: the default), bit 24 the
// odd factor of M in the row length rather than the column length.
constexpr uint32_t SPLIT_ODD_ROW = 1u << 24;
inline uint32_t split_code(uint32_t lm, int lg2, bool odd_row = false)
{
    return lm | ((uint32_t)lg2 << 16) | (odd_row ? SPLIT_ODD_ROW : 0u);
}

// M = L1 * Lm * L2: the smallest power of two Lm (the middle pass of the
// three-pass split; 1 = two passes) that keeps the column length L1 <= 1024,
// or the forced split.
inline bool split_M3(uint64_t M, uint32_t force, uint32_t& L1, uint32_t& Lm, uint32_t& L2)
{
    const uint32_t force_lm = force & 0xffffu;
    const int force_lg = (int)((force >> 16) & 0xffu);
    const bool odd_row = (force & SPLIT_ODD_ROW) != 0;
    if (force_lm >= 1 && (force_lm > 1 || force_lg || odd_row)) {
        Lm = force_lm;
        return (Lm & (Lm - 1)) == 0 && Lm <= LM_MAX && M % Lm == 0 &&
               split_M(M / Lm, L1, L2, force_lg, odd_row) && L1 <= 1024;
    }
    for (Lm = 1; Lm <= LM_MAX; Lm *= 2) {
        if (M % Lm != 0) return false;
        if (split_M(M / Lm, L1, L2, force_lg, odd_row) && L1 <= 1024) return true;
    }
    return false;
}

// smallest N in {2^a, 3*2^a, 5*2^(a>=5), 7*2^(a>=5)}, N >= max(x, 64)
inline uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 64;
    while (p < x) p *= 2;
    return p;
}

inline uint64_t next_smooth(uint64_t x)
{
    if (x < 64) x = 64;
    uint64_t best = UINT64_MAX;
    for (int a = 0; a < 62; a++) {
        const uint64_t p2 = 1ull << a;
        if (p2 >= x && p2 < best) best = p2;
        if (a < 60 && 3 * p2 >= x && 3 * p2 < best) best = 3 * p2;
        // 5 * 2^a from a = 5 on, so that M = N/2 keeps a row length of 16
        if (a >= 5 && a < 59 && 5 * p2 >= x && 5 * p2 < best) best = 5 * p2;
        if (a >= 5 && a < 59 && 7 * p2 >= x && 7 * p2 < best) best = 7 * p2;
    }
    return best;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Digit sizes of the FP32 path (double-float FFT passes, about 48 bits
// against FP64's 53, measured 2^-47 relative error per transform): the
// rounding error grows as the unit roundoff times 2^(3b) for the truncated
// products and 2^(2b) for the full product (the bounds on the convolution's
// coefficients, Sections 2.3 and 3.4), so keeping the FP64 plans' margin
// costs ceil(6/3) = 2 bits of b (11 -> 9) and ceil(6/2) = 3 bits (16 -> 13).
constexpr int B_TRUNC_DF = 9;
constexpr int B_FULL_DF = 13;

// (L1, L2) splits with a fused small-size instance (K0): the planner's
// default split of every length M = N/2 <= 4096 of the menu.
#define TM_K0_LIST(X)                                                                               \
    X(2, 16) X(3, 16) X(4, 16) X(5, 16) X(6, 16) X(7, 16) X(8, 16) X(10, 16) X(12, 16) X(14, 16)   \
    X(16, 16) X(10, 32) X(12, 32) X(14, 32) X(16, 32) X(20, 32) X(24, 32) X(28, 32) X(32, 32)      \
    X(20, 64) X(24, 64) X(28, 64) X(32, 64) X(40, 64) X(48, 64) X(56, 64) X(64, 64)
inline bool k0_supported(uint32_t L1, uint32_t L2)
{
#define X(A, B) if (L1 == A && L2 == B) return true;
    TM_K0_LIST(X)
#undef X
    return false;
}

// Build the plan.  b_trunc / b_full: digit sizes (0 = default).  via_full:
// serve a low or high product by the full product plus extraction at any n
// (the checked entry point's last fallback).  df: the FP32 path (power-of-two
// lengths, double-float FFT passes).  Returns false if unsupported.
inline bool make_plan(int kind, uint64_t n, int b_trunc, int b_full, Plan& P, uint32_t force = 0,
                      bool via_full = false, bool df = false, bool allow_fused = false)
{
    if (n == 0 || kind < 0 || kind > 2) return false;
    P = Plan();
    P.req_kind = kind;
    P.n = n;
    P.L = (n + 63) / 64;
    P.df = df;
    const int bt = b_trunc ? b_trunc : df ? B_TRUNC_DF : B_TRUNC;
    const int bf = b_full ? b_full : df ? B_FULL_DF : B_FULL;
    uint64_t (*next_len)(uint64_t) = df ? next_pow2 : next_smooth;
    if (df && (force & SPLIT_ODD_ROW)) return false;
    if (bt < B_MIN || bt > B_MAX || bf < B_MIN || bf > B_MAX) return false;
    P.via_full = kind != TM_FULL && (n < TRUNC_MIN_BITS || via_full);
    P.kind = P.via_full ? TM_FULL : kind;

    if (P.kind == TM_FULL) {
        P.b = bf;
        P.lam = 0;
        uint64_t nd = (n + P.b - 1) / P.b;
        P.N = next_len(2 * nd);
        P.digits = P.N / 2;
        P.ncoef = P.N;
        if (kind == TM_FULL) { P.off = 0; P.out_bits = 128 * P.L; P.out_limbs = 2 * P.L; }
        else if (kind == TM_LO) { P.off = 0; P.out_bits = n; P.out_limbs = P.L; }
        else { P.off = n; P.out_bits = n; P.out_limbs = P.L; }
    } else {
        P.b = bt;
        const int b = P.b;
        if (kind == TM_LO) {
            P.N = next_len((n + b - 1) / b);
            P.digits = P.N;
            P.ncoef = P.N;
        } else {
            uint64_t N = next_len((n + b - 1) / b);
            while ((N + 1) * (uint64_t)b < n + (uint64_t)lg_ceil(N) + 2) N = next_len(N + 1);
            P.N = N;
            P.digits = N + 1;
            P.ncoef = N + 1;
            P.shift = (int64_t)((N + 1) * (uint64_t)b - n);
        }
        // series length: truncation below 2^-8 after scaling by 2^b, from
        // |coef_{k,r}| <= 2^-rb and ||conv|| <= N ||F|| ||G||
        P.lam = (lg_ceil(P.N) + 3 * b + 8 + b - 1) / b;
        if (P.lam < 2) P.lam = 2;
        if (P.lam > 9) return false;
        P.jmax = (80 + b - 1) / b;
        if (P.lam + (int)P.jmax > 32) return false;  // wrap terms must fit the K4 halo
        if (P.N < (uint64_t)(2 * P.lam + P.jmax + 2)) return false;
        P.off = kind == TM_LO ? (uint64_t)b : (P.N + 3) * (uint64_t)b - n;
        P.out_bits = n;
        P.out_limbs = P.L;
    }
    P.M = P.N / 2;
    if (!split_M3(P.M, force, P.L1, P.Lm, P.L2)) return false;
    P.fused = allow_fused && !df && P.Lm == 1 && P.M <= 4096 && k0_supported(P.L1, P.L2);
    uint64_t need = (P.off + P.out_bits + P.b - 1) / P.b + 2;
    uint64_t cov = P.ncoef > need ? P.ncoef : need;
    P.ncover = (cov + DPW_HOST - 1) / DPW_HOST * DPW_HOST;
    P.nstatus = (uint32_t)(P.ncover / DPW_HOST);
    if (P.ncover > 0xFFFFFFFFull) return false;

    size_t o = 0;
    P.o_za = o; o = align256(o + P.M * 16);
    P.o_zb = o; o = align256(o + P.M * 16);
    P.o_status = o; o = align256(o + (size_t)P.nstatus * 32);
    P.o_ticket = o; o = align256(o + 8);
    P.o_guard = o; o = align256(o + sizeof(tm_guard));
    P.o_theta = o; o = align256(o + 2 * sizeof(double));
    P.ws_bytes = o;
    return true;
}

// ------------------------------------------------------- guaranteed mode
//
// The default digit sizes are chosen statistically (Section 5 picks its
// parameters by testing; the rounding guard catches the rest).  Guaranteed
// mode instead takes the largest b whose worst-case rounding error bound
// stays below 0.45:
//   * digits |U_i| <= 2^(b-1) (the top digit <= 2^b), map outputs
//     |G_j| <= g 2^(b-1) with g = 1 + 4 2^-b (the series coefficients are
//     bounded by 2^-rb, Sections 3.2 and 4.2, and the wrap and recovery terms
//     add factors 1 + O(2^-b));
//   * the FFT convolution differs from the exact one by at most
//     ||G_u||_2 ||G_v||_2 eta, eta = (1+u)^(3k) (1+sqrt5 u)^(3k+1) (1+t)^(3k) - 1
//     (the error bound of FFT-based convolution of length 2^k in Brent and
//     Zimmermann, "Modern Computer Arithmetic", Theorem 3.6, the explicit
//     bound Section 2.1 points to for Convolution; unit roundoff u = 2^-53,
//     twiddle error t), taken with k = ceil(lg M) + 4 to
//     cover the radix-3/16 codelets, the packed real transform, the
//     inter-pass twiddles and the 1/M scaling, and t = 2^-49;
//   * the truncated products scale by 2^b and the back map's gain g, and the
//     series truncation adds at most 2^-8 (the choice of lambda).
inline double conv_eta(uint64_t M, bool df = false)
{
    // double-float: unit roundoff 2^-47 per operation (measured relative
    // error of a whole transform), twiddles split from FP64 (2^-47 too)
    const double u = ldexp(1.0, df ? -47 : -53), t = ldexp(1.0, df ? -47 : -49);
    const double k = (double)(lg_ceil(M) + 4);
    return expm1(3 * k * log1p(u) + (3 * k + 1) * log1p(sqrt(5.0) * u) + 3 * k * log1p(t));
}

// Bound on |x - exact| over all rounded values x of plan P (see above).
inline double rounding_bound(const Plan& P)
{
    const double eta = conv_eta(P.M, P.df);
    if (P.kind == TM_FULL) {
        const double nrm2 = (double)(P.digits - 1) * ldexp(1.0, 2 * P.b - 2) + ldexp(1.0, 2 * P.b);
        return nrm2 * eta;
    }
    const double g = 1.0 + 4.0 * ldexp(1.0, -P.b);
    const double nrm2 = g * g * ((double)(P.N - 1) * ldexp(1.0, 2 * P.b - 2) + ldexp(1.0, 2 * P.b));
    return ldexp(g * nrm2 * eta, P.b) + ldexp(1.0, -8);
}

constexpr double GUARANTEED_MAX = 0.45;

// The guaranteed plan: the largest b (at most the default) whose bound is
// below GUARANTEED_MAX; false if none with b >= 8 exists.  via_full: the
// full product's guaranteed plan serving a low or high product by
// extraction (exists wherever the full product's does, n <= 2^30 and more).
inline bool make_plan_guaranteed(int kind, uint64_t n, Plan& P, bool via_full = false)
{
    for (int b = B_FULL; b >= B_MIN; b--) {
        Plan Q;
        const bool trunc = kind != TM_FULL && !via_full && n >= TRUNC_MIN_BITS;
        if (trunc && b > B_TRUNC) continue;
        if (!make_plan(kind, n, b, b, Q, 0, via_full)) continue;
        if (rounding_bound(Q) <= GUARANTEED_MAX) {
            P = Q;
            return true;
        }
    }
    return false;
}

// A run of a plan whose worst-case bound is below 1/2 is exact when the
// guard reports nothing but distances within that bound: every rounded
// value then lies within the bound of its integer, so rounding returns it.
inline bool exact_by_bound(const Plan& P, const tm_guard& g)
{
    const double bound = rounding_bound(P);
    return bound <= GUARANTEED_MAX && (g.flags & ~TM_GUARD_DIST) == 0 && g.max_dist <= bound;
}

}  // namespace tmul
