// Planner: (kind, n) -> digit size b, convolution length N, series length
// lambda, FFT split and workspace layout.  Host only, deterministic.
//
// Constraints (Theorems on the full, low and high product):
//   full: N_digits b >= n, convolution length 2 N_digits;
//   low:  b >= 4, N >= 3, N b >= n;
//   high: b >= 4, N >= 3, (N + 1) b >= n + lg N + 2.
// Lengths are restricted to {2^a, 3 * 2^a} (smooth lengths, Section 2.2)
// and split as M = N/2 = L1 * L2 for the two-pass FFT.
#pragma once
#include <stdint.h>
#include <stddef.h>

#include "tmul.h"

namespace tmul {

constexpr int B_TRUNC = 11;          // digit size of the truncated products (8..15)
constexpr int B_FULL = 16;           // digit size of the full product
constexpr uint64_t TRUNC_MIN_BITS = 1025;  // below: full product + extraction
constexpr uint32_t L2_MAX = 1024, L1_MAX = 4096, LM_MAX = 256;
#ifndef TM_NT4
#define TM_NT4 512
#endif
#ifndef TM_DPT
#define TM_DPT 8
#endif
constexpr int DPW_HOST = TM_DPT * TM_NT4;  // coefficients per K4 workgroup

struct Plan {
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
    uint64_t y = x % 3 == 0 ? x / 3 : x;
    return (y & (y - 1)) == 0;
}

// M = L1 * L2 with L2 a power of two in [16, 1024] near sqrt(M)
inline bool split_M(uint64_t M, uint32_t& L1, uint32_t& L2)
{
    if (M < 32) return false;
    int a = 0;
    while (((M >> a) & 1) == 0) a++;
    uint64_t odd = M >> a;
    if (odd != 1 && odd != 3) return false;
    int lg = (lg_ceil(M) + 1) / 2;
    if (lg < 4) lg = 4;
    if (lg > 10) lg = 10;
    if (lg > a) lg = a;
    L2 = 1u << lg;
    uint64_t l1 = M / L2;
    if (!l1_supported(l1)) return false;
    L1 = (uint32_t)l1;
    return true;
}

// M = L1 * Lm * L2: the smallest power of two Lm (the middle pass of the
// three-pass split; 1 = two passes) that keeps the column length L1 <= 1024,
// or the forced Lm.
inline bool split_M3(uint64_t M, uint32_t force_lm, uint32_t& L1, uint32_t& Lm, uint32_t& L2)
{
    if (force_lm > 1) {
        Lm = force_lm;
        return (Lm & (Lm - 1)) == 0 && Lm <= LM_MAX && M % Lm == 0 && split_M(M / Lm, L1, L2) &&
               L1 <= 1024;
    }
    for (Lm = 1; Lm <= LM_MAX; Lm *= 2) {
        if (M % Lm != 0) return false;
        if (split_M(M / Lm, L1, L2) && L1 <= 1024) return true;
    }
    return false;
}

// smallest N in {2^a, 3*2^a}, N >= max(x, 64)
inline uint64_t next_smooth(uint64_t x)
{
    if (x < 64) x = 64;
    uint64_t best = UINT64_MAX;
    for (int a = 0; a < 62; a++) {
        uint64_t p2 = 1ull << a;
        if (p2 >= x && p2 < best) best = p2;
        if (a < 60 && 3 * p2 >= x && 3 * p2 < best) best = 3 * p2;
    }
    return best;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Build the plan.  b_trunc / b_full: digit sizes (0 = default).
// Returns false if unsupported.
inline bool make_plan(int kind, uint64_t n, int b_trunc, int b_full, Plan& P, uint32_t force_lm = 0)
{
    if (n == 0 || kind < 0 || kind > 2) return false;
    P = Plan();
    P.req_kind = kind;
    P.n = n;
    P.L = (n + 63) / 64;
    const int bt = b_trunc ? b_trunc : B_TRUNC;
    const int bf = b_full ? b_full : B_FULL;
    if (bt < 8 || bt > 15 || bf < 8 || bf > 16) return false;
    P.via_full = kind != TM_FULL && n < TRUNC_MIN_BITS;
    P.kind = P.via_full ? TM_FULL : kind;

    if (P.kind == TM_FULL) {
        P.b = bf;
        P.lam = 0;
        uint64_t nd = (n + P.b - 1) / P.b;
        P.N = next_smooth(2 * nd);
        P.digits = P.N / 2;
        P.ncoef = P.N;
        if (kind == TM_FULL) { P.off = 0; P.out_bits = 128 * P.L; P.out_limbs = 2 * P.L; }
        else if (kind == TM_LO) { P.off = 0; P.out_bits = n; P.out_limbs = P.L; }
        else { P.off = n; P.out_bits = n; P.out_limbs = P.L; }
    } else {
        P.b = bt;
        const int b = P.b;
        if (kind == TM_LO) {
            P.N = next_smooth((n + b - 1) / b);
            P.digits = P.N;
            P.ncoef = P.N;
        } else {
            uint64_t N = next_smooth((n + b - 1) / b);
            while ((N + 1) * (uint64_t)b < n + (uint64_t)lg_ceil(N) + 2) N = next_smooth(N + 1);
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
    if (!split_M3(P.M, force_lm, P.L1, P.Lm, P.L2)) return false;
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

}  // namespace tmul
