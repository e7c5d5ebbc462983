// Workgroup-level FP64 complex DFTs on a tile held in LDS (gfx950).
//
// This is the building block of the Convolution step (Section 2.1: real
// FFTs, pointwise product, inverse FFT).  A tile holds NB independent
// sequences of length P; a Stockham autosort schedule of radix-3/5/7/16/8/4/2
// stages transforms all of them in place, one LDS round trip per stage
// (radix 16 runs as 4 x 4 in registers).  Each butterfly reads one stage
// twiddle from an LDS copy of exp(-2 pi i e / P) and forms the others as
// its powers, so no stage waits on global memory.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmul {

struct Tw {
    const double2* lo;   // lo[e0] = exp(-2 pi i e0 / M), e0 < 2^shift
    const double2* hi;   // hi[e1] = exp(-2 pi i e1 2^shift / M)
    uint32_t shift;
    uint32_t mask;
};

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 mul_mi(double2 a)
{
    return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// exp(-2 pi i e / M), or its conjugate for the inverse direction, from the
// two-level global table (used outside the LDS tiles)
template <bool INV>
__device__ __forceinline__ double2 tw_get(const Tw& t, uint32_t e)
{
    double2 w = cmul(t.lo[e & t.mask], t.hi[e >> t.shift]);
    return INV ? cconj(w) : w;
}

}  // namespace tmul

#include "dfloat.hpp"

namespace tmul {

// Twiddles base * step^q, q < Q, for a thread whose elements form an
// arithmetic progression of exponents.  base and step are fetched from the
// global FP64 table at kernel start (their latency hides behind the tile
// work); powers use at most four products each, in the tile's arithmetic C.
template <int Q, typename C = double2>
struct TwSeq {
    C pw[4];
    C base;
    __device__ __forceinline__ void init(double2 b, double2 step)
    {
        base = to_elem<C>(b);
        pw[0] = to_elem<C>(step);
#pragma unroll
        for (int i = 1; i < 4; i++) pw[i] = cmul(pw[i - 1], pw[i - 1]);
    }
    __device__ __forceinline__ C at(int q) const
    {
        C w = base;
#pragma unroll
        for (int i = 0; i < 4; i++)
            if ((1 << i) < Q && ((q >> i) & 1)) w = cmul(w, pw[i]);
        return w;
    }
};

// ------------------------------------------------------------- codelets

template <bool INV>
__device__ __forceinline__ void dft2(double2* v)
{
    double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(double2* v)
{
    const double h = 0.86602540378443864676;  // sin(2 pi / 3)
    double2 s = cadd(v[1], v[2]);
    double2 d = csub(v[1], v[2]);
    double2 t = make_double2(fma(-0.5, s.x, v[0].x), fma(-0.5, s.y, v[0].y));
    double2 u = mul_mi<INV>(cscale(d, h));  // -i h d (forward)
    v[0] = cadd(v[0], s);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
}

template <bool INV>
__device__ __forceinline__ void dft5(double2* v)
{
    const double c1 = 0.30901699437494742410;   // cos(2 pi / 5)
    const double c2 = -0.80901699437494742410;  // cos(4 pi / 5)
    const double s1 = 0.95105651629515357212;   // sin(2 pi / 5)
    const double s2 = 0.58778525229247312917;   // sin(4 pi / 5)
    const double2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const double2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const double2 a1 = make_double2(fma(c2, t2.x, fma(c1, t1.x, v[0].x)), fma(c2, t2.y, fma(c1, t1.y, v[0].y)));
    const double2 a2 = make_double2(fma(c1, t2.x, fma(c2, t1.x, v[0].x)), fma(c1, t2.y, fma(c2, t1.y, v[0].y)));
    // -i (forward) or +i (inverse) times b1 = s1 t3 + s2 t4, b2 = s2 t3 - s1 t4
    const double2 b1 = mul_mi<INV>(make_double2(fma(s2, t4.x, s1 * t3.x), fma(s2, t4.y, s1 * t3.y)));
    const double2 b2 = mul_mi<INV>(make_double2(fma(-s1, t4.x, s2 * t3.x), fma(-s1, t4.y, s2 * t3.y)));
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
}

// 7-point DFT from the symmetric sums a_k = v_k + v_(7-k) and differences
// d_k = v_k - v_(7-k), k = 1..3: X_m = v_0 + sum_k a_k cos(2 pi k m / 7)
// -+ i sum_k d_k sin(2 pi k m / 7), and X_(7-m) with the opposite sign of
// the sine part (forward: minus).
template <bool INV>
__device__ __forceinline__ void dft7(double2* v)
{
    const double c1 = 0.62348980185873353053, c2 = -0.22252093395631440429;
    const double c3 = -0.90096886790241912624;
    const double s1 = 0.78183148246802980871, s2 = 0.97492791218182360702;
    const double s3 = 0.43388373911755812048;
    const double2 a1 = cadd(v[1], v[6]), a2 = cadd(v[2], v[5]), a3 = cadd(v[3], v[4]);
    const double2 d1 = csub(v[1], v[6]), d2 = csub(v[2], v[5]), d3 = csub(v[3], v[4]);
    const double2 x0 = v[0];
    // cosine parts: rows (c1 c2 c3), (c2 c3 c1), (c3 c1 c2)
    const double2 r1 = make_double2(fma(c3, a3.x, fma(c2, a2.x, fma(c1, a1.x, x0.x))),
                                    fma(c3, a3.y, fma(c2, a2.y, fma(c1, a1.y, x0.y))));
    const double2 r2 = make_double2(fma(c1, a3.x, fma(c3, a2.x, fma(c2, a1.x, x0.x))),
                                    fma(c1, a3.y, fma(c3, a2.y, fma(c2, a1.y, x0.y))));
    const double2 r3 = make_double2(fma(c2, a3.x, fma(c1, a2.x, fma(c3, a1.x, x0.x))),
                                    fma(c2, a3.y, fma(c1, a2.y, fma(c3, a1.y, x0.y))));
    // sine parts: rows (s1 s2 s3), (s2 -s3 -s1), (s3 -s1 s2), times -i
    // (forward) or +i (inverse)
    const double2 i1 = mul_mi<INV>(make_double2(fma(s3, d3.x, fma(s2, d2.x, s1 * d1.x)),
                                                fma(s3, d3.y, fma(s2, d2.y, s1 * d1.y))));
    const double2 i2 = mul_mi<INV>(make_double2(fma(-s1, d3.x, fma(-s3, d2.x, s2 * d1.x)),
                                                fma(-s1, d3.y, fma(-s3, d2.y, s2 * d1.y))));
    const double2 i3 = mul_mi<INV>(make_double2(fma(s2, d3.x, fma(-s1, d2.x, s3 * d1.x)),
                                                fma(s2, d3.y, fma(-s1, d2.y, s3 * d1.y))));
    v[0] = cadd(x0, cadd(a1, cadd(a2, a3)));
    v[1] = cadd(r1, i1);
    v[6] = csub(r1, i1);
    v[2] = cadd(r2, i2);
    v[5] = csub(r2, i2);
    v[3] = cadd(r3, i3);
    v[4] = csub(r3, i3);
}

template <bool INV>
__device__ __forceinline__ void dft4(double2* v)
{
    double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    double2 t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(double2* v)
{
    const double c = 0.70710678118654752440;
    double2 e[4] = {v[0], v[2], v[4], v[6]};
    double2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    if (!INV) {
        o[1] = make_double2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
        o[2] = make_double2(o[2].y, -o[2].x);
        o[3] = make_double2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
    } else {
        o[1] = make_double2(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y));
        o[2] = make_double2(-o[2].y, o[2].x);
        o[3] = make_double2(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y));
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        v[k] = cadd(e[k], o[k]);
        v[k + 4] = csub(e[k], o[k]);
    }
}

// v * exp(-+2 pi i M / 16) with the trivial factors done without products
template <int M, bool INV>
__device__ __forceinline__ double2 tw16(double2 v)
{
    constexpr int m = M & 15;
    constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
    constexpr double H = 0.70710678118654752440;   // cos(pi/4)
    constexpr double cs[16] = {1, C1, H, S1, 0, -S1, -H, -C1, -1, -C1, -H, -S1, 0, S1, H, C1};
    constexpr double cc = cs[m], sn = cs[(m + 12) & 15];  // cos(2 pi m/16), sin(2 pi m/16)
    if constexpr (m == 0) return v;
    else if constexpr (m == 4) return mul_mi<INV>(v);
    else if constexpr (m == 8) return make_double2(-v.x, -v.y);
    else if constexpr (m == 12) return mul_mi<!INV>(v);
    else {
        // forward: (cc - i sn) v; inverse: (cc + i sn) v
        const double s = INV ? sn : -sn;
        return make_double2(fma(cc, v.x, -s * v.y), fma(cc, v.y, s * v.x));
    }
}

// 16-point DFT as 4 x 4: inner DFT4 over n2 (n = n1 + 4 n2), twiddles
// w16^(n1 k2), outer DFT4 over n1; output index k2 + 4 k1.
template <bool INV>
__device__ __forceinline__ void dft16(double2* v)
{
    double2 y[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; n1++) {
        double2 t[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
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
        double2 t[4] = {y[0][k2], y[1][k2], y[2][k2], y[3][k2]};
        dft4<INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; k1++) v[k2 + 4 * k1] = t[k1];
    }
}

template <int R, bool INV, typename C>
__device__ __forceinline__ void dftR(C* v)
{
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 3) dft3<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 5) dft5<INV>(v);
    else if constexpr (R == 7) dft7<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
    else dft16<INV>(v);
}

// w^1 .. w^(R-1) from w: each power is one product of two earlier ones
// (error grows with log2 r, not r)
template <int R, typename C>
__device__ __forceinline__ void tw_powers(C w, C* pw)
{
    pw[1] = w;
#pragma unroll
    for (int r = 2; r < R; r++) pw[r] = cmul(pw[r / 2], pw[r - r / 2]);
}

// radix of the next stage given the remaining length: 16 and 8 first, so
// the first stage (which needs no twiddles) is the widest one and the small
// odd radices come last, where their twiddles are few (384-point K2 rows:
// 16, 8, 3 measured 5% faster than 3, 16, 8)
constexpr int pick_radix(int rem)
{
    return rem % 16 == 0  ? 16
           : rem % 8 == 0 ? 8
           : rem % 3 == 0 ? 3
           : rem % 5 == 0 ? 5
           : rem % 7 == 0 ? 7
           : rem % 4 == 0 ? 4
                          : 2;
}

// LDS tiles are padded by one element after every 2^PS (16 by default),
// which spreads the power-of-two strides of the Stockham stages over the
// LDS banks.
#ifndef TM_PAD_SHIFT
#define TM_PAD_SHIFT 4
#endif
// (PS: log2 of the elements between pads, 0 for none; per kernel)
template <int PS = TM_PAD_SHIFT>
__device__ __forceinline__ int pidx(int e) { return PS ? e + (e >> PS) : e; }
template <int PS = TM_PAD_SHIFT>
constexpr int padded(int n) { return PS ? n + (n >> PS) + 1 : n; }

// Element (j, c) of the tile: sequence c, position j.
//   COLS: sequences interleaved (index j*NB + c)  - column tiles
//   rows: sequences contiguous  (index c*RS + j)   - row tiles
template <bool COLS, int NB, int RS, int PS>
__device__ __forceinline__ int tile_addr(int j, int c)
{
    return pidx<PS>(COLS ? j * NB + c : c * RS + j);
}

// LDS twiddle table length for a sub-transform of length P, and lookup of
// exp(-2 pi i e / P), e < P.
constexpr int twl_size(int P) { return P % 2 == 0 ? P / 2 : P; }
template <int P, typename C>
__device__ __forceinline__ C tw_half(const C* twl, int e)
{
    if constexpr (P % 2 == 0) {
        const C w = twl[e < P / 2 ? e : e - P / 2];
        return e < P / 2 ? w : cneg(w);
    } else {
        return twl[e];
    }
}

// Stage twiddles: every one read from the LDS table (TM_TW_DIRECT=1, LDS
// reads for VALU work), or one read per butterfly and the others formed as
// its powers (0).
#ifndef TM_TW_DIRECT
#define TM_TW_DIRECT 0
#endif
constexpr bool TW_DIRECT = TM_TW_DIRECT != 0;

// Synchronisation between the read and write halves of a stage and between
// stages: the whole workgroup, or (WAVE) only the wavefront that owns the
// tile.  A wavefront's LDS operations execute in program order, so a tile
// transformed by one wavefront needs no hardware barrier: the fences keep
// the compiler from moving LDS accesses across the stage boundary.
template <bool WAVE>
__device__ __forceinline__ void stage_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One Stockham stage of radix R after NS points have been combined.  WAVE:
// the tile belongs to one wavefront (NT = 64, lanes as threads).
template <int P, int R, int NS, int NB, int NT, bool INV, bool COLS, int RS, int PS, bool WAVE, typename C>
__device__ __forceinline__ void fft_stage(C* buf, const C* twl)
{
    static_assert(!WAVE || NT == 64, "a wavefront tile has 64 threads");
    constexpr int BF = P / R;
    constexpr int TOT = BF * NB;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr uint32_t ESTEP = P / (NS * R);
    C v[PER][R];
    int jj[PER], cc[PER];
    const int tid = WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        int idx = tid + q * NT;
        jj[q] = COLS ? idx / NB : idx % BF;
        cc[q] = COLS ? idx % NB : idx / BF;
        if (TOT % NT == 0 || idx < TOT) {
#pragma unroll
            for (int r = 0; r < R; r++) v[q][r] = buf[tile_addr<COLS, NB, RS, PS>(jj[q] + r * BF, cc[q])];
        }
    }
    stage_sync<WAVE>();
#pragma unroll
    for (int q = 0; q < PER; q++) {
        int idx = tid + q * NT;
        if (TOT % NT == 0 || idx < TOT) {
            const int j = jj[q];
            const int k = (NS == 1) ? 0 : j % NS;
            if (NS > 1 && k != 0) {
                if constexpr (TW_DIRECT) {
                    // every twiddle read from the LDS table (r k ESTEP < P)
#pragma unroll
                    for (int r = 1; r < R; r++) {
                        const C w = tw_half<P>(twl, r * k * (int)ESTEP);
                        v[q][r] = cmul(v[q][r], INV ? cconj(w) : w);
                    }
                } else {
                    // one table read per butterfly, the other twiddles as powers
                    const C w1 = tw_half<P>(twl, k * ESTEP);
                    C pw[R];
                    tw_powers<R>(INV ? cconj(w1) : w1, pw);
#pragma unroll
                    for (int r = 1; r < R; r++) v[q][r] = cmul(v[q][r], pw[r]);
                }
            }
            dftR<R, INV>(v[q]);
            const int out = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; r++) buf[tile_addr<COLS, NB, RS, PS>(out + r * NS, cc[q])] = v[q][r];
        }
    }
    stage_sync<WAVE>();
}

template <int P, int NS, int NB, int NT, bool INV, bool COLS, int RS, int PS, bool WAVE, typename C>
__device__ __forceinline__ void fft_stages(C* buf, const C* twl)
{
    if constexpr (NS < P) {
        constexpr int R = pick_radix(P / NS);
        fft_stage<P, R, NS, NB, NT, INV, COLS, RS, PS, WAVE>(buf, twl);
        fft_stages<P, NS * R, NB, NT, INV, COLS, RS, PS, WAVE>(buf, twl);
    }
}

// Exchange of FP64 complex values between lanes of a wavefront, one 32-bit
// word at a time: HALVES swaps lanes 32..63 of a with lanes 0..31 of b
// (permlane32_swap), otherwise the odd 16-lane rows of a with the even rows
// of b (permlane16_swap).
template <bool HALVES>
__device__ __forceinline__ void lane_swap(double2& a, double2& b)
{
    uint32_t wa[4], wb[4];
    __builtin_memcpy(wa, &a, 16);
    __builtin_memcpy(wb, &b, 16);
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if constexpr (HALVES) {
            const auto r = __builtin_amdgcn_permlane32_swap(wa[i], wb[i], false, false);
            wa[i] = r[0];
            wb[i] = r[1];
        } else {
            const auto r = __builtin_amdgcn_permlane16_swap(wa[i], wb[i], false, false);
            wa[i] = r[0];
            wb[i] = r[1];
        }
    }
    __builtin_memcpy(&a, wa, 16);
    __builtin_memcpy(&b, wb, 16);
}

// 1024-point DFT of one LDS row by one wavefront, stages of radix 16, 16
// and 4.  The first exchange goes through LDS; the last stays in registers.
// After the second stage lane (a, k) = 16 a + k holds points 256 a + k +
// 16 r, r < 16, and the third stage's butterfly k + 16 r takes point r of
// the four lanes (a, k), a < 4: a 4 x 4 transpose of register blocks
// across the lane rows (permlane swaps on lane bit 5, then bit 4) gives
// lane (a, k) the inputs of butterflies k + 16 (4 q + a), q < 4.
template <bool INV, int PS>
__device__ __forceinline__ void row1024_wave(double2* buf, const double2* twl)
{
    constexpr int P = 1024;
    fft_stage<P, 16, 1, 1, 64, INV, false, P, PS, true>(buf, twl);
    const int lane = (int)(threadIdx.x & 63);
    const int k = lane & 15, a = lane >> 4;
    double2 y[16];
#pragma unroll
    for (int r = 0; r < 16; r++) y[r] = buf[pidx<PS>(lane + 64 * r)];
    if (k != 0) {
        const double2 w1 = tw_half<P>(twl, k * 4);
        double2 pw[16];
        tw_powers<16>(INV ? cconj(w1) : w1, pw);
#pragma unroll
        for (int r = 1; r < 16; r++) y[r] = cmul(y[r], pw[r]);
    }
    dftR<16, INV>(y);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        lane_swap<true>(y[4 * q], y[4 * q + 2]);
        lane_swap<true>(y[4 * q + 1], y[4 * q + 3]);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        lane_swap<false>(y[4 * q], y[4 * q + 1]);
        lane_swap<false>(y[4 * q + 2], y[4 * q + 3]);
    }
    stage_sync<true>();  // every read of the row precedes the writes below
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int j = k + 64 * q + 16 * a;
        double2* x = y + 4 * q;
        if (j != 0) {
            const double2 w1 = tw_half<P>(twl, j);
            double2 pw[4];
            tw_powers<4>(INV ? cconj(w1) : w1, pw);
#pragma unroll
            for (int e = 1; e < 4; e++) x[e] = cmul(x[e], pw[e]);
        }
        dftR<4, INV>(x);
#pragma unroll
        for (int e = 0; e < 4; e++) buf[pidx<PS>(j + 256 * e)] = x[e];
    }
    stage_sync<true>();
}

// In-place DFT of NB sequences of length P in LDS; twl is an LDS table of
// exp(-2 pi i e / P), e < P.  Caller must __syncthreads() before (data and
// table written); the routine ends with a barrier.
template <int P, int NB, int NT, bool INV, bool COLS, int RS = P, int PS = TM_PAD_SHIFT, bool WAVE = false,
          typename C>
__device__ __forceinline__ void tile_fft(C* buf, const C* twl)
{
    fft_stages<P, 1, NB, NT, INV, COLS, RS, PS, WAVE>(buf, twl);
}

// Copy the sub-transform table into LDS: the first half only when P is even
// (exp(-2 pi i (e + P/2) / P) = -exp(-2 pi i e / P)).
template <int P, int NT, typename C>
__device__ __forceinline__ void load_twl(C* twl, const double2* src)
{
    constexpr int H = twl_size(P);
#pragma unroll
    for (int q = 0; q < (H + NT - 1) / NT; q++) {
        const int e = threadIdx.x + q * NT;
        if (H % NT == 0 || e < H) twl[e] = to_elem<C>(src[e]);
    }
}

}  // namespace tmul
