// HIP kernels of the truncated / full product path (gfx950, FP64).
//
// One multiplication is four launches on one stream (six with the middle
// pass of the three-pass split):
//   K1 split + ring map + forward column pass   (Alg. low/high steps 2-3,
//      first half of the forward FFTs of step 4; Alg. full steps 2-3)
//   [k_mid_col forward middle pass]
//   K2 forward row pass, pointwise product, inverse row pass (step 4)
//   [k_mid_col inverse middle pass]
//   K3 inverse column pass                       (end of step 4)
//   K4 back-map, rounding, guard, carry propagation, extraction (steps 5-6)
//
// The real convolution of length N is computed with complex FFTs of length
// M = N/2: a real sequence G is packed as y_m = G_2m + i G_2m+1.  The two
// operands are transformed separately; their length-N real spectra are
// recovered from the bins k and M-k of the packed transforms, multiplied,
// and repacked for a length-M inverse, all in K2.  M = L1 * Lm * L2 is split
// four-step style: K1/K3 do the L1-point column DFTs (stride R = Lm L2), the
// middle pass the Lm-point DFTs inside each row, K2 the L2-point row DFTs;
// the spectrum stays in a "scrambled" order (row (k1, km), position k2
// holds bin k1 + L1 (km + Lm k2)), so no transpose pass exists.
//
// Build-time knobs (defaults are the measured best on MI355X): TM_NT1,
// TM_NT2, TM_NT3, TM_NT4, TM_NTM threads per workgroup of K1, K2, K3, K4 and
// the middle pass; TM_TILE1 / TM_TILE3 complex elements per K1 / K3 column
// tile; TM_DPT coefficients per K4 thread; TM_PAD_SHIFT LDS tile padding
// (TM_PAD_K2 for K2's row tiles); TM_K2_WAVE wavefront-owned 1024-point K2
// rows, TM_K2_SHUFFLE their last exchange by lane swaps; TM_K4_WAVES K4's
// register bound, TM_K4_PREV_TOP its carry from the previous workgroup's
// recomputed top limb, TM_K4_DPP its wavefront scans by DPP lane moves.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fft_tile.hpp"
#include "tmul.h"

namespace tmul {

enum { K_FULL = 0, K_LO = 1, K_HI = 2 };

#ifndef TM_NT2
#define TM_NT2 256
#endif
#ifndef TM_NTM
#define TM_NTM 256
#endif
constexpr int NT2 = TM_NT2;     // threads per K2 workgroup
constexpr int NTM = TM_NTM;     // threads per middle-pass workgroup
constexpr int LMAX = 9;         // largest supported series length lambda
#ifndef TM_NT4
#define TM_NT4 1024
#endif
#ifndef TM_PAD_K2
#define TM_PAD_K2 5
#endif
constexpr int PAD2 = TM_PAD_K2;  // K2 row tiles: one pad element per 32 (measured best)
#ifndef TM_K2_WAVE
#define TM_K2_WAVE 1
#endif
// K2 row transforms of 1024 points: one wavefront per row (measured 4%
// faster there; slower for 384- and 768-point rows, which keep the
// workgroup-wide transform)
constexpr bool K2_WAVE = TM_K2_WAVE != 0;
#ifndef TM_K2_SHUFFLE
#define TM_K2_SHUFFLE 1
#endif
// wavefront-owned 1024-point rows: the last Stockham exchange by lane swaps
// instead of LDS (FP64 tiles; full product's K2 at n = 2^30 3% faster)
constexpr bool K2_SHUFFLE = TM_K2_SHUFFLE != 0;
#ifndef TM_NT3
#define TM_NT3 256
#endif
#ifndef TM_DPT
#define TM_DPT 8
#endif
constexpr int DPT = TM_DPT;     // coefficients per thread in K4
constexpr int NT4 = TM_NT4;     // threads per K4 workgroup
constexpr int NT3 = TM_NT3;     // threads per K3 workgroup
constexpr int DPW = DPT * NT4;  // coefficients per workgroup in K4
#ifndef TM_K4_WAVES
#define TM_K4_WAVES 8
#endif
constexpr int K4_WAVES = TM_K4_WAVES;  // K4 register bound: waves per SIMD
#ifndef TM_K4_PREV_TOP
#define TM_K4_PREV_TOP 1
#endif
// K4: carry into a workgroup from the previous workgroup's recomputed top
// limb when that fixes it, before any look-back
constexpr bool K4_PREV_TOP = TM_K4_PREV_TOP != 0;
#ifndef TM_TILE1
#define TM_TILE1 4096
#endif
#ifndef TM_TILE3
#define TM_TILE3 4096
#endif
#ifndef TM_NT1
#define TM_NT1 256
#endif
constexpr int TILE1 = TM_TILE1;  // complex elements per K1 column tile
constexpr int TILE3 = TM_TILE3;  // complex elements per K3 column tile
constexpr int NT1 = TM_NT1;      // threads per K1 workgroup
constexpr uint32_t SPIN_LIMIT = 1u << 22;
constexpr int K4_HALO = 32;        // q values staged below a K4 workgroup's range
constexpr int64_t K4_CMAX = 1ll << 57;  // bound on the carries between limbs
// K4 staging index with one pad double after every 8: the per-thread runs
// of 8 coefficients then start 9 doubles apart, on different LDS banks
__host__ __device__ constexpr int padq(int e) { return e + (e >> 3); }

struct KParams {
    const uint64_t* u;
    const uint64_t* v;
    uint64_t* w;
    uint64_t n;         // operand bits
    uint64_t L;         // operand limbs
    int32_t b;          // digit bits
    int32_t lam;        // series length (truncated products)
    uint32_t N;         // real convolution length
    uint32_t digits;    // digits per operand (low: N, high: N+1, full: N/2)
    uint32_t M, L1, L2; // complex length and its split M = L1 * Lm * L2
    uint32_t Lm, R;     // middle pass length (1: two-pass) and row length R = Lm * L2
    uint32_t jmax;      // powers 2^-jb kept in the high-product wrap terms
    int64_t shift;      // high product: s = (N+1) b - n
    uint64_t off;       // output = bits [off, off+out_bits) of S
    uint64_t out_bits;
    uint64_t out_limbs;
    uint32_t ncoef;     // rounded coefficients (low N, high N+1, full N)
    uint32_t ncover;    // digit positions carried (multiple of DPW)
    uint32_t nstatus;   // K4 workgroups
    uint32_t fused;     // 1: K0 replaces K1, K2, K3 (small sizes)
    double invN, invM;
    double cf[LMAX];        // c_r of the forward map: alpha (-eps)^r/r!, gamma eps^r/r!
    double cb[LMAX];        // c_r of the back map: beta eps^r/r!, delta (-eps)^r/r!
    double nf[LMAX][2];     // forward map in nested form: factor nf[r][0] y + nf[r][1]
    double nb[LMAX][2];     // back map as a chain: factor nb[r][0] x + nb[r][1]
    double bscale;          // 2^b / M (truncated products), 1 / M (full product)
    double2* za;        // operand u spectrum / convolution result
    double2* zb;        // operand v spectrum
    uint64_t* status;   // K4 look-back records, 2 words each
    uint32_t* ticket;   // K4 dynamic workgroup counter
    tm_guard* guard;
    double* theta;      // high product: theta_U, theta_V (written by K1)
    Tw tw;
    const double2* tw1; // exp(-2 pi i e / L1), e < L1
    const double2* tw2; // exp(-2 pi i e / L2), e < L2
    const double2* twm; // exp(-2 pi i e / Lm), e < Lm
    int64_t* dbg_c;     // diagnostic outputs (tm_coefficients) or null
    double* dbg_x;
};

// ------------------------------------------------------- workgroup indices

// A workgroup's position in its own multiplication's grid.  A plain launch
// takes it from the hardware ids; a packed launch (several multiplications
// in one 1-D grid) from its request's entry in the group table.
struct Blk {
    uint32_t x, y, z;  // workgroup index
    uint32_t nx, ny;   // grid extent in x and y
};

__device__ __forceinline__ Blk blk_hw()
{
    return Blk{blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gridDim.y};
}

// One entry per request of a packed launch: its first workgroup in the 1-D
// grid, its own grid extent (nx, ny; nz follows from the block count) and
// the index of its parameters.  Entries are in increasing `start` order,
// start[0] = 0, at most 64 per launch.
struct GroupEnt {
    uint32_t start, nx, ny, pi;
};
struct Group {
    const KParams* ps;
    const GroupEnt* ent;
    uint32_t nr;
};
constexpr int GROUP_MAX = 64;

// The group table is written by the host before the launch and only read by
// the kernels, so its uniform entry is loaded through the constant address
// space (a scalar load).
typedef const __attribute__((address_space(4))) GroupEnt* GroupEntC;

// Parameters of request pi of a packed launch, read in place (a private
// copy would go to scratch memory where the maps index its tables).
__device__ __forceinline__ const KParams& group_params(const Group& g, uint32_t pi)
{
    return g.ps[pi];
}

// The request of this workgroup: one entry per lane, a ballot of the
// entries that start at or before this workgroup, and the last of them.
__device__ __forceinline__ Blk group_block(const Group& g, uint32_t& pi)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t st = lane < g.nr ? g.ent[lane].start : 0xffffffffu;
    const uint64_t m = __ballot(st <= blockIdx.x);
    const uint32_t r = (uint32_t)__builtin_amdgcn_readfirstlane(__popcll(m) - 1);
#if defined(__HIP_DEVICE_COMPILE__)
    const GroupEnt e = ((GroupEntC)g.ent)[r];
#else
    const GroupEnt e = g.ent[r];
#endif
    const uint32_t local = blockIdx.x - e.start;
    Blk b;
    b.nx = e.nx;
    b.ny = e.ny;
    b.x = local % e.nx;
    b.y = (local / e.nx) % e.ny;
    b.z = local / (e.nx * e.ny);
    pi = e.pi;
    return b;
}

// ---------------------------------------------------------------- digits

// bits [pos, pos+nb) of (x mod 2^n); positions outside [0, n) read as zero
__device__ __forceinline__ uint64_t get_bits(const uint64_t* x, uint64_t L, uint64_t n,
                                             int64_t pos, int nb)
{
    if (pos >= (int64_t)n || pos + nb <= 0) return 0;
    const int64_t p0 = pos < 0 ? 0 : pos;
    const uint64_t li = (uint64_t)p0 >> 6;
    const int sh = (int)(p0 & 63);
    uint64_t lo = x[li];
    uint64_t hi = (li + 1 < L) ? x[li + 1] : 0;
    uint64_t w = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
    int64_t end = pos + nb < (int64_t)n ? pos + nb : (int64_t)n;
    int cnt = (int)(end - p0);
    if (cnt < 64) w &= (1ull << cnt) - 1;
    return w << (p0 - pos);
}

// Balanced digit i of x 2^shift (signed digits of Section 5):
// U_i = d_i - 2^b [d_i >= 2^(b-1)] + [d_(i-1) >= 2^(b-1)]; the top digit
// (i = ndig-1) keeps its carry when top_keep.
__device__ __forceinline__ int64_t bal_digit(const KParams& p, const uint64_t* x, int64_t i,
                                             uint32_t ndig, bool top_keep)
{
    const int b = p.b;
    uint64_t w = get_bits(x, p.L, p.n, (i - 1) * b - p.shift, 2 * b);
    const int64_t mask = (1ll << b) - 1, h = 1ll << (b - 1);
    int64_t dprev = (int64_t)(w & mask);
    int64_t d = (int64_t)(w >> b);
    int64_t cin = dprev >= h ? 1 : 0;
    if (top_keep && i == (int64_t)ndig - 1) return d + cin;
    return d - (d >= h ? (1ll << b) : 0) + cin;
}

// Series coefficients (Sections 3.2 and 4.2) with eps = 2^-b, x = k/N and
// the (k + r) factor of the binomial definitions cancelled:
//   alpha_{k,r} = c_r x prod_{j=1}^{r-1} ((k+r)/N - j),  c_r = (-eps)^r / r!
//   gamma_{k,r} = c_r x prod_{j=1}^{r-1} ((k+r)/N + j),  c_r =   eps^r  / r!
//   beta_{k,r}  = c_r prod_{j=0}^{r-1} (x + j),          c_r =   eps^r  / r!
//   delta_{k,r} = c_r prod_{j=0}^{r-1} (x - j),          c_r = (-eps)^r / r!
// These product forms serve the few indices next to the cyclic wrap; the
// bulk of both maps uses the factored forms of row_map_fast / back_chain.
template <int KIND>
__device__ __forceinline__ double coef_fwd(const KParams& p, uint32_t k, int r)
{
    if (r == 0) return 1.0;
    const double x = (double)k * p.invN, y = (double)(k + (uint32_t)r) * p.invN;
    double v = x * p.cf[r];
    for (int j = 1; j < r; j++) v *= KIND == K_LO ? y - (double)j : y + (double)j;
    return v;
}

template <int KIND>
__device__ __forceinline__ double coef_back(const KParams& p, uint32_t k, int r)
{
    if (r == 0) return 1.0;
    const double x = (double)k * p.invN;
    double v = p.cb[r];
    for (int j = 0; j < r; j++) v *= KIND == K_LO ? x + (double)j : x - (double)j;
    return v;
}

// Clear the per-call state that K4 accumulates into (guard, look-back
// records, ticket, and the output limbs K4 ORs into).  Done by K1.
// K4 workgroup g owns limbs [g LPW, (g+1) LPW) of S (LPW = DPW b / 64) and
// writes output limb i (bits [64 i + off, 64 i + off + 64) of S) with a
// plain store when those bits lie in its own limbs.  Only three kinds of
// output limb are OR-ed and need a zero start: one that straddles two
// workgroups (off not a multiple of 64 and S limb i + off/64 + 1 a
// multiple of LPW), the last limb when it is partial, and any limb beyond
// the workgroups' limbs.
__device__ __forceinline__ void clear_state(const KParams& p, uint32_t gid, uint32_t gsize)
{
    const uint64_t lpw = (uint64_t)(DPW / 64) * (uint64_t)p.b;
    const uint64_t q = p.off >> 6;
    if (p.off & 63) {
        for (uint64_t j = 1 + gid; j <= p.nstatus; j += gsize) {
            const uint64_t s1 = j * lpw;  // S limb above the boundary
            if (s1 >= q + 1 && s1 - q - 1 < p.out_limbs) p.w[s1 - q - 1] = 0;
        }
    }
    const uint64_t covered = (uint64_t)p.nstatus * lpw;  // S limbs written by K4
    const uint64_t first_out = covered > q + 1 ? covered - q - 1 : 0;
    for (uint64_t i = first_out + gid; i < p.out_limbs; i += gsize) p.w[i] = 0;
    if (gid == 0 && (p.out_bits & 63) && p.out_limbs) p.w[p.out_limbs - 1] = 0;
    for (uint64_t i = gid; i < 2ull * p.nstatus; i += gsize) p.status[i] = 0;
    if (gid == 0) {
        *p.ticket = 0;
        tm_guard g;
        g.max_dist = 0.0;
        g.max_abs = 0.0;
        g.flags = 0;
        g.b = (uint32_t)p.b;
        g.lambda = (uint32_t)p.lam;
        g.kind = 0;
        g.N = p.N;
        *p.guard = g;
    }
}

// ------------------------------------------------------------------- K1

// Column tiles c and c+1 share 128-byte lines (W complex doubles = 16 W
// bytes per row segment).  Workgroups are dispatched round-robin over the 8
// XCDs, each with its own L2; map workgroup id -> tile so that consecutive
// tiles run on the same XCD and a line is fetched once.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t ntiles)
{
    if (ntiles % 8 != 0) return bid;
    return (bid % 8) * (ntiles / 8) + bid / 8;
}

// Digits of one K1 tile row.  A row holds complex points m0 .. m0+W-1, i.e.
// reals 2 m0 .. 2 m0 + 2W - 1; the truncated products' stencil also reads
// the LB - 1 digits below, LB being the largest series length an instance
// serves (LB_FIXED for the instances with a compile-time digit size B,
// LMAX for the generic ones).  The limbs under every row of a tile are
// staged in LDS once; digits are cut from there.
constexpr int LB_FIXED = 7;
constexpr int k1_lb(int KIND, int B) { return KIND == K_FULL ? 1 : B ? LB_FIXED : LMAX; }
constexpr int k1_lo(int KIND, int B) { return k1_lb(KIND, B) - 1; }
constexpr int k1_nd(int W, int KIND, int B) { return 2 * W + k1_lo(KIND, B); }
constexpr int k1_nlw(int ND, int B)
{
    return B ? ((ND + 1) * B + 64 + 63) / 64 : ((ND + 1) * 16 + 63) / 64 + 1;
}

template <int NLW>
__device__ __forceinline__ uint64_t pick_limb(const uint64_t (&lim)[NLW], int i)
{
    uint64_t r = 0;
#pragma unroll
    for (int k = 0; k < NLW; k++) r = (k == i) ? lim[k] : r;
    return r;
}

// Window start of a row: first field at bit p0 = (kf - 1) b - shift, limb
// l0 = floor(p0 / 64), relative offset rel0 = p0 - 64 l0.
__device__ __forceinline__ void row_window(const KParams& p, int64_t kf, int64_t& l0, int& rel0)
{
    const int64_t p0 = (kf - 1) * p.b - p.shift;
    l0 = p0 >= 0 ? p0 >> 6 : -((63 - p0) >> 6);
    rel0 = (int)(p0 - l0 * 64);
}

// limb li of x mod 2^n (zero outside [0, L))
__device__ __forceinline__ uint64_t limb_at(const KParams& p, const uint64_t* x, int64_t li)
{
    uint64_t v = (li >= 0 && li < (int64_t)p.L) ? x[li] : 0;
    if (li == (int64_t)p.L - 1 && (p.n & 63)) v &= (1ull << (p.n & 63)) - 1;
    return v;
}

// Balanced digits from the b-bit fields f_i = d_(kf-1+i) of a window:
// U = d - 2^b [d >= 2^(b-1)] + [d_prev >= 2^(b-1)], i.e. the field read as
// a signed b-bit number plus the sign bit of the field below.

// Compile-time digit size B: the window is aligned once (funnel shifts by
// the row's bit offset), then every field sits at a fixed bit position.
template <int ND, int B, int NLW>
__device__ __forceinline__ void row_digits_fixed(const uint64_t* slimb, int rel0, int32_t (&d)[ND])
{
    constexpr int NF = ND + 1;
    constexpr int NA = (NF * B + 31) / 32;
    static_assert(NA + 2 <= 2 * NLW, "staged window too short");
    uint32_t w[2 * NLW];
#pragma unroll
    for (int i = 0; i < NLW; i++) {
        const uint64_t l = slimb[i];
        w[2 * i] = (uint32_t)l;
        w[2 * i + 1] = (uint32_t)(l >> 32);
    }
    const bool odd = rel0 >= 32;
    const uint32_t sh = (uint32_t)rel0 & 31u;
    uint32_t a[NA + 1];
#pragma unroll
    for (int k = 0; k <= NA; k++) a[k] = odd ? w[k + 1] : w[k];
#pragma unroll
    for (int k = 0; k < NA; k++) a[k] = __builtin_amdgcn_alignbit(a[k + 1], a[k], sh);
    int32_t f[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) {
        const int pos = i * B, wi = pos >> 5, o = pos & 31;
        const uint32_t v = o + B <= 32 ? a[wi] >> o : __builtin_amdgcn_alignbit(a[wi + 1], a[wi], o);
        f[i] = (int32_t)(v << (32 - B)) >> (32 - B);
    }
#pragma unroll
    for (int t = 0; t < ND; t++) d[t] = f[t + 1] + (int32_t)((uint32_t)f[t] >> 31);
}

// Runtime digit size, staged window.
template <int ND>
__device__ __forceinline__ void row_digits_var(const KParams& p, const uint64_t* slimb, int rel0,
                                               int32_t (&d)[ND])
{
    const int b = p.b;
    const int64_t mask = (1ll << b) - 1, h = 1ll << (b - 1);
#pragma unroll
    for (int t = 0; t < ND; t++) {
        const int rel = rel0 + t * b;
        const int li = rel >> 6, sh = rel & 63;
        const uint64_t lo = slimb[li], hi = slimb[li + 1];
        const uint64_t w = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
        const int64_t dprev = (int64_t)(w & mask), dd = (int64_t)((w >> b) & mask);
        d[t] = (int32_t)(dd - (dd >= h ? (1ll << b) : 0) + (dprev >= h ? 1 : 0));
    }
}

// Runtime digit size, limbs fetched into registers (tiles too small to
// stage the limbs).
template <int ND>
__device__ __forceinline__ void row_digits_reg(const KParams& p, const uint64_t* x, int64_t kf,
                                               int32_t (&d)[ND])
{
    constexpr int NLW = k1_nlw(ND, 0);
    const int b = p.b;
    int64_t l0;
    int rel0;
    row_window(p, kf, l0, rel0);
    uint64_t lim[NLW];
#pragma unroll
    for (int i = 0; i < NLW; i++) lim[i] = limb_at(p, x, l0 + i);
    const int64_t mask = (1ll << b) - 1, h = 1ll << (b - 1);
#pragma unroll
    for (int t = 0; t < ND; t++) {
        const int rel = rel0 + t * b;
        const int li = rel >> 6, sh = rel & 63;
        const uint64_t lo = pick_limb(lim, li), hi = pick_limb(lim, li + 1);
        const uint64_t w = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
        const int64_t dprev = (int64_t)(w & mask), dd = (int64_t)((w >> b) & mask);
        d[t] = (int32_t)(dd - (dd >= h ? (1ll << b) : 0) + (dprev >= h ? 1 : 0));
    }
}

// Digits of a row that touches index 0 or the top: cyclic mod N for the
// truncated products (their digits are all of the plain kind below N); for
// the full product the top digit keeps its carry and indices >= digits are
// zero.
template <int ND, int KIND>
__device__ __forceinline__ void row_digits_edge(const KParams& p, const uint64_t* x, int64_t kf,
                                                int32_t (&d)[ND])
{
    const int64_t top = (int64_t)p.digits - 1;
#pragma unroll
    for (int t = 0; t < ND; t++) {
        int64_t k = kf + t;
        if (KIND == K_FULL) {
            d[t] = (k >= 0 && k <= top) ? (int32_t)bal_digit(p, x, k, p.digits, true) : 0;
        } else {
            if (k < 0) k += p.N;
            d[t] = (int32_t)bal_digit(p, x, k, p.digits, false);
        }
    }
}

// G_j, j = j0 .. j0 + 2W - 1 (j0 = kf + LB - 1), away from the wrap:
//   low:  G = alpha* U  (Prop. approximating alpha*),
//   high: G = gamma* F' (Prop. approximating gamma-dagger; F'_k = F_k for
//         k >= jmax).
// With y = j/N the coefficient alpha_{j-r,r} = c_r x_(j-r) pi_(r-1)(y),
// pi_m(y) = prod_{i=1}^m (y - i) (gamma: y + i), so with V_k = x_k U_k
//   G_j = U_j + c_1 (V_(j-1) + k_1 (y -+ 1) (V_(j-2) + k_2 (y -+ 2) (...)))
// where k_r = c_(r+1) / c_r: two FMAs per series term.  The host zeroes
// the factors from r = lam - 1 on, which cuts the nest at the plan's lam.
template <int W, int ND, int LB>
__device__ __forceinline__ void row_map_fast(const KParams& p, int64_t kf, const int32_t (&d)[ND],
                                             double2* g)
{
    constexpr int LO = LB - 1;
    static_assert(ND == 2 * W + LO, "row digits");
    double v[ND];
    const double x0 = (double)kf * p.invN;
#pragma unroll
    for (int i = 0; i < ND; i++) v[i] = fma((double)i, p.invN, x0) * (double)d[i];
    const double y0 = (double)(kf + LO) * p.invN;
    double o[2 * W];
#pragma unroll
    for (int t = 0; t < 2 * W; t++) {
        const double y = fma((double)t, p.invN, y0);
        double s = v[t];
#pragma unroll
        for (int r = LB - 2; r >= 1; r--) s = fma(fma(p.nf[r][0], y, p.nf[r][1]), s, v[t + LO - r]);
        o[t] = fma(p.cf[1], s, (double)d[t + LO]);
    }
#pragma unroll
    for (int c = 0; c < W; c++) g[c] = make_double2(o[2 * c], o[2 * c + 1]);
}

// The same maps term by term, for rows next to the wrap: cyclic indices,
// and for the high product F'_k = F_k + 2^(-kb) F_N (F mod C by eq.
// reduction-modC with rho ~ 2^b).
template <int W, int KIND, int ND, int LB>
__device__ __forceinline__ void row_map_edge(const KParams& p, uint32_t m0, double FN,
                                             const int32_t (&d)[ND], double2* g)
{
    constexpr int LO = LB - 1;
    const uint32_t N = p.N;
#pragma unroll
    for (int c = 0; c < W; c++) {
        double s[2] = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < 2; e++) {
            const uint32_t j = 2 * m0 + 2 * c + e;
#pragma unroll
            for (int r = 0; r < LB; r++) {
                if (r < p.lam) {
                    const uint32_t k = j >= (uint32_t)r ? j - r : j + N - r;
                    double f = (double)d[2 * c + e - r + LO];
                    if (KIND == K_HI && k < p.jmax) f += ldexp(FN, -(int)k * p.b);
                    s[e] = fma(coef_fwd<KIND>(p, k, r), f, s[e]);
                }
            }
        }
        g[c] = make_double2(s[0], s[1]);
    }
}

// K1: split + map + column FFT for one column tile of the L1 x R matrix
// (M = L1 R, R = Lm L2; element (k1, col) is point m = k1 R + col).
// B: compile-time digit size (0: runtime p.b).
template <int L1, int W, int KIND, int B, typename C = double2>
__device__ __forceinline__ void k1_body(const KParams& p, const Blk bk)
{
    static_assert(L1 * W <= TILE1, "tile too large");
    constexpr int PER = (L1 * W + NT1 - 1) / NT1;
    constexpr int LB = k1_lb(KIND, B), LO = LB - 1, ND = k1_nd(W, KIND, B), NLW = k1_nlw(ND, B);
    constexpr int TE = padded(L1 * W);
    // limb windows staged in the tile area when they fit
    // staged rows are NLWP limbs apart: an odd stride puts the rows that
    // neighbouring lanes read on different LDS banks
    constexpr int NLWP = NLW | 1;
    constexpr bool STAGE = L1 * NLWP * 8 <= TE * 16;
    static_assert(STAGE || B == 0, "compile-time digit sizes need staged limbs");
    constexpr int RPT = (L1 + NT1 - 1) / NT1;
    __shared__ C tile[TE];
    __shared__ C twl[twl_size(L1)];
    __shared__ double s_th[LMAX + 8];  // terms of theta (high product, tile 0)
    const int op = bk.y;
    const uint64_t* x = op ? p.v : p.u;
    C* dst = reinterpret_cast<C*>(op ? p.zb : p.za);
    const uint32_t L2 = p.R;  // row length of the L1 x R matrix
    const uint32_t c0 = xcd_tile(bk.x, bk.nx) * W;
    const int tid = threadIdx.x;

    load_twl<L1, NT1>(twl, p.tw1);
    // inter-pass twiddles exp(-2 pi i col k1 / M): this thread's elements
    // share col = c0 + tid % W and step k1 by NT1 / W
    static_assert(NT1 % W == 0, "W must divide NT1");
    const uint32_t colt = c0 + tid % W;
    const uint32_t eb = (uint32_t)((uint64_t)colt * (uint32_t)(tid / W) % p.M);
    const uint32_t es = (uint32_t)((uint64_t)colt * (uint32_t)(NT1 / W) % p.M);
    const double2 tb0 = p.tw.lo[eb & p.tw.mask], tb1 = p.tw.hi[eb >> p.tw.shift];
    const double2 ts0 = p.tw.lo[es & p.tw.mask], ts1 = p.tw.hi[es >> p.tw.shift];
    if (op == 0) clear_state(p, bk.x * NT1 + tid, bk.nx * NT1);
    if (KIND == K_HI && bk.x == 0 && tid <= (int)p.jmax && tid <= (int)p.N)
        s_th[tid] = ldexp((double)bal_digit(p, x, (int64_t)p.N - tid, p.digits, true), -tid * p.b);
    // When a row of the tile spans a whole number of limbs (2 R b bits a
    // multiple of 64), every row's digit window starts at the same bit
    // offset rel_u and row j1's window at limb l_u + j1 (2 R b / 64).
    int64_t l_u;
    int rel_u;
    row_window(p, 2 * (int64_t)c0 - LO, l_u, rel_u);
    const uint64_t row_bits = 2ull * L2 * (uint64_t)(B ? B : p.b);
    const int64_t row_limbs = (int64_t)(row_bits >> 6);
    // ... and if every staged limb lies below the operand's top limb, no
    // bounds checks or top-limb mask are needed
    const bool inner = (row_bits & 63) == 0 && l_u >= 0 && l_u + (L1 - 1) * row_limbs + NLW < (int64_t)p.L;
    if constexpr (STAGE) {
        uint64_t* slimb = reinterpret_cast<uint64_t*>(tile);
        constexpr int PL = (L1 * NLW + NT1 - 1) / NT1;
        uint64_t lv[PL];
        if (inner) {
#pragma unroll
            for (int q = 0; q < PL; q++) {
                const int e = tid + q * NT1;
                if (L1 * NLW % NT1 == 0 || e < L1 * NLW) lv[q] = x[l_u + (e / NLW) * row_limbs + e % NLW];
            }
        } else {
#pragma unroll
            for (int q = 0; q < PL; q++) {
                const int e = tid + q * NT1;
                if (L1 * NLW % NT1 == 0 || e < L1 * NLW) {
                    const int row = e / NLW, i = e % NLW;
                    int64_t l0;
                    int rel0;
                    row_window(p, 2 * ((int64_t)row * L2 + c0) - LO, l0, rel0);
                    lv[q] = limb_at(p, x, l0 + i);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < PL; q++) {
            const int e = tid + q * NT1;
            if (L1 * NLW % NT1 == 0 || e < L1 * NLW) slimb[(e / NLW) * NLWP + e % NLW] = lv[q];
        }
    }
    // Row 0 of tile 0 of a truncated product touches index 0: its map takes
    // the term-by-term form with cyclic indices.  Its digits are read here,
    // one per thread, while the staging loads are in flight, and its 2W
    // outputs are formed by 2W threads below (one thread doing all of them
    // cost about 5 us at n = 2^16).
    const bool erow = KIND != K_FULL && c0 == 0;
    __shared__ int32_t s_ed[ND];
    __shared__ double s_efn;
    __shared__ double s_eo[2 * W];
    static_assert(2 * W <= NT1 && ND < NT1, "one thread per edge digit and output");
    if (erow) {
        if (tid < ND) {
            int64_t k = tid - (int64_t)LO;  // kf + tid with kf = -LO
            if (k < 0) k += p.N;
            s_ed[tid] = (int32_t)bal_digit(p, x, k, p.digits, false);
        }
        if (KIND == K_HI && tid == ND) s_efn = (double)bal_digit(p, x, p.N, p.digits, true);
    }
    __syncthreads();
    if (KIND == K_HI && bk.x == 0 && tid == 0) {
        // theta = rho^-N F(rho), rho ~ 2^b: sum_j 2^(-jb) F_(N-j), j <= jmax
        double th = 0.0;
        for (int j = 0; j <= (int)p.jmax && j <= (int)p.N; j++) th += s_th[j];
        p.theta[op] = th;
        if (bk.ny == 1) p.theta[1] = th;  // squaring: theta_V = theta_U
    }
    // rows away from index 0 (and, for the full product, from the top digit)
    // take the fast path; the others the term-by-term one
    const int64_t kf_min = KIND == K_HI ? (int64_t)p.jmax : 0;
    const int64_t top = (int64_t)p.digits - 1;
    if (erow && tid < 2 * W) {
        // output j = tid of the row, as row_map_edge forms it
        const uint32_t j = (uint32_t)tid;
        double sj = 0.0;
#pragma unroll
        for (int r = 0; r < LB; r++) {
            if (r < p.lam) {
                const uint32_t k = j >= (uint32_t)r ? j - r : j + p.N - r;
                double f = (double)s_ed[tid - r + LO];
                if (KIND == K_HI && k < p.jmax) f += ldexp(s_efn, -(int)k * p.b);
                sj = fma(coef_fwd<KIND>(p, k, r), f, sj);
            }
        }
        s_eo[tid] = sj;
    }
    double2 g[RPT][W];
#pragma unroll
    for (int rr = 0; rr < RPT; rr++) {
        const int j1 = tid + rr * NT1;
        if ((L1 % NT1 == 0 || j1 < L1) && !(erow && j1 == 0)) {
            const uint32_t m0 = (uint32_t)j1 * L2 + c0;
            const int64_t kf = 2 * (int64_t)m0 - LO;
            const bool fast = kf >= kf_min && (KIND != K_FULL || kf + ND <= top);
            int32_t d[ND];
            if (fast) {
                if constexpr (STAGE) {
                    int64_t l0;
                    int rel0 = rel_u;
                    if (!inner) row_window(p, kf, l0, rel0);
                    const uint64_t* sl = reinterpret_cast<const uint64_t*>(tile) + j1 * NLWP;
                    if constexpr (B > 0)
                        row_digits_fixed<ND, B, NLW>(sl, rel0, d);
                    else
                        row_digits_var<ND>(p, sl, rel0, d);
                } else {
                    row_digits_reg<ND>(p, x, kf, d);
                }
                if constexpr (KIND == K_FULL) {
#pragma unroll
                    for (int c = 0; c < W; c++)
                        g[rr][c] = make_double2((double)d[2 * c], (double)d[2 * c + 1]);
                } else {
                    row_map_fast<W, ND, LB>(p, kf, d, g[rr]);
                }
            } else {
                row_digits_edge<ND, KIND>(p, x, kf, d);
                if constexpr (KIND == K_FULL) {
#pragma unroll
                    for (int c = 0; c < W; c++)
                        g[rr][c] = make_double2((double)d[2 * c], (double)d[2 * c + 1]);
                } else {
                    const double FN = KIND == K_HI ? (double)bal_digit(p, x, p.N, p.digits, true) : 0.0;
                    row_map_edge<W, KIND, ND, LB>(p, m0, FN, d, g[rr]);
                }
            }
        }
    }
    if (STAGE || erow) __syncthreads();
#pragma unroll
    for (int rr = 0; rr < RPT; rr++) {
        const int j1 = tid + rr * NT1;
        if ((L1 % NT1 == 0 || j1 < L1) && !(erow && j1 == 0)) {
#pragma unroll
            for (int c = 0; c < W; c++) tile[pidx(j1 * W + c)] = to_elem<C>(g[rr][c]);
        }
    }
    if (erow && tid < W) tile[pidx(tid)] = to_elem<C>(make_double2(s_eo[2 * tid], s_eo[2 * tid + 1]));
    __syncthreads();
    tile_fft<L1, W, NT1, false, true>(tile, twl);
    TwSeq<PER, C> tws;
    tws.init(cmul(tb0, tb1), cmul(ts0, ts1));
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int e = tid + q * NT1;
        if (L1 * W % NT1 == 0 || e < L1 * W) {
            const int k1 = e / W;
            dst[(size_t)k1 * L2 + colt] = cmul(tile[pidx(e)], tws.at(q));
        }
    }
}

template <int L1, int W, int KIND, int B, typename C = double2>
__global__ __launch_bounds__(NT1) void k1_split_map_col(KParams p)
{
    k1_body<L1, W, KIND, B, C>(p, blk_hw());
}

template <int L1, int W, int KIND, int B>
__global__ __launch_bounds__(NT1) void k1_split_map_col_g(Group g)
{
    uint32_t pi;
    const Blk bk = group_block(g, pi);
    const KParams& p = group_params(g, pi);
    k1_body<L1, W, KIND, B>(p, bk);
}

// ------------------------------------------------------------------- K2

// Spectra of the two real operands from the packed transforms, product, and
// repacking for the half-length inverse.  With Y the packed transform and
// M - k the mirror bin: E_k = (Y_k + conj Y_(M-k))/2, O_k = (Y_k - conj
// Y_(M-k))/(2i) (even / odd sample spectra); the product spectrum's even
// and odd parts are E'_k = Ea Eb + w^k Oa Ob and O'_k = Ea Ob + Oa Eb with
// w = exp(-2 pi i / M), and Q_k = E'_k + i O'_k is the length-M transform of
// (W_2m + i W_2m+1) (times M).
template <typename C>
__device__ __forceinline__ C pointwise_bin(C Ya, C Yam, C Yb, C Ybm, C wk)
{
    C Ea = cscale(cadd(Ya, cconj(Yam)), 0.5);
    C Oa = cscale(csub(Ya, cconj(Yam)), 0.5);
    Oa = mul_mi<false>(Oa);  // divide by i
    C Eb = cscale(cadd(Yb, cconj(Ybm)), 0.5);
    C Ob = cscale(csub(Yb, cconj(Ybm)), 0.5);
    Ob = mul_mi<false>(Ob);
    C X = cadd(cmul(Ea, Eb), cmul(wk, cmul(Oa, Ob)));
    C Yv = cadd(cmul(Ea, Ob), cmul(Oa, Eb));
    return cadd(X, mul_mi<true>(Yv));  // X + i Yv
}

// A bin and its mirror from one unpacking: the mirror's even and odd
// spectra are the conjugates of the bin's and so is its twiddle
// (w^(M-k) = conj w^k), so its X and Yv are the conjugates too.
template <typename C>
__device__ __forceinline__ void pointwise_pair(C Ya, C Yam, C Yb, C Ybm, C wk, C& q, C& qm)
{
    C Ea = cscale(cadd(Ya, cconj(Yam)), 0.5);
    C Oa = cscale(csub(Ya, cconj(Yam)), 0.5);
    Oa = mul_mi<false>(Oa);
    C Eb = cscale(cadd(Yb, cconj(Ybm)), 0.5);
    C Ob = cscale(csub(Yb, cconj(Ybm)), 0.5);
    Ob = mul_mi<false>(Ob);
    C X = cadd(cmul(Ea, Eb), cmul(wk, cmul(Oa, Ob)));
    C Yv = cadd(cmul(Ea, Ob), cmul(Oa, Eb));
    q = cadd(X, mul_mi<true>(Yv));
    qm = cadd(cconj(X), mul_mi<true>(cconj(Yv)));
}

// Row pairs of K2.  Row (k1, km) (k1 < L1, km < Lm) holds bins
// k = k1 + L1 (km + Lm k2), k2 < L2, at positions ((k1 Lm + km) L2 + k2).
// The mirror bin M - k lies in row (L1 - k1, Lm - 1 - km) at L2 - 1 - k2 when
// k1 != 0, in row (0, Lm - km) at L2 - 1 - k2 when k1 = 0 and km != 0, and
// row (0, 0) is its own mirror with k2 -> (L2 - k2) mod L2.  Besides (0, 0),
// one more row is its own mirror: (0, Lm/2) for even Lm, else (L1/2,
// (Lm-1)/2) for even L1 (none when both are odd).  Workgroup g < G-1 takes
// the g-th row of a pair of distinct rows whose index does not exceed its
// mirror's (A rows with 0 < k1 < L1/2, B with k1 = L1/2, C with k1 = 0);
// the last workgroup takes both self-mirrored rows, so that no workgroup
// loads a row twice.
struct K2Rows {
    uint32_t rowa, rowb;  // row indices k1 Lm + km of the two rows
    uint32_t rhoa, rhob;  // their first bins k1 + L1 km
    bool self;            // each row is its own mirror
};

__host__ __device__ inline uint32_t k2_groups(uint32_t L1, uint32_t Lm)
{
    const uint32_t A = (L1 - 1) / 2 * Lm;
    const uint32_t B = L1 % 2 == 0 ? Lm / 2 : 0;
    return A + B + (Lm - 1) / 2 + 1;
}

__device__ __forceinline__ K2Rows k2_rows_of(uint32_t g, uint32_t L1, uint32_t Lm)
{
    const uint32_t A = (L1 - 1) / 2 * Lm;
    const uint32_t B = L1 % 2 == 0 ? Lm / 2 : 0;
    const uint32_t C = (Lm - 1) / 2;
    K2Rows r;
    r.self = g >= A + B + C;
    uint32_t k1, km, k1m, kmm;
    if (r.self) {
        k1 = km = 0;
        if (Lm % 2 == 0) {
            k1m = 0;
            kmm = Lm / 2;
        } else if (L1 % 2 == 0) {
            k1m = L1 / 2;
            kmm = (Lm - 1) / 2;
        } else {
            k1m = kmm = 0;
        }
    } else {
        if (g < A) {
            k1 = 1 + g / Lm;
            km = g % Lm;
        } else if (g < A + B) {
            k1 = L1 / 2;
            km = g - A;
        } else {
            k1 = 0;
            km = 1 + (g - A - B);
        }
        k1m = k1 ? L1 - k1 : 0;
        kmm = k1 ? Lm - 1 - km : Lm - km;
    }
    r.rowa = k1 * Lm + km;
    r.rowb = k1m * Lm + kmm;
    r.rhoa = k1 + L1 * km;
    r.rhob = k1m + L1 * kmm;
    return r;
}

template <int L2, typename C = double2>
__device__ __forceinline__ void k2_body(const KParams& p, const Blk bk)
{
    // rows 0,1: operands u,v at row (k1, km); rows 2,3: at the mirror row
    __shared__ C rows[padded<PAD2>(4 * L2)];
    __shared__ C twl[twl_size(L2)];
    C* za = reinterpret_cast<C*>(p.za);
    const C* zb = reinterpret_cast<const C*>(p.zb);
    const uint32_t L1 = p.L1, Lm = p.Lm;
    const K2Rows rr = k2_rows_of(bk.x, L1, Lm);
    const uint32_t rowa = rr.rowa, rowb = rr.rowb;
    load_twl<L2, NT2>(twl, p.tw2);
    // exp(-2 pi i k / M) for bin k = rho + L1 Lm k2 (rho = k1 + L1 km) is
    // exp(-2 pi i rho / M) times exp(-2 pi i k2 / L2): one table value per row
    const uint32_t rhoa = rr.rhoa, rhob = rr.rhob;
    const double2 wr0a = p.tw.lo[rhoa & p.tw.mask], wr0b = p.tw.hi[rhoa >> p.tw.shift];
    const double2 wr1a = p.tw.lo[rhob & p.tw.mask], wr1b = p.tw.hi[rhob >> p.tw.shift];
    {
        constexpr int PL = (4 * L2 + NT2 - 1) / NT2;
        C v[PL];
#pragma unroll
        for (int q = 0; q < PL; q++) {
            const int e = threadIdx.x + q * NT2;
            if (4 * L2 % NT2 == 0 || e < 4 * L2) {
                const int r = e / L2, j2 = e % L2;
                const uint32_t row = r < 2 ? rowa : rowb;
                const C* src = (r & 1) ? zb : za;
                v[q] = src[(size_t)row * L2 + j2];
            }
        }
#pragma unroll
        for (int q = 0; q < PL; q++) {
            const int e = threadIdx.x + q * NT2;
            if (4 * L2 % NT2 == 0 || e < 4 * L2) rows[pidx<PAD2>(e)] = v[q];
        }
    }
    __syncthreads();
    // forward row DFTs of the four rows: one wavefront per row (no
    // workgroup barriers inside the transforms), or the whole workgroup
    constexpr bool WAVE_ROWS = K2_WAVE && NT2 == 256 && L2 == 1024;
    static_assert(!WAVE_ROWS || L2 % (1 << PAD2) == 0, "a row starts on a pad boundary");
    if constexpr (WAVE_ROWS) {
        C* row = rows + pidx<PAD2>((int)(threadIdx.x >> 6) * L2);
        if constexpr (K2_SHUFFLE && std::is_same<C, double2>::value)
            row1024_wave<false, PAD2>(row, twl);
        else
            tile_fft<L2, 1, 64, false, false, L2, PAD2, true>(row, twl);
        __syncthreads();
    } else {
        tile_fft<L2, 4, NT2, false, false, L2, PAD2>(rows, twl);
    }

    constexpr int PER = (2 * L2 + NT2 - 1) / NT2;
    const C wrow0 = to_elem<C>(cmul(wr0a, wr0b)), wrow1 = to_elem<C>(cmul(wr1a, wr1b));
    if (!rr.self) {
        // distinct rows: bin (row a, k2) with its mirror (row b, L2 - 1 - k2)
        constexpr int PP = (L2 + NT2 - 1) / NT2;
        C qa[PP], qb[PP];
#pragma unroll
        for (int t = 0; t < PP; t++) {
            const int k2 = threadIdx.x + t * NT2;
            if (L2 % NT2 == 0 || k2 < L2) {
                const int mk2 = L2 - 1 - k2;
                pointwise_pair(rows[pidx<PAD2>(k2)], rows[pidx<PAD2>(2 * L2 + mk2)], rows[pidx<PAD2>(L2 + k2)],
                               rows[pidx<PAD2>(3 * L2 + mk2)], cmul(wrow0, tw_half<L2>(twl, k2)), qa[t], qb[t]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PP; t++) {
            const int k2 = threadIdx.x + t * NT2;
            if (L2 % NT2 == 0 || k2 < L2) {
                rows[pidx<PAD2>(k2)] = qa[t];
                rows[pidx<PAD2>(2 * L2 + L2 - 1 - k2)] = qb[t];
            }
        }
    } else {
        // the workgroup of the self-mirrored rows: one bin at a time (row
        // (0, 0) in slot 0 pairs with itself with k2 -> (L2 - k2) mod L2, the
        // other self-mirrored row with k2 -> L2 - 1 - k2)
        C qv[PER];
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = threadIdx.x + t * NT2;
            if (e < 2 * L2) {
                const int pr = e / L2, k2 = e % L2;
                const int mk2 = pr == 0 ? (L2 - k2) % L2 : L2 - 1 - k2;
                qv[t] = pointwise_bin(rows[pidx<PAD2>((2 * pr) * L2 + k2)], rows[pidx<PAD2>((2 * pr) * L2 + mk2)],
                                      rows[pidx<PAD2>((2 * pr + 1) * L2 + k2)], rows[pidx<PAD2>((2 * pr + 1) * L2 + mk2)],
                                      cmul(pr ? wrow1 : wrow0, tw_half<L2>(twl, k2)));
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = threadIdx.x + t * NT2;
            if (e < 2 * L2) {
                const int pr = e / L2, k2 = e % L2;
                rows[pidx<PAD2>((2 * pr) * L2 + k2)] = qv[t];
            }
        }
    }
    __syncthreads();
    // inverse row DFTs of rows 0 and 2 (row stride 2*L2)
    if constexpr (WAVE_ROWS) {
        const int w = (int)(threadIdx.x >> 6);
        if (w < 2) {
            C* row = rows + pidx<PAD2>(2 * w * L2);
            if constexpr (K2_SHUFFLE && std::is_same<C, double2>::value)
                row1024_wave<true, PAD2>(row, twl);
            else
                tile_fft<L2, 1, 64, true, false, L2, PAD2, true>(row, twl);
        }
        __syncthreads();
    } else {
        tile_fft<L2, 2, NT2, true, false, 2 * L2, PAD2>(rows, twl);
    }
    for (int e = threadIdx.x; e < 2 * L2; e += NT2) {
        const int pr = e / L2, j2 = e % L2;
        if (pr == 1 && rowb == rowa) continue;
        za[(size_t)(pr ? rowb : rowa) * L2 + j2] = rows[pidx<PAD2>((2 * pr) * L2 + j2)];
    }
}

// rows of up to 512 points fit four workgroups per CU in LDS; the second
// bound (waves per SIMD) keeps their registers within that occupancy
template <int L2, typename C = double2>
__global__ __launch_bounds__(NT2, L2 <= 512 ? 4 : 2) void k2_rows_pointwise(KParams p)
{
    k2_body<L2, C>(p, blk_hw());
}

template <int L2>
__global__ __launch_bounds__(NT2, L2 <= 512 ? 4 : 2) void k2_rows_pointwise_g(Group g)
{
    uint32_t pi;
    const Blk bk = group_block(g, pi);
    const KParams& p = group_params(g, pi);
    k2_body<L2>(p, bk);
}

// ------------------------------------------------------------ middle pass

// Middle column pass of the three-pass split (Lm > 1): inside each row k1
// of the L1 x R matrix (R = Lm L2), Lm-point DFTs over jm (stride L2) for W
// adjacent columns j2.  Forward: DFT, then exp(-2 pi i j2 km / R), in place
// on both operands.  Inverse: exp(+2 pi i j2 km / R), then inverse DFT, on
// the product.  grid = (L2 / W, L1, operands).
template <int LM, int W, bool INV, typename C = double2>
__device__ __forceinline__ void mid_body(const KParams& p, const Blk bk)
{
    constexpr int PER = (LM * W + NTM - 1) / NTM;
    static_assert(NTM % W == 0, "W must divide NTM");
    __shared__ C tile[padded(LM * W)];
    __shared__ C twl[twl_size(LM)];
    const uint32_t L2 = p.L2;
    // tile and row of this workgroup: with both grid extents multiples of
    // 8, the workgroups of one XCD (bk.x mod 8 under the round-robin
    // dispatch) take whole rows of each group of eight rows, so one XCD
    // streams contiguous row segments (4% faster than XCD-contiguous column
    // tiles within every row for 384-point rows; equal for 1024)
    uint32_t xt = xcd_tile(bk.x, bk.nx), yr = bk.y;
    if (bk.nx % 8 == 0 && bk.ny % 8 == 0) {
        xt = bk.x / 8 + (bk.nx / 8) * (bk.y % 8);
        yr = (bk.y & ~7u) + bk.x % 8;
    }
    const uint32_t c0 = xt * W;
    C* a = reinterpret_cast<C*>(bk.z ? p.zb : p.za) + (size_t)yr * p.R;
    const int tid = threadIdx.x;
    load_twl<LM, NTM>(twl, p.twm);
    // twiddle exponents on the R-th root, as exponents of the M-th root (x L1)
    const uint32_t colt = c0 + tid % W;
    const uint32_t eb = (uint32_t)(((uint64_t)colt * (uint32_t)(tid / W) * p.L1) % p.M);
    const uint32_t es = (uint32_t)(((uint64_t)colt * (uint32_t)(NTM / W) * p.L1) % p.M);
    const double2 tb0 = p.tw.lo[eb & p.tw.mask], tb1 = p.tw.hi[eb >> p.tw.shift];
    const double2 ts0 = p.tw.lo[es & p.tw.mask], ts1 = p.tw.hi[es >> p.tw.shift];
    C v[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int e = tid + q * NTM;
        if (LM * W % NTM == 0 || e < LM * W) v[q] = a[(size_t)(e / W) * L2 + colt];
    }
    TwSeq<PER, C> tws;
    if (INV) tws.init(cconj(cmul(tb0, tb1)), cconj(cmul(ts0, ts1)));
    else tws.init(cmul(tb0, tb1), cmul(ts0, ts1));
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int e = tid + q * NTM;
        if (LM * W % NTM == 0 || e < LM * W) tile[pidx(e)] = INV ? cmul(v[q], tws.at(q)) : v[q];
    }
    __syncthreads();
    tile_fft<LM, W, NTM, INV, true>(tile, twl);
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int e = tid + q * NTM;
        if (LM * W % NTM == 0 || e < LM * W) {
            const C t = tile[pidx(e)];
            a[(size_t)(e / W) * L2 + colt] = INV ? t : cmul(t, tws.at(q));
        }
    }
}

template <int LM, int W, bool INV, typename C = double2>
__global__ __launch_bounds__(NTM) void k_mid_col(KParams p)
{
    mid_body<LM, W, INV, C>(p, blk_hw());
}

template <int LM, int W, bool INV>
__global__ __launch_bounds__(NTM) void k_mid_col_g(Group g)
{
    uint32_t pi;
    const Blk bk = group_block(g, pi);
    const KParams& p = group_params(g, pi);
    mid_body<LM, W, INV>(p, bk);
}

// ------------------------------------------------------------------- K3

template <int L1, int W, typename C = double2>
__device__ __forceinline__ void k3_body(const KParams& p, const Blk bk)
{
    __shared__ C tile[padded(L1 * W)];
    __shared__ C twl[twl_size(L1)];
    C* za = reinterpret_cast<C*>(p.za);
    const uint32_t L2 = p.R;  // row length of the L1 x R matrix
    const uint32_t c0 = xcd_tile(bk.x, bk.nx) * W;
    load_twl<L1, NT3>(twl, p.tw1);
    constexpr int PER = (L1 * W + NT3 - 1) / NT3;
    static_assert(NT3 % W == 0, "W must divide NT3");
    const int tid = threadIdx.x;
    const uint32_t colt = c0 + tid % W;
    const uint32_t eb = (uint32_t)((uint64_t)colt * (uint32_t)(tid / W) % p.M);
    const uint32_t es = (uint32_t)((uint64_t)colt * (uint32_t)(NT3 / W) % p.M);
    const double2 tb0 = p.tw.lo[eb & p.tw.mask], tb1 = p.tw.hi[eb >> p.tw.shift];
    const double2 ts0 = p.tw.lo[es & p.tw.mask], ts1 = p.tw.hi[es >> p.tw.shift];
    {
        C v[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int e = tid + q * NT3;
            if (L1 * W % NT3 == 0 || e < L1 * W) v[q] = za[(size_t)(e / W) * L2 + colt];
        }
        // inverse inter-pass twiddles exp(+2 pi i col k1 / M)
        TwSeq<PER, C> tws;
        tws.init(cconj(cmul(tb0, tb1)), cconj(cmul(ts0, ts1)));
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int e = tid + q * NT3;
            if (L1 * W % NT3 == 0 || e < L1 * W) tile[pidx(e)] = cmul(v[q], tws.at(q));
        }
    }
    __syncthreads();
    tile_fft<L1, W, NT3, true, true>(tile, twl);
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int e = threadIdx.x + q * NT3;
        if (L1 * W % NT3 == 0 || e < L1 * W) za[(size_t)(e / W) * L2 + c0 + e % W] = tile[pidx(e)];
    }
}

template <int L1, int W, typename C = double2>
__global__ __launch_bounds__(NT3) void k3_col_inverse(KParams p)
{
    k3_body<L1, W, C>(p, blk_hw());
}

template <int L1, int W>
__global__ __launch_bounds__(NT3) void k3_col_inverse_g(Group g)
{
    uint32_t pi;
    const Blk bk = group_block(g, pi);
    const KParams& p = group_params(g, pi);
    k3_body<L1, W>(p, bk);
}

// ------------------------------------------------------------------- K0

// Fused small-size pass: one workgroup computes both operands' digits and
// maps, their whole length-M transforms (M = L1 L2 <= 4096: both packed
// spectra fit in LDS), the pointwise product and the whole inverse
// transform, and writes the real convolution for K4 (which then rounds and
// carries).  It replaces K1, K2 and K3 of the four-step path, so a small
// product is two launches, and a packed batch of small products is one K0
// launch (one workgroup per product) plus one K4 launch.
constexpr int NT0 = 256;
constexpr uint32_t K0_MAX_M = 4096;

template <int L1, int L2, int KIND>
__device__ __forceinline__ void k0_body(const KParams& p)
{
    constexpr int M = L1 * L2;
    static_assert(M <= (int)K0_MAX_M, "fused pass holds both spectra in LDS");
    constexpr int LB = k1_lb(KIND, 0), LO = LB - 1;
    constexpr int WC = 8;                   // complex points per digit row
    static_assert(L2 % WC == 0, "row chunks");
    constexpr int ND = k1_nd(WC, KIND, 0);
    constexpr int CH = L2 / WC;
    constexpr int UNITS = 2 * L1 * CH;      // (operand, row, chunk)
    __shared__ double2 A[padded(M)], B[padded(M)];
    __shared__ double2 tw1[twl_size(L1)], tw2[twl_size(L2)];
    __shared__ double s_th[2][LMAX + 8];
    const int tid = threadIdx.x;
    const bool square = p.zb == p.za;

    clear_state(p, tid, NT0);
    load_twl<L1, NT0>(tw1, p.tw1);
    load_twl<L2, NT0>(tw2, p.tw2);
    if (KIND == K_HI && tid <= (int)p.jmax && tid <= (int)p.N) {
        s_th[0][tid] = ldexp((double)bal_digit(p, p.u, (int64_t)p.N - tid, p.digits, true), -tid * p.b);
        s_th[1][tid] = ldexp((double)bal_digit(p, p.v, (int64_t)p.N - tid, p.digits, true), -tid * p.b);
    }
    // G = alpha* U / gamma-dagger F (truncated products) or the digits (full
    // product) of both operands, element (j1, col) at index j1 L2 + col.
    // The loop is unrolled so that every unit's limb loads are in flight
    // together.
    const int64_t kf_min = KIND == K_HI ? (int64_t)p.jmax : 0;
    const int64_t top = (int64_t)p.digits - 1;
    constexpr int PU = (UNITS + NT0 - 1) / NT0;
#pragma unroll
    for (int qu = 0; qu < PU; qu++) {
        const int ux = tid + qu * NT0;
        if (UNITS % NT0 != 0 && ux >= UNITS) continue;
        const int op = ux / (L1 * CH);
        const int rem = ux % (L1 * CH);
        const uint32_t m0 = (uint32_t)(rem / CH) * L2 + (uint32_t)(rem % CH) * WC;
        const uint64_t* x = op ? p.v : p.u;
        const int64_t kf = 2 * (int64_t)m0 - LO;
        const bool fast = kf >= kf_min && (KIND != K_FULL || kf + ND <= top);
        int32_t d[ND];
        double2 g[WC];
        if (fast) row_digits_reg<ND>(p, x, kf, d);
        else row_digits_edge<ND, KIND>(p, x, kf, d);
        if constexpr (KIND == K_FULL) {
#pragma unroll
            for (int c = 0; c < WC; c++) g[c] = make_double2((double)d[2 * c], (double)d[2 * c + 1]);
        } else if (fast) {
            row_map_fast<WC, ND, LB>(p, kf, d, g);
        } else {
            const double FN = KIND == K_HI ? (double)bal_digit(p, x, p.N, p.digits, true) : 0.0;
            row_map_edge<WC, KIND, ND, LB>(p, m0, FN, d, g);
        }
        double2* dst = op ? B : A;
#pragma unroll
        for (int c = 0; c < WC; c++) dst[pidx(m0 + c)] = g[c];
    }
    __syncthreads();
    if (KIND == K_HI && tid == 0) {
        // theta = rho^-N F(rho), rho ~ 2^b: sum_j 2^(-jb) F_(N-j), j <= jmax
        double t0 = 0.0, t1 = 0.0;
        for (int j = 0; j <= (int)p.jmax && j <= (int)p.N; j++) {
            t0 += s_th[0][j];
            t1 += s_th[1][j];
        }
        p.theta[0] = t0;
        p.theta[1] = square ? t0 : t1;
    }
    // forward: L1-point column DFTs, twiddles exp(-2 pi i col k1 / M),
    // L2-point row DFTs; position (k1, k2) then holds bin k1 + L1 k2
    // Twiddles of this thread's elements e = tid + q NT0: L2 divides NT0, so
    // col = e mod L2 is fixed and k1 = e / L2 steps by NT0 / L2; the
    // exponents col k1 (inter-pass) and k1 + L1 col (pointwise bin) are
    // arithmetic progressions in q, formed from two table values each.
    static_assert(NT0 % L2 == 0, "row length divides the workgroup");
    constexpr int PE = (M + NT0 - 1) / NT0;
    const uint32_t col = (uint32_t)(tid % L2), r1 = (uint32_t)(tid / L2), dk = (uint32_t)(NT0 / L2);
    TwSeq<PE> tip, tbin;
    tip.init(tw_get<false>(p.tw, (col * r1) % M), tw_get<false>(p.tw, (col * dk) % M));
    tbin.init(tw_get<false>(p.tw, (r1 + L1 * col) % M), tw_get<false>(p.tw, dk % M));
    tile_fft<L1, L2, NT0, false, true>(A, tw1);
    tile_fft<L1, L2, NT0, false, true>(B, tw1);
#pragma unroll
    for (int q = 0; q < PE; q++) {
        const int e = tid + q * NT0;
        if (M % NT0 == 0 || e < M) {
            const double2 w = tip.at(q);
            A[pidx(e)] = cmul(A[pidx(e)], w);
            B[pidx(e)] = cmul(B[pidx(e)], w);
        }
    }
    __syncthreads();
    tile_fft<L2, L1, NT0, false, false, L2>(A, tw2);
    tile_fft<L2, L1, NT0, false, false, L2>(B, tw2);
    // pointwise product over mirror pairs (bin k, bin M - k), each pair
    // read and written by one thread
#pragma unroll
    for (int q = 0; q < PE; q++) {
        const int e = tid + q * NT0;
        if (M % NT0 != 0 && e >= M) continue;
        const int k1 = e / L2, k2 = e % L2;
        const int mk1 = k1 ? L1 - k1 : 0, mk2 = k1 ? L2 - 1 - k2 : (L2 - k2) % L2;
        const int em = mk1 * L2 + mk2;
        if (e > em) continue;
        // exp(-2 pi i k / M) for bin k = k1 + L1 k2, and its conjugate for M - k
        const double2 wk = tbin.at(q);
        const double2 Ya = A[pidx(e)], Yam = A[pidx(em)], Yb = B[pidx(e)], Ybm = B[pidx(em)];
        const double2 qe = pointwise_bin(Ya, Yam, Yb, Ybm, wk);
        if (em != e) {
            const double2 qm = pointwise_bin(Yam, Ya, Ybm, Yb, cconj(wk));
            A[pidx(em)] = qm;
        }
        A[pidx(e)] = qe;
    }
    __syncthreads();
    // inverse: row DFTs, twiddles exp(+2 pi i j2 k1 / M), column DFTs;
    // position (j1, j2) then holds point j1 L2 + j2 of the product
    tile_fft<L2, L1, NT0, true, false, L2>(A, tw2);
#pragma unroll
    for (int q = 0; q < PE; q++) {
        const int e = tid + q * NT0;
        if (M % NT0 == 0 || e < M) A[pidx(e)] = cmul(A[pidx(e)], cconj(tip.at(q)));
    }
    __syncthreads();
    tile_fft<L1, L2, NT0, true, true>(A, tw1);
#pragma unroll
    for (int q = 0; q < PE; q++) {
        const int e = tid + q * NT0;
        if (M % NT0 == 0 || e < M) p.za[e] = A[pidx(e)];
    }
}

template <int L1, int L2, int KIND>
__global__ __launch_bounds__(NT0) void k0_fused(KParams p)
{
    k0_body<L1, L2, KIND>(p);
}

template <int L1, int L2, int KIND>
__global__ __launch_bounds__(NT0) void k0_fused_g(Group g)
{
    uint32_t pi;
    (void)group_block(g, pi);
    k0_body<L1, L2, KIND>(group_params(g, pi));
}

// ------------------------------------------------------------------- K4

// Carry function of a block of digits: carry_out = A + [carry_in >= T]
// (T = INT64_MAX: constant A; T = INT64_MIN: constant A + 1).
struct CarryF {
    int64_t A, T;
};

// g after f (f acts first)
__device__ __forceinline__ CarryF compose(CarryF f, CarryF g)
{
    CarryF r;
    if (f.A >= g.T) { r.A = g.A + 1; r.T = INT64_MAX; }
    else if (f.A + 1 < g.T) { r.A = g.A; r.T = INT64_MAX; }
    else { r.A = g.A; r.T = f.T; }
    return r;
}

__device__ __forceinline__ int64_t apply(CarryF f, int64_t c) { return f.A + (c >= f.T ? 1 : 0); }

// Look-back records are 64-bit words holding a 2-bit state (0 empty,
// 1 aggregate, 2 inclusive, 3 constant aggregate) and a 62-bit
// two's-complement value.  A constant aggregate (almost every workgroup's,
// since one constant limb function makes the composition constant) is one
// word holding its carry-out, so a reader needs no second load.  Each word
// is written once per state by a single relaxed device-scope atomic store
// and polled with relaxed device-scope atomic loads: no acquire/release
// fences, which on this GPU would write back or invalidate the whole L2.
__device__ __forceinline__ uint64_t ld_rlx(uint64_t* a)
{
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint64_t* a, uint64_t v)
{
    __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
constexpr int64_t V62_MAX = (1ll << 61) - 1, V62_MIN = -(1ll << 61);
__device__ __forceinline__ uint64_t pack62(uint64_t state, int64_t v)
{
    v = v > V62_MAX ? V62_MAX : v < V62_MIN ? V62_MIN : v;
    return (state << 62) | ((uint64_t)v & ((1ull << 62) - 1));
}
__device__ __forceinline__ int64_t unpack62(uint64_t w) { return (int64_t)(w << 2) >> 2; }
// Lane moves by DPP (data-parallel primitives, GFX9 controls): row_shr:d
// (0x110 + d) within 16-lane rows, row_bcast:15 / row_bcast:31 (0x142 /
// 0x143: the last lane of a row into the next row(s), rows chosen by ROWS),
// wave_shr:1 (0x138), quad_perm (0x00..0xff), row_half_mirror (0x141) and
// row_mirror (0x140).  A lane with no source, or in a row outside ROWS,
// gets `old`.  They run at VALU speed, where ds_bpermute / ds_swizzle
// shuffles take an LDS round trip per step.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint64_t dpp64(uint64_t old, uint64_t v)
{
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)old, (int)(uint32_t)v, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(old >> 32), (int)(uint32_t)(v >> 32), CTRL, ROWS,
                                               0xf, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_keep(double v)  // lanes with no source keep v
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return __longlong_as_double((long long)dpp64<CTRL, ROWS>(u, u));
}

// Maximum over the wavefront, returned in every lane: quad, half-row and
// row mirrors, then the rows' maxima carried into lane 63 by the row
// broadcasts, then read from lane 63.
#ifndef TM_K4_DPP
#define TM_K4_DPP 1
#endif
__device__ __forceinline__ double wave_max(double v)
{
    if (!TM_K4_DPP) {
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        return v;
    }
    v = fmax(v, dpp_keep<0xb1>(v));        // quad_perm [1,0,3,2]
    v = fmax(v, dpp_keep<0x4e>(v));        // quad_perm [2,3,0,1]
    v = fmax(v, dpp_keep<0x141>(v));       // row_half_mirror
    v = fmax(v, dpp_keep<0x140>(v));       // row_mirror
    v = fmax(v, dpp_keep<0x142, 0xa>(v));  // row_bcast:15 into rows 1, 3
    v = fmax(v, dpp_keep<0x143, 0xc>(v));  // row_bcast:31 into rows 2, 3
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Inclusive scan of carry functions over the wavefront (lane l ends with
// f_l o ... o f_0): the rows of 16 by row shifts, then each row composed
// after the rows below it by the row broadcasts.
__device__ __forceinline__ CarryF wave_scan(CarryF f, int lane)
{
    if (!TM_K4_DPP) {
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t pa = __shfl_up(f.A, d), pt = __shfl_up(f.T, d);
            if (lane >= d) f = compose(CarryF{pa, pt}, f);
        }
        return f;
    }
    // a constant function (T = INT64_MAX) absorbs every function before it,
    // so lane l ends with f_l when f_l is constant, and with f_l o f_(l-1)
    // when only f_(l-1) is: while no two neighbouring lanes hold
    // non-constant functions (the usual case) one lane shift is the scan
    const bool nc = f.T != INT64_MAX;
    const uint64_t m = __ballot(nc);
    if ((m & (m << 1)) == 0) {
        const CarryF q = {(int64_t)dpp64<0x138>(0, (uint64_t)f.A), (int64_t)dpp64<0x138>(0, (uint64_t)f.T)};
        if (nc && lane > 0) f = compose(q, f);
        return f;
    }
    const int lr = lane & 15;
#define TM_SCAN_STEP(CTRL, ROWS, COND)                                             \
    {                                                                              \
        const CarryF q = {(int64_t)dpp64<CTRL, ROWS>(0, (uint64_t)f.A),            \
                          (int64_t)dpp64<CTRL, ROWS>(0, (uint64_t)f.T)};           \
        if (COND) f = compose(q, f);                                               \
    }
    TM_SCAN_STEP(0x111, 0xf, lr >= 1)
    TM_SCAN_STEP(0x112, 0xf, lr >= 2)
    TM_SCAN_STEP(0x114, 0xf, lr >= 4)
    TM_SCAN_STEP(0x118, 0xf, lr >= 8)
    TM_SCAN_STEP(0x142, 0xa, (lane & 16) != 0)
    TM_SCAN_STEP(0x143, 0xc, (lane & 32) != 0)
#undef TM_SCAN_STEP
    return f;
}

// x_i, the value rounded to c_i (see tm_guard), from the LDS copy of q
// (sq[padq(o + K4_HALO)] = q at index base + o, cyclically: workgroup 0 holds the
// top of q below its range):
//   full: W_i                                       (Alg. full, step 4)
//   low:  2^b W-bar_i, W-bar = beta* W mod A        (Prop. approximating
//         beta*): sum_r beta_{i-r,r} W_(i-r) with cyclic indices, minus
//         2^-b sum_{r>=i} beta_{N+i-1-r,r} W_(N+i-1-r) for 1 <= i < lam
//         (X^(N+s) = X^s - 2^-b X^(s+1) mod A)
//   high: 2^b J_i, J = (1 - 2^-b X) H + psi C(X), H = delta* W mod C,
//         psi ~ theta_W, C_j ~ -2^(-jb)  (eq. crt-sum, Remark on Newton):
//         H_i = sum_r delta_{i-r,r} W_(i-r) (r <= i) + sum_j 2^(-jb)
//         sum_{r > i-j} delta_{N+i-j-r,r} W_(N+i-j-r)  (X^(N+s) = sum_j
//         2^(-jb) X^(s+j) mod C)
// The sums use the unnormalised q = M W.  edge_part / edge_sum evaluate them term by
// term for the indices next to the wrap (i < K4_HALO) and the top index
// i = N of the high product; all other indices use back_chain.
// Parts of the sum at index i next to the wrap (workgroup 0: o = i), one
// per thread; edge_sum combines them in a fixed order.
//   low:  part 0 = sum_r beta_{(i-r) mod N, r} q_((i-r) mod N),
//         part 1 = sum_{r>=i} beta_{N+i-1-r,r} q_(N+i-1-r)  (1 <= i < lam)
//   high: part K4_EP-1 = sum_{r<=i} delta_{i-r,r} q_(i-r),
//         part j (j <= min(i, jmax)) = sum_{r>i-j} delta_{N+i-j-r,r} q_(N+i-j-r)
constexpr int K4_EP = 12;  // parts per index (jmax + 2 <= 12 for b >= 8)
template <int KIND>
__device__ double edge_part(const KParams& p, const double* sq, uint32_t i, int part)
{
    const int o = (int)i + K4_HALO;
    double s = 0.0;
    if (KIND == K_LO) {
        if (part == 0) {
            for (int r = 0; r < p.lam && r <= (int)i; r++)
                s = fma(coef_back<KIND>(p, i - r, r), sq[padq(o - r)], s);
            for (int r = (int)i + 1; r < p.lam; r++)
                s = fma(coef_back<KIND>(p, p.N + i - r, r), sq[padq(o - r)], s);
        } else if (part == 1 && i >= 1 && i < (uint32_t)p.lam) {
            for (int r = (int)i; r < p.lam; r++)
                s = fma(coef_back<KIND>(p, p.N + i - 1 - r, r), sq[padq(o - 1 - r)], s);
        }
    } else {
        if (part == K4_EP - 1) {
            for (int r = 0; r < p.lam && r <= (int)i; r++)
                s = fma(coef_back<KIND>(p, i - r, r), sq[padq(o - r)], s);
        } else if (part <= (int)i && part <= (int)p.jmax) {
            const int j = part;
            for (int r = (int)i - j + 1; r < p.lam; r++)
                s = fma(coef_back<KIND>(p, p.N + i - j - r, r), sq[padq(o - j - r)], s);
        }
    }
    return s;
}

template <int KIND>
__device__ __forceinline__ double edge_sum(const KParams& p, const double* ep, uint32_t i)
{
    if (KIND == K_LO) {
        double s = ep[0];
        if (i >= 1 && i < (uint32_t)p.lam) s = fma(-ldexp(1.0, -p.b), ep[1], s);
        return s;
    }
    double s = ep[K4_EP - 1];
    for (int j = 0; j <= (int)i && j <= (int)p.jmax; j++) s = fma(ldexp(1.0, -j * p.b), ep[j], s);
    return s;
}

// x_i for i < K4_HALO (workgroup 0) from se[i + 1] = the sum of
// edge_sum at index i (se[0] = 0: the index below 0).
template <int KIND>
__device__ __forceinline__ double back_edge(const KParams& p, const double* se, uint32_t i, double thW)
{
    if (KIND == K_LO) return ldexp(se[i + 1] * p.invM, p.b);
    return ldexp(fma(-ldexp(1.0, -p.b), se[i], se[i + 1]) * p.invM - ldexp(thW, -(int)i * p.b), p.b);
}

// The back maps away from the wrap, as a chain per input: with x = k/N,
// beta_{k,r} = c_r prod_{j<r} (x + j) (delta: x - j), so the contributions
// tau_r = 2^b/M beta_{k,r} q_k of input k to outputs k + r follow from
// tau_(r+1) = tau_r (c_(r+1)/c_r) (x +- r): two FMAs per term.  The host
// zeroes the factor at r = lam - 1, ending every chain at the plan's lam.
// acc[o] = 2^b/M (beta* q)_(i0 - OFF + o), o < NOUT.
template <int LB, int NOUT, int OFF>
__device__ __forceinline__ void back_chain(const KParams& p, const double* sq, int s0, int64_t k0,
                                           double (&acc)[NOUT])
{
    // every operation as written (no contraction), so that prev_top_carry's
    // per-output recomputation gives the same bits
#pragma clang fp contract(off)
    constexpr int NIN = NOUT + LB - 1;
#pragma unroll
    for (int o = 0; o < NOUT; o++) acc[o] = 0.0;
    const double x0 = (double)k0 * p.invN;
#pragma unroll
    for (int e = 0; e < NIN; e++) {
        double tau = sq[padq(s0 + e)] * p.bscale;
        const double xk = fma((double)e, p.invN, x0);
#pragma unroll
        for (int r = 0; r < LB; r++) {
            const int o = e + r - (LB - 1);
            if (o >= 0 && o < NOUT) acc[o] += tau;
            if (r + 1 < LB && o + 1 < NOUT) tau *= fma(p.nb[r][0], xk, p.nb[r][1]);
        }
    }
}

// Real element i of the packed convolution result (real parts at even i,
// imaginary parts at odd i), in FP64.
__device__ __forceinline__ double real_at(const double2* z, int64_t i)
{
    return reinterpret_cast<const double*>(z)[i];
}
__device__ __forceinline__ double real_at(const dfc* z, int64_t i)
{
    const dfc c = z[i >> 1];
    return df_to((i & 1) ? c.y : c.x);
}

// Carry function of one limb of S from its 128-bit sum T = thi 2^64 + tlo:
// carry out = floor((T + cin) / 2^64) = A + [cin >= T'].  Every carry is
// below 2^57 in magnitude (|c_i| < 2^51, at most 8 per limb), so a
// threshold beyond that decides the carry alone: such functions are made
// constant (T' = INT64_MAX).
__device__ __forceinline__ CarryF limb_carry_fn(uint64_t tlo, int64_t thi)
{
    CarryF f;
    if (tlo >= (1ull << 63)) {
        f.A = thi;
        f.T = tlo == (1ull << 63) ? INT64_MAX : (int64_t)(0 - tlo);
    } else {
        f.A = thi - 1;
        f.T = -(int64_t)tlo;
    }
    if (f.T > K4_CMAX) {
        f.T = INT64_MAX;
    } else if (f.T < -K4_CMAX) {
        f.A += 1;
        f.T = INT64_MAX;
    }
    return f;
}

// Carry out of the previous workgroup's top limb (limb j0 - 1, j0 = the
// first limb of this workgroup), from that workgroup's last DPT
// coefficients recomputed here by one wavefront, lane t taking output t of
// the previous workgroup's last thread: its inputs lie in this workgroup's
// staged halo, and the sum runs over the same inputs in the same order with
// the same operations as back_chain, so the values are the same bits.  The
// coefficients that start in limb j0 - 1 are among them since b >= 8.
// When that limb's carry function is constant it is the carry into this
// workgroup, whatever lies further back, and the look-back is not needed;
// pk = false otherwise, or when a value is not clearly rounded (then the
// look-back decides).  For workgroups g >= 1 whose first index base <= N
// (the previous one holds neither the wrap's edge indices nor the high
// product's top index N); called by a whole wavefront.
template <int KIND, int B>
__device__ void prev_top_carry(const KParams& p, const double* sq, uint64_t base, int b, int lane,
                               bool& pk, int64_t& pc)
{
#pragma clang fp contract(off)
    constexpr int LB = KIND == K_FULL ? 1 : B ? LB_FIXED : LMAX;
    constexpr int OFF = KIND == K_HI ? 1 : 0;
    constexpr int NOUT = DPT + OFF;
    constexpr double RMAG = 6755399441055744.0;
    static_assert(DPT * 8 >= 64, "digits of b >= 8 bits: one limb's coefficients lie among the last DPT");
    static_assert(NOUT <= 64 && K4_HALO >= DPT + OFF + LMAX - 1, "one lane per output, inputs in the halo");
    const uint64_t i0 = base - DPT;  // first index of the previous workgroup's last thread
    const int o = lane < NOUT ? lane : NOUT - 1;
    double x;
    if constexpr (KIND == K_FULL) {
        x = sq[padq(K4_HALO - DPT + o)] * p.bscale;
    } else {
        // back_chain's acc[o]: inputs e = o .. o + LB - 1 in that order, input
        // e scaled by r = o + LB - 1 - e factors
        const int s0 = K4_HALO - DPT - OFF - (LB - 1);
        const int64_t k0 = (int64_t)i0 - OFF - (LB - 1);
        const double x0 = (double)k0 * p.invN;
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < LB; d++) {
            const int e = o + d;
            const int r = LB - 1 - d;
            double tau = sq[padq(s0 + e)] * p.bscale;
            const double xk = fma((double)e, p.invN, x0);
#pragma unroll
            for (int q = 0; q < LB - 1; q++)
                if (q < r) tau *= fma(p.nb[q][0], xk, p.nb[q][1]);
            acc += tau;
        }
        if constexpr (KIND == K_LO) {
            x = acc;
        } else {
            const double nxt = __shfl_down(acc, 1);
            x = fma(-ldexp(1.0, -b), acc, nxt);
        }
    }
    // rounding as in k4_body
    const double xs = lane < DPT && i0 + lane < p.ncoef ? x : 0.0;
    const double sh = xs + RMAG;
    const double rr = sh - RMAG;
    int64_t c = (int64_t)__double_as_longlong(sh) - (int64_t)__double_as_longlong(RMAG);
    const bool clear = fabs(xs - rr) < 0.25 && fabs(xs) < 1125899906842624.0;
    if (KIND == K_HI && lane < DPT) {
        const uint64_t dm1 = p.off - 1;
        const uint64_t ih = dm1 / (uint64_t)b;
        if (ih == i0 + lane) c += 1ll << (dm1 - ih * (uint64_t)b);
    }
    pk = false;
    pc = 0;
    if (__ballot(!clear) != 0) return;
    // limb j0 - 1: the coefficients i >= ia, summed in 128 bits
    const int64_t j = (int64_t)(base * (uint64_t)b / 64) - 1;
    const int64_t ia = (64 * j + b - 1) / b;
    uint64_t tlo = 0;
    int64_t thi = 0;
#pragma unroll
    for (int t = 0; t < DPT; t++) {
        const int64_t ct = __shfl(c, t);
        const int64_t i = (int64_t)i0 + t;
        if (i >= ia) {
            const int shf = (int)(i * b - 64 * j);
            const uint64_t plo = (uint64_t)ct << shf;
            const int64_t phi = shf ? ct >> (64 - shf) : (ct >> 63);
            const uint64_t nlo = tlo + plo;
            thi += phi + (nlo < plo ? 1 : 0);
            tlo = nlo;
        }
    }
    const CarryF f = limb_carry_fn(tlo, thi);
    pk = f.T == INT64_MAX;
    pc = f.A;
}

template <int KIND, bool DIAG, int B, typename C = double2>
__device__ __forceinline__ void k4_body(const KParams& p, const Blk bk)
{
    constexpr int NW = NT4 / 64;
    constexpr int LB = KIND == K_FULL ? 1 : B ? LB_FIXED : LMAX;
    __shared__ uint32_t s_g;
    __shared__ int64_t s_cin;
    __shared__ uint32_t s_pk;  // the previous workgroup's top limb fixed the carry
    __shared__ int64_t s_pc;   // (and that carry)
    __shared__ double s_thW;
    __shared__ double sq[padq(DPW + K4_HALO) + 1];
    __shared__ int64_t sWA[NW], sWT[NW];
    __shared__ double sGD[NW], sGA[NW];
    __shared__ uint32_t sGF;
    __shared__ double s_edge[K4_HALO + 1];
    __shared__ double sc_edge[K4_HALO * K4_EP];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const C* q = reinterpret_cast<const C*>(p.za);

    if (tid == 0) {
        s_pk = 0;
        s_g = DIAG ? bk.x : atomicAdd(p.ticket, 1u);
        if (KIND == K_HI) s_thW = p.theta[0] * p.theta[1];
    }
    __syncthreads();
    const uint32_t g = s_g;
    const double thW = KIND == K_HI ? s_thW : 0.0;
    const uint64_t base = (uint64_t)g * DPW;
    const uint64_t i0 = base + (uint64_t)tid * DPT;
    const int b = B ? B : p.b;

    // stage q[base - HALO, base + DPW) (zero outside [0, N))
    if (tid == 0) sGF = 0;
    if (std::is_same<C, double2>::value && base >= (uint64_t)K4_HALO && base + DPW <= p.N) {
        // away from both ends: every index in range, no wrap
        const double2* qh = reinterpret_cast<const double2*>(p.za) + (base - K4_HALO) / 2;
        for (int e = 2 * tid; e < DPW + K4_HALO; e += 2 * NT4) {
            const double2 z = qh[e >> 1];
            sq[padq(e)] = z.x;
            sq[padq(e + 1)] = z.y;
        }
    } else if constexpr (std::is_same<C, double2>::value) {
        // pairs (i, i + 1) with i even (base, K4_HALO and N are even): one
        // 16-byte load of the packed result per pair
        for (int e = 2 * tid; e < DPW + K4_HALO; e += 2 * NT4) {
            int64_t i = (int64_t)base - K4_HALO + e;
            if (i < 0 && KIND != K_FULL) i += p.N;  // cyclic: wrapped terms of the maps
            const double2 z = (i >= 0 && i < (int64_t)p.N) ? q[i >> 1] : make_double2(0.0, 0.0);
            sq[padq(e)] = z.x;
            sq[padq(e + 1)] = z.y;
        }
    } else {
        for (int e = tid; e < DPW + K4_HALO; e += NT4) {
            int64_t i = (int64_t)base - K4_HALO + e;
            if (i < 0 && KIND != K_FULL) i += p.N;
            sq[padq(e)] = (i >= 0 && i < (int64_t)p.N) ? real_at(q, i) : 0.0;
        }
    }
    __syncthreads();
    // the previous workgroup's top limb, while its inputs are staged (the
    // last wavefront; the others meet it at the next barrier)
    if (K4_PREV_TOP && !DIAG && wv == NW - 1 && g > 0 && base <= (uint64_t)p.N) {
        bool pk;
        int64_t pc;
        prev_top_carry<KIND, B>(p, sq, base, b, lane, pk, pc);
        if (lane == 0 && pk) {
            s_pc = pc;
            s_pk = 1;
        }
    }

    // x_i (see back_edge / back_chain) and rounded coefficients, with the guard
    double xv[DPT];
    if constexpr (KIND == K_FULL) {
#pragma unroll
        for (int t = 0; t < DPT; t++) xv[t] = sq[padq(tid * DPT + t + K4_HALO)] * p.bscale;
    } else {
        constexpr int OFF = KIND == K_HI ? 1 : 0;
        constexpr int NOUT = DPT + OFF;
        double acc[NOUT];
        const int s0 = tid * DPT + K4_HALO - OFF - (LB - 1);
        back_chain<LB, NOUT, OFF>(p, sq, s0, (int64_t)i0 - OFF - (LB - 1), acc);
        if constexpr (KIND == K_LO) {
#pragma unroll
            for (int t = 0; t < DPT; t++) xv[t] = acc[t];
        } else {
            const double eps = ldexp(1.0, -b);
#pragma unroll
            for (int t = 0; t < DPT; t++) xv[t] = fma(-eps, acc[t], acc[t + 1]);
            // top coefficient: 2^b J_N = -2^-b 2^b H_(N-1) + 2^b theta_W
            if (base + DPW > p.N) {
#pragma unroll
                for (int t = 0; t < DPT; t++)
                    if (i0 + t == p.N) xv[t] = fma(-eps, acc[t], ldexp(thW, b));
            }
        }
        if (base == 0) {
            // indices next to the wrap: parts spread over threads, then one
            // fixed-order combination per index
            static_assert(K4_HALO * K4_EP <= NT4, "edge parts need one thread each");
            double* s_ep = reinterpret_cast<double*>(sc_edge);
            if (tid < K4_HALO * K4_EP)
                s_ep[tid] = edge_part<KIND>(p, sq, (uint32_t)(tid / K4_EP), tid % K4_EP);
            __syncthreads();
            if (tid <= K4_HALO)
                s_edge[tid] = tid ? edge_sum<KIND>(p, s_ep + (tid - 1) * K4_EP, (uint32_t)tid - 1) : 0.0;
            __syncthreads();
#pragma unroll
            for (int t = 0; t < DPT; t++)
                if (i0 + t < (uint64_t)K4_HALO) xv[t] = back_edge<KIND>(p, s_edge, (uint32_t)(i0 + t), thW);
        }
    }

    // rint by the 1.5 2^52 shift (exact and ties-to-even for |x| < 2^51;
    // larger |x| trip the guard's 2^50 bound)
    constexpr double RMAG = 6755399441055744.0;
    int64_t c[DPT];
    double dmax = 0.0, amax = 0.0;
    uint32_t gflags = 0;
    auto round_at = [&](int t, bool live) {
        const uint64_t i = i0 + t;
        const double xs = live ? xv[t] : 0.0;
        const double sh = xs + RMAG;
        const double r = sh - RMAG;
        c[t] = (int64_t)__double_as_longlong(sh) - (int64_t)__double_as_longlong(RMAG);
        dmax = fmax(dmax, fabs(xs - r));
        amax = fmax(amax, fabs(xs));
        if (DIAG && live) {
            p.dbg_c[i] = c[t];
            if (p.dbg_x) p.dbg_x[i] = xs;
        }
    };
    if (base + DPW <= p.ncoef) {  // every coefficient of the workgroup exists
#pragma unroll
        for (int t = 0; t < DPT; t++) round_at(t, true);
    } else {
#pragma unroll
        for (int t = 0; t < DPT; t++) round_at(t, i0 + t < p.ncoef);
    }
    if (KIND != K_FULL && i0 == 0 && (c[0] & ((1ll << b) - 1)) != 0) gflags |= TM_GUARD_C0;
    // guard: reduce over the workgroup (published at the end)
    dmax = wave_max(dmax);
    amax = wave_max(amax);
    if (gflags) atomicOr(&sGF, gflags);
    if (lane == 0) {
        sGD[wv] = dmax;
        sGA[wv] = amax;
    }
    // (read by the guard's publication after later barriers; the diagnostic
    // variant publishes here)
    if (DIAG) __syncthreads();
    // guard: one atomic per field and only when it raises the stored
    // maximum (non-negative doubles order like their bit patterns).  Done by
    // wave 1 during the look-back, off the other waves' path.
    auto publish_guard = [&]() {
        double dm = sGD[0], am = sGA[0];
        for (int w2 = 1; w2 < NW; w2++) {
            dm = fmax(dm, sGD[w2]);
            am = fmax(am, sGA[w2]);
        }
        uint64_t* gd = reinterpret_cast<uint64_t*>(&p.guard->max_dist);
        uint64_t* ga = reinterpret_cast<uint64_t*>(&p.guard->max_abs);
        const uint64_t bd = (uint64_t)__double_as_longlong(dm);
        const uint64_t ba = (uint64_t)__double_as_longlong(am);
        if (bd > ld_rlx(gd)) atomicMax(reinterpret_cast<unsigned long long*>(gd), (unsigned long long)bd);
        if (ba > ld_rlx(ga)) atomicMax(reinterpret_cast<unsigned long long*>(ga), (unsigned long long)ba);
        const uint32_t f = sGF | (dm >= 0.25 ? TM_GUARD_DIST : 0u) |
                           (am >= 1125899906842624.0 ? TM_GUARD_ABS : 0u);
        if (f) atomicOr(&p.guard->flags, f);
    };
    if (DIAG) {
        if (tid == 0) publish_guard();
        return;
    }

    if (KIND == K_HI) {
        // round(t) = floor((S + 2^(D-1)) / 2^D): add 2^(D-1) at its digit
        const uint64_t dm1 = p.off - 1;
        const uint64_t ih = dm1 / (uint64_t)b;
        if (ih >= i0 && ih < i0 + DPT) c[ih - i0] += 1ll << (dm1 - ih * (uint64_t)b);
    }

    // S = sum_i c_i 2^(ib).  This workgroup's DPW coefficients start in its
    // LPW = DPW b / 64 limbs of S (S limbs g LPW ..), limb j taking the c_i
    // that start in bits [64 j, 64 j + 64):  T_j = sum c_i 2^(ib - 64j), a
    // signed 128-bit value whose high half carries into limb j + 1.
    int64_t* sc = reinterpret_cast<int64_t*>(sq);  // coefficients reuse the q staging area
    __syncthreads();
#pragma unroll
    for (int t = 0; t < DPT; t++) sc[padq(tid * DPT + t)] = c[t];
    __syncthreads();
    const int LPW = DPW / 64 * b;
    // limbs per thread: lpt or lpt + 1 (threads below ex), at most MLPT
    constexpr int MLPT = (DPW / 64 * 16 + NT4 - 1) / NT4;
    static_assert(DPW % 64 == 0 && DPW / 64 * 8 >= NT4, "every thread holds a limb for b >= 8");
    const int lpt = LPW / NT4, ex = LPW % NT4;
    const int j0 = tid * lpt + (tid < ex ? tid : ex);
    const int nl = lpt + (tid < ex ? 1 : 0);
    uint64_t tlo[MLPT];
    int64_t thi[MLPT];
    CarryF fl[MLPT];
#pragma unroll
    for (int k = 0; k < MLPT; k++) {
        tlo[k] = 0;
        thi[k] = 0;
        fl[k] = CarryF{0, INT64_MAX};
        if (k < nl) {
            const int j = j0 + k;
            // c_i, ia <= i < ib, start in limb j: at most ceil(64 / b) of them
            const int ia = (64 * j + b - 1) / b, ib = (64 * (j + 1) + b - 1) / b;
            unsigned __int128 tacc = 0;
#pragma unroll
            for (int u = 0; u < (B ? (64 + B - 1) / B : 8); u++) {
                const int i = ia + u;
                if (i < ib) {
                    // c_i 2^sh as a 128-bit two's-complement term: the low
                    // word c_i << sh, the high word floor(c_i 2^sh / 2^64)
                    const int64_t cv = sc[padq(i)];
                    const int sh = i * b - 64 * j;
                    const uint64_t plo = (uint64_t)cv << sh;
                    const uint64_t phi = (uint64_t)((cv >> 1) >> (63 - sh));
                    tacc += ((unsigned __int128)phi << 64) | plo;
                }
            }
            tlo[k] = (uint64_t)tacc;
            thi[k] = (int64_t)(uint64_t)(tacc >> 64);
            fl[k] = limb_carry_fn(tlo[k], thi[k]);
        }
    }
    CarryF f = fl[0];
#pragma unroll
    for (int k = 1; k < MLPT; k++)
        if (k < nl) f = compose(f, fl[k]);

    // inclusive scan of carry functions: within each wave by DPP lane moves,
    // then across the NW waves through LDS
    f = wave_scan(f, lane);
    if (lane == 63) {
        sWA[wv] = f.A;
        sWT[wv] = f.T;
    }
    __syncthreads();
    // prefix of the waves below, from the nearest one down, stopping at the
    // first constant composition (which the waves further down cannot change)
    CarryF pre = {0, INT64_MAX};
    const bool have_pre = wv > 0;
    for (int w2 = wv - 1; w2 >= 0; w2--) {
        const CarryF t = {sWA[w2], sWT[w2]};
        pre = w2 == wv - 1 ? t : compose(t, pre);
        if (pre.T == INT64_MAX) break;
    }
    if (have_pre) f = compose(pre, f);
    // exclusive prefix of this thread
    const int64_t ea = (int64_t)dpp64<0x138>(0, (uint64_t)f.A);  // wave_shr:1
    const int64_t et = (int64_t)dpp64<0x138>(0, (uint64_t)f.T);
    CarryF excl = lane > 0 ? CarryF{ea, et} : pre;
    const bool have_excl = lane > 0 || have_pre;

    // the guard's global atomics go out from wave 1 while wave 0 looks back
    if (wv == 1 && lane == 0) publish_guard();

    // decoupled look-back, one wavefront.  status[2g] = state | A (aggregate),
    // state | C (inclusive or constant aggregate: the carry-out), and for a
    // non-constant aggregate status[2g+1] = state | T.  Values
    // are carries (|c| < 2^53) and thresholds clamped to +-2^61, which act
    // as +-infinity for such carries.
    if (wv == 0) {
        CarryF agg = {sWA[NW - 1], sWT[NW - 1]};
        for (int w2 = NW - 2; w2 >= 0 && agg.T != INT64_MAX; w2--) agg = compose(CarryF{sWA[w2], sWT[w2]}, agg);
        uint64_t* st = p.status;
        int64_t cin = 0;
        // the previous workgroup's top limb usually fixes the carry alone
        const bool known = K4_PREV_TOP && s_pk != 0;
        if (known) cin = s_pc;
        if (g > 0 && !known) {
            if (lane == 0) {
                if (agg.T == INT64_MAX || agg.T == INT64_MIN) {
                    st_rlx(&st[2 * g + 0], pack62(3, apply(agg, 0)));
                } else {
                    st_rlx(&st[2 * g + 1], pack62(1, agg.T));
                    st_rlx(&st[2 * g + 0], pack62(1, agg.A));
                }
            }
            CarryF acc = {0, INT64_MAX};
            bool have_acc = false;
            int64_t e = (int64_t)g - 1;
            bool timed_out = false;
            uint32_t spins = 0;
            // Window of the 64 records below e, read without blocking.  A
            // record absorbs when it fixes the carry by itself: an inclusive
            // record, a constant aggregate, or the start of the number.  The
            // window is usable as soon as the nearest absorbing record and
            // every record between it and e are published: records further
            // back cannot change the carry, so they are not waited for.
            while (true) {
                const int64_t idx = e - 63 + lane;
                bool ready = true, absorb = true;
                CarryF fv = {0, INT64_MAX};  // before the number: carry 0
                if (idx >= 0) {
                    const uint64_t wa = ld_rlx(&st[2 * idx]);
                    const uint64_t sa = wa >> 62;
                    if (sa >= 2) {  // inclusive, or constant aggregate: the carry-out
                        fv.A = unpack62(wa);
                    } else if (sa == 1) {
                        const uint64_t wt = ld_rlx(&st[2 * idx + 1]);
                        if ((wt >> 62) == 0) {
                            ready = absorb = false;
                        } else {
                            fv.A = unpack62(wa);
                            fv.T = unpack62(wt);
                            fv.T = fv.T <= V62_MIN ? INT64_MIN : fv.T >= V62_MAX ? INT64_MAX : fv.T;
                            absorb = fv.T == INT64_MAX || fv.T == INT64_MIN;
                        }
                    } else {
                        ready = absorb = false;
                    }
                }
                const uint64_t mr = __ballot(ready), ma = __ballot(absorb);
                const int top = ma ? 63 - __clzll((long long)ma) : 0;  // nearest absorbing lane
                const uint64_t need = ~0ull << top;                      // lanes top .. 63
                if ((mr & need) != need) {
                    if (++spins > SPIN_LIMIT) {
                        timed_out = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                    continue;
                }
                CarryF r;
                if (ma >> 63) {
                    // the nearest record (the usual case) fixes the carry
                    r.A = __shfl(fv.A, 63);
                    r.T = __shfl(fv.T, 63);
                } else {
                    if (ma && lane < top) fv = CarryF{0, INT64_MAX};  // absorbed: any constant
                    // ordered reduction: lane 0 ends with f_(idx 63) o ... o f_(idx 0)
                    r = fv;
#pragma unroll
                    for (int d = 1; d < 64; d <<= 1) {
                        const int64_t oa = __shfl_down(r.A, d), ot = __shfl_down(r.T, d);
                        if ((lane & (2 * d - 1)) == 0) r = compose(r, CarryF{oa, ot});
                    }
                    r.A = __shfl(r.A, 0);
                    r.T = __shfl(r.T, 0);
                }
                const CarryF tot = have_acc ? compose(r, acc) : r;
                // done at an absorbing record, or as soon as the carry no
                // longer depends on what lies further back (constant function)
                if (ma || tot.T == INT64_MAX) {
                    cin = apply(tot, 0);
                    break;
                }
                acc = tot;
                have_acc = true;
                e -= 64;
                spins = 0;
            }
            if (__ballot(timed_out) != 0 && lane == 0) atomicOr(&p.guard->flags, TM_GUARD_SPIN);
        }
        if (lane == 0) {
            st_rlx(&st[2 * g + 0], pack62(2, apply(agg, cin)));
            s_cin = cin;
        }
    }
    // the carry into this workgroup: from the previous workgroup's top limb
    // (known to every wave, no wait for wave 0), else from the look-back
    // (after a barrier).  Every read of sc ended before the scan's barrier,
    // so the limb values sS may reuse the space.
    const bool cknown = K4_PREV_TOP && s_pk != 0;
    if (!cknown) __syncthreads();
    const int64_t cwg = cknown ? s_pc : s_cin;
    int64_t cin = have_excl ? apply(excl, cwg) : cwg;
    uint64_t* sS = reinterpret_cast<uint64_t*>(sq);
#pragma unroll
    for (int k = 0; k < MLPT; k++) {
        if (k < nl) {
            sS[j0 + k] = tlo[k] + (uint64_t)cin;
            cin = apply(fl[k], cin);
        }
    }
    __syncthreads();

    // extraction: output bit j = bit (j + off) of S; output limbs that
    // straddle two workgroups' limbs are OR-ed together (K1 zeroed them)
    const int64_t sb0 = (int64_t)g * LPW * 64, sb1 = sb0 + (int64_t)LPW * 64;
    const int64_t ob0 = sb0 - (int64_t)p.off, ob1 = sb1 - (int64_t)p.off;
    const int64_t lo_o = ob0 > 0 ? ob0 : 0;
    const int64_t hi_o = ob1 < (int64_t)p.out_bits ? ob1 : (int64_t)p.out_bits;
    if (hi_o > lo_o) {
    const int64_t l0 = lo_o >> 6, l1 = (hi_o - 1) >> 6;
    const int r = (int)(p.off & 63);
    for (int64_t li = l0 + tid; li <= l1; li += NT4) {
        const int64_t sl = li * 64 + (int64_t)p.off;  // S bit of output bit 64 li
        const int64_t jl = (sl >> 6) - (int64_t)g * LPW;
        uint64_t val = 0;
        if (jl >= 0 && jl < LPW) val |= sS[jl] >> r;
        if (r && jl + 1 >= 0 && jl + 1 < LPW) val |= sS[jl + 1] << (64 - r);
        if ((uint64_t)(li + 1) * 64 > p.out_bits) {
            const int keep = (int)(p.out_bits - (uint64_t)li * 64);
            val &= (1ull << keep) - 1;
        }
        const bool full = sl >= sb0 && sl + 64 <= sb1 && (uint64_t)(li + 1) * 64 <= p.out_bits;
        if (full) p.w[li] = val;
        else atomicOr(reinterpret_cast<unsigned long long*>(&p.w[li]), (unsigned long long)val);
    }
    }
}

// eight waves per SIMD (two 1024-thread workgroups per CU, as the LDS
// allows).  Every workgroup takes one ticket, an atomic on a single address
// that serialises at roughly 13 ns per ticket; 8192 coefficients per
// workgroup keep that below the kernel's other work (with 4096 it bounded
// the full product's K4 at n = 2^30)
template <int KIND, bool DIAG, int B, typename C = double2>
__global__ __launch_bounds__(NT4, K4_WAVES) void k4_backmap_carry(KParams p)
{
    k4_body<KIND, DIAG, B, C>(p, blk_hw());
}

template <int KIND, int B>
__global__ __launch_bounds__(NT4, K4_WAVES) void k4_backmap_carry_g(Group g)
{
    uint32_t pi;
    const Blk bk = group_block(g, pi);
    const KParams& p = group_params(g, pi);
    k4_body<KIND, false, B>(p, bk);
}

}  // namespace tmul
