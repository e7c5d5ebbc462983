// HIP kernels of the truncated / full product path (gfx950, FP64).
//
// One multiplication is four launches on one stream:
//   K1 split + ring map + forward column pass   (Alg. low/high steps 2-3,
//      first half of the forward FFTs of step 4; Alg. full steps 2-3)
//   K2 forward row pass, pointwise product, inverse row pass (step 4)
//   K3 inverse column pass                       (end of step 4)
//   K4 back-map, rounding, guard, carry propagation, extraction (steps 5-6)
//
// The real convolution of length N is computed with complex FFTs of length
// M = N/2: a real sequence G is packed as y_m = G_2m + i G_2m+1.  The two
// operands are transformed separately; their length-N real spectra are
// recovered from the bins k and M-k of the packed transforms, multiplied,
// and repacked for a length-M inverse, all in K2.  M = L1 * L2 is split
// four-step style: K1/K3 do the L1-point column DFTs (stride L2), K2 the
// L2-point row DFTs; the spectrum stays in the row-major "scrambled" order
// (position k1*L2 + k2 holds bin k1 + L1*k2), so no transpose pass exists.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_tile.hpp"
#include "tmul.h"

namespace tmul {

enum { K_FULL = 0, K_LO = 1, K_HI = 2 };

constexpr int NT = 256;         // threads per workgroup, every kernel
constexpr int LMAX = 9;         // largest supported series length lambda
constexpr int DPT = 7;          // digits per thread in K4
constexpr int DPW = DPT * NT;   // digits per workgroup in K4
constexpr int TILE = 4096;      // complex elements per column tile (64 KiB)
constexpr uint32_t SPIN_LIMIT = 1u << 22;

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
    uint32_t M, L1, L2; // complex length and its split
    uint32_t jmax;      // powers 2^-jb kept in the high-product wrap terms
    int64_t shift;      // high product: s = (N+1) b - n
    uint64_t off;       // output = bits [off, off+out_bits) of S
    uint64_t out_bits;
    uint64_t out_limbs;
    uint32_t ncoef;     // rounded coefficients (low N, high N+1, full N)
    uint32_t ncover;    // digit positions carried (multiple of DPW)
    uint32_t nstatus;   // K4 workgroups
    uint32_t pad0;
    double invN, invM;
    double cf[LMAX];    // (-eps)^r / r! or eps^r / r! for the forward map
    double cb[LMAX];    // same for the back map
    double2* za;        // operand u spectrum / convolution result
    double2* zb;        // operand v spectrum
    uint64_t* status;   // K4 look-back records, 4 words each
    uint32_t* ticket;   // K4 dynamic workgroup counter
    tm_guard* guard;
    Tw tw;
    int64_t* dbg_c;     // diagnostic outputs (tm_coefficients) or null
    double* dbg_x;
};

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

// Series coefficients (closed forms of the binomial definitions, Sections
// 3.2 and 4.2); c = (-+eps)^r / r! supplied by the host.
//   alpha_{k,r} = c (k/N) prod_{j=1}^{r-1} ((k+r)/N - j)
//   gamma_{k,r} = c (k/N) prod_{j=1}^{r-1} ((k+r)/N + j)
//   beta_{k,r}  = c prod_{j=0}^{r-1} (k/N + j)
//   delta_{k,r} = c prod_{j=0}^{r-1} (k/N - j)
__device__ __forceinline__ double coef_fwd(int kind, uint32_t k, int r, double invN, double c)
{
    if (r == 0) return 1.0;
    const double x = (double)k * invN, y = (double)(k + (uint32_t)r) * invN;
    double p = x;
    if (kind == K_LO) {
        for (int j = 1; j < r; j++) p *= (y - (double)j);
    } else {
        for (int j = 1; j < r; j++) p *= (y + (double)j);
    }
    return p * c;
}

__device__ __forceinline__ double coef_back(int kind, uint32_t k, int r, double invN, double c)
{
    if (r == 0) return 1.0;
    const double x = (double)k * invN;
    double p = 1.0;
    if (kind == K_LO) {
        for (int j = 0; j < r; j++) p *= (x + (double)j);
    } else {
        for (int j = 0; j < r; j++) p *= (x - (double)j);
    }
    return p * c;
}

// Top digit F_N of the high-product split and theta = rho^-N F(rho) with
// rho ~ 2^b (Remark on Newton's method): theta = sum_j 2^(-jb) F_(N-j).
__device__ __forceinline__ double hi_theta(const KParams& p, const uint64_t* x)
{
    double t = 0.0;
    for (int j = 0; j <= (int)p.jmax && j <= (int)p.N; j++) {
        double f = (double)bal_digit(p, x, (int64_t)p.N - j, p.digits, true);
        t += ldexp(f, -j * p.b);
    }
    return t;
}

// G_j and G_(j+1) of the sequence fed to the convolution:
//   full: the digits themselves (zero beyond the digit count);
//   low:  G = alpha* U   (Prop. approximating alpha*), cyclic indices;
//   high: G = gamma* F'  with F'_k = F_k + 2^(-kb) F_N  (F mod C by eq.
//         reduction-modC with rho ~ 2^b, Prop. approximating gamma-dagger).
template <int KIND>
__device__ __forceinline__ void gen_pair(const KParams& p, const uint64_t* x, uint32_t j,
                                         double FN, double& g0, double& g1)
{
    if constexpr (KIND == K_FULL) {
        g0 = j < p.digits ? (double)bal_digit(p, x, j, p.digits, true) : 0.0;
        g1 = j + 1 < p.digits ? (double)bal_digit(p, x, j + 1, p.digits, true) : 0.0;
    } else {
        const uint32_t N = p.N;
        const int lam = p.lam;
        // d[t] = F'_(k) with k = (j + 1 - lam + t) mod N, t = 0..lam
        double d[LMAX + 1];
#pragma unroll
        for (int t = 0; t <= LMAX; t++) {
            if (t <= lam) {
                uint32_t k = (uint32_t)(((int64_t)j + 1 - lam + t + (int64_t)N) % N);
                double f = (double)bal_digit(p, x, k, p.digits, KIND == K_HI);
                if (KIND == K_HI && k < p.jmax) f += ldexp(FN, -(int)k * p.b);
                d[t] = f;
            }
        }
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int r = LMAX - 1; r >= 0; r--) {
            if (r < lam) {
                // G_j gets F'_(j-r) = d[lam-1-r]; G_(j+1) gets F'_(j+1-r) = d[lam-r]
                uint32_t k0 = (uint32_t)(((int64_t)j - r + (int64_t)N) % N);
                uint32_t k1 = (uint32_t)(((int64_t)j + 1 - r + (int64_t)N) % N);
                s0 = fma(coef_fwd(KIND, k0, r, p.invN, p.cf[r]), d[lam - 1 - r], s0);
                s1 = fma(coef_fwd(KIND, k1, r, p.invN, p.cf[r]), d[lam - r], s1);
            }
        }
        g0 = s0;
        g1 = s1;
    }
}

// Clear the per-call state that K4 accumulates into (output limbs for the
// partial-limb OR, guard, look-back records, ticket).  Done by K1.
__device__ __forceinline__ void clear_state(const KParams& p, uint32_t gid, uint32_t gsize)
{
    for (uint64_t i = gid; i < p.out_limbs; i += gsize) p.w[i] = 0;
    for (uint64_t i = gid; i < 4ull * p.nstatus; i += gsize) p.status[i] = 0;
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

template <int L1, int W, int KIND>
__global__ __launch_bounds__(NT) void k1_split_map_col(KParams p)
{
    static_assert(L1 * W <= TILE, "tile too large");
    __shared__ double2 tile[L1 * W];
    __shared__ double s_FN;
    const int op = blockIdx.y;
    const uint64_t* x = op ? p.v : p.u;
    double2* dst = op ? p.zb : p.za;
    const uint32_t L2 = p.L2;
    const uint32_t c0 = blockIdx.x * W;

    if (op == 0) clear_state(p, blockIdx.x * NT + threadIdx.x, gridDim.x * NT);
    if (KIND == K_HI && threadIdx.x == 0) s_FN = (double)bal_digit(p, x, p.N, p.digits, true);
    __syncthreads();
    const double FN = KIND == K_HI ? s_FN : 0.0;

    for (int e = threadIdx.x; e < L1 * W; e += NT) {
        const int c = e % W, j1 = e / W;
        const uint32_t m = (uint32_t)j1 * L2 + c0 + c;
        double g0, g1;
        gen_pair<KIND>(p, x, 2 * m, FN, g0, g1);
        tile[e] = make_double2(g0, g1);
    }
    __syncthreads();
    tile_fft<L1, W, NT, false, true>(tile, p.tw, p.M / L1);
    for (int e = threadIdx.x; e < L1 * W; e += NT) {
        const int c = e % W, k1 = e / W;
        const uint32_t col = c0 + c;
        double2 val = tile[e];
        if (k1 != 0 && col != 0) val = cmul(val, tw_get<false>(p.tw, col * (uint32_t)k1));
        dst[(size_t)k1 * L2 + col] = val;
    }
}

// ------------------------------------------------------------------- K2

// Spectra of the two real operands from the packed transforms, product, and
// repacking for the half-length inverse.  With Y the packed transform and
// M - k the mirror bin: E_k = (Y_k + conj Y_(M-k))/2, O_k = (Y_k - conj
// Y_(M-k))/(2i) (even / odd sample spectra); the product spectrum's even
// and odd parts are E'_k = Ea Eb + w^k Oa Ob and O'_k = Ea Ob + Oa Eb with
// w = exp(-2 pi i / M), and Q_k = E'_k + i O'_k is the length-M transform of
// (W_2m + i W_2m+1) (times M).
__device__ __forceinline__ double2 pointwise_bin(double2 Ya, double2 Yam, double2 Yb, double2 Ybm,
                                                 double2 wk)
{
    double2 Ea = cscale(cadd(Ya, cconj(Yam)), 0.5);
    double2 Oa = cscale(csub(Ya, cconj(Yam)), 0.5);
    Oa = make_double2(Oa.y, -Oa.x);  // divide by i
    double2 Eb = cscale(cadd(Yb, cconj(Ybm)), 0.5);
    double2 Ob = cscale(csub(Yb, cconj(Ybm)), 0.5);
    Ob = make_double2(Ob.y, -Ob.x);
    double2 X = cadd(cmul(Ea, Eb), cmul(wk, cmul(Oa, Ob)));
    double2 Yv = cadd(cmul(Ea, Ob), cmul(Oa, Eb));
    return make_double2(X.x - Yv.y, X.y + Yv.x);  // X + i Yv
}

template <int L2>
__global__ __launch_bounds__(NT) void k2_rows_pointwise(KParams p)
{
    // rows 0,1: operands u,v at row k1; rows 2,3: at the mirror row
    __shared__ double2 rows[4 * L2];
    const uint32_t L1 = p.L1;
    const uint32_t k1 = blockIdx.x;
    const uint32_t k1m = (L1 - k1) % L1;
    for (int e = threadIdx.x; e < 4 * L2; e += NT) {
        const int r = e / L2, j2 = e % L2;
        const uint32_t row = r < 2 ? k1 : k1m;
        const double2* src = (r & 1) ? p.zb : p.za;
        rows[e] = src[(size_t)row * L2 + j2];
    }
    __syncthreads();
    tile_fft<L2, 4, NT, false, false, L2>(rows, p.tw, p.M / L2);

    constexpr int PER = (2 * L2 + NT - 1) / NT;
    double2 qv[PER];
#pragma unroll
    for (int t = 0; t < PER; t++) {
        const int e = threadIdx.x + t * NT;
        if (e < 2 * L2) {
            const int pr = e / L2, k2 = e % L2;
            const uint32_t rho = pr ? k1m : k1;
            const int mk2 = rho == 0 ? (L2 - k2) % L2 : L2 - 1 - k2;
            const int mr = 1 - pr;
            const uint32_t k = rho + L1 * (uint32_t)k2;
            qv[t] = pointwise_bin(rows[(2 * pr) * L2 + k2], rows[(2 * mr) * L2 + mk2],
                                  rows[(2 * pr + 1) * L2 + k2], rows[(2 * mr + 1) * L2 + mk2],
                                  tw_get<false>(p.tw, k));
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; t++) {
        const int e = threadIdx.x + t * NT;
        if (e < 2 * L2) {
            const int pr = e / L2, k2 = e % L2;
            rows[(2 * pr) * L2 + k2] = qv[t];
        }
    }
    __syncthreads();
    // inverse row DFTs of rows 0 and 2 (row stride 2*L2)
    tile_fft<L2, 2, NT, true, false, 2 * L2>(rows, p.tw, p.M / L2);
    for (int e = threadIdx.x; e < 2 * L2; e += NT) {
        const int pr = e / L2, j2 = e % L2;
        if (pr == 1 && k1m == k1) continue;
        const uint32_t rho = pr ? k1m : k1;
        double2 val = rows[(2 * pr) * L2 + j2];
        if (rho != 0 && j2 != 0) val = cmul(val, tw_get<true>(p.tw, (uint32_t)j2 * rho));
        p.za[(size_t)rho * L2 + j2] = val;
    }
}

// ------------------------------------------------------------------- K3

template <int L1, int W>
__global__ __launch_bounds__(NT) void k3_col_inverse(KParams p)
{
    __shared__ double2 tile[L1 * W];
    const uint32_t L2 = p.L2;
    const uint32_t c0 = blockIdx.x * W;
    for (int e = threadIdx.x; e < L1 * W; e += NT) {
        const int c = e % W, k1 = e / W;
        tile[e] = p.za[(size_t)k1 * L2 + c0 + c];
    }
    __syncthreads();
    tile_fft<L1, W, NT, true, true>(tile, p.tw, p.M / L1);
    for (int e = threadIdx.x; e < L1 * W; e += NT) {
        const int c = e % W, j1 = e / W;
        p.za[(size_t)j1 * L2 + c0 + c] = tile[e];
    }
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

__device__ __forceinline__ uint64_t ld_acq(uint64_t* a)
{
    return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t* a, uint64_t v)
{
    __hip_atomic_store(a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rlx(uint64_t* a)
{
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint64_t* a, uint64_t v)
{
    __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// x_i: the value rounded to c_i (see tm_guard)
//   full: W_i                                       (Alg. full, step 4)
//   low:  2^b W-bar_i with W-bar = beta* W (mod A)  (Prop. approximating
//         beta*; X^(N+s) = X^s - 2^-b X^(s+1) for the wrapped terms)
//   high: 2^b J_i, J = (1 - 2^-b X) H + psi C(X), H = delta* W (mod C),
//         psi ~ theta_W, C_j ~ -2^(-jb)  (eq. crt-sum, Remark on Newton)
template <int KIND>
__device__ __forceinline__ double x_value(const KParams& p, const double* q, uint32_t i, double thW)
{
    const uint32_t N = p.N;
    const int lam = p.lam, b = p.b;
    if constexpr (KIND == K_FULL) {
        return q[i] * p.invM;
    } else if constexpr (KIND == K_LO) {
        double s = 0.0;
        for (int r = 0; r < lam; r++) {
            if ((uint32_t)r <= i) s = fma(coef_back(K_LO, i - r, r, p.invN, p.cb[r]), q[i - r], s);
            else s = fma(coef_back(K_LO, N + i - r, r, p.invN, p.cb[r]), q[N + i - r], s);
        }
        if (i >= 1 && i < (uint32_t)lam) {
            double t = 0.0;
            for (int r = (int)i; r < lam; r++)
                t = fma(coef_back(K_LO, N + i - 1 - r, r, p.invN, p.cb[r]), q[N + i - 1 - r], t);
            s = fma(-ldexp(1.0, -b), t, s);
        }
        return ldexp(s * p.invM, b);
    } else {
        // H_i for i < N (H on the unnormalised q)
        auto H = [&](uint32_t ii) -> double {
            double s = 0.0;
            for (int r = 0; r < lam && (uint32_t)r <= ii; r++)
                s = fma(coef_back(K_HI, ii - r, r, p.invN, p.cb[r]), q[ii - r], s);
            if (ii < (uint32_t)lam + p.jmax) {
                // X^(N+s') = sum_j 2^(-jb) X^(s'+j) mod C: target ii = s' + j
                for (int j = 0; j <= (int)ii && j <= (int)p.jmax; j++) {
                    double t = 0.0;
                    for (int r = (int)ii - j + 1; r < lam; r++)
                        t = fma(coef_back(K_HI, N + ii - j - r, r, p.invN, p.cb[r]), q[N + ii - j - r], t);
                    s = fma(ldexp(1.0, -j * b), t, s);
                }
            }
            return s;
        };
        const double eps = ldexp(1.0, -b);
        double J;
        if (i < N) {
            double h = H(i);
            double hm = i ? H(i - 1) : 0.0;
            J = fma(-eps, hm, h) * p.invM - ldexp(thW, -(int)i * b);
        } else {
            J = -eps * H(N - 1) * p.invM + thW;
        }
        return ldexp(J, b);
    }
}

template <int KIND, bool DIAG>
__global__ __launch_bounds__(NT) void k4_backmap_carry(KParams p)
{
    __shared__ uint32_t s_g;
    __shared__ int64_t s_cin;
    __shared__ double s_thW;
    __shared__ int64_t sA[NT], sT[NT];
    __shared__ uint16_t sd[DPW];
    const int tid = threadIdx.x;
    const double* q = reinterpret_cast<const double*>(p.za);

    if (tid == 0) {
        s_g = DIAG ? blockIdx.x : atomicAdd(p.ticket, 1u);
        if (KIND == K_HI) s_thW = hi_theta(p, p.u) * hi_theta(p, p.v);
    }
    __syncthreads();
    const uint32_t g = s_g;
    const double thW = KIND == K_HI ? s_thW : 0.0;
    const uint64_t base = (uint64_t)g * DPW;
    const uint64_t i0 = base + (uint64_t)tid * DPT;
    const int b = p.b;

    // rounded coefficients and guard
    int64_t c[DPT];
    double dmax = 0.0, amax = 0.0;
    uint32_t gflags = 0;
#pragma unroll
    for (int t = 0; t < DPT; t++) {
        const uint64_t i = i0 + t;
        c[t] = 0;
        if (i < p.ncoef) {
            const double xv = x_value<KIND>(p, q, (uint32_t)i, thW);
            const double r = rint(xv);
            const double ax = fabs(xv);
            dmax = fmax(dmax, fabs(xv - r));
            amax = fmax(amax, ax);
            if (ax < 4503599627370496.0) c[t] = (int64_t)r;  // |x| < 2^52
            if (DIAG) {
                p.dbg_c[i] = c[t];
                if (p.dbg_x) p.dbg_x[i] = xv;
            }
            if (KIND != K_FULL && i == 0 && (c[t] & ((1ll << b) - 1)) != 0) gflags |= TM_GUARD_C0;
        }
    }
    dmax = wave_max(dmax);
    amax = wave_max(amax);
    if ((tid & 63) == 0) {
        atomicMax(reinterpret_cast<unsigned long long*>(&p.guard->max_dist),
                  (unsigned long long)__double_as_longlong(dmax));
        atomicMax(reinterpret_cast<unsigned long long*>(&p.guard->max_abs),
                  (unsigned long long)__double_as_longlong(amax));
        uint32_t f = (dmax >= 0.25 ? TM_GUARD_DIST : 0u) | (amax >= 1125899906842624.0 ? TM_GUARD_ABS : 0u);
        if (f) atomicOr(&p.guard->flags, f);
    }
    if (gflags) atomicOr(&p.guard->flags, gflags);
    if (DIAG) return;

    if (KIND == K_HI) {
        // round(t) = floor((S + 2^(D-1)) / 2^D): add 2^(D-1) at its digit
        const uint64_t dm1 = p.off - 1;
        const uint64_t ih = dm1 / (uint64_t)b;
        if (ih >= i0 && ih < i0 + DPT) c[ih - i0] += 1ll << (dm1 - ih * (uint64_t)b);
    }

    // carry function of this thread's digits: digit sweep with carry 0
    const int64_t mask = (1ll << b) - 1;
    int64_t carry = 0;
    unsigned __int128 l = 0;
#pragma unroll
    for (int t = 0; t < DPT; t++) {
        int64_t s = c[t] + carry;
        l |= (unsigned __int128)(uint64_t)(s & mask) << (t * b);
        carry = s >> b;
    }
    const int B = DPT * b;
    CarryF f;
    if (l < ((unsigned __int128)1 << (B - 1))) {
        f.A = carry - 1;
        f.T = l > (unsigned __int128)INT64_MAX ? INT64_MIN : -(int64_t)(uint64_t)l;
    } else {
        unsigned __int128 t = ((unsigned __int128)1 << B) - l;
        f.A = carry;
        f.T = t > (unsigned __int128)INT64_MAX ? INT64_MAX : (int64_t)(uint64_t)t;
    }

    // inclusive scan of carry functions over the workgroup (Hillis-Steele)
    sA[tid] = f.A;
    sT[tid] = f.T;
    __syncthreads();
    for (int d = 1; d < NT; d <<= 1) {
        CarryF mine = {sA[tid], sT[tid]};
        CarryF prev = {0, 0};
        if (tid >= d) prev = CarryF{sA[tid - d], sT[tid - d]};
        __syncthreads();
        if (tid >= d) {
            CarryF r = compose(prev, mine);
            sA[tid] = r.A;
            sT[tid] = r.T;
        }
        __syncthreads();
    }

    // decoupled look-back over workgroups: status[4g..4g+3] = flag, A, T, C
    if (tid == 0) {
        const CarryF agg = {sA[NT - 1], sT[NT - 1]};
        uint64_t* st = p.status;
        st_rlx(&st[4 * g + 1], (uint64_t)agg.A);
        st_rlx(&st[4 * g + 2], (uint64_t)agg.T);
        st_rel(&st[4 * g + 0], 1);
        int64_t cin = 0;
        if (g > 0) {
            bool have = false;
            CarryF acc = {0, 0};
            int64_t j = (int64_t)g - 1;
            while (true) {
                uint64_t fl;
                uint32_t spins = 0;
                while ((fl = ld_acq(&st[4 * j])) == 0) {
                    if (++spins > SPIN_LIMIT) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                if (fl == 0) {
                    atomicOr(&p.guard->flags, TM_GUARD_SPIN);
                    cin = 0;
                    break;
                }
                if (fl == 2) {
                    int64_t C = (int64_t)ld_rlx(&st[4 * j + 3]);
                    cin = have ? apply(acc, C) : C;
                    break;
                }
                CarryF fj = {(int64_t)ld_rlx(&st[4 * j + 1]), (int64_t)ld_rlx(&st[4 * j + 2])};
                acc = have ? compose(fj, acc) : fj;
                have = true;
                if (j == 0) {  // the number starts with carry 0
                    cin = apply(acc, 0);
                    break;
                }
                j--;
            }
        }
        const int64_t cout = apply(agg, cin);
        st_rlx(&st[4 * g + 3], (uint64_t)cout);
        st_rel(&st[4 * g + 0], 2);
        s_cin = cin;
    }
    __syncthreads();

    // final digits with the true carry-in
    int64_t cin = s_cin;
    if (tid > 0) cin = apply(CarryF{sA[tid - 1], sT[tid - 1]}, cin);
    carry = cin;
#pragma unroll
    for (int t = 0; t < DPT; t++) {
        int64_t s = c[t] + carry;
        sd[tid * DPT + t] = (uint16_t)(s & mask);
        carry = s >> b;
    }
    __syncthreads();

    // extraction: output bit j = bit (j + off) of S
    const int64_t sb0 = (int64_t)(base * b), sb1 = (int64_t)((base + DPW) * b);
    const int64_t ob0 = sb0 - (int64_t)p.off, ob1 = sb1 - (int64_t)p.off;
    const int64_t lo_o = ob0 > 0 ? ob0 : 0;
    const int64_t hi_o = ob1 < (int64_t)p.out_bits ? ob1 : (int64_t)p.out_bits;
    if (hi_o <= lo_o) return;
    const int64_t l0 = lo_o >> 6, l1 = (hi_o - 1) >> 6;
    for (int64_t li = l0 + tid; li <= l1; li += NT) {
        const int64_t sl = li * 64 + (int64_t)p.off;  // S bit of output bit 64 li
        const int64_t a = sl > sb0 ? sl : sb0;
        const int64_t z = sl + 64 < sb1 ? sl + 64 : sb1;
        uint64_t val = 0;
        for (int64_t i = a / b; i * b < z; i++) {
            const uint64_t dv = sd[i - (int64_t)base];
            const int64_t sh = i * b - sl;
            val |= sh >= 0 ? (dv << sh) : (dv >> (-sh));
        }
        if ((uint64_t)(li + 1) * 64 > p.out_bits) {
            const int keep = (int)(p.out_bits - (uint64_t)li * 64);
            val &= (1ull << keep) - 1;
        }
        const bool full = sl >= sb0 && sl + 64 <= sb1 && (uint64_t)(li + 1) * 64 <= p.out_bits;
        if (full) p.w[li] = val;
        else atomicOr(reinterpret_cast<unsigned long long*>(&p.w[li]), (unsigned long long)val);
    }
}

// twiddle table: lo[e] = exp(-2 pi i e/M) for e < S, hi[e] = exp(-2 pi i e S/M)
__global__ void k_twiddles(double2* lo, double2* hi, uint32_t M, uint32_t S, uint32_t nhi)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) {
        double s, c;
        sincospi(-2.0 * ((double)i / (double)M), &s, &c);
        lo[i] = make_double2(c, s);
    }
    if (i < nhi) {
        const uint64_t e = ((uint64_t)i * S) % M;
        double s, c;
        sincospi(-2.0 * ((double)e / (double)M), &s, &c);
        hi[i] = make_double2(c, s);
    }
}

}  // namespace tmul
