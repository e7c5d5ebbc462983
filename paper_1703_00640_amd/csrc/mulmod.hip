// Barrett modular multiplication on top of the truncated products (see
// tm_mulmod in include/tmul.h).
//
// r = a b mod m for an n-bit modulus m (2^(n-1) < m < 2^n) and the caller's
// mu = floor(2^(2n) / m):
//   x  = a b                                   full product, 2n bits
//   q1 = floor(x / 2^(n-1))                    n + 1 bits
//   w  = high product of q1 and mu at n + 1 bits: |q1 mu - 2^(n+1) w| < 2^(n+1)
//   y  = w m mod 2^(n+2)                       low product at n + 2 bits
//   r  = x - y mod 2^(n+2)                     the true x - w m, in (-m, 3m)
//   r += m if r < 0; r -= m while r >= m (at most twice)
// Barrett's quotient estimate floor(q1 mu / 2^(n+1)) is at most 2 below
// floor(x / m) and never above it; w is that estimate or one more, so
// x - w m lies in [-m, 3m) and fits (n+2)-bit two's complement.  These are
// the uses of the truncated products that Section 1 names (the high product
// for the quotient, the low product for the remainder).
//
// The additions and subtractions on (n+2)-bit numbers are three launches
// each, without any inter-workgroup waiting: per 1024-limb chunk the carry
// function (generate, propagate), one workgroup's scan of the chunk
// functions, then each chunk applies its carry in.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "tmul.h"

namespace {

constexpr int NTA = 256;             // threads per add / bits workgroup
constexpr int LPT = 4;               // limbs per thread
constexpr int CH = NTA * LPT;        // limbs per chunk
constexpr int NTS = 1024;            // threads of the chunk scan

// carry function of a run of limbs: carry out = g | (p & carry in)
struct GP {
    uint32_t g, p;
};
__device__ __forceinline__ GP gp_then(GP lo, GP hi) { return GP{hi.g | (hi.p & lo.g), hi.p & lo.p}; }

enum Pred : uint32_t { P_ALWAYS = 0, P_SIGN = 1, P_NO_BORROW = 2 };

// dst[i] = bits [lo + 64 i, lo + 64 i + 64) of src (ls limbs, zero above),
// with bits >= keep of dst cleared
__global__ __launch_bounds__(NTA) void k_bits(uint64_t* dst, uint64_t nd, const uint64_t* src, uint64_t ls,
                                              uint64_t lo, uint64_t keep)
{
    for (uint64_t i = (uint64_t)blockIdx.x * NTA + threadIdx.x; i < nd; i += (uint64_t)gridDim.x * NTA) {
        const uint64_t pos = lo + 64 * i, li = pos >> 6;
        const int sh = (int)(pos & 63);
        uint64_t v = li < ls ? src[li] >> sh : 0;
        if (sh && li + 1 < ls) v |= src[li + 1] << (64 - sh);
        const uint64_t b0 = 64 * i;
        if (b0 >= keep) v = 0;
        else if (keep - b0 < 64) v &= (1ull << (keep - b0)) - 1;
        dst[i] = v;
    }
}

// limb i of y or its complement
__device__ __forceinline__ uint64_t yv(const uint64_t* y, uint64_t i, bool sub) { return sub ? ~y[i] : y[i]; }

// ordered workgroup scan of NTA carry functions in LDS: returns the
// composition of threads 0 .. tid-1 (exclusive); *total: all of them
__device__ __forceinline__ GP gp_scan_excl(GP mine, GP* s, GP* total)
{
    const int tid = threadIdx.x;
    s[tid] = mine;
    __syncthreads();
    for (int d = 1; d < NTA; d *= 2) {
        GP t = s[tid];
        if (tid >= d) t = gp_then(s[tid - d], t);
        __syncthreads();
        s[tid] = t;
        __syncthreads();
    }
    const GP incl = s[tid];
    *total = s[NTA - 1];
    const GP ex = tid ? s[tid - 1] : GP{0u, 1u};
    (void)incl;
    __syncthreads();
    return ex;
}

// phase 1: carry function of every chunk of x + (y or ~y)
__global__ __launch_bounds__(NTA) void k_add_chunks(const uint64_t* x, const uint64_t* y, uint64_t nl, int sub,
                                                    uint32_t* gp)
{
    __shared__ GP s[NTA];
    const uint64_t base = (uint64_t)blockIdx.x * CH + (uint64_t)threadIdx.x * LPT;
    GP f{0u, 1u};
    for (int k = 0; k < LPT; k++) {
        const uint64_t i = base + k;
        if (i < nl) {
            const uint64_t a = x[i], s1 = a + yv(y, i, sub != 0);
            f = gp_then(f, GP{s1 < a ? 1u : 0u, s1 == ~0ull ? 1u : 0u});
        }
    }
    GP total;
    gp_scan_excl(f, s, &total);
    if (threadIdx.x == 0) {
        gp[2 * blockIdx.x] = total.g;
        gp[2 * blockIdx.x + 1] = total.p;
    }
}

// phase 2 (one workgroup): carry into every chunk, and whether phase 3
// applies the operation: always, if bit `sign_bit` of x is set, or if the
// subtraction does not borrow (x >= y)
__global__ __launch_bounds__(NTS) void k_add_scan(const uint32_t* gp, uint32_t nch, uint32_t cin0,
                                                  const uint64_t* x, uint64_t sign_bit, uint32_t pred,
                                                  uint32_t* cin, uint32_t* apply)
{
    __shared__ GP s[NTS];
    const int tid = threadIdx.x;
    const uint32_t per = (nch + NTS - 1) / NTS;
    const uint32_t c0 = tid * per;
    GP f{0u, 1u};
    for (uint32_t c = c0; c < c0 + per && c < nch; c++) f = gp_then(f, GP{gp[2 * c], gp[2 * c + 1]});
    s[tid] = f;
    __syncthreads();
    for (int d = 1; d < NTS; d *= 2) {
        GP t = s[tid];
        if (tid >= d) t = gp_then(s[tid - d], t);
        __syncthreads();
        s[tid] = t;
        __syncthreads();
    }
    const GP ex = tid ? s[tid - 1] : GP{0u, 1u};
    uint32_t c_in = ex.g | (ex.p & cin0);
    for (uint32_t c = c0; c < c0 + per && c < nch; c++) {
        cin[c] = c_in;
        c_in = gp[2 * c] | (gp[2 * c + 1] & c_in);
    }
    if (tid == NTS - 1) {
        const GP t = s[NTS - 1];
        const uint32_t cout = t.g | (t.p & cin0);
        uint32_t a = 1;
        if (pred == P_SIGN) a = (uint32_t)((x[sign_bit >> 6] >> (sign_bit & 63)) & 1);
        else if (pred == P_NO_BORROW) a = cout;
        *apply = a;
    }
}

// phase 3: dst = x + (y or ~y) + carries, bits >= keep cleared, when *apply
__global__ __launch_bounds__(NTA) void k_add_apply(uint64_t* dst, const uint64_t* x, const uint64_t* y,
                                                   uint64_t nl, int sub, const uint32_t* cin,
                                                   const uint32_t* apply, uint64_t keep)
{
    __shared__ GP s[NTA];
    if (*apply == 0) return;  // uniform over the grid
    const uint64_t base = (uint64_t)blockIdx.x * CH + (uint64_t)threadIdx.x * LPT;
    uint64_t a[LPT], b[LPT];
    GP f{0u, 1u};
    for (int k = 0; k < LPT; k++) {
        const uint64_t i = base + k;
        a[k] = i < nl ? x[i] : 0;
        b[k] = i < nl ? yv(y, i, sub != 0) : 0;
        const uint64_t s1 = a[k] + b[k];
        f = gp_then(f, GP{s1 < a[k] ? 1u : 0u, s1 == ~0ull ? 1u : 0u});
    }
    GP total;
    const GP ex = gp_scan_excl(f, s, &total);
    uint32_t c = ex.g | (ex.p & cin[blockIdx.x]);
    for (int k = 0; k < LPT; k++) {
        const uint64_t i = base + k;
        if (i >= nl) break;
        const uint64_t s1 = a[k] + b[k];
        const uint64_t s2 = s1 + c;
        c = (s1 < a[k] || s2 < s1) ? 1u : 0u;
        uint64_t v = s2;
        const uint64_t b0 = 64 * i;
        if (b0 >= keep) v = 0;
        else if (keep - b0 < 64) v &= (1ull << (keep - b0)) - 1;
        dst[i] = v;
    }
}

uint64_t nlimbs(uint64_t n) { return (n + 63) / 64; }
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct MLayout {
    size_t mulws, x, q1, w, mext, wext, y, r, gp, cin, flag, total;
    uint64_t L, L1, L2, nch;
};

bool mlayout(uint64_t n, MLayout& o)
{
    if (n < 2 || n > (1ull << 31)) return false;
    const size_t f = tm_workspace_bytes(TM_FULL, n), h = tm_workspace_bytes(TM_HI, n + 1),
                 l = tm_workspace_bytes(TM_LO, n + 2);
    if (!f || !h || !l) return false;
    o.L = nlimbs(n);
    o.L1 = nlimbs(n + 1);
    o.L2 = nlimbs(n + 2);
    o.nch = (o.L2 + CH - 1) / CH;
    size_t m = f > h ? f : h;
    m = m > l ? m : l;
    size_t p = 0;
    o.mulws = p; p = al(p + m);
    o.x = p; p = al(p + 16 * o.L);
    o.q1 = p; p = al(p + 8 * o.L1);
    o.w = p; p = al(p + 8 * o.L1);
    o.mext = p; p = al(p + 8 * o.L2);
    o.wext = p; p = al(p + 8 * o.L2);
    o.y = p; p = al(p + 8 * o.L2);
    o.r = p; p = al(p + 8 * o.L2);
    o.gp = p; p = al(p + 8 * o.nch);
    o.cin = p; p = al(p + 4 * o.nch);
    o.flag = p; p = al(p + 4);
    o.total = p;
    return true;
}

dim3 grid_for(uint64_t nl)
{
    uint64_t g = (nl + NTA - 1) / NTA;
    return dim3((unsigned)(g < 4096 ? (g ? g : 1) : 4096));
}

// dst = x +- y (mod 2^keep) when the predicate holds (three launches)
void addsub(uint64_t* dst, const uint64_t* x, const uint64_t* y, const MLayout& lay, char* ws, bool sub,
            Pred pred, uint64_t sign_bit, uint64_t keep, hipStream_t s)
{
    uint32_t* gp = reinterpret_cast<uint32_t*>(ws + lay.gp);
    uint32_t* cin = reinterpret_cast<uint32_t*>(ws + lay.cin);
    uint32_t* flag = reinterpret_cast<uint32_t*>(ws + lay.flag);
    const unsigned nch = (unsigned)lay.nch;
    hipLaunchKernelGGL(k_add_chunks, dim3(nch), dim3(NTA), 0, s, x, y, lay.L2, sub ? 1 : 0, gp);
    hipLaunchKernelGGL(k_add_scan, dim3(1), dim3(NTS), 0, s, gp, nch, sub ? 1u : 0u, x, sign_bit,
                       (uint32_t)pred, cin, flag);
    hipLaunchKernelGGL(k_add_apply, dim3(nch), dim3(NTA), 0, s, dst, x, y, lay.L2, sub ? 1 : 0, cin, flag, keep);
}

}  // namespace

extern "C" {

size_t tm_workspace_bytes_mulmod(uint64_t n_bits)
{
    MLayout l;
    return mlayout(n_bits, l) ? l.total : 0;
}

tm_status tm_mulmod(uint64_t* r, const uint64_t* a, const uint64_t* b, const uint64_t* m, const uint64_t* mu,
                    uint64_t n_bits, void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    MLayout lay;
    if (!r || !a || !b || !m || !mu || !workspace) return TM_ERR_INVALID;
    if (!mlayout(n_bits, lay)) return n_bits < 2 ? TM_ERR_INVALID : TM_ERR_UNSUPPORTED;
    if (workspace_bytes < lay.total || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return TM_ERR_INVALID;
    const uint64_t n = n_bits;
    char* ws = static_cast<char*>(workspace);
    uint64_t* x = reinterpret_cast<uint64_t*>(ws + lay.x);
    uint64_t* q1 = reinterpret_cast<uint64_t*>(ws + lay.q1);
    uint64_t* w = reinterpret_cast<uint64_t*>(ws + lay.w);
    uint64_t* mext = reinterpret_cast<uint64_t*>(ws + lay.mext);
    uint64_t* wext = reinterpret_cast<uint64_t*>(ws + lay.wext);
    uint64_t* y = reinterpret_cast<uint64_t*>(ws + lay.y);
    uint64_t* rr = reinterpret_cast<uint64_t*>(ws + lay.r);
    void* mws = ws + lay.mulws;
    const size_t mwsb = lay.x - lay.mulws;
    tm_status st = tm_mul(TM_FULL, x, a, b, n, mws, mwsb, stream, nullptr);
    if (st != TM_OK) return st;
    hipLaunchKernelGGL(k_bits, grid_for(lay.L1), dim3(NTA), 0, stream, q1, lay.L1, x, 2 * lay.L, n - 1, n + 1);
    st = tm_mul(TM_HI, w, q1, mu, n + 1, mws, mwsb, stream, nullptr);
    if (st != TM_OK) return st;
    hipLaunchKernelGGL(k_bits, grid_for(lay.L2), dim3(NTA), 0, stream, wext, lay.L2, w, lay.L1, 0, n + 2);
    hipLaunchKernelGGL(k_bits, grid_for(lay.L2), dim3(NTA), 0, stream, mext, lay.L2, m, lay.L, 0, n);
    st = tm_mul(TM_LO, y, wext, mext, n + 2, mws, mwsb, stream, nullptr);
    if (st != TM_OK) return st;
    hipLaunchKernelGGL(k_bits, grid_for(lay.L2), dim3(NTA), 0, stream, rr, lay.L2, x, 2 * lay.L, 0, n + 2);
    addsub(rr, rr, y, lay, ws, true, P_ALWAYS, 0, n + 2, stream);
    addsub(rr, rr, mext, lay, ws, false, P_SIGN, n + 1, n + 2, stream);
    addsub(rr, rr, mext, lay, ws, true, P_NO_BORROW, 0, n + 2, stream);
    addsub(rr, rr, mext, lay, ws, true, P_NO_BORROW, 0, n + 2, stream);
    hipLaunchKernelGGL(k_bits, grid_for(lay.L), dim3(NTA), 0, stream, r, lay.L, rr, lay.L2, 0, n);
    return hipGetLastError() == hipSuccess ? TM_OK : TM_ERR_HIP;
}

}  // extern "C"
