// C-ABI of the truncated-multiplication library (see include/tmul.h).
// Host code: planning, twiddle cache, template dispatch, launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "tmul.h"
#include "plan.hpp"

#ifndef TM_NOALLOC_SCRATCH_BYTES
#define TM_NOALLOC_SCRATCH_BYTES (48u << 20)
#endif
#include "kernels.hpp"
#include "dispatch.hpp"

using namespace tmul;

static_assert(DPW == DPW_HOST, "K4 digits per workgroup must match the planner");

namespace {

thread_local std::string g_last_error;

tm_status hip_fail(hipError_t e, const char* what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_last_error = buf;
    return TM_ERR_HIP;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

// ------------------------------------------------------------ twiddles

}  // namespace

namespace tmul {

// sub-transform table: t[e] = exp(-2 pi i e / P), e < P
__global__ void k_subtwiddles(double2* t, uint32_t P)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) {
        const int64_t ee = i > P / 2 ? (int64_t)i - (int64_t)P : (int64_t)i;
        double s, c;
        sincospi(-2.0 * ((double)ee / (double)P), &s, &c);
        t[i] = make_double2(c, s);
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

namespace {


struct TwEntry {
    double2* buf = nullptr;
    Tw tw{};
    const double2* sub1 = nullptr;  // exp(-2 pi i e / L1), e < L1
    const double2* sub2 = nullptr;  // exp(-2 pi i e / L2), e < L2
    const double2* subm = nullptr;  // exp(-2 pi i e / Lm), e < Lm
};

std::mutex g_tw_mu;
std::map<std::tuple<int, uint64_t, uint32_t, uint32_t>, TwEntry> g_tw;

// Twiddle tables for transform length M = L1 * Lm * L2, built once per
// device and split (the sub-transform tables depend on L1, Lm and L2).
// build = false: look up only (callers that may not allocate).
tm_status get_twiddles(uint64_t M, uint32_t L1, uint32_t Lm, uint32_t L2, hipStream_t s, TwEntry& out,
                       bool build = true)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tw_mu);
    const auto key = std::make_tuple(dev, M, Lm, L2);
    auto it = g_tw.find(key);
    if (it != g_tw.end()) {
        out = it->second;
        return TM_OK;
    }
    if (!build) {
        g_last_error = "twiddle tables for this size are not built: call tm_prepare first";
        return TM_ERR_INVALID;
    }
    // building a table allocates and synchronises: not allowed while the
    // stream is being captured into a graph (tm_prepare the size first)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) {
        g_last_error = "twiddle tables for this size are not built: call tm_prepare before capturing";
        return TM_ERR_INVALID;
    }
    uint32_t sh = (uint32_t)((lg_ceil(M) + 1) / 2);
    uint32_t S = 1u << sh;
    uint32_t nhi = (uint32_t)((M + S - 1) / S);
    TwEntry e;
    HIP_TRY(hipMalloc(&e.buf, (size_t)(S + nhi + L1 + L2 + Lm) * sizeof(double2)));
    uint32_t n = S > nhi ? S : nhi;
    hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, e.buf, e.buf + S,
                       (uint32_t)M, S, nhi);
    hipLaunchKernelGGL(k_subtwiddles, dim3((L1 + 255) / 256), dim3(256), 0, s, e.buf + S + nhi, L1);
    hipLaunchKernelGGL(k_subtwiddles, dim3((L2 + 255) / 256), dim3(256), 0, s, e.buf + S + nhi + L1, L2);
    hipLaunchKernelGGL(k_subtwiddles, dim3((Lm + 255) / 256), dim3(256), 0, s, e.buf + S + nhi + L1 + L2, Lm);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    e.tw.lo = e.buf;
    e.tw.hi = e.buf + S;
    e.tw.shift = sh;
    e.tw.mask = S - 1;
    e.sub1 = e.buf + S + nhi;
    e.sub2 = e.buf + S + nhi + L1;
    e.subm = e.buf + S + nhi + L1 + L2;
    g_tw[key] = e;
    out = e;
    return TM_OK;
}

// ------------------------------------------------------------ dispatch

bool launch_k3(uint32_t L1, const KParams& p, hipStream_t s)
{
    switch (L1) {
#define X(V) \
    case V:                                                                                              \
        if (wide_tiles(p))                                                                               \
            hipLaunchKernelGGL((k3_col_inverse<V, w3_for(V, true)>), dim3(p.R / w3_for(V, true)), dim3(NT3), 0, s, p); \
        else                                                                                             \
            hipLaunchKernelGGL((k3_col_inverse<V, w3_for(V, false)>), dim3(p.R / w3_for(V, false)), dim3(NT3), 0, s, p); \
        return true;
        TM_L1_LIST(X)
#undef X
    }
    return false;
}

bool launch_k2(uint32_t L2, const KParams& p, hipStream_t s)
{
    dim3 g(k2_groups(p.L1, p.Lm));
    switch (L2) {
    case 16: hipLaunchKernelGGL((k2_rows_pointwise<16>), g, dim3(NT2), 0, s, p); return true;
    case 32: hipLaunchKernelGGL((k2_rows_pointwise<32>), g, dim3(NT2), 0, s, p); return true;
    case 64: hipLaunchKernelGGL((k2_rows_pointwise<64>), g, dim3(NT2), 0, s, p); return true;
    case 128: hipLaunchKernelGGL((k2_rows_pointwise<128>), g, dim3(NT2), 0, s, p); return true;
    case 256: hipLaunchKernelGGL((k2_rows_pointwise<256>), g, dim3(NT2), 0, s, p); return true;
    case 512: hipLaunchKernelGGL((k2_rows_pointwise<512>), g, dim3(NT2), 0, s, p); return true;
    case 1024: hipLaunchKernelGGL((k2_rows_pointwise<1024>), g, dim3(NT2), 0, s, p); return true;
    case 96: hipLaunchKernelGGL((k2_rows_pointwise<96>), g, dim3(NT2), 0, s, p); return true;
    case 192: hipLaunchKernelGGL((k2_rows_pointwise<192>), g, dim3(NT2), 0, s, p); return true;
    case 384: hipLaunchKernelGGL((k2_rows_pointwise<384>), g, dim3(NT2), 0, s, p); return true;
    case 768: hipLaunchKernelGGL((k2_rows_pointwise<768>), g, dim3(NT2), 0, s, p); return true;
    }
    return false;
}

constexpr int w_mid(int LM) { return 4096 / LM < 64 ? 4096 / LM : 64; }

template <bool INV>
bool launch_mid(const KParams& p, hipStream_t s)
{
    const int W = (int)p.L2 < w_mid((int)p.Lm) ? (int)p.L2 : w_mid((int)p.Lm);
    dim3 g(p.L2 / W, p.L1, INV || p.zb == p.za ? 1 : 2);
#define MIDW(LM, WW) \
    if (p.Lm == LM && W == WW) { hipLaunchKernelGGL((k_mid_col<LM, WW, INV>), g, dim3(NTM), 0, s, p); return true; }
#define MID(LM) MIDW(LM, 16) MIDW(LM, 32) MIDW(LM, 64)
    MID(2) MID(4) MID(8) MID(16) MID(32) MID(64) MIDW(128, 16) MIDW(128, 32) MIDW(256, 16)
#undef MID
#undef MIDW
    return false;
}

template <bool DIAG, int KIND, int BF>
void launch_k4_k(const KParams& p, hipStream_t s)
{
    dim3 g(p.nstatus);
    if (fixed_b(KIND, p)) hipLaunchKernelGGL((k4_backmap_carry<KIND, DIAG, BF>), g, dim3(NT4), 0, s, p);
    else hipLaunchKernelGGL((k4_backmap_carry<KIND, DIAG, 0>), g, dim3(NT4), 0, s, p);
}

template <bool DIAG>
void launch_k4(int kind, const KParams& p, hipStream_t s)
{
    if (kind == TM_FULL) launch_k4_k<DIAG, K_FULL, B_FULL>(p, s);
    else if (kind == TM_LO) launch_k4_k<DIAG, K_LO, B_TRUNC>(p, s);
    else launch_k4_k<DIAG, K_HI, B_TRUNC>(p, s);
}

bool launch_k1_any(int kind, const KParams& p, hipStream_t s)
{
    if (kind == TM_FULL) return launch_k1_full(p.L1, p, s);
    if (kind == TM_LO) return launch_k1_lo(p.L1, p, s);
    return launch_k1_hi(p.L1, p, s);
}

// ------------------------------------------------------------ packed launches
//
// Requests whose plans select the same kernel instance for a stage share one
// launch of that instance; each workgroup finds its request in the group
// table (see group_block).

int mid_w(const KParams& p) { return (int)p.L2 < w_mid((int)p.Lm) ? (int)p.L2 : w_mid((int)p.Lm); }

bool launch_k2g(uint32_t L2, const Group& g, uint32_t blocks, hipStream_t s)
{
    switch (L2) {
#define X(V) \
    case V: hipLaunchKernelGGL((k2_rows_pointwise_g<V>), dim3(blocks), dim3(NT2), 0, s, g); return true;
        X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(96) X(192) X(384) X(768)
#undef X
    }
    return false;
}

template <bool INV>
bool launch_midg(uint32_t Lm, int W, const Group& g, uint32_t blocks, hipStream_t s)
{
#define MIDW(LM, WW) \
    if (Lm == LM && W == WW) { hipLaunchKernelGGL((k_mid_col_g<LM, WW, INV>), dim3(blocks), dim3(NTM), 0, s, g); return true; }
#define MID(LM) MIDW(LM, 16) MIDW(LM, 32) MIDW(LM, 64)
    MID(2) MID(4) MID(8) MID(16) MID(32) MID(64) MIDW(128, 16) MIDW(128, 32) MIDW(256, 16)
#undef MID
#undef MIDW
    return false;
}

bool launch_k3g(uint32_t L1, bool wide, const Group& g, uint32_t blocks, hipStream_t s)
{
    switch (L1) {
#define X(V)                                                                                          \
    case V:                                                                                           \
        if (wide)                                                                                     \
            hipLaunchKernelGGL((k3_col_inverse_g<V, w3_for(V, true)>), dim3(blocks), dim3(NT3), 0, s, g); \
        else                                                                                          \
            hipLaunchKernelGGL((k3_col_inverse_g<V, w3_for(V, false)>), dim3(blocks), dim3(NT3), 0, s, g); \
        return true;
        TM_L1_LIST(X)
#undef X
    }
    return false;
}

void launch_k4g(int kind, int fb, const Group& g, uint32_t blocks, hipStream_t s)
{
    if (kind == TM_FULL) {
        if (fb) hipLaunchKernelGGL((k4_backmap_carry_g<K_FULL, B_FULL>), dim3(blocks), dim3(NT4), 0, s, g);
        else hipLaunchKernelGGL((k4_backmap_carry_g<K_FULL, 0>), dim3(blocks), dim3(NT4), 0, s, g);
    } else if (kind == TM_LO) {
        if (fb) hipLaunchKernelGGL((k4_backmap_carry_g<K_LO, B_TRUNC>), dim3(blocks), dim3(NT4), 0, s, g);
        else hipLaunchKernelGGL((k4_backmap_carry_g<K_LO, 0>), dim3(blocks), dim3(NT4), 0, s, g);
    } else {
        if (fb) hipLaunchKernelGGL((k4_backmap_carry_g<K_HI, B_TRUNC>), dim3(blocks), dim3(NT4), 0, s, g);
        else hipLaunchKernelGGL((k4_backmap_carry_g<K_HI, 0>), dim3(blocks), dim3(NT4), 0, s, g);
    }
}

bool launch_k1g_any(int kind, uint32_t L1, int fb, bool wide, const Group& g, uint32_t blocks, hipStream_t s)
{
    if (kind == TM_FULL) return launch_k1g_full(L1, fb, wide, g, blocks, s);
    if (kind == TM_LO) return launch_k1g_lo(L1, fb, wide, g, blocks, s);
    return launch_k1g_hi(L1, fb, wide, g, blocks, s);
}

// Stages of one multiplication in launch order; the middle passes exist
// only for three-pass splits, and fused plans have K0 in place of K1 and no
// K2 or K3.
enum Stage { ST_K1, ST_MIDF, ST_K2, ST_MIDI, ST_K3, ST_K4, ST_COUNT };

// Kernel instance (key) and grid of request p at stage st; false if the
// request has no launch at that stage.
bool stage_shape(int st, int kind, const KParams& p, uint64_t& key, uint32_t& nx, uint32_t& ny,
                 uint32_t& nz)
{
    const int fb = fixed_b(kind, p) ? 1 : 0;
    const bool wide = wide_tiles(p);
    nx = ny = nz = 1;
    if (p.fused) {
        // K0: one workgroup per request
        if (st == ST_K1) {
            key = (1ull << 50) | ((uint64_t)kind << 40) | ((uint64_t)p.L1 << 16) | p.L2;
            return true;
        }
        if (st != ST_K4) return false;
    }
    switch (st) {
    case ST_K1:
        key = ((uint64_t)wide << 42) | ((uint64_t)kind << 40) | ((uint64_t)fb << 32) | p.L1;
        nx = p.R / (uint32_t)w1_for(kind, (int)p.L1, wide);
        ny = p.zb == p.za ? 1 : 2;
        return true;
    case ST_MIDF:
    case ST_MIDI: {
        if (p.Lm <= 1) return false;
        const int W = mid_w(p);
        key = ((uint64_t)p.Lm << 16) | (uint32_t)W;
        nx = p.L2 / (uint32_t)W;
        ny = p.L1;
        nz = st == ST_MIDF && p.zb != p.za ? 2 : 1;
        return true;
    }
    case ST_K2:
        key = p.L2;
        nx = k2_groups(p.L1, p.Lm);
        return true;
    case ST_K3:
        key = ((uint64_t)wide << 32) | p.L1;
        nx = p.R / (uint32_t)w3_for((int)p.L1, wide);
        return true;
    default:
        key = ((uint64_t)kind << 1) | (uint64_t)fb;
        nx = p.nstatus;
        return true;
    }
}


// Device metadata of a packed batch: parameters, then the group tables of
// every stage (at most one entry per request and stage).
size_t meta_params_bytes(size_t count) { return align256(count * sizeof(KParams)); }
size_t meta_bytes_for(size_t count)
{
    return meta_params_bytes(count) + align256(count * ST_COUNT * sizeof(GroupEnt));
}

// Pinned host buffers for metadata uploads, per device.  A buffer is reused
// once the event recorded after its upload has completed.
struct StageBuf {
    char* host = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};
std::mutex g_stage_mu;
std::map<int, std::vector<StageBuf>> g_stage;
constexpr size_t kStageBufs = 32;

// Caller holds g_stage_mu.
tm_status stage_acquire(int dev, size_t bytes, StageBuf*& out)
{
    auto& v = g_stage[dev];
    for (auto& b : v) {
        if (b.bytes < bytes) continue;
        if (b.pending) {
            hipError_t e = hipEventQuery(b.ev);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
            b.pending = false;
        }
        out = &b;
        return TM_OK;
    }
    StageBuf* b;
    if (v.size() < kStageBufs) {
        v.emplace_back();
        b = &v.back();
        HIP_TRY(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming));
    } else {
        // every buffer busy or too small: wait for the first one
        b = &v.front();
        if (b->pending) HIP_TRY(hipEventSynchronize(b->ev));
        b->pending = false;
    }
    if (b->bytes < bytes) {
        if (b->host) HIP_TRY(hipHostFree(b->host));
        b->host = nullptr;
        b->bytes = 0;
        const size_t nb = bytes < (64u << 10) ? (64u << 10) : bytes;
        HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&b->host), nb, hipHostMallocDefault));
        b->bytes = nb;
    }
    out = b;
    return TM_OK;
}

struct Launch {
    int st;
    int kind, fb;
    bool wide;          // K1/K3: wide column tiles (three-pass split)
    bool fused;         // K1 stage of a fused request: K0
    uint32_t a, b;      // instance: K1/K3 L1, K2 L2, middle Lm and W
    uint32_t ent0, nr;  // first table entry, requests
    uint32_t blocks;
};


// ------------------------------------------------------------ params

// Series constants.  c_r: alpha (-eps)^r/r!, gamma eps^r/r! (forward),
// beta eps^r/r!, delta (-eps)^r/r! (back).  Forward nested form (see
// row_map_fast): factor k_r (y -+ r), k_r = c_(r+1)/c_r, for 1 <= r <= lam-2.
// Back chain (see back_chain): factor k_r (x +- r) for 0 <= r <= lam-2.
// Factors from r = lam - 1 on are zero.
void fill_series(const Plan& P, KParams& p)
{
    const double eps = ldexp(1.0, -P.b);
    const bool lo = P.kind == TM_LO;
    double e = 1.0, fact = 1.0;
    for (int r = 0; r < LMAX; r++) {
        if (r > 0) {
            e *= eps;
            fact *= r;
        }
        const double sgn = (r & 1) ? -1.0 : 1.0;
        p.cf[r] = (lo ? sgn : 1.0) * e / fact;
        p.cb[r] = (lo ? 1.0 : sgn) * e / fact;
    }
    for (int r = 0; r < LMAX; r++) {
        p.nf[r][0] = p.nf[r][1] = 0.0;
        p.nb[r][0] = p.nb[r][1] = 0.0;
        if (P.kind == TM_FULL || r + 1 >= P.lam || r + 1 >= LMAX) continue;
        const double kf = p.cf[r + 1] / p.cf[r];  // (-+eps) / (r + 1)
        const double kb = p.cb[r + 1] / p.cb[r];
        if (r >= 1) {
            p.nf[r][0] = kf;
            p.nf[r][1] = kf * (lo ? -(double)r : (double)r);
        }
        p.nb[r][0] = kb;
        p.nb[r][1] = kb * (lo ? (double)r : -(double)r);
    }
    p.bscale = P.kind == TM_FULL ? 1.0 / (double)P.M : ldexp(1.0 / (double)P.M, P.b);
}

void fill_params(const Plan& P, const uint64_t* u, const uint64_t* v, uint64_t* w, void* ws,
                 tm_guard* guard, const TwEntry& tw, KParams& p)
{
    memset(&p, 0, sizeof p);
    char* base = static_cast<char*>(ws);
    p.u = u;
    p.v = v;
    p.w = w;
    p.n = P.n;
    p.L = P.L;
    p.b = P.b;
    p.lam = P.lam;
    p.N = (uint32_t)P.N;
    p.digits = (uint32_t)P.digits;
    p.M = (uint32_t)P.M;
    p.L1 = P.L1;
    p.L2 = P.L2;
    p.Lm = P.Lm;
    p.R = P.Lm * P.L2;
    p.jmax = P.jmax;
    p.shift = P.shift;
    p.off = P.off;
    p.out_bits = P.out_bits;
    p.out_limbs = P.out_limbs;
    p.ncoef = (uint32_t)P.ncoef;
    p.ncover = (uint32_t)P.ncover;
    p.nstatus = P.nstatus;
    p.fused = P.fused ? 1u : 0u;
    p.invN = 1.0 / (double)P.N;
    p.invM = 1.0 / (double)P.M;
    fill_series(P, p);
    p.za = reinterpret_cast<double2*>(base + P.o_za);
    // squaring (u == v): one forward transform, both spectra read from za
    p.zb = u == v ? p.za : reinterpret_cast<double2*>(base + P.o_zb);
    p.status = reinterpret_cast<uint64_t*>(base + P.o_status);
    p.ticket = reinterpret_cast<uint32_t*>(base + P.o_ticket);
    p.guard = guard ? guard : reinterpret_cast<tm_guard*>(base + P.o_guard);
    p.theta = reinterpret_cast<double*>(base + P.o_theta);
    p.tw = tw.tw;
    p.tw1 = tw.sub1;
    p.tw2 = tw.sub2;
    p.twm = tw.subm;
}

// Splits chosen by tm_autotune: (kind, n) -> split code (middle length Lm
// and row length L2, see split_code; 0: the planner's own choice).  The
// split changes only the FFT schedule, not N or b, so tuned and untuned
// calls return the same products.
std::mutex g_tune_mu;
std::map<std::pair<int, uint64_t>, uint32_t> g_tuned;

uint32_t tuned_split(tm_kind kind, uint64_t n)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_pair((int)kind, n));
    return it == g_tuned.end() ? 0u : it->second;
}

tm_status plan_for(tm_kind kind, uint64_t n, Plan& P, int bt = 0, int bf = 0)
{
    if (kind != TM_FULL && kind != TM_LO && kind != TM_HI) {
        g_last_error = "invalid kind";
        return TM_ERR_INVALID;
    }
    if (n == 0) {
        g_last_error = "n_bits must be positive";
        return TM_ERR_INVALID;
    }
    if (!bt) {
        const char* e = getenv("TM_FORCE_B");
        if (e && *e) bt = atoi(e);
    }
    if (!bf) {
        const char* e = getenv("TM_FORCE_B_FULL");
        if (e && *e) bf = atoi(e);
    }
    uint32_t flm = 0;
    {
        // forced split (tests, experiments): middle length, log2 row length
        // (of its power-of-two part), odd factor in the row length
        const char* e = getenv("TM_FORCE_LM");
        if (e && *e) flm = (uint32_t)atoi(e);
        const char* e2 = getenv("TM_FORCE_LG2");
        if (e2 && *e2) flm = split_code(flm, atoi(e2));
        const char* e3 = getenv("TM_FORCE_ODD_ROW");
        if (e3 && *e3 == '1') flm |= SPLIT_ODD_ROW;
    }
    if (!flm) flm = tuned_split(kind, n);
    // fused small-size pass (K0) on request only (TM_FUSED=1): one
    // workgroup per product is latency-bound and measured slower than the
    // four-step kernels at these sizes
    const char* fe = getenv("TM_FUSED");
    const bool fused_ok = fe && *fe == '1';
    if (!make_plan((int)kind, n, bt, bf, P, flm, false, false, fused_ok)) {
        g_last_error = "unsupported size";
        return TM_ERR_UNSUPPORTED;
    }
    return TM_OK;
}

// Plan of the FP32 path: the planner with double-float digit sizes and
// power-of-two lengths; forced digit sizes and splits from the same
// environment variables as the FP64 plans (odd-row splits do not apply).
tm_status plan_fp32c(tm_kind kind, uint64_t n, Plan& P)
{
    if (kind != TM_FULL && kind != TM_LO && kind != TM_HI) {
        g_last_error = "invalid kind";
        return TM_ERR_INVALID;
    }
    if (n == 0) {
        g_last_error = "n_bits must be positive";
        return TM_ERR_INVALID;
    }
    int bt = 0, bf = 0;
    const char* e = getenv("TM_FORCE_B");
    if (e && *e) bt = atoi(e);
    e = getenv("TM_FORCE_B_FULL");
    if (e && *e) bf = atoi(e);
    uint32_t flm = 0;
    e = getenv("TM_FORCE_LM");
    if (e && *e) flm = (uint32_t)atoi(e);
    e = getenv("TM_FORCE_LG2");
    if (e && *e) flm = split_code(flm, atoi(e));
    if (!make_plan((int)kind, n, bt, bf, P, flm, false, true)) {
        g_last_error = "unsupported size";
        return TM_ERR_UNSUPPORTED;
    }
    return TM_OK;
}

enum Mode { RUN, DIAG_RUN };

tm_status run(const Plan& P, uint64_t* w, const uint64_t* u, const uint64_t* v, void* ws,
              size_t ws_bytes, hipStream_t s, tm_guard* guard, Mode mode, int64_t* dc,
              double* dx, hipEvent_t* ev, bool build_tables = true)
{
    if (!u || !v || !ws || (mode == RUN && !w) || (mode == DIAG_RUN && !dc)) {
        g_last_error = "null pointer";
        return TM_ERR_INVALID;
    }
    if (ws_bytes < P.ws_bytes) {
        g_last_error = "workspace too small";
        return TM_ERR_INVALID;
    }
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) {
        g_last_error = "workspace must be 256-byte aligned";
        return TM_ERR_INVALID;
    }
    TwEntry tw;
    tm_status st = get_twiddles(P.M, P.L1, P.Lm, P.L2, s, tw, build_tables);
    if (st != TM_OK) return st;
    KParams p;
    fill_params(P, u, v, w, ws, guard, tw, p);
    if (mode == DIAG_RUN) {
        // K1 clears out_limbs of w; point it at the coefficient buffer's
        // storage only when no output exists: use zero output limbs instead
        p.w = reinterpret_cast<uint64_t*>(dc);
        p.out_limbs = 0;
        p.dbg_c = dc;
        p.dbg_x = dx;
    }
    // FP64 path, or the FP32 path's double-float instances (P.df)
    int ne = 0;
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    if (P.fused) {
        // small sizes: one workgroup per product does K1, K2 and K3
        if (!launch_k0(P.kind, P.L1, P.L2, p, s)) {
            g_last_error = "no fused kernel for the split";
            return TM_ERR_UNSUPPORTED;
        }
        if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
        if (mode == DIAG_RUN) launch_k4<true>(P.kind, p, s);
        else launch_k4<false>(P.kind, p, s);
        if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
        HIP_TRY(hipGetLastError());
        return TM_OK;
    }
    if (!(P.df ? launch_k1_fp32c(P.kind, P.L1, p, s) : launch_k1_any(P.kind, p, s))) {
        g_last_error = "no kernel for L1";
        return TM_ERR_UNSUPPORTED;
    }
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    if (P.Lm > 1) {
        if (!(P.df ? launch_mid_fp32c<false>(p, s) : launch_mid<false>(p, s))) {
            g_last_error = "no kernel for Lm";
            return TM_ERR_UNSUPPORTED;
        }
        if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    }
    if (!(P.df ? launch_k2_fp32c(P.L2, p, s) : launch_k2(P.L2, p, s))) {
        g_last_error = "no kernel for L2";
        return TM_ERR_UNSUPPORTED;
    }
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    if (P.Lm > 1) {
        if (!(P.df ? launch_mid_fp32c<true>(p, s) : launch_mid<true>(p, s))) {
            g_last_error = "no kernel for Lm";
            return TM_ERR_UNSUPPORTED;
        }
        if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    }
    if (!(P.df ? launch_k3_fp32c(P.L1, p, s) : launch_k3(P.L1, p, s))) {
        g_last_error = "no kernel for L1";
        return TM_ERR_UNSUPPORTED;
    }
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    if (P.df) {
        if (mode == DIAG_RUN) launch_k4_fp32c<true>(P.kind, p, s);
        else launch_k4_fp32c<false>(P.kind, p, s);
    } else if (mode == DIAG_RUN) {
        launch_k4<true>(P.kind, p, s);
    } else {
        launch_k4<false>(P.kind, p, s);
    }
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    HIP_TRY(hipGetLastError());
    return TM_OK;
}

tm_status run_packed(const tm_request* reqs, size_t count, void* const* ws, const size_t* ws_bytes,
                     tm_guard* const* guards, void* meta, size_t meta_bytes, hipStream_t s,
                     void* host_staging = nullptr, size_t host_staging_bytes = 0)
{
    if (count == 0) return TM_OK;
    if (!reqs || !ws || !ws_bytes || !meta) {
        g_last_error = "null pointer";
        return TM_ERR_INVALID;
    }
    if (meta_bytes < meta_bytes_for(count) || (reinterpret_cast<uintptr_t>(meta) & 255) != 0) {
        g_last_error = "metadata area too small or not 256-byte aligned";
        return TM_ERR_INVALID;
    }
    const size_t pbytes = meta_params_bytes(count);
    std::vector<KParams> ps(count);
    std::vector<int> kinds(count);
    for (size_t i = 0; i < count; i++) {
        const tm_request& r = reqs[i];
        Plan P;
        tm_status st = plan_for((tm_kind)r.kind, r.n_bits, P);
        if (st != TM_OK) return st;
        if (!r.u || !r.v || !r.w || !ws[i]) {
            g_last_error = "null pointer";
            return TM_ERR_INVALID;
        }
        if ((reinterpret_cast<uintptr_t>(ws[i]) & 255) != 0) {
            g_last_error = "workspace must be 256-byte aligned";
            return TM_ERR_INVALID;
        }
        if (ws_bytes[i] < P.ws_bytes) {
            g_last_error = "workspace too small";
            return TM_ERR_INVALID;
        }
        TwEntry tw;
        st = get_twiddles(P.M, P.L1, P.Lm, P.L2, s, tw);
        if (st != TM_OK) return st;
        fill_params(P, r.u, r.v, r.w, ws[i], guards ? guards[i] : nullptr, tw, ps[i]);
        kinds[i] = P.kind;
    }
    // group tables: per stage, requests sorted by kernel instance, at most
    // GROUP_MAX per launch
    std::vector<GroupEnt> ents;
    std::vector<Launch> launches;
    std::vector<std::pair<uint64_t, uint32_t>> order;
    for (int st = 0; st < ST_COUNT; st++) {
        order.clear();
        for (size_t i = 0; i < count; i++) {
            uint64_t key;
            uint32_t nx, ny, nz;
            if (stage_shape(st, kinds[i], ps[i], key, nx, ny, nz)) order.emplace_back(key, (uint32_t)i);
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<uint64_t, uint32_t>& x, const std::pair<uint64_t, uint32_t>& y) {
                             return x.first < y.first;
                         });
        for (size_t k = 0; k < order.size();) {
            Launch L{};
            L.st = st;
            L.ent0 = (uint32_t)ents.size();
            const uint64_t key = order[k].first;
            const KParams& p0 = ps[order[k].second];
            L.kind = kinds[order[k].second];
            L.fb = fixed_b(L.kind, p0) ? 1 : 0;
            L.wide = wide_tiles(p0);
            L.fused = p0.fused != 0;
            L.a = st == ST_K2 ? p0.L2 : (st == ST_MIDF || st == ST_MIDI) ? p0.Lm : p0.L1;
            L.b = (st == ST_MIDF || st == ST_MIDI) ? (uint32_t)mid_w(p0) : 0;
            if (L.fused && st == ST_K1) L.b = p0.L2;  // K0 instance: (L1, L2)
            uint64_t blocks = 0;
            while (k < order.size() && order[k].first == key && L.nr < (uint32_t)GROUP_MAX) {
                const uint32_t i = order[k].second;
                uint64_t kk;
                uint32_t nx, ny, nz;
                stage_shape(st, kinds[i], ps[i], kk, nx, ny, nz);
                ents.push_back(GroupEnt{(uint32_t)blocks, nx, ny, i});
                blocks += (uint64_t)nx * ny * nz;
                L.nr++;
                k++;
            }
            if (blocks >= 0xffffffffull) {
                g_last_error = "packed launch too large";
                return TM_ERR_UNSUPPORTED;
            }
            L.blocks = (uint32_t)blocks;
            launches.push_back(L);
        }
    }
    // one upload of parameters and tables through a pinned staging buffer:
    // the caller's (which it keeps until the batch has run: safe under stream
    // capture) or one of the library's, reused once its upload completed
    const size_t used = pbytes + ents.size() * sizeof(GroupEnt);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (host_staging) {
        if (host_staging_bytes < used) {
            g_last_error = "host staging buffer too small";
            return TM_ERR_INVALID;
        }
        char* h = static_cast<char*>(host_staging);
        memcpy(h, ps.data(), count * sizeof(KParams));
        memcpy(h + pbytes, ents.data(), ents.size() * sizeof(GroupEnt));
        HIP_TRY(hipMemcpyAsync(meta, h, used, hipMemcpyHostToDevice, s));
    } else {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        StageBuf* sb = nullptr;
        tm_status st = stage_acquire(dev, used, sb);
        if (st != TM_OK) return st;
        memcpy(sb->host, ps.data(), count * sizeof(KParams));
        memcpy(sb->host + pbytes, ents.data(), ents.size() * sizeof(GroupEnt));
        HIP_TRY(hipMemcpyAsync(meta, sb->host, used, hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(sb->ev, s));
        sb->pending = true;
    }
    const KParams* dps = static_cast<const KParams*>(meta);
    const GroupEnt* dent = reinterpret_cast<const GroupEnt*>(static_cast<const char*>(meta) + pbytes);
    for (const Launch& L : launches) {
        const Group g{dps, dent + L.ent0, L.nr};
        bool ok = true;
        switch (L.st) {
        case ST_K1:
            ok = L.fused ? launch_k0g(L.kind, L.a, L.b, g, L.blocks, s)
                         : launch_k1g_any(L.kind, L.a, L.fb, L.wide, g, L.blocks, s);
            break;
        case ST_MIDF: ok = launch_midg<false>(L.a, (int)L.b, g, L.blocks, s); break;
        case ST_K2: ok = launch_k2g(L.a, g, L.blocks, s); break;
        case ST_MIDI: ok = launch_midg<true>(L.a, (int)L.b, g, L.blocks, s); break;
        case ST_K3: ok = launch_k3g(L.a, L.wide, g, L.blocks, s); break;
        default: launch_k4g(L.kind, L.fb, g, L.blocks, s); break;
        }
        if (!ok) {
            g_last_error = "no packed kernel for a stage of the batch";
            return TM_ERR_UNSUPPORTED;
        }
    }
    HIP_TRY(hipGetLastError());
    return TM_OK;
}

// Fallback plan of tm_mul_checked, exact for every input by its worst-case
// bound: the guaranteed plan of the requested kind when it has smaller
// digits than the plan that tripped, else (the truncated products beyond
// the sizes where a guaranteed truncated plan exists) the full product's
// guaranteed plan with extraction of the requested bits.
bool fallback_plan(tm_kind kind, uint64_t n_bits, const Plan& P, Plan& F)
{
    if (make_plan_guaranteed((int)kind, n_bits, F) && F.b < P.b) return true;
    if (kind == TM_FULL) return false;
    return make_plan_guaranteed((int)kind, n_bits, F, true);
}

tm_status plan_guaranteed(tm_kind kind, uint64_t n, Plan& P)
{
    if ((int)kind < 0 || (int)kind > 2 || n == 0) {
        g_last_error = "invalid kind or size";
        return TM_ERR_INVALID;
    }
    if (!make_plan_guaranteed((int)kind, n, P)) {
        g_last_error = "no digit size >= 8 meets the guaranteed bound at this size";
        return TM_ERR_UNSUPPORTED;
    }
    return TM_OK;
}

void fill_info(tm_kind kind, uint64_t n_bits, const Plan& P, tm_plan_info* out)
{
    out->kind = (uint32_t)kind;
    out->via_full = P.via_full ? 1u : 0u;
    out->b = (uint32_t)P.b;
    out->lambda = (uint32_t)P.lam;
    out->n_bits = n_bits;
    out->N = P.N;
    out->digits = P.digits;
    out->M = P.M;
    out->L1 = P.L1;
    out->L2 = P.L2;
    out->workspace_bytes = P.ws_bytes;
    out->Lm = P.Lm;
    out->rounding_bound = rounding_bound(P);
    out->guaranteed = out->rounding_bound <= GUARANTEED_MAX ? 1u : 0u;
    out->fused = P.fused ? 1u : 0u;
    out->reserved = 0;
}

// ------------------------------------------------------------ static scratch
//
// Workspace of tm_mul_noalloc: a file-scope device array, one copy per GPU,
// held until the process ends.  In host code its name is a host-side
// stand-in, not a device address: every host use goes through the address
// hipGetSymbolAddress returns for the current device, taken once per device.
constexpr size_t NOALLOC_MAX = TM_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[NOALLOC_MAX];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch;

tm_status scratch_ptr(void*& out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        out = it->second;
        return TM_OK;
    }
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0) {
        g_last_error = "static scratch has no usable device address";
        return TM_ERR_HIP;
    }
    g_scratch[dev] = ptr;
    out = ptr;
    return TM_OK;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

size_t tm_workspace_bytes(tm_kind kind, uint64_t n_bits)
{
    Plan P;
    if (plan_for(kind, n_bits, P) != TM_OK) return 0;
    return P.ws_bytes;
}

tm_status tm_plan_query(tm_kind kind, uint64_t n_bits, tm_plan_info* out)
{
    if (!out) {
        g_last_error = "null pointer";
        return TM_ERR_INVALID;
    }
    Plan P;
    tm_status st = plan_for(kind, n_bits, P);
    if (st != TM_OK) return st;
    fill_info(kind, n_bits, P, out);
    return TM_OK;
}

tm_status tm_autotune(tm_kind kind, uint64_t n_bits, hipStream_t stream, tm_plan_info* chosen)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned.erase(std::make_pair((int)kind, n_bits));
    }
    Plan P0;
    tm_status st = plan_for(kind, n_bits, P0);
    if (st != TM_OK) return st;
    // candidates: the planner's split, every forced middle length with the
    // odd factor of M in the column length or in the row length, and for
    // each of these the row lengths twice and half its own
    std::vector<uint32_t> cand{0};
    std::vector<std::pair<uint32_t, uint32_t>> seen{{P0.Lm, P0.L2}};
    for (uint32_t lm = 1; lm <= LM_MAX; lm *= 2) {
        for (bool odd_row : {false, true}) {
            Plan Q;
            if (!make_plan((int)kind, n_bits, 0, 0, Q, split_code(lm, 0, odd_row)) || Q.Lm != lm) continue;
            uint32_t odd = Q.L2;
            while (odd % 2 == 0) odd /= 2;
            const int lg = lg_ceil(Q.L2 / odd);  // log2 of the row length's power-of-two part
            for (int lg2 : {0, lg + 1, lg - 1}) {
                Plan S;
                const uint32_t code = split_code(lm, lg2, odd_row);
                if (!make_plan((int)kind, n_bits, 0, 0, S, code)) continue;
                const std::pair<uint32_t, uint32_t> key{S.Lm, S.L2};
                bool dup = false;
                for (auto& k : seen) dup = dup || k == key;
                if (dup) continue;
                seen.push_back(key);
                cand.push_back(code);
            }
        }
    }
    uint32_t best = 0;
    if (cand.size() > 1) {
        // pseudo-random operands (carry patterns like real data), own buffers
        const size_t L = (n_bits + 63) / 64;
        std::vector<uint64_t> h(2 * L);
        uint64_t x = 0x9E3779B97F4A7C15ull;
        for (auto& w : h) {
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            w = x;
        }
        void *du = nullptr, *dw = nullptr, *dws = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto cleanup = [&]() {
            if (du) (void)hipFree(du);
            if (dw) (void)hipFree(dw);
            if (dws) (void)hipFree(dws);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        };
        const size_t wsb = P0.ws_bytes;
        if (hipMalloc(&du, 2 * L * 8) != hipSuccess || hipMalloc(&dw, 2 * L * 8) != hipSuccess ||
            hipMalloc(&dws, wsb) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess) {
            cleanup();
            return hip_fail(hipGetLastError(), "tm_autotune buffers");
        }
        if (hipMemcpy(du, h.data(), 2 * L * 8, hipMemcpyHostToDevice) != hipSuccess) {
            cleanup();
            return hip_fail(hipGetLastError(), "tm_autotune operands");
        }
        const uint64_t* u = static_cast<const uint64_t*>(du);
        float best_ms = 0.0f;
        for (uint32_t lm : cand) {
            Plan Q;
            if (!make_plan((int)kind, n_bits, 0, 0, Q, lm)) continue;
            // one untimed run, then the fastest of five timed ones
            float tot = 0.0f;
            for (int rep = 0; rep < 6 && st == TM_OK; rep++) {
                if (rep > 0) st = hipEventRecord(e0, stream) == hipSuccess ? TM_OK : TM_ERR_HIP;
                if (st == TM_OK)
                    st = run(Q, static_cast<uint64_t*>(dw), u, u + L, dws, wsb, stream, nullptr, RUN,
                             nullptr, nullptr, nullptr);
                float t = 0.0f;
                if (st == TM_OK && rep > 0 &&
                    (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                     hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                    st = TM_ERR_HIP;
                if (st == TM_OK && rep > 0 && (tot == 0.0f || t < tot)) tot = t;
            }
            if (st != TM_OK) break;
            if (best_ms == 0.0f || tot < best_ms) {
                best_ms = tot;
                best = lm;
            }
        }
        cleanup();
        if (st != TM_OK) return st;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_pair((int)kind, n_bits)] = best;
    }
    if (chosen) return tm_plan_query(kind, n_bits, chosen);
    return TM_OK;
}

size_t tm_workspace_bytes_guaranteed(tm_kind kind, uint64_t n_bits)
{
    Plan P;
    return plan_guaranteed(kind, n_bits, P) == TM_OK ? P.ws_bytes : 0;
}

tm_status tm_plan_query_guaranteed(tm_kind kind, uint64_t n_bits, tm_plan_info* out)
{
    if (!out) {
        g_last_error = "null pointer";
        return TM_ERR_INVALID;
    }
    Plan P;
    tm_status st = plan_guaranteed(kind, n_bits, P);
    if (st != TM_OK) return st;
    fill_info(kind, n_bits, P, out);
    return TM_OK;
}

tm_status tm_mul_guaranteed(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                            uint64_t n_bits, void* workspace, size_t workspace_bytes,
                            hipStream_t stream, tm_guard* guard_dev)
{
    Plan P;
    tm_status st = plan_guaranteed(kind, n_bits, P);
    if (st != TM_OK) return st;
    return run(P, w, u, v, workspace, workspace_bytes, stream, guard_dev, RUN, nullptr, nullptr,
               nullptr);
}

tm_status tm_mul(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                 uint64_t n_bits, void* workspace, size_t workspace_bytes, hipStream_t stream,
                 tm_guard* guard_dev)
{
    Plan P;
    tm_status st = plan_for(kind, n_bits, P);
    if (st != TM_OK) return st;
    return run(P, w, u, v, workspace, workspace_bytes, stream, guard_dev, RUN, nullptr, nullptr,
               nullptr);
}

size_t tm_workspace_bytes_fp32c(tm_kind kind, uint64_t n_bits)
{
    Plan P;
    return plan_fp32c(kind, n_bits, P) == TM_OK ? P.ws_bytes : 0;
}

tm_status tm_plan_query_fp32c(tm_kind kind, uint64_t n_bits, tm_plan_info* out)
{
    if (!out) {
        g_last_error = "null pointer";
        return TM_ERR_INVALID;
    }
    Plan P;
    tm_status st = plan_fp32c(kind, n_bits, P);
    if (st != TM_OK) return st;
    fill_info(kind, n_bits, P, out);
    return TM_OK;
}

tm_status tm_mul_fp32c(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                       uint64_t n_bits, void* workspace, size_t workspace_bytes, hipStream_t stream,
                       tm_guard* guard_dev)
{
    Plan P;
    tm_status st = plan_fp32c(kind, n_bits, P);
    if (st != TM_OK) return st;
    return run(P, w, u, v, workspace, workspace_bytes, stream, guard_dev, RUN, nullptr, nullptr,
               nullptr);
}

tm_status tm_coefficients_fp32c(tm_kind kind, int64_t* coeffs, double* x, uint64_t coeffs_len,
                                const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                                void* workspace, size_t workspace_bytes, hipStream_t stream,
                                tm_guard* guard_dev)
{
    Plan P;
    tm_status st = plan_fp32c(kind, n_bits, P);
    if (st != TM_OK) return st;
    if (coeffs_len < P.ncoef) {
        g_last_error = "coefficient buffer too small";
        return TM_ERR_INVALID;
    }
    return run(P, nullptr, u, v, workspace, workspace_bytes, stream, guard_dev, DIAG_RUN, coeffs,
               x, nullptr);
}

size_t tm_noalloc_max_bytes(void) { return NOALLOC_MAX; }

tm_status tm_mul_noalloc(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                         uint64_t n_bits, hipStream_t stream, tm_guard* guard_dev)
{
    Plan P;
    tm_status st = plan_for(kind, n_bits, P);
    if (st != TM_OK) return st;
    if (P.ws_bytes > NOALLOC_MAX) {
        char buf[160];
        snprintf(buf, sizeof buf, "tm_mul_noalloc: needs %zu bytes of scratch, the static maximum is %zu",
                 P.ws_bytes, NOALLOC_MAX);
        g_last_error = buf;
        return TM_ERR_UNSUPPORTED;
    }
    void* ws = nullptr;
    st = scratch_ptr(ws);
    if (st != TM_OK) return st;
    // same kernels as tm_mul; K1 clears the look-back records, ticket and
    // guard at the start of every call, so nothing carries over between calls
    return run(P, w, u, v, ws, NOALLOC_MAX, stream, guard_dev, RUN, nullptr, nullptr, nullptr,
               false);
}

tm_status tm_prepare(tm_kind kind, uint64_t n_bits, hipStream_t stream)
{
    Plan P;
    tm_status st = plan_for(kind, n_bits, P);
    if (st != TM_OK) return st;
    TwEntry tw;
    return get_twiddles(P.M, P.L1, P.Lm, P.L2, stream, tw);
}

tm_status tm_mul_full(uint64_t* w, const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                      void* workspace, size_t workspace_bytes, hipStream_t stream,
                      tm_guard* guard_dev)
{
    return tm_mul(TM_FULL, w, u, v, n_bits, workspace, workspace_bytes, stream, guard_dev);
}

tm_status tm_mul_lo(uint64_t* w, const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                    void* workspace, size_t workspace_bytes, hipStream_t stream,
                    tm_guard* guard_dev)
{
    return tm_mul(TM_LO, w, u, v, n_bits, workspace, workspace_bytes, stream, guard_dev);
}

tm_status tm_mul_hi(uint64_t* w, const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                    void* workspace, size_t workspace_bytes, hipStream_t stream,
                    tm_guard* guard_dev)
{
    return tm_mul(TM_HI, w, u, v, n_bits, workspace, workspace_bytes, stream, guard_dev);
}

size_t tm_workspace_bytes_batched(const tm_request* reqs, size_t count)
{
    if (!reqs && count) return 0;
    size_t m = 0;
    for (size_t i = 0; i < count; i++) {
        size_t b = tm_workspace_bytes((tm_kind)reqs[i].kind, reqs[i].n_bits);
        if (b == 0) return 0;
        m += align256(b);
    }
    return m + meta_bytes_for(count);
}

size_t tm_batch_meta_bytes(size_t count) { return meta_bytes_for(count); }

tm_status tm_mul_packed(const tm_request* reqs, size_t count, void* const* workspaces,
                        const size_t* workspace_bytes, void* meta, size_t meta_bytes,
                        hipStream_t stream, tm_guard* const* guards_dev)
{
    return run_packed(reqs, count, workspaces, workspace_bytes, guards_dev, meta, meta_bytes, stream);
}

tm_status tm_mul_packed_staged(const tm_request* reqs, size_t count, void* const* workspaces,
                               const size_t* workspace_bytes, void* meta, size_t meta_bytes,
                               void* host_staging, size_t host_staging_bytes, hipStream_t stream,
                               tm_guard* const* guards_dev)
{
    if (count && !host_staging) {
        g_last_error = "null host staging buffer";
        return TM_ERR_INVALID;
    }
    return run_packed(reqs, count, workspaces, workspace_bytes, guards_dev, meta, meta_bytes, stream,
                      host_staging, host_staging_bytes);
}

tm_status tm_mul_batched(const tm_request* reqs, size_t count, void* workspace,
                         size_t workspace_bytes, hipStream_t stream, tm_guard* guards_dev)
{
    if (count == 0) return TM_OK;
    if (!reqs || !workspace) {
        g_last_error = "null pointer";
        return TM_ERR_INVALID;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
        g_last_error = "workspace must be 256-byte aligned";
        return TM_ERR_INVALID;
    }
    const size_t need = tm_workspace_bytes_batched(reqs, count);
    if (need == 0) {
        g_last_error = "unsupported request in batch";
        return TM_ERR_UNSUPPORTED;
    }
    if (workspace_bytes < need) {
        g_last_error = "workspace too small";
        return TM_ERR_INVALID;
    }
    // carve: one workspace per request, then the metadata area
    std::vector<void*> ws(count);
    std::vector<size_t> wsb(count);
    std::vector<tm_guard*> gs(count);
    char* base = static_cast<char*>(workspace);
    size_t o = 0;
    for (size_t i = 0; i < count; i++) {
        ws[i] = base + o;
        wsb[i] = tm_workspace_bytes((tm_kind)reqs[i].kind, reqs[i].n_bits);
        o += align256(wsb[i]);
        gs[i] = guards_dev ? guards_dev + i : nullptr;
    }
    return run_packed(reqs, count, ws.data(), wsb.data(), gs.data(), base + o, need - o, stream);
}

size_t tm_workspace_bytes_checked(tm_kind kind, uint64_t n_bits)
{
    Plan P, F;
    if (plan_for(kind, n_bits, P) != TM_OK) return 0;
    size_t m = P.ws_bytes;
    if (fallback_plan(kind, n_bits, P, F)) m = F.ws_bytes > m ? F.ws_bytes : m;
    return m;
}

tm_status tm_mul_checked(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                         uint64_t n_bits, void* workspace, size_t workspace_bytes,
                         hipStream_t stream, tm_guard* guard_host)
{
    Plan P;
    tm_status st = plan_for(kind, n_bits, P);
    if (st != TM_OK) return st;
    tm_guard g;
    for (int attempt = 0; attempt < 2; attempt++) {
        st = run(P, w, u, v, workspace, workspace_bytes, stream, nullptr, RUN, nullptr, nullptr,
                 nullptr);
        if (st != TM_OK) return st;
        HIP_TRY(hipMemcpyAsync(&g, static_cast<char*>(workspace) + P.o_guard, sizeof g,
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (guard_host) *guard_host = g;
        if (g.flags == 0 || exact_by_bound(P, g)) return TM_OK;
        if (attempt == 0) {
            Plan F;
            if (!fallback_plan(kind, n_bits, P, F)) {
                g_last_error = "rounding guard tripped and no guaranteed plan exists at this size";
                return TM_ERR_PRECISION;
            }
            P = F;
        }
    }
    g_last_error = "rounding guard tripped in the guaranteed fallback plan";
    return TM_ERR_PRECISION;
}

tm_status tm_coefficients(tm_kind kind, int64_t* coeffs, double* x, uint64_t coeffs_len,
                          const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                          void* workspace, size_t workspace_bytes, hipStream_t stream,
                          tm_guard* guard_dev)
{
    Plan P;
    tm_status st = plan_for(kind, n_bits, P);
    if (st != TM_OK) return st;
    if (coeffs_len < P.ncoef) {
        g_last_error = "coefficient buffer too small";
        return TM_ERR_INVALID;
    }
    return run(P, nullptr, u, v, workspace, workspace_bytes, stream, guard_dev, DIAG_RUN, coeffs,
               x, nullptr);
}

tm_status tm_profile_stages(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                            uint64_t n_bits, void* workspace, size_t workspace_bytes,
                            hipStream_t stream, float* stage_ms, const char** names, int cap,
                            int* n_stages)
{
    static const char* kNames2[4] = {"split_map_colfft", "rowfft_pointwise_rowifft", "col_ifft",
                                     "backmap_round_carry"};
    static const char* kNames3[6] = {"split_map_colfft", "mid_colfft", "rowfft_pointwise_rowifft",
                                     "mid_colifft", "col_ifft", "backmap_round_carry"};
    if (!stage_ms || !n_stages || cap < 6) {
        g_last_error = "stage buffer too small";
        return TM_ERR_INVALID;
    }
    Plan P;
    tm_status st = plan_for(kind, n_bits, P);
    if (st != TM_OK) return st;
    static const char* kNamesF[2] = {"fused_fft", "backmap_round_carry"};
    const int ns = P.fused ? 2 : P.Lm > 1 ? 6 : 4;
    const char** nm = P.fused ? kNamesF : P.Lm > 1 ? kNames3 : kNames2;
    hipEvent_t ev[7];
    for (int i = 0; i <= ns; i++) HIP_TRY(hipEventCreate(&ev[i]));
    st = run(P, w, u, v, workspace, workspace_bytes, stream, nullptr, RUN, nullptr, nullptr, ev);
    if (st == TM_OK) {
        hipError_t e = hipEventSynchronize(ev[ns]);
        if (e != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
        for (int i = 0; st == TM_OK && i < ns; i++) {
            e = hipEventElapsedTime(&stage_ms[i], ev[i], ev[i + 1]);
            if (e != hipSuccess) st = hip_fail(e, "hipEventElapsedTime");
            if (names) names[i] = nm[i];
        }
        *n_stages = ns;
    }
    for (int i = 0; i <= ns; i++) (void)hipEventDestroy(ev[i]);
    return st;
}

const char* tm_status_string(tm_status s)
{
    switch (s) {
    case TM_OK: return "ok";
    case TM_ERR_INVALID: return "invalid argument";
    case TM_ERR_HIP: return "HIP error";
    case TM_ERR_PRECISION: return "rounding guard tripped";
    case TM_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

const char* tm_last_error(void) { return g_last_error.c_str(); }

void tm_release_caches(void)
{
    {
        // work still queued on any stream may read the tables: wait for
        // each device that holds some before freeing them
        std::lock_guard<std::mutex> lk(g_tw_mu);
        int cur = 0;
        const bool have_cur = hipGetDevice(&cur) == hipSuccess;
        int last = -1;
        for (auto& kv : g_tw) {
            const int dev = std::get<0>(kv.first);
            if (dev != last && hipSetDevice(dev) == hipSuccess) (void)hipDeviceSynchronize();
            last = dev;
            (void)hipFree(kv.second.buf);
        }
        g_tw.clear();
        if (have_cur) (void)hipSetDevice(cur);
    }
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (auto& kv : g_stage)
        for (auto& b : kv.second) {
            if (b.pending) (void)hipEventSynchronize(b.ev);
            (void)hipEventDestroy(b.ev);
            if (b.host) (void)hipHostFree(b.host);
        }
    g_stage.clear();
}

}  // extern "C"
