// C-ABI of the truncated-multiplication library (see include/tmul.h).
// Host code: planning, twiddle cache, template dispatch, launch sequence.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "tmul.h"
#include "plan.hpp"
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
std::map<std::pair<int, uint64_t>, TwEntry> g_tw;

// Twiddle tables for transform length M = L1 * L2 (the plan fixes L1, L2
// from M), built once per device.
tm_status get_twiddles(uint64_t M, uint32_t L1, uint32_t Lm, uint32_t L2, hipStream_t s, TwEntry& out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tw_mu);
    auto key = std::make_pair(dev, M * 512 + Lm);
    auto it = g_tw.find(key);
    if (it != g_tw.end()) {
        out = it->second;
        return TM_OK;
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
    case V: hipLaunchKernelGGL((k3_col_inverse<V, w3_for(V)>), dim3(p.R / w3_for(V)), dim3(NT3), 0, s, p); return true;
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

// Splits chosen by tm_autotune: (kind, n) -> middle length Lm (0: the
// planner's own choice).  The split changes only the FFT schedule, not N or
// b, so tuned and untuned calls return the same products.
std::mutex g_tune_mu;
std::map<std::pair<int, uint64_t>, uint32_t> g_tuned;

uint32_t tuned_lm(tm_kind kind, uint64_t n)
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
        const char* e = getenv("TM_FORCE_LM");
        if (e && *e) flm = (uint32_t)atoi(e);
    }
    if (!flm) flm = tuned_lm(kind, n);
    if (!make_plan((int)kind, n, bt, bf, P, flm)) {
        g_last_error = "unsupported size";
        return TM_ERR_UNSUPPORTED;
    }
    return TM_OK;
}

enum Mode { RUN, DIAG_RUN };

tm_status run(const Plan& P, uint64_t* w, const uint64_t* u, const uint64_t* v, void* ws,
              size_t ws_bytes, hipStream_t s, tm_guard* guard, Mode mode, int64_t* dc,
              double* dx, hipEvent_t* ev)
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
    tm_status st = get_twiddles(P.M, P.L1, P.Lm, P.L2, s, tw);
    if (st != TM_OK) return st;
    KParams p;
    uint64_t dummy_out = 0;
    (void)dummy_out;
    fill_params(P, u, v, w, ws, guard, tw, p);
    if (mode == DIAG_RUN) {
        // K1 clears out_limbs of w; point it at the coefficient buffer's
        // storage only when no output exists: use zero output limbs instead
        p.w = reinterpret_cast<uint64_t*>(dc);
        p.out_limbs = 0;
        p.dbg_c = dc;
        p.dbg_x = dx;
    }
    int ne = 0;
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    if (!launch_k1_any(P.kind, p, s)) {
        g_last_error = "no kernel for L1";
        return TM_ERR_UNSUPPORTED;
    }
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    if (P.Lm > 1) {
        if (!launch_mid<false>(p, s)) {
            g_last_error = "no kernel for Lm";
            return TM_ERR_UNSUPPORTED;
        }
        if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    }
    if (!launch_k2(P.L2, p, s)) {
        g_last_error = "no kernel for L2";
        return TM_ERR_UNSUPPORTED;
    }
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    if (P.Lm > 1) {
        launch_mid<true>(p, s);
        if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    }
    launch_k3(P.L1, p, s);
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    if (mode == DIAG_RUN) launch_k4<true>(P.kind, p, s);
    else launch_k4<false>(P.kind, p, s);
    if (ev) HIP_TRY(hipEventRecord(ev[ne++], s));
    HIP_TRY(hipGetLastError());
    return TM_OK;
}

// Fallback plan of tm_mul_checked: the guaranteed plan if there is one with
// smaller digits, else two bits smaller digits for the truncated products
// and four bits smaller for the full product.
bool fallback_plan(tm_kind kind, uint64_t n_bits, const Plan& P, Plan& F)
{
    if (make_plan_guaranteed((int)kind, n_bits, F) && F.b < P.b) return true;
    int bt = P.kind == TM_FULL ? 0 : P.b - 2;
    int bf = P.kind == TM_FULL ? P.b - 4 : 0;
    return make_plan((int)kind, n_bits, bt, bf, F);
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
    // candidates: the planner's split and every forced middle length
    std::vector<uint32_t> cand{0};
    for (uint32_t lm = 2; lm <= LM_MAX; lm *= 2) {
        Plan Q;
        if (make_plan((int)kind, n_bits, 0, 0, Q, lm) && Q.Lm != P0.Lm) cand.push_back(lm);
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
            float tot = 0.0f;
            for (int rep = 0; rep < 4 && st == TM_OK; rep++) {
                if (rep == 1) st = hipEventRecord(e0, stream) == hipSuccess ? TM_OK : TM_ERR_HIP;
                if (st == TM_OK)
                    st = run(Q, static_cast<uint64_t*>(dw), u, u + L, dws, wsb, stream, nullptr, RUN,
                             nullptr, nullptr, nullptr);
            }
            if (st == TM_OK && (hipEventRecord(e1, stream) != hipSuccess ||
                                hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&tot, e0, e1) != hipSuccess))
                st = TM_ERR_HIP;
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
    size_t m = 0;
    if (!reqs) return 0;
    for (size_t i = 0; i < count; i++) {
        size_t b = tm_workspace_bytes((tm_kind)reqs[i].kind, reqs[i].n_bits);
        if (b == 0) return 0;
        if (b > m) m = b;
    }
    return m;
}

tm_status tm_mul_batched(const tm_request* reqs, size_t count, void* workspace,
                         size_t workspace_bytes, hipStream_t stream, tm_guard* guards_dev)
{
    if (!reqs && count) {
        g_last_error = "null pointer";
        return TM_ERR_INVALID;
    }
    for (size_t i = 0; i < count; i++) {
        tm_status st = tm_mul((tm_kind)reqs[i].kind, reqs[i].w, reqs[i].u, reqs[i].v,
                              reqs[i].n_bits, workspace, workspace_bytes, stream,
                              guards_dev ? guards_dev + i : nullptr);
        if (st != TM_OK) return st;
    }
    return TM_OK;
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
        if (g.flags == 0) return TM_OK;
        if (attempt == 0) {
            Plan F;
            if (!fallback_plan(kind, n_bits, P, F)) break;
            P = F;
        }
    }
    g_last_error = "rounding guard tripped after fallback";
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
    const int ns = P.Lm > 1 ? 6 : 4;
    const char** nm = P.Lm > 1 ? kNames3 : kNames2;
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
    std::lock_guard<std::mutex> lk(g_tw_mu);
    for (auto& kv : g_tw) (void)hipFree(kv.second.buf);
    g_tw.clear();
}

}  // extern "C"
