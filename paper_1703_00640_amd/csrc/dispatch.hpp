// Template dispatch shared by the host translation units: column tile
// widths, the list of column lengths L1 with kernel instances, the choice of
// compile-time digit size, and the K1 launchers (one translation unit per
// kind, so the instances compile in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "plan.hpp"

namespace tmul {

// column tile width: the largest power of two W <= wmax with L1 W <= tile.
// With the three-pass split (large transforms, many column tiles) K3 and
// the full product's K1 take up to 16 columns: 256-byte row segments are
// 25-30% faster than 128-byte ones at n = 2^30 for columns up to 256.
// Two-pass splits (smaller sizes) keep 8, which gives twice the workgroups
// and lower latency; so does the truncated products' K1 always (its digit
// rows with the map halo need the registers).
constexpr int w_for(int L1, int tile, int wmax)
{
    int lim = tile / L1 < wmax ? tile / L1 : wmax;
    int w = 1;
    while (w * 2 <= lim) w *= 2;
    return w;
}
#ifndef TM_K1_TRUNC_WIDE
#define TM_K1_TRUNC_WIDE 0
#endif
constexpr int w1_for(int kind, int L1, bool wide)
{
    return w_for(L1, TILE1, (kind == K_FULL || TM_K1_TRUNC_WIDE) && wide ? 16 : 8);
}
constexpr int w3_for(int L1, bool wide) { return w_for(L1, TILE3, wide ? 16 : 8); }
inline bool wide_tiles(const KParams& p) { return p.Lm > 1; }

#define TM_L1_LIST(X) \
    X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) \
    X(256) X(384) X(512) X(768) X(1024) X(5) X(10) X(20) X(40) X(80) X(160) X(320) X(640) \
    X(7) X(14) X(28) X(56) X(112) X(224) X(448) X(896)

// Compile-time digit size of the K1 / K4 instances for a plan: the default
// sizes (b = 11 truncated with lam <= LB_FIXED, b = 16 full) have their own
// instances; every other plan runs the generic ones (B = 0).
inline int fixed_b(int kind, const KParams& p)
{
    if (kind == TM_FULL) return p.b == B_FULL ? B_FULL : 0;
    return p.b == B_TRUNC && p.lam <= LB_FIXED ? B_TRUNC : 0;
}

template <int KIND, int B>
bool launch_k1_b(uint32_t L1, const KParams& p, hipStream_t s)
{
    switch (L1) {
#define X(V) \
    case V:                                                                                              \
        if (wide_tiles(p))                                                                               \
            hipLaunchKernelGGL((k1_split_map_col<V, w1_for(KIND, V, true), KIND, B>),                    \
                               dim3(p.R / w1_for(KIND, V, true), p.zb == p.za ? 1 : 2), dim3(NT1), 0, s, p); \
        else                                                                                             \
            hipLaunchKernelGGL((k1_split_map_col<V, w1_for(KIND, V, false), KIND, B>),                   \
                               dim3(p.R / w1_for(KIND, V, false), p.zb == p.za ? 1 : 2), dim3(NT1), 0, s, p); \
        return true;
        TM_L1_LIST(X)
#undef X
    }
    return false;
}

template <int KIND, int BF>
bool launch_k1(uint32_t L1, const KParams& p, hipStream_t s)
{
    return fixed_b(KIND, p) ? launch_k1_b<KIND, BF>(L1, p, s) : launch_k1_b<KIND, 0>(L1, p, s);
}

// Packed launch of one K1 instance over the requests of group g (`blocks`
// workgroups in total); fb: the requests' common fixed_b().
template <int KIND, int B>
bool launch_k1g_b(uint32_t L1, bool wide, const Group& g, uint32_t blocks, hipStream_t s)
{
    switch (L1) {
#define X(V)                                                                                                  \
    case V:                                                                                                   \
        if (wide)                                                                                             \
            hipLaunchKernelGGL((k1_split_map_col_g<V, w1_for(KIND, V, true), KIND, B>), dim3(blocks), dim3(NT1), 0, s, g); \
        else                                                                                                  \
            hipLaunchKernelGGL((k1_split_map_col_g<V, w1_for(KIND, V, false), KIND, B>), dim3(blocks), dim3(NT1), 0, s, g); \
        return true;
        TM_L1_LIST(X)
#undef X
    }
    return false;
}

template <int KIND, int BF>
bool launch_k1g(uint32_t L1, int fb, bool wide, const Group& g, uint32_t blocks, hipStream_t s)
{
    return fb ? launch_k1g_b<KIND, BF>(L1, wide, g, blocks, s) : launch_k1g_b<KIND, 0>(L1, wide, g, blocks, s);
}

// defined in k1_full.hip, k1_lo.hip, k1_hi.hip
bool launch_k1_full(uint32_t L1, const KParams& p, hipStream_t s);
bool launch_k1_lo(uint32_t L1, const KParams& p, hipStream_t s);
bool launch_k1_hi(uint32_t L1, const KParams& p, hipStream_t s);
bool launch_k1g_full(uint32_t L1, int fb, bool wide, const Group& g, uint32_t blocks, hipStream_t s);
bool launch_k1g_lo(uint32_t L1, int fb, bool wide, const Group& g, uint32_t blocks, hipStream_t s);
bool launch_k1g_hi(uint32_t L1, int fb, bool wide, const Group& g, uint32_t blocks, hipStream_t s);

// fused small-size pass, defined in k0_small.hip
bool launch_k0(int kind, uint32_t L1, uint32_t L2, const KParams& p, hipStream_t s);
bool launch_k0g(int kind, uint32_t L1, uint32_t L2, const Group& g, uint32_t blocks, hipStream_t s);

// FP32 path (double-float FFT passes), defined in fp32c.hip
bool launch_k1_fp32c(int kind, uint32_t L1, const KParams& p, hipStream_t s);
bool launch_k2_fp32c(uint32_t L2, const KParams& p, hipStream_t s);
template <bool INV>
bool launch_mid_fp32c(const KParams& p, hipStream_t s);
bool launch_k3_fp32c(uint32_t L1, const KParams& p, hipStream_t s);
template <bool DIAG>
bool launch_k4_fp32c(int kind, const KParams& p, hipStream_t s);

}  // namespace tmul
