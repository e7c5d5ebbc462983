// Kernel instances of the FP32 path: the same stages as the FP64 path with
// the FFT passes in double-float arithmetic (element type dfc, see
// dfloat.hpp).  Digits, ring maps, theta, the 2^b scaling, rounding and the
// carry stay in FP64 and integers.  Transform lengths are powers of two, so
// only power-of-two column, middle and row lengths have instances; digit
// sizes are runtime values (generic digit windows).
#include "dispatch.hpp"

namespace tmul {

#define TM_L1_POW2(X) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024)

template <int KIND>
static bool k1_fp32c(uint32_t L1, const KParams& p, hipStream_t s)
{
    switch (L1) {
#define X(V)                                                                                    \
    case V:                                                                                     \
        hipLaunchKernelGGL((k1_split_map_col<V, w1_for(KIND, V, false), KIND, 0, dfc>),         \
                           dim3(p.R / w1_for(KIND, V, false), p.zb == p.za ? 1 : 2), dim3(NT1), 0, s, p); \
        return true;
        TM_L1_POW2(X)
#undef X
    }
    return false;
}

bool launch_k1_fp32c(int kind, uint32_t L1, const KParams& p, hipStream_t s)
{
    if (kind == TM_FULL) return k1_fp32c<K_FULL>(L1, p, s);
    if (kind == TM_LO) return k1_fp32c<K_LO>(L1, p, s);
    return k1_fp32c<K_HI>(L1, p, s);
}

bool launch_k2_fp32c(uint32_t L2, const KParams& p, hipStream_t s)
{
    const dim3 g(k2_groups(p.L1, p.Lm));
    switch (L2) {
#define X(V) \
    case V: hipLaunchKernelGGL((k2_rows_pointwise<V, dfc>), g, dim3(NT2), 0, s, p); return true;
        X(16) X(32) X(64) X(128) X(256) X(512) X(1024)
#undef X
    }
    return false;
}

// middle pass: 16 columns per tile for every middle length
template <bool INV>
bool launch_mid_fp32c(const KParams& p, hipStream_t s)
{
    constexpr int W = 16;
    if (p.L2 % W != 0) return false;
    const dim3 g(p.L2 / W, p.L1, INV || p.zb == p.za ? 1 : 2);
    switch (p.Lm) {
#define X(V) \
    case V: hipLaunchKernelGGL((k_mid_col<V, W, INV, dfc>), g, dim3(NTM), 0, s, p); return true;
        X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256)
#undef X
    }
    return false;
}
template bool launch_mid_fp32c<false>(const KParams&, hipStream_t);
template bool launch_mid_fp32c<true>(const KParams&, hipStream_t);

bool launch_k3_fp32c(uint32_t L1, const KParams& p, hipStream_t s)
{
    switch (L1) {
#define X(V)                                                                                            \
    case V:                                                                                             \
        hipLaunchKernelGGL((k3_col_inverse<V, w3_for(V, false), dfc>), dim3(p.R / w3_for(V, false)),     \
                           dim3(NT3), 0, s, p);                                                         \
        return true;
        TM_L1_POW2(X)
#undef X
    }
    return false;
}

template <bool DIAG>
bool launch_k4_fp32c(int kind, const KParams& p, hipStream_t s)
{
    const dim3 g(p.nstatus);
    if (kind == TM_FULL) hipLaunchKernelGGL((k4_backmap_carry<K_FULL, DIAG, 0, dfc>), g, dim3(NT4), 0, s, p);
    else if (kind == TM_LO) hipLaunchKernelGGL((k4_backmap_carry<K_LO, DIAG, 0, dfc>), g, dim3(NT4), 0, s, p);
    else hipLaunchKernelGGL((k4_backmap_carry<K_HI, DIAG, 0, dfc>), g, dim3(NT4), 0, s, p);
    return true;
}
template bool launch_k4_fp32c<false>(int, const KParams&, hipStream_t);
template bool launch_k4_fp32c<true>(int, const KParams&, hipStream_t);

}  // namespace tmul
