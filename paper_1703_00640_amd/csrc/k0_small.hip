// Instances of the fused small-size pass K0 (one workgroup per product,
// whole transform in LDS), for every split of the planner's lengths
// M <= 4096, plain and packed.
#include "dispatch.hpp"

namespace tmul {

template <int KIND>
static bool k0_plain(uint32_t L1, uint32_t L2, const KParams& p, hipStream_t s)
{
#define X(A, B)                                                                        \
    if (L1 == A && L2 == B) {                                                          \
        hipLaunchKernelGGL((k0_fused<A, B, KIND>), dim3(1), dim3(NT0), 0, s, p);     \
        return true;                                                                   \
    }
    TM_K0_LIST(X)
#undef X
    return false;
}

template <int KIND>
static bool k0_packed(uint32_t L1, uint32_t L2, const Group& g, uint32_t blocks, hipStream_t s)
{
#define X(A, B)                                                                            \
    if (L1 == A && L2 == B) {                                                              \
        hipLaunchKernelGGL((k0_fused_g<A, B, KIND>), dim3(blocks), dim3(NT0), 0, s, g);  \
        return true;                                                                       \
    }
    TM_K0_LIST(X)
#undef X
    return false;
}

bool launch_k0(int kind, uint32_t L1, uint32_t L2, const KParams& p, hipStream_t s)
{
    if (kind == TM_FULL) return k0_plain<K_FULL>(L1, L2, p, s);
    if (kind == TM_LO) return k0_plain<K_LO>(L1, L2, p, s);
    return k0_plain<K_HI>(L1, L2, p, s);
}

bool launch_k0g(int kind, uint32_t L1, uint32_t L2, const Group& g, uint32_t blocks, hipStream_t s)
{
    if (kind == TM_FULL) return k0_packed<K_FULL>(L1, L2, g, blocks, s);
    if (kind == TM_LO) return k0_packed<K_LO>(L1, L2, g, blocks, s);
    return k0_packed<K_HI>(L1, L2, g, blocks, s);
}

}  // namespace tmul
