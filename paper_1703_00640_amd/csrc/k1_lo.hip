// K1 instances (split + map + column FFT) of the low product.
#include "dispatch.hpp"

namespace tmul {

bool launch_k1_lo(uint32_t L1, const KParams& p, hipStream_t s)
{
    return launch_k1<K_LO, B_TRUNC>(L1, p, s);
}

bool launch_k1g_lo(uint32_t L1, int fb, bool wide, const Group& g, uint32_t blocks, hipStream_t s)
{
    return launch_k1g<K_LO, B_TRUNC>(L1, fb, wide, g, blocks, s);
}

}  // namespace tmul
