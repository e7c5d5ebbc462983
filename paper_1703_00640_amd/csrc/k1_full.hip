// K1 instances (split + map + column FFT) of the full product.
#include "dispatch.hpp"

namespace tmul {

bool launch_k1_full(uint32_t L1, const KParams& p, hipStream_t s)
{
    return launch_k1<K_FULL, B_FULL>(L1, p, s);
}

bool launch_k1g_full(uint32_t L1, int fb, bool wide, const Group& g, uint32_t blocks, hipStream_t s)
{
    return launch_k1g<K_FULL, B_FULL>(L1, fb, wide, g, blocks, s);
}

}  // namespace tmul
