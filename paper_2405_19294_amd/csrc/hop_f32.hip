// Hopping-kernel instances with float storage.
#include "hop_impl.h"

namespace hrw {
template <>
hipError_t launch_hop<float>(int nr, bool dagger, int epi, const HopArgs<float> &a, hipStream_t st)
{
    return launch_hop_impl<float>(nr, dagger, epi, a, st);
}
}  // namespace hrw
