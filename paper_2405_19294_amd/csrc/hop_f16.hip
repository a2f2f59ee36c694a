// Hopping-kernel instances with f16_t storage.
#include "hop_impl.h"

namespace hrw {
template <>
hipError_t launch_hop<f16_t>(int nr, bool dagger, int epi, const HopArgs<f16_t> &a, hipStream_t st)
{
    return launch_hop_impl<f16_t>(nr, dagger, epi, a, st);
}
template <>
hipError_t launch_hop_fused<f16_t>(int nc, int rep, bool dagger, int epi, const HopArgs<f16_t> &a, hipStream_t st)
{
    return launch_hop_fused_impl<f16_t>(nc, rep, dagger, epi, a, st);
}
template <>
hipError_t launch_hop_su3<f16_t>(bool dagger, int epi, const HopArgs<f16_t> &a, hipStream_t st)
{
    return launch_hop_su3_impl<f16_t>(dagger, epi, a, st);
}
}  // namespace hrw
