// Hopping-kernel instances with double storage.
#include "hop_impl.h"

namespace hrw {
template <>
hipError_t launch_hop<double>(int nr, bool dagger, int epi, const HopArgs<double> &a, hipStream_t st)
{
    return launch_hop_impl<double>(nr, dagger, epi, a, st);
}
template <>
hipError_t launch_hop_fused<double>(int nc, int rep, bool dagger, int epi, const HopArgs<double> &a, hipStream_t st)
{
    return launch_hop_fused_impl<double>(nc, rep, dagger, epi, a, st);
}
template <>
hipError_t launch_hop_su3<double>(bool dagger, int epi, const HopArgs<double> &a, hipStream_t st)
{
    return launch_hop_su3_impl<double>(dagger, epi, a, st);
}
}  // namespace hrw
