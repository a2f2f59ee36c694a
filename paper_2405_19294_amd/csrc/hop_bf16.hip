// Hopping-kernel instances with bf16_t storage.
#include "hop_impl.h"

namespace hrw {
template <>
hipError_t launch_hop<bf16_t>(int nr, bool dagger, int epi, const HopArgs<bf16_t> &a, hipStream_t st)
{
    return launch_hop_impl<bf16_t>(nr, dagger, epi, a, st);
}
template <>
hipError_t launch_hop_fused<bf16_t>(int nc, int rep, bool dagger, int epi, const HopArgs<bf16_t> &a, hipStream_t st)
{
    return launch_hop_fused_impl<bf16_t>(nc, rep, dagger, epi, a, st);
}
template <>
hipError_t launch_hop_su3<bf16_t>(bool dagger, int epi, const HopArgs<bf16_t> &a, hipStream_t st)
{
    return launch_hop_su3_impl<bf16_t>(dagger, epi, a, st);
}
}  // namespace hrw
