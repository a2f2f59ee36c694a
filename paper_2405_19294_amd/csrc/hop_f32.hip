// Hopping-kernel instances with float storage; several sources of the
// two-index representations of SU(3)/SU(4) (N_R = 6) run on the matrix cores.
#include "hop_mfma.h"

namespace hrw {
template <>
hipError_t launch_hop<float>(int nr, bool dagger, int epi, const HopArgs<float> &a, hipStream_t st)
{
    if (hop_uses_mfma(nr, 1, a.n_rhs)) return launch_hop_mfma<6>(dagger, epi, a, st);
    return launch_hop_impl<float>(nr, dagger, epi, a, st);
}
template <>
hipError_t launch_hop_fused<float>(int nc, int rep, bool dagger, int epi, const HopArgs<float> &a, hipStream_t st)
{
    return launch_hop_fused_impl<float>(nc, rep, dagger, epi, a, st);
}
template <>
hipError_t launch_hop_su3<float>(bool dagger, int epi, const HopArgs<float> &a, hipStream_t st)
{
    return launch_hop_su3_impl<float>(dagger, epi, a, st);
}
}  // namespace hrw
