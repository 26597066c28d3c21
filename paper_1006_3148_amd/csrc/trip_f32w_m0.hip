// Trip kernel instantiations: FP32 with right-hand side, weighted sweeps (the
// multigrid smoother), mode 0.
#include "trip_kernel.h"

namespace jacobi_impl {
hipError_t trip_dispatch_f32w_m0(const TripConfig& c, const TripParams& p, hipStream_t s)
{
    return dispatch_unit<float, true, 0, true>(c, p, s);
}
}  // namespace jacobi_impl
