// Trip kernel instantiations: FP32, with right-hand side, mode 0.
#include "trip_kernel.h"

namespace jacobi_impl {
hipError_t trip_dispatch_f32rhs_m0(const TripConfig& c, const TripParams& p, hipStream_t s)
{
    return dispatch_unit<float, true, 0>(c, p, s);
}
}  // namespace jacobi_impl
