// Trip kernel instantiations: FP64, no right-hand side, mode 1, k-mirrored
// view (backward compressed trips).
#include "trip_kernel.h"

namespace jacobi_impl {
hipError_t trip_dispatch_f64_m1r(const TripConfig& c, const TripParams& p, hipStream_t s)
{
    return dispatch_unit<double, false, 1, false, true>(c, p, s);
}
}  // namespace jacobi_impl
