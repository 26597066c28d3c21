// Trip kernel instantiations: FP64, no right-hand side, mode 3 (several
// trips in one persistent launch).
#include "trip_kernel.h"

namespace jacobi_impl {
hipError_t trip_dispatch_f64_m3(const TripConfig& c, const TripParams& p, hipStream_t s)
{
    return dispatch_unit<double, false, 3>(c, p, s);
}
}  // namespace jacobi_impl
