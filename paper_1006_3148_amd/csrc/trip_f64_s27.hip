// Trip kernel instantiations: FP64, 27-point update, mode 0 (whole columns or
// segments) and mode 4 (the segmented tail columns of a split trip).
#include "trip_kernel.h"

namespace jacobi_impl {
hipError_t trip_dispatch_f64_s27(const TripConfig& c, const TripParams& p, hipStream_t s)
{
#define JACOBI_CASE(T_, R_, W_)                                                               \
    if (c.T == T_ && c.R == R_ && c.W == W_)                                                  \
        return p.mode == 4                                                                    \
                   ? launch_mode<double, T_, R_, W_, kPrefetch, false, 4, false, false, true>(p, s) \
                   : launch_mode<double, T_, R_, W_, kPrefetch, false, 0, false, false, true>(p, s);
    JACOBI_S27_CFGS(JACOBI_CASE)
#undef JACOBI_CASE
    return hipErrorInvalidValue;
}
}  // namespace jacobi_impl
