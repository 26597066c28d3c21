// Trip kernel dispatch: picks the instantiation unit (trip_*.hip) for a
// launch's precision, right-hand side and mode.  The kernel itself is in
// trip_kernel.h.

#include "internal.h"
#include "trip_configs.h"

namespace jacobi_impl {

hipError_t trip_dispatch_f64_m0(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f64_m1(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f64_m1r(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f64_m2(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f64_m3(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f64_s27(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f32_m0(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f32_m2(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f32rhs_m0(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f32rhs_m2(const TripConfig&, const TripParams&, hipStream_t);
hipError_t trip_dispatch_f32w_m0(const TripConfig&, const TripParams&, hipStream_t);

bool trip_config_supported(int dtype_f32, const TripConfig& c)
{
    (void)dtype_f32;
#define JACOBI_SUP(T_, R_, W_) \
    if (c.T == T_ && c.R == R_ && c.W == W_) return true;
    JACOBI_TRIP_CFGS(JACOBI_SUP)
#undef JACOBI_SUP
    return false;
}

bool trip_config_supported_s27(const TripConfig& c)
{
#define JACOBI_SUP(T_, R_, W_) \
    if (c.T == T_ && c.R == R_ && c.W == W_) return true;
    JACOBI_S27_CFGS(JACOBI_SUP)
#undef JACOBI_SUP
    return false;
}

hipError_t launch_trip_f64(const TripConfig& c, const TripParams& p,
                           hipStream_t s)
{
    if (p.s27)
        return p.mode == 0 || p.mode == 4 ? trip_dispatch_f64_s27(c, p, s) : hipErrorInvalidValue;
    switch (p.mode) {
    case 0: return trip_dispatch_f64_m0(c, p, s);
    case 1: return p.krev ? trip_dispatch_f64_m1r(c, p, s) : trip_dispatch_f64_m1(c, p, s);
    case 2: return trip_dispatch_f64_m2(c, p, s);
    case 3: return trip_dispatch_f64_m3(c, p, s);
    default: return hipErrorInvalidValue;
    }
}

// FP32 sweeps run on dense A/B correction grids (mode 0) or in a batch
// (mode 2); there is no compressed FP32 layout.
hipError_t launch_trip_f32(const TripConfig& c, const TripParams& p,
                           hipStream_t s)
{
    const bool rhs = p.rhs || p.rhs_in_table;
    if (p.weighted) return rhs && p.mode == 0 ? trip_dispatch_f32w_m0(c, p, s) : hipErrorInvalidValue;
    switch (p.mode) {
    case 0: return rhs ? trip_dispatch_f32rhs_m0(c, p, s) : trip_dispatch_f32_m0(c, p, s);
    case 2: return rhs ? trip_dispatch_f32rhs_m2(c, p, s) : trip_dispatch_f32_m2(c, p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace jacobi_impl
