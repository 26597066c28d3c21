// Internal declarations shared by the HIP translation units of libjacobi.
// Not part of the public C-ABI (that is include/jacobi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace jacobi_impl {

// Geometry and pointers of one trip launch (t fused sweeps, one pass through
// HBM).  All pointers address logical cell (0,0,0) of their frame; cell
// (i,j,k) of a frame lives at origin + k*py + j*px + i.
struct TripParams {
    const void* src;   // input frame (current iterate)
    void* dst;         // output frame (next iterate; == src frame shifted for
                       // the compressed layout, the other grid for A/B)
    const float* rhs;  // FP32 right-hand side frame (correction sweeps) or null
    int64_t px, py;    // pitches of src/dst (elements)
    int64_t rpx, rpy;  // pitches of rhs
    int nx, ny, nz;    // interior dims
    int tiles_x, tiles_y, segs, seg_len;
    int ntiles;
    int mode;          // 0: blockIdx tiles (A/B); 1: tickets + flags (compressed)
    int dir;           // +1 forward shift (-t), -1 backward shift (+t); mode 1
    int* flags;        // per-tile progress words, stride kFlagStride ints
    int* ticket;       // ticket counter (zeroed before the launch)
    int* err;          // error word: 0 ok, nonzero = watchdog fired
    int64_t spin_limit;
};

constexpr int kFlagStride = 32;  // ints per flag (128 B line each)

// Trip kernel configurations (tile = 64 x R*W columns, T stages).
struct TripConfig {
    int T, R, W;
};

// Launches one trip.  Returns hipSuccess or the launch error.  `cfg` must be
// one of the compiled configurations (see trip_config_supported).
hipError_t launch_trip_f64(const TripConfig& cfg, const TripParams& p,
                           hipStream_t s);
hipError_t launch_trip_f32(const TripConfig& cfg, const TripParams& p,
                           hipStream_t s);
bool trip_config_supported(int dtype_f32, const TripConfig& cfg);

// ---- auxiliary kernels (kernels_aux.hip) ----
hipError_t launch_fill_i32(int* p, int value, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float value, int64_t n, hipStream_t s);

// Residual r = fold(nbrs) - 6u on the interior.  Pass 1 writes per-block
// partial sums of r^2 (and max |r|) into `partials` (2*nblocks doubles);
// pass 2 reduces them in fixed order into out[0] = ||r||_2, out[1] = max|r|.
int residual_blocks(int nx, int ny, int nz);
hipError_t launch_residual(const double* u, int64_t px, int64_t py, int nx,
                           int ny, int nz, double* partials, double* out,
                           hipStream_t s);

// FP32 refinement helpers.
//  rhs = fl32(r * 2^-s) with s = frexp exponent of out[1] (max|r|) read on the
//  device; the exponent is stored in *scale_exp.
hipError_t launch_make_rhs(const double* u, int64_t px, int64_t py, int nx,
                           int ny, int nz, const double* maxabs,
                           int* scale_exp, float* rhs, int64_t rpx,
                           int64_t rpy, hipStream_t s);
//  u(interior) += fl64(e) * 2^scale_exp
hipError_t launch_apply_correction(double* u, int64_t px, int64_t py, int nx,
                                   int ny, int nz, const float* e,
                                   int64_t epx, int64_t epy,
                                   const int* scale_exp, hipStream_t s);

// Box copy between frames of the same logical dims (used to seed the second
// grid and for compressed-layout moves).
hipError_t launch_copy_box_f64(const double* src, int64_t spx, int64_t spy,
                               double* dst, int64_t dpx, int64_t dpy, int nx2,
                               int ny2, int nz2, hipStream_t s);

// Bandwidth probes: STREAM-like copy b[i] = a[i] and in-place update
// a[i] += 1.0 (the paper's array-update benchmark).
hipError_t launch_stream_copy(const double* a, double* b, int64_t n,
                              hipStream_t s);
hipError_t launch_stream_update(double* a, int64_t n, hipStream_t s);

}  // namespace jacobi_impl
