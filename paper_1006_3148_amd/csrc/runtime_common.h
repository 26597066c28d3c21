// Host-side helpers shared by the single-problem and batched runtimes.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "internal.h"
#include "jacobi.h"

namespace jacobi_impl {

// Sets the thread-local error message and returns `code`.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
const char* last_error_text();

constexpr int kCUs = 256;  // MI355X compute units

struct Plan {
    TripConfig cfg{1, 4, 16};
    int tiles_x = 0, tiles_y = 0, segs = 0, seg_len = 0, ntiles = 0;
    // Split trip (A/B, 27-point): the first ntiles columns run whole (one
    // segment), then tail_cols columns from column ntiles on run in a second
    // launch, in segments of tail_len planes (tail_tiles tiles).
    int tail_cols = 0, tail_len = 0, tail_tiles = 0;
};

// Default tile shape for T sweeps per trip (register state fits without
// spilling; measured best on MI355X at 512^3); s27: of the 27-point update.
TripConfig default_cfg(int T, bool compressed = false, bool s27 = false);

// Tiling of one (nx, ny, nz) box for `cfg`.  seg_req > 0 fixes the k segment
// length; `compressed` enforces tiles and segments >= 2T (the shift safety
// condition of the compressed grid) and segments >= min_seg.  `target_tiles`
// is the tile count the segment heuristic aims to fill (concurrent
// workgroups).  False if the shape cannot cover the box.
bool make_plan(int64_t nx, int64_t ny, int64_t nz, const TripConfig& cfg,
               int seg_req, bool compressed, int target_tiles, Plan* out,
               int min_seg = 0);

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

}  // namespace jacobi_impl
