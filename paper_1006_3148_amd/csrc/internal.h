// Internal declarations shared by the HIP translation units of libjacobi.
// Not part of the public C-ABI (that is include/jacobi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace jacobi_impl {

// One problem of a batch (device-resident table, MODE 2 of the trip kernel).
// grid[0], grid[1]: logical (0,0,0) of the two A/B frames; tile_base: number
// of tiles of all earlier problems in the table.
struct BatchProblem {
    void* grid[2];
    const float* rhs;
    int64_t px, py;
    int nx, ny, nz;
    int tiles_x, tiles_y, segs, seg_len;
    int tile_base;
};

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
    int mode;          // 0: blockIdx tiles (A/B); 1: tickets + flags
                       // (compressed); 2: batch table, tickets; 3: several
                       // trips (teams) in one persistent launch (A/B);
                       // 4: segmented tail columns of a split trip (A/B,
                       // 27-point)
    int dir;           // +1 forward shift (-t), -1 backward shift (+t); mode 1
    int* flags;        // per-tile progress words, stride kFlagStride ints
    int* ticket;       // ticket counter (zeroed before the launch)
    int* err;          // error word: 0 ok, nonzero = watchdog fired
    int64_t spin_limit;
    const BatchProblem* table;  // mode 2: problems (device memory)
    int count;                  // mode 2: number of problems
    const int* parity;          // mode 2: A/B parity word (device memory)
    int rhs_in_table;           // mode 2: FP32 rhs pointers are in the table
    int teams;                  // mode 3: trips in the launch (team r reads
                                // src for even r, dst for odd r)
    int looseness;              // mode 3: d_u (< 0: no bound)
    int* done;                  // mode 3: per-team count of finished tiles,
                                // stride kFlagStride ints (zeroed)
    int weighted;               // FP32 with rhs: weighted sweeps (multigrid
                                // smoother) with weight omega
    float omega;
    int groups;                 // mode 1: per-XCD claim groups (> 1) or one
                                // ticket counter (1); mode 4: tail columns
    int chunk;                  // mode 1 groups: tiles per chunk (set at
                                // launch); mode 0: > 0 selects band order;
                                // mode 4: first tail column
    int* gcnt;                  // mode 1 groups: kClaimGroups counters, stride
                                // kFlagStride ints (zeroed)
    int zshift;                 // mode 1: k shift of dst against src
                                // (planes, >= T)
    int krev;                   // mode 1, dir -1: src/dst are k-mirrored
                                // views (origin at plane nz+1, py < 0)
    int s27;                    // mode 0 FP64: the 27-point update
};

// Claim groups of a compressed-grid launch (one per XCD).
constexpr int kClaimGroups = 8;

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
// Tile shapes compiled for the 27-point update (FP64, A/B).
bool trip_config_supported_s27(const TripConfig& cfg);

// ---- auxiliary kernels (kernels_aux.hip) ----
hipError_t launch_fill_i32(int* p, int value, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float value, int64_t n, hipStream_t s);

// One problem for the residual / refinement kernels.  u[par]: logical
// (0,0,0) of the FP64 iterate (par = *parity when a parity word is given,
// else 0); e[0..1], rhs: dense FP32 boxes of the refinement (may be null).
struct AuxProblem {
    const double* u[2];
    float* e[2];
    float* rhs;
    int64_t px, py;     // pitches of u
    int64_t epx, epy;   // pitches of e / rhs
    int nx, ny, nz;
    int rtx, rty, rsegs, rseg_len;  // residual tiling (62 x 16 columns x seg)
    int rblocks, rblock_base;       // residual blocks of this problem, prefix
};

// Fills the residual tiling fields of `a` (rtx..rblocks); returns rblocks.
int residual_plan(AuxProblem* a);

// Residual r = fold(nbrs) - 6u on the interior of each problem.
// Pass 1 (k-streaming, one block per 62x16-column tile and k segment) writes
// (sum r^2, max|r|) per block into partials[2*b], partials[2*b+1]; pass 2
// reduces each problem's blocks in fixed order into out[2*q] = ||r||_2,
// out[2*q+1] = max|r|.  `table` (device) with `count` problems, or `table`
// null and the single problem `one` passed by value.  `total_blocks` = sum of
// rblocks.
hipError_t launch_residual_tab(const AuxProblem* table, int count,
                               const AuxProblem& one, const int* parity,
                               int total_blocks, double* partials, double* out,
                               hipStream_t s);

// FP32 refinement helpers, per problem q: rhs_q = fl32(r_q * 2^-s_q) with s_q
// the frexp exponent of out[2q+1] (max |r|), written to scale_exp[q].
hipError_t launch_make_rhs_tab(const AuxProblem* table, int count,
                               const AuxProblem& one, const int* parity,
                               const double* out, int* scale_exp,
                               hipStream_t s);
// u_q(interior) += fl64(e_q[which]) * 2^scale_exp[q]
hipError_t launch_apply_correction_tab(const AuxProblem* table, int count,
                                       const AuxProblem& one,
                                       const int* parity, int which,
                                       const int* scale_exp, hipStream_t s);
// e_q[0] = 0 (whole box) for every problem.
hipError_t launch_zero_e_tab(const AuxProblem* table, int count,
                             const AuxProblem& one, hipStream_t s);
// *word ^= 1 (A/B parity flip between batched trips) and ticket = 0.
hipError_t launch_flip_parity(int* word, int* ticket, hipStream_t s);
hipError_t launch_set_int(int* word, int value, hipStream_t s);

// Box copy between frames of the same logical dims (used to seed the second
// grid and for compressed-layout moves).
hipError_t launch_copy_box_f64(const double* src, int64_t spx, int64_t spy,
                               double* dst, int64_t dpx, int64_t dpy, int nx2,
                               int ny2, int nz2, hipStream_t s);

// Multigrid correction solve (kernels_mg.hip), FP32 dense (n+2)^3 boxes with
// n = 2^k - 1: r = (fold(e nbrs) + rhs) - 6e; coarse rhs = 4 x full
// weighting of r; e += trilinear prolongation of the coarse correction.
hipError_t launch_mg_residual(const float* e, const float* rhs, float* r, int n, hipStream_t s);
hipError_t launch_mg_restrict(const float* r, int n, float* rc, hipStream_t s);
hipError_t launch_mg_prolong_add(const float* ec, float* e, int n, hipStream_t s);

// One FP64 sweep of a small A/B box, one thread per interior cell (the
// boundary layers of both grids already hold the boundary).
hipError_t launch_sweep1_f64(const double* a, double* b, int64_t px, int64_t py, int nx,
                             int ny, int nz, hipStream_t s);
constexpr int64_t kSmallBoxCells = 128 * 128 * 128;

// Bandwidth probes: STREAM-like copy b[i] = a[i] and in-place update
// a[i] += 1.0 (the paper's array-update benchmark).
hipError_t launch_stream_copy(const double* a, double* b, int64_t n,
                              hipStream_t s);
hipError_t launch_stream_update(double* a, int64_t n, hipStream_t s);

}  // namespace jacobi_impl
