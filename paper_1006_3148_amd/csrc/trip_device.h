// Device helpers of the trip kernel (kernels_trip.hip): constants, DPP lane
// shifts, the XCD-aware tile map, progress-word access and raw buffer loads
// and stores.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace jacobi_impl {
namespace {

template <typename Real>
struct Sixth;
template <>
struct Sixth<double> {
    static constexpr double v = 1.0 / 6.0;
};
template <>
struct Sixth<float> {
    static constexpr float v = 1.0f / 6.0f;
};

// DPP wave shifts (GFX9 family): wave_shr:1 gives lane L the value of lane
// L-1, wave_shl:1 the value of lane L+1.  Lanes without a source read 0
// (bound_ctrl).
__device__ __forceinline__ int lane_from_left(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ int lane_from_right(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ float from_left(float v)
{
    return __int_as_float(lane_from_left(__float_as_int(v)));
}
__device__ __forceinline__ float from_right(float v)
{
    return __int_as_float(lane_from_right(__float_as_int(v)));
}
__device__ __forceinline__ double from_left(double v)
{
    int lo = lane_from_left(__double2loint(v));
    int hi = lane_from_left(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v)
{
    int lo = lane_from_right(__double2loint(v));
    int hi = lane_from_right(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Workgroup b is dispatched to XCD b % 8.  Give each XCD a contiguous range
// of the tile order so that tiles sharing ghost cells share an L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    const int x = b & 7, idx = b >> 3;
    const int q = ntiles >> 3, r = ntiles & 7;
    return x * q + min(x, r) + idx;
}

// Band order of a multi-generation A/B launch: the first bands*256 workgroups
// run generation g = idx / 32 of XCD x = b % 8 (idx = b / 8) on tiles
// g*256 + x*32 + idx % 32, so each generation covers 256 consecutive tiles,
// 32 per XCD; the tail (a partial generation) is split into eight contiguous
// ranges like xcd_tile.
__device__ __forceinline__ int band_tile(int b, int ntiles)
{
    const int full = (ntiles >> 8) << 8;
    if (b >= full) return full + xcd_tile(b - full, ntiles - full);
    const int x = b & 7, idx = b >> 3;
    return ((idx >> 5) << 8) + (x << 5) + (idx & 31);
}

__device__ __forceinline__ int flag_load(const int* f)
{
    return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_store(int* f, int v)
{
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kDone = 0x7fffffff;

// Tile claim of the compressed-grid launch with per-XCD groups.  The tile
// order O of a forward trip (row-major: segment, row, column; a backward trip
// mirrors the index) is cut into chunks of `chunk` consecutive tiles (the
// workgroups one XCD holds), and chunk c belongs to group c mod 8: at any time
// the eight XCDs work on eight consecutive chunks, each on a run of whole tile
// rows as in the A/B map, so the ghost cells of neighbouring tiles are shared
// in that XCD's L2 and the memory streams stay row-long.  A workgroup on XCD
// x (workgroup b is dispatched to XCD b mod 8) takes the next tile of group x
// with one atomic add.  Every tile waits only for tiles earlier in O; a group
// hands out its tiles in O order, so the earliest unfinished tile is claimed
// as soon as a workgroup of its group is free, and its dependees are done:
// the launch completes once every group has a workgroup resident.  When
// every tile is resident at once (chunk = 0; one workgroup per tile), group
// x is instead the x-th of eight near-equal ranges, sized like the
// workgroups on XCD x: chunks of grid/8 would leave the remainder tiles to
// one group, whose trip then takes two tile times.  Returns the tile in O
// numbering, or ntiles when the group is exhausted.
__device__ __forceinline__ int claim_grouped(int* gcnt, int xcd, int chunk, int ntiles)
{
    const int k = atomicAdd(gcnt + xcd * kFlagStride, 1);
    if (chunk == 0) {
        const int q = ntiles >> 3, r = ntiles & 7;
        return k < q + (xcd < r ? 1 : 0) ? xcd * q + min(xcd, r) + k : ntiles;
    }
    const int64_t v = ((int64_t)(k / chunk) * kClaimGroups + xcd) * chunk + k % chunk;
    return v < ntiles ? (int)v : ntiles;
}

// Planes in flight per tile (register ring depth).
#ifndef JACOBI_PREFETCH
#define JACOBI_PREFETCH 2
#endif
constexpr int kPrefetch = JACOBI_PREFETCH;

// Raw buffer accesses (GFX9 buffer resource, stride 0, 32-bit data format).
// An access whose byte offset is at or past the descriptor's record count is
// dropped by the hardware: a load returns 0 and a store writes nothing.  Plane
// loads and stores therefore need no branches, and the compiler can count
// outstanding memory operations exactly (a branch around a load makes it
// wait for all of them).
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;
constexpr uint32_t kOob = 0xFFFF0000u;  // past every plane descriptor's range

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                             (int)bytes, kRsrcWord3);
}
template <typename Real>
__device__ __forceinline__ Real buf_load(Rsrc r, uint32_t off);
template <>
__device__ __forceinline__ double buf_load<double>(Rsrc r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(Rsrc r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store(double v, Rsrc r, uint32_t off)
{
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(float v, Rsrc r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}

// Geometry and pointers of the problem a tile belongs to.
struct Geo {
    const void* src;
    void* dst;
    const float* rhs;
    int64_t px, py, rpx, rpy;
    int nx, ny, nz;
    int tiles_x, tiles_y, segs, seg_len;
};

}  // namespace
}  // namespace jacobi_impl
