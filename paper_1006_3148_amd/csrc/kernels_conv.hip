// Stride-1 3x3x3 convolutions of the learned-guess network (16 -> 16
// channels, zero padding) on v_mfma_f32_16x16x16_bf16, for gfx950.
//
// One workgroup (4 waves) computes a 16 x 16 (x, y) output tile over a run of
// z planes.  It streams the input along z through four LDS plane slots of the
// 18 x 18 halo region: three are read while the fourth is filled from the
// registers the next plane was prefetched into.  The 27 taps' weight
// fragments stay in registers for the whole launch.  Each wave computes four
// output rows of 16 voxels per plane as D[channel][voxel] = sum over taps of
// W_t[channel][c] x[voxel + d_t][c]: 27 MFMAs per row.  The lane layout of
// the 16x16x16 MFMA: lane l supplies A[m = l%16][k = 4(l/16)+j] and
// B[k = 4(l/16)+j][n = l%16] and receives D[m = 4(l/16)+j][n = l%16],
// j = 0..3.  With m the output channel and n the voxel, every lane ends up
// holding four consecutive channels of one voxel: one 8-byte (BF16) or
// 16-byte (FP32) store per row.
//
// LDS plane slot: [channel quarter kq][y][x] 8-byte words (four BF16
// channels).  The 16 lanes of one quarter read 16 consecutive words, so the
// reads are free of bank conflicts.
//
// Forward: input BF16 activations, output BF16 after bias and ReLU, or the
// FP32 accumulator plus bias.  Data gradient: dx[v][ci] = sum over taps t of
// sum_co w[t][co][ci] dy[v - d_t][co].  That is the same stream with the taps
// mirrored and each tap's weights transposed, the FP32 input rounded to BF16
// as it enters LDS, and an FP32 output.  The output is optionally added to
// the existing dx and masked by a ReLU output (mask > 0).

#include <hip/hip_runtime.h>

#include "nn_internal.h"

namespace jacobi_impl {
namespace nn {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kT = 16;            // output tile edge in x and y
constexpr int kH = kT + 2;        // with the one-voxel halo
constexpr int kSlots = 4;
constexpr int kSlotWords = 4 * kH * kH;

// Round to the nearest BF16, ties to even (NaN stays a quiet NaN); branch-free.
__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t q = (u >> 16) | 0x40u;
    return (uint16_t)(((u & 0x7fffffffu) > 0x7f800000u) ? q : r);
}
__device__ __forceinline__ uint64_t pack4(float a, float b, float c, float d)
{
    return (uint64_t)bf16_rne(a) | ((uint64_t)bf16_rne(b) << 16) |
           ((uint64_t)bf16_rne(c) << 32) | ((uint64_t)bf16_rne(d) << 48);
}

// One halo voxel of the next plane, held in registers until it is stored
// into its LDS slot: four words of four BF16 channels (zero outside the
// volume).
template <bool IN_F32>
struct Voxel {
    uint64_t q[4];
};

template <bool IN_F32>
__device__ __forceinline__ void load_voxel(const void* __restrict__ xin, int d, int gx, int gy,
                                           int gz, Voxel<IN_F32>& v)
{
    const bool in = (unsigned)gx < (unsigned)d && (unsigned)gy < (unsigned)d &&
                    (unsigned)gz < (unsigned)d;
    const int64_t vox = in ? (((int64_t)gz * d + gy) * d + gx) : 0;
    if (IN_F32) {
        const float4* p = reinterpret_cast<const float4*>(xin) + vox * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float4 f = in ? p[k] : make_float4(0.f, 0.f, 0.f, 0.f);
            v.q[k] = pack4(f.x, f.y, f.z, f.w);
        }
    } else {
        const uint4* p = reinterpret_cast<const uint4*>(xin) + vox * 2;
        const uint4 a = in ? p[0] : make_uint4(0, 0, 0, 0);
        const uint4 b = in ? p[1] : make_uint4(0, 0, 0, 0);
        v.q[0] = (uint64_t)a.x | ((uint64_t)a.y << 32);
        v.q[1] = (uint64_t)a.z | ((uint64_t)a.w << 32);
        v.q[2] = (uint64_t)b.x | ((uint64_t)b.y << 32);
        v.q[3] = (uint64_t)b.z | ((uint64_t)b.w << 32);
    }
}

// EPI 0: y = bf16(relu(acc + bias)); 1: y = acc + bias (FP32);
// 2: dx = (accum ? dx : 0) + acc, zeroed where mask <= 0 (FP32).
// Three waves per SIMD (three workgroups of 41 KB LDS per CU).
template <bool IN_F32, int EPI, bool FLIP>
__global__ __launch_bounds__(256, 3) void conv3_s1_kernel(
    const void* __restrict__ xin, int d, const uint16_t* __restrict__ w,
    const float* __restrict__ bias, void* __restrict__ yout, int accum,
    const uint16_t* __restrict__ mask, int zseg)
{
    __shared__ __align__(16) uint64_t lds[kSlots][kSlotWords];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int tiles_x = (d + kT - 1) / kT;
    const int x0 = (blockIdx.x % tiles_x) * kT;
    const int y0 = (blockIdx.x / tiles_x) * kT;
    const int z0 = blockIdx.y * zseg;
    const int z1 = min(z0 + zseg, d);
    if (z0 >= d) return;

    // A fragments of the 27 taps: lane (m, kq) holds channels 4kq..4kq+3 of
    // output row m.  Forward: w[t][m][4kq + j].  Data gradient, tap t reads
    // dy at v + d_t, i.e. original tap 26 - t: w[26 - t][4kq + j][m].
    v4s wa[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        if (!FLIP) {
            wa[t] = __builtin_bit_cast(
                v4s, *reinterpret_cast<const uint2*>(w + (t * 16 + m) * 16 + 4 * kq));
        } else {
            const uint16_t* p = w + (26 - t) * 256 + (4 * kq) * 16 + m;
            wa[t][0] = (short)p[0];
            wa[t][1] = (short)p[16];
            wa[t][2] = (short)p[32];
            wa[t][3] = (short)p[48];
        }
    }
    float bq[4] = {0.f, 0.f, 0.f, 0.f};
    if (EPI != 2) {
#pragma unroll
        for (int j = 0; j < 4; ++j) bq[j] = bias[4 * kq + j];
    }

    // halo voxels of a plane handled by this thread: q = tid, tid + 256
    constexpr int kHalo = kH * kH;
    auto stage_load = [&](int gz, Voxel<IN_F32> (&v)[2]) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int q = threadIdx.x + r * 256;
            if (q < kHalo)
                load_voxel<IN_F32>(xin, d, x0 - 1 + q % kH, y0 - 1 + q / kH, gz, v[r]);
        }
    };
    auto stage_store = [&](int slot, const Voxel<IN_F32> (&v)[2]) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int q = threadIdx.x + r * 256;
            if (q < kHalo) {
#pragma unroll
                for (int k = 0; k < 4; ++k) lds[slot][k * kHalo + q] = v[r].q[k];
            }
        }
    };

    {
        Voxel<IN_F32> v[2];
        for (int gz = z0 - 1; gz <= z0 + 1; ++gz) {
            stage_load(gz, v);
            stage_store((gz + 4) & 3, v);
        }
    }
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 2 <= z1;  // plane z+2 feeds output plane z+1
        Voxel<IN_F32> nxt[2];
        if (more) stage_load(z + 2, nxt);
        // The four output rows of this wave at once: every input fragment
        // (x row 4*wave + yo of plane z+dz, shift dx) is read from LDS once
        // and feeds the taps of up to three output rows.  Each row still sums
        // its taps in ascending order.
        v4f acc4[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc4[r] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
            for (int yo = -1; yo <= 4; ++yo) {
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const v4s bv = __builtin_bit_cast(
                        v4s,
                        lds[(z + dz + 4) & 3][(kq * kH + 4 * wave + yo + 1) * kH + m + 1 + dx]);
#pragma unroll
                    for (int dy = 1; dy >= -1; --dy) {
                        const int r = yo - dy;
                        if (r < 0 || r > 3) continue;
                        const int t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                        acc4[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[t], bv, acc4[r],
                                                                             0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int yr = 4 * wave + r;
            const v4f acc = acc4[r];
            const int gx = x0 + m, gy = y0 + yr;
            if (gx < d && gy < d) {
                const int64_t base = ((((int64_t)z * d + gy) * d + gx) << 4) + 4 * kq;
                if (EPI == 0) {
                    const float v0 = fmaxf(acc[0] + bq[0], 0.f), v1 = fmaxf(acc[1] + bq[1], 0.f),
                                v2 = fmaxf(acc[2] + bq[2], 0.f), v3 = fmaxf(acc[3] + bq[3], 0.f);
                    *reinterpret_cast<uint64_t*>(static_cast<uint16_t*>(yout) + base) =
                        pack4(v0, v1, v2, v3);
                } else if (EPI == 1) {
                    *reinterpret_cast<float4*>(static_cast<float*>(yout) + base) =
                        make_float4(acc[0] + bq[0], acc[1] + bq[1], acc[2] + bq[2],
                                    acc[3] + bq[3]);
                } else {
                    float4* o = reinterpret_cast<float4*>(static_cast<float*>(yout) + base);
                    float4 v = make_float4(acc[0], acc[1], acc[2], acc[3]);
                    if (accum) {
                        const float4 old = *o;
                        v.x += old.x;
                        v.y += old.y;
                        v.z += old.z;
                        v.w += old.w;
                    }
                    if (mask) {
                        const uint2 mk = *reinterpret_cast<const uint2*>(mask + base);
                        // bf16 > 0: sign bit clear and not zero
                        if (!((mk.x & 0x8000u) == 0 && (mk.x & 0x7fffu) != 0)) v.x = 0.f;
                        if (!((mk.x >> 31) == 0 && (mk.x & 0x7fff0000u) != 0)) v.y = 0.f;
                        if (!((mk.y & 0x8000u) == 0 && (mk.y & 0x7fffu) != 0)) v.z = 0.f;
                        if (!((mk.y >> 31) == 0 && (mk.y & 0x7fff0000u) != 0)) v.w = 0.f;
                    }
                    *o = v;
                }
            }
        }
        if (more) stage_store((z + 2) & 3, nxt);
        __syncthreads();
    }
}

template <bool IN_F32, int EPI, bool FLIP>
hipError_t launch_s1(const void* x, int d, const uint16_t* w, const float* b, void* y,
                     bool accum, const uint16_t* mask, hipStream_t s)
{
    const int tiles = ((d + kT - 1) / kT) * ((d + kT - 1) / kT);
    // As many z runs as fill the resident workgroups (three per CU) in one
    // round: a launch of 1.33 rounds leaves two thirds of its second round
    // idle.
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    int zsegs = 3 * cus / tiles;
    const int max_segs = (d + 3) / 4;  // runs of at least 4 planes
    if (zsegs > max_segs) zsegs = max_segs;
    if (zsegs < 1) zsegs = 1;
    const int zseg = (d + zsegs - 1) / zsegs;
    zsegs = (d + zseg - 1) / zseg;
    hipLaunchKernelGGL((conv3_s1_kernel<IN_F32, EPI, FLIP>), dim3(tiles, zsegs), dim3(256), 0,
                       s, x, d, w, b, y, accum ? 1 : 0, mask, zseg);
    return hipGetLastError();
}

// ------------------------------------------------------ weight gradient ----
// dW[t][co][ci] = sum_v bf16(dy[v][co]) x[v + d_t][ci] and db[co] = sum_v
// dy[v][co] (FP32, unrounded) over one 16 x 16 x zseg block of voxels, as
// per-block partials.  MFMA D[m = co][n = ci] += A[co][k] B[k][ci] with the
// K index running over 16 voxels of one x-row: A from the plane of dy, B from
// the plane of x shifted by the tap.  Both planes are held in LDS channel-
// major ([c][y][x]), so a lane's four consecutive voxels are one 8-byte
// word; an x shift of one voxel is assembled from two aligned dwords with
// v_alignbit.  Each wave owns four rows of the tile and all 27 taps (27
// accumulators): one x row, read once with its three shifts, feeds the taps
// of up to three dy rows, so LDS delivers about half an operand fragment per
// MFMA instead of two.  The four waves' sums meet in LDS in a fixed order.
constexpr int kDyStride = kT * kT + 8;    // bf16 per channel, padded (banks)
constexpr int kXRow = kT + 8;             // x = -4 .. kT+3 at element x + 4
constexpr int kXPlane = kH * kXRow;       // rows y = -1 .. kT
constexpr int kXStride = kXPlane + 8;     // bf16 per channel, padded

__device__ __forceinline__ v4s words_to_v4s(uint32_t lo, uint32_t hi)
{
    return __builtin_bit_cast(v4s, make_uint2(lo, hi));
}

__global__ __launch_bounds__(256) void conv3_s1_wgrad_kernel(
    const uint16_t* __restrict__ x, const float* __restrict__ dy, int d, int zseg,
    float* __restrict__ part)
{
    __shared__ __align__(16) uint16_t xs[kSlots][16 * kXStride];
    __shared__ __align__(16) uint16_t ys[2][16 * kDyStride];
    // the bias-gradient tree reuses the x planes once the sweep is done
    float(*red)[17] = reinterpret_cast<float(*)[17]>(&xs[0][0]);
    static_assert(sizeof(float) * 256 * 17 <= sizeof(uint16_t) * kSlots * 16 * kXStride,
                  "reduction buffer must fit in the x planes");
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int tiles_x = (d + kT - 1) / kT;
    const int x0 = (blockIdx.x % tiles_x) * kT;
    const int y0 = (blockIdx.x / tiles_x) * kT;
    const int z0 = blockIdx.y * zseg;
    const int z1 = min(z0 + zseg, d);
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;

    // x pad columns are read (and discarded) by the shifted fragments: zero them
    for (int q = threadIdx.x; q < kSlots * 16 * kXStride; q += 256)
        (&xs[0][0])[q] = 0;

    v4f acc[27];
#pragma unroll
    for (int u = 0; u < 27; ++u) acc[u] = (v4f){0.f, 0.f, 0.f, 0.f};
    float dbs[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) dbs[c] = 0.f;

    // staging of one x plane (324 halo voxels, two per thread) and one dy
    // plane (256 voxels, one per thread) through registers
    uint4 xv[2][2];
    float4 yv[4];
    auto load_x = [&](int gz) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int q = threadIdx.x + r * 256;
            const int gx = x0 - 1 + q % kH, gy = y0 - 1 + q / kH;
            const bool in = q < kH * kH && (unsigned)gx < (unsigned)d &&
                            (unsigned)gy < (unsigned)d && (unsigned)gz < (unsigned)d;
            const uint4* p = reinterpret_cast<const uint4*>(x) +
                             (in ? (((int64_t)gz * d + gy) * d + gx) * 2 : 0);
            xv[r][0] = in ? p[0] : make_uint4(0, 0, 0, 0);
            xv[r][1] = in ? p[1] : make_uint4(0, 0, 0, 0);
        }
    };
    auto store_x = [&](int slot) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int q = threadIdx.x + r * 256;
            if (q < kH * kH) {
                const int e = (q / kH) * kXRow + (q % kH) + 3;  // x + 4 with x = q%kH - 1
                const uint32_t wds[8] = {xv[r][0].x, xv[r][0].y, xv[r][0].z, xv[r][0].w,
                                         xv[r][1].x, xv[r][1].y, xv[r][1].z, xv[r][1].w};
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    xs[slot][c * kXStride + e] =
                        (uint16_t)((c & 1) ? (wds[c >> 1] >> 16) : (wds[c >> 1] & 0xffff));
            }
        }
    };
    auto load_dy = [&](int gz) {
        const int gx = x0 + (threadIdx.x & 15), gy = y0 + (threadIdx.x >> 4);
        const bool in = (unsigned)gx < (unsigned)d && (unsigned)gy < (unsigned)d &&
                        (unsigned)gz < (unsigned)d;
        const float4* p = reinterpret_cast<const float4*>(dy) +
                          (in ? (((int64_t)gz * d + gy) * d + gx) * 4 : 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) yv[k] = in ? p[k] : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto store_dy = [&](int slot) {
        const int e = threadIdx.x;  // y * 16 + x
        const float f[16] = {yv[0].x, yv[0].y, yv[0].z, yv[0].w, yv[1].x, yv[1].y,
                             yv[1].z, yv[1].w, yv[2].x, yv[2].y, yv[2].z, yv[2].w,
                             yv[3].x, yv[3].y, yv[3].z, yv[3].w};
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            dbs[c] += f[c];
            ys[slot][c * kDyStride + e] = bf16_rne(f[c]);
        }
    };

    __syncthreads();  // pad zeroing before the first plane stores
    load_x(z0 - 1);
    store_x((z0 + 3) & 3);
    load_x(z0);
    store_x(z0 & 3);
    load_x(z0 + 1);
    store_x((z0 + 1) & 3);
    load_dy(z0);
    store_dy(z0 & 1);
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 1 < z1;
        if (more) {
            load_x(z + 2);
            load_dy(z + 1);
        }
        const uint16_t* yb = ys[z & 1];
        // dy rows 4*wave + r of this plane
        v4s A[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint2 aw = *reinterpret_cast<const uint2*>(yb + m * kDyStride +
                                                             (4 * wave + r) * kT + 4 * kq);
            A[r] = words_to_v4s(aw.x, aw.y);
        }
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
            const uint16_t* plane = xs[(z + dz + 4) & 3] + m * kXStride + 4 * kq + 4;
#pragma unroll
            for (int yo = -1; yo <= 4; ++yo) {
                // x row 4*wave + yo at shifts dx = -1, 0, +1
                const uint16_t* row = plane + (4 * wave + yo + 1) * kXRow;
                const uint32_t d0 = *reinterpret_cast<const uint32_t*>(row - 2);
                const uint2 w2 = *reinterpret_cast<const uint2*>(row);
                const uint32_t d3 = *reinterpret_cast<const uint32_t*>(row + 4);
                const v4s bm = words_to_v4s(__builtin_amdgcn_alignbit(w2.x, d0, 16),
                                            __builtin_amdgcn_alignbit(w2.y, w2.x, 16));
                const v4s b0 = words_to_v4s(w2.x, w2.y);
                const v4s bp = words_to_v4s(__builtin_amdgcn_alignbit(w2.y, w2.x, 16),
                                            __builtin_amdgcn_alignbit(d3, w2.y, 16));
#pragma unroll
                for (int dyy = -1; dyy <= 1; ++dyy) {
                    const int r = yo - dyy;  // dy row 4*wave + r meets x row 4*wave + r + dyy
                    if (r < 0 || r > 3) continue;
                    const int tb = (dz + 1) * 9 + (dyy + 1) * 3;
                    acc[tb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[r], bm, acc[tb], 0, 0, 0);
                    acc[tb + 1] =
                        __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[r], b0, acc[tb + 1], 0, 0, 0);
                    acc[tb + 2] =
                        __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[r], bp, acc[tb + 2], 0, 0, 0);
                }
            }
        }
        if (more) {
            store_x((z + 2) & 3);
            store_dy((z + 1) & 1);
        }
        __syncthreads();
    }

    // Partials D[m = co = 4kq + j][n = ci = m] of tap u, summed over the
    // waves as (w0 + w2) + (w1 + w3) through two LDS copies (the x planes are
    // no longer needed: the plane loop ended with a barrier).
    constexpr int kTapW = 27 * 256;
    float* sum2 = reinterpret_cast<float*>(&xs[0][0]);
    static_assert(2 * kTapW * sizeof(float) <= sizeof(uint16_t) * kSlots * 16 * kXStride,
                  "the wave sums must fit in the x planes");
    if (wave < 2) {
#pragma unroll
        for (int u = 0; u < 27; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                sum2[wave * kTapW + u * 256 + (4 * kq + j) * 16 + m] = acc[u][j];
    }
    __syncthreads();
    if (wave >= 2) {
#pragma unroll
        for (int u = 0; u < 27; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                sum2[(wave - 2) * kTapW + u * 256 + (4 * kq + j) * 16 + m] += acc[u][j];
    }
    __syncthreads();
    float* out = part + (int64_t)blk * kConvP;
    for (int q = threadIdx.x; q < kTapW; q += 256) out[q] = sum2[q] + sum2[kTapW + q];
    __syncthreads();  // the bias tree below reuses the same LDS
    // bias gradient: fixed-order tree over the 256 threads
#pragma unroll
    for (int c = 0; c < 16; ++c) red[threadIdx.x][c] = dbs[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < 16; ++c) red[threadIdx.x][c] += red[threadIdx.x + w][c];
        }
        __syncthreads();
    }
    if (threadIdx.x < 16) out[kConvW + threadIdx.x] = red[0][threadIdx.x];
}

// --------------------------------------------- stride-2 weight gradient ----
// dW[t][co][ci] = sum_o bf16(dy[o][co]) x[2o + d_t][ci] and db[co] = sum_o
// dy[o][co] over a 16 x 4 x zseg block of output voxels o, as per-block
// partials.  MFMA K runs over the 16 voxels of an output row.  An input row
// is held in LDS split by x parity (per channel: even columns 2j at element
// j - ox0, odd columns 2j+1 at element 24 + j - ox0, j = ox0-1 .. ox0+15), so
// the taps dx = 0 and +1 read aligned words and dx = -1 shifts the odd half by
// one element with v_alignbit.  Each wave owns one output row and all 27 taps.
constexpr int kS2Rows = 4;                   // output rows per block (one per wave)
constexpr int kS2InRows = 2 * kS2Rows + 1;   // input rows 2*oy0-1 .. 2*oy0+7
constexpr int kS2Row = 40;                   // elements per input row and channel
constexpr int kS2Chan = kS2InRows * kS2Row + 8;  // per channel, padded
constexpr int kS2DyChan = kS2Rows * kT + 8;

__global__ __launch_bounds__(256) void conv3_s2_wgrad_kernel(
    const uint16_t* __restrict__ x, int din, const float* __restrict__ dy, int dout, int zseg,
    float* __restrict__ part)
{
    __shared__ __align__(16) uint16_t xs[4][16 * kS2Chan];
    __shared__ __align__(16) uint16_t ys[16 * kS2DyChan];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int tiles_x = (dout + kT - 1) / kT;
    const int ox0 = (blockIdx.x % tiles_x) * kT;
    const int oy0 = (blockIdx.x / tiles_x) * kS2Rows;
    const int z0 = blockIdx.y * zseg;
    const int z1 = min(z0 + zseg, dout);
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;

    // the pad elements are read (and discarded) by the shifted fragments
    for (int q = threadIdx.x; q < 4 * 16 * kS2Chan; q += 256) (&xs[0][0])[q] = 0;

    v4f acc[27];
#pragma unroll
    for (int u = 0; u < 27; ++u) acc[u] = (v4f){0.f, 0.f, 0.f, 0.f};
    float dbs[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) dbs[c] = 0.f;

    // one input plane iz into slot: 9 rows x 33 columns (2*ox0-1 .. 2*ox0+31)
    auto stage_x = [&](int iz, int slot) {
        constexpr int kCols = 2 * kT + 1;
        for (int q = threadIdx.x; q < kS2InRows * kCols; q += 256) {
            const int r = q / kCols, cx = q % kCols;
            const int ix = 2 * ox0 - 1 + cx, iy = 2 * oy0 - 1 + r;
            const bool in = (unsigned)ix < (unsigned)din && (unsigned)iy < (unsigned)din &&
                            (unsigned)iz < (unsigned)din;
            const uint4* p = reinterpret_cast<const uint4*>(x) +
                             (in ? (((int64_t)iz * din + iy) * din + ix) * 2 : 0);
            const uint4 a = in ? p[0] : make_uint4(0, 0, 0, 0);
            const uint4 b = in ? p[1] : make_uint4(0, 0, 0, 0);
            const uint32_t wds[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
            // cx odd: even column 2j at j - ox0 = (cx - 1) / 2; cx even: odd
            // column 2j + 1 at 24 + j - ox0 = 23 + cx / 2
            const int e = r * kS2Row + ((cx & 1) ? (cx - 1) / 2 : 23 + cx / 2);
#pragma unroll
            for (int c = 0; c < 16; ++c)
                xs[slot][c * kS2Chan + e] =
                    (uint16_t)((c & 1) ? (wds[c >> 1] >> 16) : (wds[c >> 1] & 0xffff));
        }
    };
    // the dy rows of output plane oz (bias sums from the FP32 values)
    auto stage_dy = [&](int oz) {
        if (threadIdx.x < kS2Rows * kT) {
            const int r = threadIdx.x / kT, cx = threadIdx.x % kT;
            const int ox = ox0 + cx, oy = oy0 + r;
            const bool in = ox < dout && oy < dout;
            const float4* p = reinterpret_cast<const float4*>(dy) +
                              (in ? (((int64_t)oz * dout + oy) * dout + ox) * 4 : 0);
            float f[16];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float4 v = in ? p[k] : make_float4(0.f, 0.f, 0.f, 0.f);
                f[4 * k] = v.x;
                f[4 * k + 1] = v.y;
                f[4 * k + 2] = v.z;
                f[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                dbs[c] += f[c];
                ys[c * kS2DyChan + r * kT + cx] = bf16_rne(f[c]);
            }
        }
    };

    __syncthreads();  // pad zeroing before the first stores
    stage_x(2 * z0 - 1, (2 * z0 - 1 + 8) & 3);
    for (int oz = z0; oz < z1; ++oz) {
        stage_x(2 * oz, (2 * oz + 8) & 3);
        stage_x(2 * oz + 1, (2 * oz + 1 + 8) & 3);
        stage_dy(oz);
        __syncthreads();
        const uint2 aw =
            *reinterpret_cast<const uint2*>(ys + m * kS2DyChan + wave * kT + 4 * kq);
        const v4s A = words_to_v4s(aw.x, aw.y);
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
            const uint16_t* plane = xs[(2 * oz + dz + 8) & 3] + m * kS2Chan;
#pragma unroll
            for (int dyy = -1; dyy <= 1; ++dyy) {
                const uint16_t* row = plane + (2 * wave + 1 + dyy) * kS2Row;
                const uint2 ev = *reinterpret_cast<const uint2*>(row + 4 * kq);
                const uint2 od = *reinterpret_cast<const uint2*>(row + 24 + 4 * kq);
                const uint32_t d0 = *reinterpret_cast<const uint32_t*>(row + 22 + 4 * kq);
                const v4s bm = words_to_v4s(__builtin_amdgcn_alignbit(od.x, d0, 16),
                                            __builtin_amdgcn_alignbit(od.y, od.x, 16));
                const v4s b0 = words_to_v4s(ev.x, ev.y);
                const v4s bp = words_to_v4s(od.x, od.y);
                const int tb = (dz + 1) * 9 + (dyy + 1) * 3;
                acc[tb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, bm, acc[tb], 0, 0, 0);
                acc[tb + 1] =
                    __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, b0, acc[tb + 1], 0, 0, 0);
                acc[tb + 2] =
                    __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, bp, acc[tb + 2], 0, 0, 0);
            }
        }
        __syncthreads();  // the slots of planes 2oz-1 and 2oz are refilled next
    }

    // wave sums (w0 + w2) + (w1 + w3) through LDS, taps 0..13 then 14..26
    // (the two copies of all 27 would not fit in the x slots), then the bias
    // tree
    constexpr int kHalfW = 14 * 256;
    float* sum2 = reinterpret_cast<float*>(&xs[0][0]);
    static_assert(2 * kHalfW * sizeof(float) <= sizeof(uint16_t) * 4 * 16 * kS2Chan,
                  "the wave sums must fit in the x slots");
    float* out = part + (int64_t)blk * kConvP;
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        const int u0 = 14 * hf, nu = hf ? 13 : 14;
        if (wave < 2) {
#pragma unroll
            for (int u = 0; u < 27; ++u)
                if (u / 14 == hf)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        sum2[wave * kHalfW + (u - u0) * 256 + (4 * kq + j) * 16 + m] = acc[u][j];
        }
        __syncthreads();
        if (wave >= 2) {
#pragma unroll
            for (int u = 0; u < 27; ++u)
                if (u / 14 == hf)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        sum2[(wave - 2) * kHalfW + (u - u0) * 256 + (4 * kq + j) * 16 + m] +=
                            acc[u][j];
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nu * 256; q += 256)
            out[u0 * 256 + q] = sum2[q] + sum2[kHalfW + q];
        __syncthreads();
    }
    float(*red)[17] = reinterpret_cast<float(*)[17]>(&xs[0][0]);
#pragma unroll
    for (int c = 0; c < 16; ++c) red[threadIdx.x][c] = dbs[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < 16; ++c) red[threadIdx.x][c] += red[threadIdx.x + w][c];
        }
        __syncthreads();
    }
    if (threadIdx.x < 16) out[kConvW + threadIdx.x] = red[0][threadIdx.x];
}

}  // namespace

hipError_t conv_fwd_s1(const uint16_t* x, int d, const uint16_t* w, const float* b,
                       uint16_t* y, hipStream_t s)
{
    return launch_s1<false, 0, false>(x, d, w, b, y, false, nullptr, s);
}

hipError_t conv_fwd_s1_f32(const uint16_t* x, int d, const uint16_t* w, const float* b,
                           float* y, hipStream_t s)
{
    return launch_s1<false, 1, false>(x, d, w, b, y, false, nullptr, s);
}

hipError_t conv_bwd_data_s1(const float* dy, int d, const uint16_t* w, float* dx, bool accum,
                            const uint16_t* mask, hipStream_t s)
{
    return launch_s1<true, 2, true>(dy, d, w, nullptr, dx, accum, mask, s);
}

// Blocks of the stride-1 weight-gradient launch for edge d (0 when the
// 16 x 16 tiles of one plane alone exceed kMaxWgradBlocks).
int wgrad_s1_blocks(int d, int* zseg_out)
{
    const int tiles = ((d + kT - 1) / kT) * ((d + kT - 1) / kT);
    if (tiles > kMaxWgradBlocks) return 0;
    int zsegs = kMaxWgradBlocks / tiles;
    const int max_segs = (d + 3) / 4;
    if (zsegs > max_segs) zsegs = max_segs;
    if (zsegs < 1) zsegs = 1;
    const int zseg = (d + zsegs - 1) / zsegs;
    if (zseg_out) *zseg_out = zseg;
    return tiles * ((d + zseg - 1) / zseg);
}

hipError_t conv_bwd_weight_s1(const uint16_t* x, const float* dy, int d, float* part,
                              float* grad_w_b, hipStream_t s)
{
    int zseg = 1;
    const int blocks = wgrad_s1_blocks(d, &zseg);
    const int tiles = ((d + kT - 1) / kT) * ((d + kT - 1) / kT);
    hipLaunchKernelGGL(conv3_s1_wgrad_kernel, dim3(tiles, blocks / tiles), dim3(256), 0, s, x,
                       dy, d, zseg, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_partials(part, blocks, grad_w_b, s);
}

}  // namespace nn
}  // namespace jacobi_impl

namespace jacobi_impl {
namespace nn {

// Blocks of the stride-2 weight-gradient launch for output edge dout (0 when
// one plane's tiles alone exceed kMaxWgradBlocks).
int wgrad_s2_blocks(int dout, int* zseg_out)
{
    const int tiles = ((dout + kT - 1) / kT) * ((dout + kS2Rows - 1) / kS2Rows);
    if (tiles > kMaxWgradBlocks) return 0;
    int zsegs = kMaxWgradBlocks / tiles;
    if (zsegs > dout) zsegs = dout;
    if (zsegs < 1) zsegs = 1;
    const int zseg = (dout + zsegs - 1) / zsegs;
    if (zseg_out) *zseg_out = zseg;
    return tiles * ((dout + zseg - 1) / zseg);
}

hipError_t conv_bwd_weight_s2(const uint16_t* x, int din, const float* dy, int dout,
                              float* part, float* grad_w_b, hipStream_t s)
{
    int zseg = 1;
    const int blocks = wgrad_s2_blocks(dout, &zseg);
    const int tiles = ((dout + kT - 1) / kT) * ((dout + kS2Rows - 1) / kS2Rows);
    hipLaunchKernelGGL(conv3_s2_wgrad_kernel, dim3(tiles, blocks / tiles), dim3(256), 0, s, x,
                       din, dy, dout, zseg, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_partials(part, blocks, grad_w_b, s);
}

}  // namespace nn
}  // namespace jacobi_impl
