// Kernels of the learned initial guess (a small 3D U-Net) for gfx950.
//
// The guess only supplies the starting field of the Jacobi method (Sect. 1.1
// of the paper); the paper itself starts from a fixed field.  Numerics: BF16
// weights and activations, FP32 accumulation on MFMA, FP32 gradients.
//
// Layouts: activations [D][H][W][16] bfloat16 (channel last, 32 B per voxel);
// activation gradients [D][H][W][16] float; conv weights [27][Cout][Cin]
// bfloat16 with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) and a transposed copy
// [27][Cin][Cout] for the data gradient.
//
// 3x3x3 convolutions are implicit GEMMs on v_mfma_f32_16x16x16_bf16: one wave
// computes a 16 (voxels along x) x 16 (channels) output tile and accumulates
// 27 taps x 16 input channels.  Operand lane layout of the 16x16x16 MFMA: lane
// l holds A[m = l%16][k = 4(l/16) .. 4(l/16)+3], B[k = 4(l/16)..+3][n = l%16]
// and receives D[m = 4(l/16)+i][n = l%16], i = 0..3.

#include <hip/hip_runtime.h>

#include "internal.h"
#include "nn_internal.h"

namespace jacobi_impl {
namespace nn {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}

__device__ __forceinline__ v4s load4bf(const uint16_t* p)
{
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    v4s r;
    r[0] = (short)(v.x & 0xffff);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xffff);
    r[3] = (short)(v.y >> 16);
    return r;
}
__device__ __forceinline__ v4s f4_to_bf(const float* p)
{
    const float4 v = *reinterpret_cast<const float4*>(p);
    v4s r;
    r[0] = (short)f2bf(v.x);
    r[1] = (short)f2bf(v.y);
    r[2] = (short)f2bf(v.z);
    r[3] = (short)f2bf(v.w);
    return r;
}

__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- lift ----
// x[k][j][i][c] for the interior of an (n+2)^3 FP64 box: six face values,
// three centred coordinates, the inverse-distance blend of the six face
// values (also written to blend[v] in FP32: the network output is blend +
// head), zeros.
__global__ __launch_bounds__(256) void lift_kernel(const double* __restrict__ box,
                                                   int n, uint16_t* __restrict__ x,
                                                   float* __restrict__ blend)
{
    const int64_t nv = (int64_t)n * n * n;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int i = (int)(v % n), j = (int)((v / n) % n), k = (int)(v / ((int64_t)n * n));
    const int64_t p = n + 2, pp = p * p;
    const int64_t kk = k + 1, jj = j + 1, ii = i + 1;
    double g[6];
    g[0] = box[kk * pp + jj * p + 0];
    g[1] = box[kk * pp + jj * p + (n + 1)];
    g[2] = box[kk * pp + 0 * p + ii];
    g[3] = box[kk * pp + (int64_t)(n + 1) * p + ii];
    g[4] = box[0 * pp + jj * p + ii];
    g[5] = box[(int64_t)(n + 1) * pp + jj * p + ii];
    const double w[6] = {1.0 / (i + 1), 1.0 / (n - i), 1.0 / (j + 1),
                         1.0 / (n - j), 1.0 / (k + 1), 1.0 / (n - k)};
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        num = num + g[f] * w[f];
        den = den + w[f];
    }
    const double b = num / den;
    float c[16];
#pragma unroll
    for (int f = 0; f < 6; ++f) c[f] = (float)g[f];
    c[6] = (float)((double)(i + 1) / (n + 1) - 0.5);
    c[7] = (float)((double)(j + 1) / (n + 1) - 0.5);
    c[8] = (float)((double)(k + 1) / (n + 1) - 0.5);
    c[9] = (float)b;
#pragma unroll
    for (int q = 10; q < 16; ++q) c[q] = 0.f;
    blend[v] = (float)b;
    uint32_t wd[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        wd[q] = (uint32_t)f2bf(c[2 * q]) | ((uint32_t)f2bf(c[2 * q + 1]) << 16);
    uint4* dst = reinterpret_cast<uint4*>(x + v * 16);
    dst[0] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
    dst[1] = make_uint4(wd[4], wd[5], wd[6], wd[7]);
}

// ------------------------------------------------------ conv forward ----
// y[o] = relu?(b + sum_t W_t x[S*o + d_t]); input D^3 (Din), output Dout^3.
// OUTF32: y is FP32 (accumulator + bias, no ReLU, no BF16 rounding).
template <int S, bool RELU, bool OUTF32 = false>
__global__ __launch_bounds__(256) void conv_fwd_kernel(
    const uint16_t* __restrict__ x, int din, const uint16_t* __restrict__ w,
    const float* __restrict__ bias, void* __restrict__ yv, int dout)
{
    const int lane = threadIdx.x & 63;
    const int wid = (blockIdx.x * (blockDim.x >> 6)) + (threadIdx.x >> 6);
    const int xt = (dout + 15) >> 4;
    const int64_t ntile = (int64_t)dout * dout * xt;
    if (wid >= ntile) return;
    const int ox0 = (wid % xt) * 16;
    const int oy = (wid / xt) % dout;
    const int oz = wid / (xt * dout);
    const int m = lane & 15, kq = lane >> 4;
    const int ox = ox0 + m;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const int iz = S * oz + dz, iy = S * oy + dy, ix = S * ox + dx;
        v4s a = {0, 0, 0, 0};
        if (ox < dout && (unsigned)iz < (unsigned)din && (unsigned)iy < (unsigned)din &&
            (unsigned)ix < (unsigned)din)
            a = load4bf(x + (((int64_t)iz * din + iy) * din + ix) * 16 + 4 * kq);
        const v4s bw = load4bf(w + ((int64_t)t * 16 + m) * 16 + 4 * kq);
        acc = mfma16(a, bw, acc);
    }
    const int n = lane & 15;
    const float bn = bias[n];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int vx = ox0 + 4 * kq + r;
        if (vx >= dout) continue;
        float v = acc[r] + bn;
        if (RELU) v = fmaxf(v, 0.f);
        const int64_t idx = (((int64_t)oz * dout + oy) * dout + vx) * 16 + n;
        if (OUTF32)
            static_cast<float*>(yv)[idx] = v;
        else
            static_cast<uint16_t*>(yv)[idx] = f2bf(v);
    }
}

// ---------------------------------------------------- conv data grad ----
// dx[v] (+)= sum_t W_t^T dy[(v - d_t)/S] over the taps with an integral
// in-range source; then dx *= (mask[v] > 0) if a mask (the ReLU output that
// produced this conv's input) is given.  wt: [27][Cin][Cout].  Stride 1 runs
// in conv3_s1_kernel (kernels_conv.hip).
// Stride 2: dx[v] receives tap t only where v - d_t is even in every axis,
// i.e. 1, 2, 4 or 8 taps by the parity class of v.  A wave takes 16 voxels of
// one class along x (x = 2j + px, j = j0..j0+15, fixed y and z), so it runs
// only its class's taps (27/8 on average instead of 27; the others added
// exact zeros) and its dy sources are 16 consecutive voxels.
__global__ __launch_bounds__(256) void conv_bwd_data_s2_kernel(
    const float* __restrict__ dy, int dout, const uint16_t* __restrict__ wt,
    float* __restrict__ dx, int din, int accum, const uint16_t* __restrict__ mask)
{
    const int lane = threadIdx.x & 63;
    const int wid = (blockIdx.x * (blockDim.x >> 6)) + (threadIdx.x >> 6);
    const int half = (din + 1) >> 1;   // j values per parity
    const int jt = (half + 15) >> 4;   // 16-voxel runs per (row, parity)
    const int64_t nw = (int64_t)din * din * 2 * jt;
    if (wid >= nw) return;
    const int j0 = (wid % jt) * 16;
    const int px = (wid / jt) & 1;
    const int vy = (wid / (2 * jt)) % din;
    const int vz = (int)(wid / (2 * (int64_t)jt * din));
    const int m = lane & 15, kq = lane >> 4;
    const int vx = 2 * (j0 + m) + px;  // this lane's voxel (A row m)
    const int pz = vz & 1, py = vy & 1;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    // taps in ascending order: d in {0} for an even coordinate, {-1, +1} for an odd one
    for (int dz = pz ? -1 : 0; dz <= (pz ? 1 : 0); dz += 2) {
        const int oz = (vz - dz) >> 1;
        if ((unsigned)oz >= (unsigned)dout) continue;
        for (int dyy = py ? -1 : 0; dyy <= (py ? 1 : 0); dyy += 2) {
            const int oy = (vy - dyy) >> 1;
            if ((unsigned)oy >= (unsigned)dout) continue;
            for (int dx_ = px ? -1 : 0; dx_ <= (px ? 1 : 0); dx_ += 2) {
                const int t = (dz + 1) * 9 + (dyy + 1) * 3 + dx_ + 1;
                const int ox = (vx - dx_) >> 1;
                const bool ok = vx < din && (unsigned)ox < (unsigned)dout;
                v4s a = {0, 0, 0, 0};
                if (ok) a = f4_to_bf(dy + (((int64_t)oz * dout + oy) * dout + ox) * 16 + 4 * kq);
                const v4s bw = load4bf(wt + ((int64_t)t * 16 + m) * 16 + 4 * kq);
                acc = mfma16(a, bw, acc);
            }
        }
    }
    const int n = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int x = 2 * (j0 + 4 * kq + r) + px;
        if (x >= din) continue;
        const int64_t idx = (((int64_t)vz * din + vy) * din + x) * 16 + n;
        float v = acc[r];
        if (accum) v += dx[idx];
        if (mask && !(bf2f(mask[idx]) > 0.f)) v = 0.f;
        dx[idx] = v;
    }
}

// -------------------------------------------------- conv weight grad ----
// Per block: partial dw[t][co][ci] = sum over its output voxels o of
// dy[o][co] * x[S*o + d_t][ci], and partial db[co] = sum dy[o][co].
// Voxels are taken 16 at a time by each wave (the K dimension of the MFMA).
template <int S>
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(
    const uint16_t* __restrict__ x, int din, const float* __restrict__ dy,
    int dout, float* __restrict__ part, int chunks_per_wave)
{
    __shared__ float red[4][27 * 256 + 16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int64_t nvox = (int64_t)dout * dout * dout;
    const int64_t nchunk = (nvox + 15) / 16;
    v4f acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
    float dbs = 0.f;
    const int64_t first = ((int64_t)blockIdx.x * 4 + wave) * chunks_per_wave;
    for (int c = 0; c < chunks_per_wave; ++c) {
        const int64_t ch = first + c;
        if (ch >= nchunk) break;
        // A[m = co][k = voxel 4kq..4kq+3] = dy[voxel][co]
        int oz[4], oy[4], ox[4];
        bool ov[4];
        v4s a;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t o = ch * 16 + 4 * kq + r;
            ov[r] = o < nvox;
            const int64_t oc = ov[r] ? o : 0;
            ox[r] = (int)(oc % dout);
            oy[r] = (int)((oc / dout) % dout);
            oz[r] = (int)(oc / ((int64_t)dout * dout));
            const float g = ov[r] ? dy[oc * 16 + m] : 0.f;
            dbs += g;
            a[r] = (short)f2bf(g);
        }
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int dz = t / 9 - 1, dyy = (t / 3) % 3 - 1, dx_ = t % 3 - 1;
            v4s b;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int iz = S * oz[r] + dz, iy = S * oy[r] + dyy, ix = S * ox[r] + dx_;
                uint16_t v = 0;
                if (ov[r] && (unsigned)iz < (unsigned)din && (unsigned)iy < (unsigned)din &&
                    (unsigned)ix < (unsigned)din)
                    v = x[(((int64_t)iz * din + iy) * din + ix) * 16 + m];
                b[r] = (short)v;
            }
            acc[t] = mfma16(a, b, acc[t]);
        }
    }
    // D[m = co 4kq+r][n = ci lane%16] -> red[wave][t*256 + co*16 + ci]
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave][t * 256 + (4 * kq + r) * 16 + m] = acc[t][r];
    // db: lanes with the same m (co) hold partial sums; reduce over kq
    dbs += __shfl_xor(dbs, 16, 64);
    dbs += __shfl_xor(dbs, 32, 64);
    if (lane < 16) red[wave][27 * 256 + lane] = dbs;
    __syncthreads();
    for (int q = threadIdx.x; q < 27 * 256 + 16; q += blockDim.x)
        part[(int64_t)blockIdx.x * (27 * 256 + 16) + q] =
            ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
}

// Sum of per-block partials added into the FP32 gradient, in a fixed order:
// a workgroup owns 16 consecutive entries; its 16 groups of 16 threads each
// sum every 16th block for one entry (group g takes blocks g, g+16, ...),
// then a fixed tree over the 16 groups.
__global__ __launch_bounds__(256) void reduce_partials_kernel(
    const float* __restrict__ part, int blocks, int width, float* __restrict__ grad)
{
    __shared__ float sh[16][17];
    const int e = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int q = blockIdx.x * 16 + e;
    float s = 0.f;
    if (q < width)
        for (int b = g; b < blocks; b += 16) s += part[(int64_t)b * width + q];
    sh[g][e] = s;
    __syncthreads();
    for (int w = 8; w > 0; w >>= 1) {
        if (g < w) sh[g][e] += sh[g + w][e];
        __syncthreads();
    }
    if (g == 0 && q < width) grad[q] += sh[0][e];
}

// ----------------------------------------------------- up / skip add ----
// s[v] = bf16(x[v/2] + skip[v]) on a D^3 grid (x is (D/2)^3).
__global__ __launch_bounds__(256) void up_add_kernel(
    const uint16_t* __restrict__ x, const uint16_t* __restrict__ skip,
    uint16_t* __restrict__ s, int d)
{
    const int64_t n = (int64_t)d * d * d * 16;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int c = (int)(q & 15);
    const int64_t v = q >> 4;
    const int i = (int)(v % d), j = (int)((v / d) % d), k = (int)(v / ((int64_t)d * d));
    const int h = d / 2;
    const int64_t src = ((((int64_t)(k >> 1) * h + (j >> 1)) * h + (i >> 1)) << 4) + c;
    s[q] = f2bf(bf2f(x[src]) + bf2f(skip[q]));
}

// dx[o] = mask? * sum of the 8 children of o in ds (D^3 -> (D/2)^3).
__global__ __launch_bounds__(256) void up_bwd_kernel(const float* __restrict__ ds,
                                                     float* __restrict__ dx, int d,
                                                     const uint16_t* __restrict__ mask)
{
    const int h = d / 2;
    const int64_t n = (int64_t)h * h * h * 16;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int c = (int)(q & 15);
    const int64_t v = q >> 4;
    const int i = (int)(v % h), j = (int)((v / h) % h), k = (int)(v / ((int64_t)h * h));
    float s = 0.f;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx)
                s += ds[((((int64_t)(2 * k + cz) * d + (2 * j + cy)) * d + (2 * i + cx)) << 4) + c];
    if (mask && !(bf2f(mask[q]) > 0.f)) s = 0.f;
    dx[q] = s;
}

// ------------------------------------------------------------- head ----
// out = blend + hw . x + hb (FP32).  The loss is mean((out - target)^2)
// plus, optionally, W sum_m a_m^2 with a_m = mean((out - target) v_m) over
// the eight sine modes v_m(i,j,k) = S_p(i) S_q(j) S_r(k), p,q,r in {1,2}
// (S_p(i) = sin(pi p (i+1)/(n+1)), mode index m = 4(p-1) + 2(q-1) + (r-1)).
//
// MODE 0: forward; with a target also the plain-MSE backward in the same
//         pass: dout = 2 (out - target) / nvox, dx[v][c] = dout hw[c] (masked
//         by x > 0), per-block partials of the loss and of dhw, dhb.
// MODE 1: forward, loss partials and per-block partials of sum (out-target) v_m.
// MODE 2: backward after MODE 1 and the mode reduction: dout = 2 (out -
//         target) / nvox + (2 W / nvox) sum_m a_m v_m, then dx and partials.
__device__ __forceinline__ float mode_value(const float* sines, int n, int64_t v, int m)
{
    const int i = (int)(v % n), j = (int)((v / n) % n), k = (int)(v / ((int64_t)n * n));
    const int p = m >> 2, q = (m >> 1) & 1, r = m & 1;
    return sines[p * n + i] * sines[q * n + j] * sines[r * n + k];
}

template <int MODE>
__global__ __launch_bounds__(256) void head_kernel(
    const uint16_t* __restrict__ x, int64_t nvox, int n, const float* __restrict__ hw,
    const float* __restrict__ hb, const float* __restrict__ blend,
    float* __restrict__ out, const float* __restrict__ target,
    float* __restrict__ dx, double* __restrict__ loss_part,
    float* __restrict__ gpart, const float* __restrict__ sines,
    double* __restrict__ mpart, const double* __restrict__ acoef, float wlow)
{
    __shared__ double sl[MODE == 1 ? 9 : 1][256];
    __shared__ float sg[MODE == 1 ? 1 : 17][256];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float xc[16];
    float o = 0.f;
    if (v < nvox) {
        const uint4* src = reinterpret_cast<const uint4*>(x + v * 16);
        const uint4 a = src[0], b = src[1];
        const uint32_t wds[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            xc[2 * q] = bf2f((uint16_t)(wds[q] & 0xffff));
            xc[2 * q + 1] = bf2f((uint16_t)(wds[q] >> 16));
        }
        if (MODE == 2) {
            o = out[v];
        } else {
            o = hb[0];
#pragma unroll
            for (int c = 0; c < 16; ++c) o += hw[c] * xc[c];
            o += blend[v];
            if (out) out[v] = o;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 16; ++c) xc[c] = 0.f;
    }
    if (!target) return;
    const float diff = v < nvox ? o - target[v] : 0.f;
    if (MODE == 1) {
        sl[0][threadIdx.x] = (double)diff * diff;
#pragma unroll
        for (int m = 0; m < 8; ++m)
            sl[1 + m][threadIdx.x] =
                v < nvox ? (double)diff * (double)mode_value(sines, n, v, m) : 0.0;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
#pragma unroll
                for (int m = 0; m < 9; ++m) sl[m][threadIdx.x] += sl[m][threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            loss_part[blockIdx.x] = sl[0][0];
            for (int m = 0; m < 8; ++m) mpart[(int64_t)blockIdx.x * 8 + m] = sl[1 + m][0];
        }
        return;
    }
    double l = 0.0;
    float g = 0.f;
    if (v < nvox) {
        l = (double)diff * diff;
        g = 2.f * diff / (float)nvox;
        if (MODE == 2) {
            float lowsum = 0.f;
#pragma unroll
            for (int m = 0; m < 8; ++m) lowsum += (float)acoef[m] * mode_value(sines, n, v, m);
            g += 2.f * wlow * lowsum / (float)nvox;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c)
            dx[v * 16 + c] = (xc[c] > 0.f) ? g * hw[c] : 0.f;
    }
    sl[0][threadIdx.x] = l;
#pragma unroll
    for (int c = 0; c < 16; ++c) sg[MODE == 1 ? 0 : c][threadIdx.x] = g * xc[c];
    sg[MODE == 1 ? 0 : 16][threadIdx.x] = g;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sl[0][threadIdx.x] += sl[0][threadIdx.x + w];
#pragma unroll
            for (int c = 0; c < 17; ++c)
                sg[MODE == 1 ? 0 : c][threadIdx.x] += sg[MODE == 1 ? 0 : c][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (MODE == 0) loss_part[blockIdx.x] = sl[0][0];
        for (int c = 0; c < 17; ++c)
            gpart[(int64_t)blockIdx.x * 17 + c] = sg[MODE == 1 ? 0 : c][0];
    }
}

// a_m = (sum of the per-block partials, fixed order) / nvox; adds
// W sum_m a_m^2 to the loss already summed by sum_loss_kernel.
__global__ void mode_reduce_kernel(const double* __restrict__ mpart, int blocks,
                                   int64_t nvox, float wlow, double* __restrict__ acoef,
                                   double* __restrict__ loss)
{
    __shared__ double a[8];
    const int m = threadIdx.x;
    if (m < 8) {
        double s = 0.0;
        for (int b = 0; b < blocks; ++b) s += mpart[(int64_t)b * 8 + m];
        a[m] = s / (double)nvox;
        acoef[m] = a[m];
    }
    __syncthreads();
    if (m == 0) {
        double q = 0.0;
        for (int k = 0; k < 8; ++k) q += a[k] * a[k];
        loss[0] += (double)wlow * q;
    }
}

__global__ __launch_bounds__(256) void sum_loss_kernel(const double* __restrict__ part,
                                                       int n, int64_t nvox,
                                                       double* __restrict__ out)
{
    __shared__ double s[256];
    double a = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) a += part[q];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0] / (double)nvox;
}

// Output (FP32, n^3) into the interior of an (n+2)^3 FP64 box.
__global__ __launch_bounds__(256) void write_guess_kernel(const float* __restrict__ out,
                                                          int n, double* __restrict__ box)
{
    const int64_t nv = (int64_t)n * n * n;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int i = (int)(v % n), j = (int)((v / n) % n), k = (int)(v / ((int64_t)n * n));
    const int64_t p = n + 2;
    box[((int64_t)(k + 1) * p + (j + 1)) * p + (i + 1)] = (double)out[v];
}

// --------------------------------------------------- parameters / Adam ----
// bf16 copies of every conv layer's weights: w[l][t][co][ci] and the
// transpose wt[l][t][ci][co], from the FP32 parameter vector.
__global__ __launch_bounds__(256) void prep_weights_kernel(
    const float* __restrict__ params, const int64_t* __restrict__ woff, int layers,
    uint16_t* __restrict__ w, uint16_t* __restrict__ wt)
{
    const int64_t per = 27 * 256;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= per * layers) return;
    const int l = (int)(q / per);
    const int r = (int)(q % per);
    const int t = r / 256, co = (r / 16) % 16, ci = r % 16;
    const uint16_t b = f2bf(params[woff[l] + r]);
    w[q] = b;
    wt[(int64_t)l * per + t * 256 + ci * 16 + co] = b;
}

// wt[t][ci][co] = w[t][co][ci] (bf16) for one layer.
__global__ __launch_bounds__(256) void transpose_w_kernel(const uint16_t* __restrict__ w,
                                                          uint16_t* __restrict__ wt)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 27 * 256) return;
    const int t = q / 256, co = (q / 16) % 16, ci = q % 16;
    wt[t * 256 + ci * 16 + co] = w[q];
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ m,
                                                   float* __restrict__ v, int64_t n,
                                                   float lr, float b1, float b2, float eps,
                                                   float c1, float c2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

__global__ __launch_bounds__(256) void zero_f32_kernel(float* __restrict__ p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
        p[q] = 0.f;
}

// Head parameter gradients from per-block partials: one workgroup per
// component, strided partial sums then a tree, both in a fixed order.
__global__ __launch_bounds__(256) void head_grad_kernel(const float* __restrict__ gpart,
                                                        int blocks, float* __restrict__ ghw,
                                                        float* __restrict__ ghb)
{
    __shared__ float sh[256];
    const int c = blockIdx.x;  // 0..15: hw, 16: hb
    float a = 0.f;
    for (int b = threadIdx.x; b < blocks; b += 256) a += gpart[(int64_t)b * 17 + c];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c < 16)
            ghw[c] += sh[0];
        else
            ghb[0] += sh[0];
    }
}

int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t lift(const double* box, int n, uint16_t* x, float* blend, hipStream_t s)
{
    const int64_t nv = (int64_t)n * n * n;
    hipLaunchKernelGGL(lift_kernel, dim3(blocks_for(nv, 256)), dim3(256), 0, s, box, n, x,
                       blend);
    return hipGetLastError();
}

hipError_t conv_fwd(const uint16_t* x, int din, const uint16_t* w, const float* b,
                    uint16_t* y, int stride, bool relu, hipStream_t s)
{
    if (stride == 1 && relu) return conv_fwd_s1(x, din, w, b, y, s);
    const int dout = din / stride;
    const int64_t tiles = (int64_t)dout * dout * ((dout + 15) / 16);
    const dim3 grid(blocks_for(tiles, 4));
    if (stride == 1) {
        if (relu)
            hipLaunchKernelGGL((conv_fwd_kernel<1, true>), grid, dim3(256), 0, s, x, din, w, b, y, dout);
        else
            hipLaunchKernelGGL((conv_fwd_kernel<1, false>), grid, dim3(256), 0, s, x, din, w, b, y, dout);
    } else {
        if (relu)
            hipLaunchKernelGGL((conv_fwd_kernel<2, true>), grid, dim3(256), 0, s, x, din, w, b, y, dout);
        else
            hipLaunchKernelGGL((conv_fwd_kernel<2, false>), grid, dim3(256), 0, s, x, din, w, b, y, dout);
    }
    return hipGetLastError();
}

hipError_t conv_fwd_f32(const uint16_t* x, int din, const uint16_t* w, const float* b,
                        float* y, int stride, hipStream_t s)
{
    if (stride == 1) return conv_fwd_s1_f32(x, din, w, b, y, s);
    const int dout = din / stride;
    const int64_t tiles = (int64_t)dout * dout * ((dout + 15) / 16);
    const dim3 grid(blocks_for(tiles, 4));
    if (stride == 1)
        hipLaunchKernelGGL((conv_fwd_kernel<1, false, true>), grid, dim3(256), 0, s, x, din, w, b, y, dout);
    else
        hipLaunchKernelGGL((conv_fwd_kernel<2, false, true>), grid, dim3(256), 0, s, x, din, w, b, y, dout);
    return hipGetLastError();
}

hipError_t transpose_w(const uint16_t* w, uint16_t* wt, hipStream_t s)
{
    hipLaunchKernelGGL(transpose_w_kernel, dim3(27), dim3(256), 0, s, w, wt);
    return hipGetLastError();
}

hipError_t conv_bwd_data(const float* dy, int dout, const uint16_t* w, const uint16_t* wt,
                         float* dx, int din, int stride, bool accum, const uint16_t* mask,
                         hipStream_t s)
{
    if (stride == 1) return conv_bwd_data_s1(dy, din, w, dx, accum, mask, s);
    if (stride == 2) {
        const int64_t waves = (int64_t)din * din * 2 * ((((din + 1) >> 1) + 15) >> 4);
        hipLaunchKernelGGL(conv_bwd_data_s2_kernel, dim3(blocks_for(waves, 4)), dim3(256), 0, s,
                           dy, dout, wt, dx, din, accum ? 1 : 0, mask);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

int wgrad_blocks(int dout)
{
    const int64_t nchunk = ((int64_t)dout * dout * dout + 15) / 16;
    int64_t b = (nchunk + 4 * 8 - 1) / (4 * 8);  // >= 8 chunks per wave
    if (b > 512) b = 512;
    return (int)(b < 1 ? 1 : b);
}

hipError_t reduce_partials(const float* part, int blocks, float* grad, hipStream_t s)
{
    const int width = 27 * 256 + 16;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(blocks_for(width, 16)), dim3(256), 0, s,
                       part, blocks, width, grad);
    return hipGetLastError();
}

hipError_t conv_bwd_weight(const uint16_t* x, int din, const float* dy, int dout,
                           int stride, float* part, float* grad_w_b, hipStream_t s)
{
    if (stride == 1 && wgrad_s1_blocks(din, nullptr) > 0)
        return conv_bwd_weight_s1(x, dy, din, part, grad_w_b, s);
    if (stride == 2 && wgrad_s2_blocks(dout, nullptr) > 0)
        return conv_bwd_weight_s2(x, din, dy, dout, part, grad_w_b, s);
    const int blocks = wgrad_blocks(dout);
    const int64_t nchunk = ((int64_t)dout * dout * dout + 15) / 16;
    const int cpw = (int)((nchunk + (int64_t)blocks * 4 - 1) / ((int64_t)blocks * 4));
    if (stride == 1)
        hipLaunchKernelGGL((conv_bwd_weight_kernel<1>), dim3(blocks), dim3(256), 0, s, x, din,
                           dy, dout, part, cpw);
    else
        hipLaunchKernelGGL((conv_bwd_weight_kernel<2>), dim3(blocks), dim3(256), 0, s, x, din,
                           dy, dout, part, cpw);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_partials(part, blocks, grad_w_b, s);
}

hipError_t up_add(const uint16_t* x, const uint16_t* skip, uint16_t* out, int d,
                  hipStream_t s)
{
    const int64_t n = (int64_t)d * d * d * 16;
    hipLaunchKernelGGL(up_add_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, skip, out, d);
    return hipGetLastError();
}

hipError_t up_bwd(const float* ds, float* dx, int d, const uint16_t* mask, hipStream_t s)
{
    const int64_t n = (int64_t)(d / 2) * (d / 2) * (d / 2) * 16;
    hipLaunchKernelGGL(up_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, ds, dx, d, mask);
    return hipGetLastError();
}

int head_blocks(int64_t nvox) { return blocks_for(nvox, 256); }

hipError_t head(const uint16_t* x, int64_t nvox, int n, const float* hw, const float* hb,
                const float* blend, float* out, const float* target, float* dx,
                double* loss_part, float* gpart, double* loss, float* ghw, float* ghb,
                const LowModeLoss& low, hipStream_t s)
{
    const int blocks = head_blocks(nvox);
    if (!target || low.weight == 0.f) {
        hipLaunchKernelGGL((head_kernel<0>), dim3(blocks), dim3(256), 0, s, x, nvox, n, hw,
                           hb, blend, out, target, dx, loss_part, gpart, low.sines,
                           low.mpart, low.acoef, low.weight);
        if (target)
            hipLaunchKernelGGL(sum_loss_kernel, dim3(1), dim3(256), 0, s, loss_part, blocks,
                               nvox, loss);
    } else {
        hipLaunchKernelGGL((head_kernel<1>), dim3(blocks), dim3(256), 0, s, x, nvox, n, hw,
                           hb, blend, out, target, dx, loss_part, gpart, low.sines,
                           low.mpart, low.acoef, low.weight);
        hipLaunchKernelGGL(sum_loss_kernel, dim3(1), dim3(256), 0, s, loss_part, blocks, nvox,
                           loss);
        hipLaunchKernelGGL(mode_reduce_kernel, dim3(1), dim3(64), 0, s, low.mpart, blocks,
                           nvox, low.weight, low.acoef, loss);
        hipLaunchKernelGGL((head_kernel<2>), dim3(blocks), dim3(256), 0, s, x, nvox, n, hw,
                           hb, blend, out, target, dx, loss_part, gpart, low.sines,
                           low.mpart, low.acoef, low.weight);
    }
    if (target)
        hipLaunchKernelGGL(head_grad_kernel, dim3(17), dim3(256), 0, s, gpart, blocks, ghw, ghb);
    return hipGetLastError();
}

hipError_t write_guess(const float* out, int n, double* box, hipStream_t s)
{
    const int64_t nv = (int64_t)n * n * n;
    hipLaunchKernelGGL(write_guess_kernel, dim3(blocks_for(nv, 256)), dim3(256), 0, s, out, n,
                       box);
    return hipGetLastError();
}

hipError_t prep_weights(const float* params, const int64_t* woff, int layers, uint16_t* w,
                        uint16_t* wt, hipStream_t s)
{
    const int64_t n = (int64_t)27 * 256 * layers;
    hipLaunchKernelGGL(prep_weights_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, params,
                       woff, layers, w, wt);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                float b2, float eps, int64_t step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step);
    const float c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, g, m, v, n,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t zero_f32(float* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int g = blocks_for(n, 256);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(zero_f32_kernel, dim3(g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace jacobi_impl
