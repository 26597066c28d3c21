// Auxiliary kernels of libjacobi for gfx950: residual norm (fixed-order,
// deterministic two-pass reduction), the FP32 refinement helpers, fills, box
// copies and the two bandwidth probes of the paper's Table 1 (STREAM copy and
// the array-update loop of Sect. 2.3).
//
// Residual of the discrete Laplace equation (the stopping test of the solver;
// the paper runs a fixed number of sweeps): r = fold(u nbrs) - fl(6u) with the
// neighbour fold of Eq. (1) in the order i-1, i+1, j-1, j+1, k-1, k+1.
// Compiled with -ffp-contract=off.

#include "internal.h"

namespace jacobi_impl {
namespace {

constexpr int kRedThreads = 256;
constexpr int kNoCorrection = -2147483647 - 1;
constexpr int kMaxRedBlocks = 2048;

__device__ __forceinline__ double resid_at(const double* __restrict__ u,
                                           int64_t c, int64_t px, int64_t py)
{
    double s = u[c - 1];
    s = s + u[c + 1];
    s = s + u[c - px];
    s = s + u[c + px];
    s = s + u[c - py];
    s = s + u[c + py];
    return s - 6.0 * u[c];
}

// Block tree reduction of (sum, max) in a fixed order.
__device__ __forceinline__ void block_reduce(double& sum, double& mx,
                                             double* sh_sum, double* sh_max)
{
    const int t = threadIdx.x;
    sh_sum[t] = sum;
    sh_max[t] = mx;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh_sum[t] = sh_sum[t] + sh_sum[t + w];
            sh_max[t] = fmax(sh_max[t], sh_max[t + w]);
        }
        __syncthreads();
    }
    sum = sh_sum[0];
    mx = sh_max[0];
}

// Pass 1: block b owns the interior rows (j,k) with row index = b mod
// gridDim.x; each thread owns i = 1 + t, 1 + t + 256, ...
__global__ __launch_bounds__(kRedThreads) void residual_pass1(
    const double* __restrict__ u, int64_t px, int64_t py, int nx, int ny,
    int nz, double* __restrict__ partials)
{
    __shared__ double sh_sum[kRedThreads], sh_max[kRedThreads];
    double sum = 0.0, mx = 0.0;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = 1 + (int)(row % ny);
        const int k = 1 + (int)(row / ny);
        const int64_t base = (int64_t)k * py + (int64_t)j * px;
        for (int i = 1 + threadIdx.x; i <= nx; i += kRedThreads) {
            const double r = resid_at(u, base + i, px, py);
            sum = sum + r * r;
            mx = fmax(mx, fabs(r));
        }
    }
    block_reduce(sum, mx, sh_sum, sh_max);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = sum;
        partials[gridDim.x + blockIdx.x] = mx;
    }
}

__global__ __launch_bounds__(kRedThreads) void residual_pass2(
    const double* __restrict__ partials, int nblocks, double* __restrict__ out)
{
    __shared__ double sh_sum[kRedThreads], sh_max[kRedThreads];
    double sum = 0.0, mx = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads) {
        sum = sum + partials[b];
        mx = fmax(mx, partials[nblocks + b]);
    }
    block_reduce(sum, mx, sh_sum, sh_max);
    if (threadIdx.x == 0) {
        out[0] = sqrt(sum);
        out[1] = mx;
    }
}

// rhs = fl32(r * 2^-s), s = frexp exponent of max|r|.
__global__ __launch_bounds__(256) void make_rhs_kernel(
    const double* __restrict__ u, int64_t px, int64_t py, int nx, int ny,
    int nz, const double* __restrict__ maxabs, int* __restrict__ scale_exp,
    float* __restrict__ rhs, int64_t rpx, int64_t rpy)
{
    const double m = *maxabs;
    int s = 0;
    if (m > 0.0) frexp(m, &s);
    // kNoCorrection tells the update kernel that the field is already exact.
    if (blockIdx.x == 0 && threadIdx.x == 0) *scale_exp = m > 0.0 ? s : kNoCorrection;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = 1 + (int)(row % ny);
        const int k = 1 + (int)(row / ny);
        const int64_t base = (int64_t)k * py + (int64_t)j * px;
        const int64_t rbase = (int64_t)k * rpy + (int64_t)j * rpx;
        for (int i = 1 + threadIdx.x; i <= nx; i += blockDim.x) {
            float v = 0.f;
            if (m > 0.0) v = (float)ldexp(resid_at(u, base + i, px, py), -s);
            rhs[rbase + i] = v;
        }
    }
}

__global__ __launch_bounds__(256) void apply_correction_kernel(
    double* __restrict__ u, int64_t px, int64_t py, int nx, int ny, int nz,
    const float* __restrict__ e, int64_t epx, int64_t epy,
    const int* __restrict__ scale_exp)
{
    const int s = *scale_exp;
    if (s == kNoCorrection) return;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = 1 + (int)(row % ny);
        const int k = 1 + (int)(row / ny);
        const int64_t base = (int64_t)k * py + (int64_t)j * px;
        const int64_t ebase = (int64_t)k * epy + (int64_t)j * epx;
        for (int i = 1 + threadIdx.x; i <= nx; i += blockDim.x) {
            u[base + i] = u[base + i] + ldexp((double)e[ebase + i], s);
        }
    }
}

template <typename V>
__global__ __launch_bounds__(256) void fill_kernel(V* __restrict__ p, V value,
                                                   int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += stride)
        p[x] = value;
}

__global__ __launch_bounds__(256) void copy_box_kernel(
    const double* __restrict__ src, int64_t spx, int64_t spy,
    double* __restrict__ dst, int64_t dpx, int64_t dpy, int nx2, int ny2,
    int nz2)
{
    const int64_t rows = (int64_t)ny2 * nz2;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = (int)(row % ny2);
        const int k = (int)(row / ny2);
        const double* s = src + (int64_t)k * spy + (int64_t)j * spx;
        double* d = dst + (int64_t)k * dpy + (int64_t)j * dpx;
        for (int i = threadIdx.x; i < nx2; i += blockDim.x) d[i] = s[i];
    }
}

// 16 bytes per lane per access, four independent accesses in flight per
// lane per iteration.
__global__ __launch_bounds__(256) void stream_copy_kernel(
    const double2* __restrict__ a, double2* __restrict__ b, int64_t n2)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; x + 3 * stride < n2; x += 4 * stride) {
        const double2 v0 = a[x], v1 = a[x + stride], v2 = a[x + 2 * stride],
                      v3 = a[x + 3 * stride];
        b[x] = v0;
        b[x + stride] = v1;
        b[x + 2 * stride] = v2;
        b[x + 3 * stride] = v3;
    }
    for (; x < n2; x += stride) b[x] = a[x];
}

__global__ __launch_bounds__(256) void stream_update_kernel(
    double2* __restrict__ a, int64_t n2)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; x + 3 * stride < n2; x += 4 * stride) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = a[x + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u].x = v[u].x + 1.0;
            v[u].y = v[u].y + 1.0;
            a[x + u * stride] = v[u];
        }
    }
    for (; x < n2; x += stride) {
        double2 v = a[x];
        v.x = v.x + 1.0;
        v.y = v.y + 1.0;
        a[x] = v;
    }
}

int grid_for_rows(int64_t rows)
{
    return (int)(rows < 65536 ? rows : 65536);
}

int grid_for_elems(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int residual_blocks(int nx, int ny, int nz)
{
    (void)nx;
    const int64_t rows = (int64_t)ny * nz;
    return (int)(rows < kMaxRedBlocks ? rows : kMaxRedBlocks);
}

hipError_t launch_residual(const double* u, int64_t px, int64_t py, int nx,
                           int ny, int nz, double* partials, double* out,
                           hipStream_t s)
{
    const int nb = residual_blocks(nx, ny, nz);
    hipLaunchKernelGGL(residual_pass1, dim3(nb), dim3(kRedThreads), 0, s, u, px,
                       py, nx, ny, nz, partials);
    hipLaunchKernelGGL(residual_pass2, dim3(1), dim3(kRedThreads), 0, s,
                       partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_make_rhs(const double* u, int64_t px, int64_t py, int nx,
                           int ny, int nz, const double* maxabs,
                           int* scale_exp, float* rhs, int64_t rpx,
                           int64_t rpy, hipStream_t s)
{
    hipLaunchKernelGGL(make_rhs_kernel, dim3(grid_for_rows((int64_t)ny * nz)),
                       dim3(256), 0, s, u, px, py, nx, ny, nz, maxabs,
                       scale_exp, rhs, rpx, rpy);
    return hipGetLastError();
}

hipError_t launch_apply_correction(double* u, int64_t px, int64_t py, int nx,
                                   int ny, int nz, const float* e,
                                   int64_t epx, int64_t epy,
                                   const int* scale_exp, hipStream_t s)
{
    hipLaunchKernelGGL(apply_correction_kernel,
                       dim3(grid_for_rows((int64_t)ny * nz)), dim3(256), 0, s,
                       u, px, py, nx, ny, nz, e, epx, epy, scale_exp);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int value, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel<int>, dim3(grid_for_elems(n)), dim3(256), 0,
                       s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float value, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel<float>, dim3(grid_for_elems(n)), dim3(256),
                       0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_copy_box_f64(const double* src, int64_t spx, int64_t spy,
                               double* dst, int64_t dpx, int64_t dpy, int nx2,
                               int ny2, int nz2, hipStream_t s)
{
    hipLaunchKernelGGL(copy_box_kernel,
                       dim3(grid_for_rows((int64_t)ny2 * nz2)), dim3(256), 0, s,
                       src, spx, spy, dst, dpx, dpy, nx2, ny2, nz2);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const double* a, double* b, int64_t n,
                              hipStream_t s)
{
    const int64_t n2 = n / 2;
    hipLaunchKernelGGL(stream_copy_kernel, dim3(grid_for_elems(n2 / 8)),
                       dim3(256), 0, s, reinterpret_cast<const double2*>(a),
                       reinterpret_cast<double2*>(b), n2);
    return hipGetLastError();
}

hipError_t launch_stream_update(double* a, int64_t n, hipStream_t s)
{
    const int64_t n2 = n / 2;
    hipLaunchKernelGGL(stream_update_kernel, dim3(grid_for_elems(n2 / 8)),
                       dim3(256), 0, s, reinterpret_cast<double2*>(a), n2);
    return hipGetLastError();
}

}  // namespace jacobi_impl
