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
#include "trip_device.h"

namespace jacobi_impl {
namespace {

constexpr int kRedThreads = 256;
constexpr int kNoCorrection = -2147483647 - 1;
// Residual block: 4 waves of kRR j-rows each; a wave's 64 lanes span 62
// output i-columns plus one halo column on each side.
constexpr int kRR = 4;
constexpr int kRX = 62, kRY = kRR * (kRedThreads / 64);

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

// Problem owning global residual block b (binary search over rblock_base).
__device__ __forceinline__ const AuxProblem* find_rblock(const AuxProblem* tab,
                                                        int count, int b)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].rblock_base <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return tab + lo;
}

// Pass 1: k-streaming residual.  Wave w of a block owns kRR consecutive
// interior rows j of a 62-column strip and one k segment; lane L holds column
// i = 62 tx + L (lanes 1..62 are outputs, 0 and 63 their i-halo).  Per plane
// a wave loads its rows and the row above and below them (kRR + 2 row loads
// for kRR output rows); i-neighbours come from the adjacent lanes (DPP), j
// neighbours from the wave's own rows, k-1 / k / k+1 from the rows of three
// planes.  Planes are loaded four at a time, every load of a group issued
// before any use, with indices clamped to the box (no branch around a load).
__global__ __launch_bounds__(kRedThreads) void residual_pass1(
    const AuxProblem* __restrict__ tab, int count, AuxProblem one,
    const int* __restrict__ parity, double* __restrict__ partials)
{
    __shared__ double sh_sum[kRedThreads], sh_max[kRedThreads];
    const AuxProblem Pv = tab ? *find_rblock(tab, count, blockIdx.x) : one;
    const AuxProblem* P = &Pv;
    const int lb = blockIdx.x - P->rblock_base;
    const int tx = lb % P->rtx;
    const int rest = lb / P->rtx;
    const int ty = rest % P->rty;
    const int sg = rest / P->rty;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = tx * kRX + lane;
    const int j0 = 1 + ty * kRY + wave * kRR;
    const int k0 = 1 + sg * P->rseg_len;
    const int k1 = min(k0 + P->rseg_len, P->nz + 1);
    const int64_t px = P->px, py = P->py;
    const int kmax = P->nz + 1;
    const double* __restrict__ u = ((parity && (*parity & 1)) ? P->u[1] : P->u[0]);
    // Row offsets of rows j0-1 .. j0+kRR (clamped to the box; clamped rows
    // and columns feed no output).
    const double* rowp[kRR + 2];
#pragma unroll
    for (int r = 0; r < kRR + 2; ++r)
        rowp[r] = u + (int64_t)min(j0 - 1 + r, P->ny + 1) * px + min(i, P->nx + 1);
    const bool lane_out = lane >= 1 && lane <= kRX && i <= P->nx;
    bool out[kRR];
#pragma unroll
    for (int r = 0; r < kRR; ++r) out[r] = lane_out && j0 + r <= P->ny;

    // cur: plane k (rows -1..kRR), prev: plane k-1 (output rows)
    double cur[kRR + 2], prev[kRR];
#pragma unroll
    for (int r = 0; r < kRR + 2; ++r) cur[r] = rowp[r][(int64_t)k0 * py];
#pragma unroll
    for (int r = 0; r < kRR; ++r) prev[r] = rowp[r + 1][(int64_t)(k0 - 1) * py];
    double sum = 0.0, mx = 0.0;
    for (int k = k0; k < k1; k += 4) {
        double nxt[4][kRR + 2];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < kRR + 2; ++r)
                nxt[q][r] = rowp[r][(int64_t)min(k + 1 + q, kmax) * py];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (k + q < k1) {
#pragma unroll
                for (int r = 0; r < kRR; ++r) {
                    const double c = cur[r + 1];
                    double t = from_left(c);
                    t = t + from_right(c);
                    t = t + cur[r];
                    t = t + cur[r + 2];
                    t = t + prev[r];
                    t = t + nxt[q][r + 1];
                    const double res = t - 6.0 * c;
                    sum = out[r] ? sum + res * res : sum;
                    mx = out[r] ? fmax(mx, fabs(res)) : mx;
                }
            }
#pragma unroll
            for (int r = 0; r < kRR; ++r) prev[r] = cur[r + 1];
#pragma unroll
            for (int r = 0; r < kRR + 2; ++r) cur[r] = nxt[q][r];
        }
    }
    block_reduce(sum, mx, sh_sum, sh_max);
    if (threadIdx.x == 0) {
        partials[2 * (int64_t)blockIdx.x] = sum;
        partials[2 * (int64_t)blockIdx.x + 1] = mx;
    }
}

// Pass 2: block q reduces problem q's partials in a fixed order.
__global__ __launch_bounds__(kRedThreads) void residual_pass2(
    const AuxProblem* __restrict__ tab, AuxProblem one,
    const double* __restrict__ partials, double* __restrict__ out)
{
    __shared__ double sh_sum[kRedThreads], sh_max[kRedThreads];
    const AuxProblem Pv = tab ? tab[blockIdx.x] : one;
    const AuxProblem* P = &Pv;
    double sum = 0.0, mx = 0.0;
    for (int b = threadIdx.x; b < P->rblocks; b += kRedThreads) {
        const int64_t g = P->rblock_base + b;
        sum = sum + partials[2 * g];
        mx = fmax(mx, partials[2 * g + 1]);
    }
    block_reduce(sum, mx, sh_sum, sh_max);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = sqrt(sum);
        out[2 * blockIdx.x + 1] = mx;
    }
}

__device__ __forceinline__ double resid_plain(const double* __restrict__ u,
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

// rhs = fl32(r * 2^-s), s = frexp exponent of max|r|; blockIdx.y = problem.
__global__ __launch_bounds__(256) void make_rhs_kernel(
    const AuxProblem* __restrict__ tab, AuxProblem one,
    const int* __restrict__ parity, const double* __restrict__ out,
    int* __restrict__ scale_exp)
{
    const int q = blockIdx.y;
    const AuxProblem Pv = tab ? tab[q] : one;
    const AuxProblem* P = &Pv;
    const double m = out[2 * q + 1];
    int s = 0;
    if (m > 0.0) frexp(m, &s);
    // kNoCorrection tells the update kernel that the field is already exact.
    if (blockIdx.x == 0 && threadIdx.x == 0)
        scale_exp[q] = m > 0.0 ? s : kNoCorrection;
    const double* __restrict__ u = ((parity && (*parity & 1)) ? P->u[1] : P->u[0]);
    float* __restrict__ rhs = P->rhs;
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = 1 + (int)(row % ny);
        const int k = 1 + (int)(row / ny);
        const int64_t base = (int64_t)k * P->py + (int64_t)j * P->px;
        const int64_t rbase = (int64_t)k * P->epy + (int64_t)j * P->epx;
        for (int i = 1 + threadIdx.x; i <= nx; i += blockDim.x) {
            float v = 0.f;
            if (m > 0.0) v = (float)ldexp(resid_plain(u, base + i, P->px, P->py), -s);
            rhs[rbase + i] = v;
        }
    }
}

__global__ __launch_bounds__(256) void apply_correction_kernel(
    const AuxProblem* __restrict__ tab, AuxProblem one,
    const int* __restrict__ parity, int which,
    const int* __restrict__ scale_exp)
{
    const int q = blockIdx.y;
    const AuxProblem Pv = tab ? tab[q] : one;
    const AuxProblem* P = &Pv;
    const int s = scale_exp[q];
    if (s == kNoCorrection) return;
    double* __restrict__ u = const_cast<double*>(((parity && (*parity & 1)) ? P->u[1] : P->u[0]));
    const float* __restrict__ e = which ? P->e[1] : P->e[0];
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = 1 + (int)(row % ny);
        const int k = 1 + (int)(row / ny);
        const int64_t base = (int64_t)k * P->py + (int64_t)j * P->px;
        const int64_t ebase = (int64_t)k * P->epy + (int64_t)j * P->epx;
        for (int i = 1 + threadIdx.x; i <= nx; i += blockDim.x)
            u[base + i] = u[base + i] + ldexp((double)e[ebase + i], s);
    }
}

__global__ __launch_bounds__(256) void zero_e_kernel(
    const AuxProblem* __restrict__ tab, AuxProblem one)
{
    const AuxProblem Pv = tab ? tab[blockIdx.y] : one;
    float* __restrict__ e = Pv.e[0];
    const AuxProblem* P = &Pv;
    const int64_t n = P->epy * (P->nz + 2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += stride)
        e[x] = 0.f;
}

__global__ void flip_parity_kernel(int* word, int* ticket)
{
    if (threadIdx.x == 0) {
        *word = *word ^ 1;
        *ticket = 0;
    }
}

__global__ void set_int_kernel(int* word, int value)
{
    if (threadIdx.x == 0) *word = value;
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

// Bandwidth probes.  Each workgroup streams one contiguous chunk of
// kProbeChunk 16-byte elements, eight independent 16-byte accesses in flight
// per lane, with non-temporal loads and stores (the data is touched once).
// This form measured fastest among grid-stride and chunked variants with 4,
// 8 and 16 accesses per lane, with and without the non-temporal hint.
typedef double dv2 __attribute__((ext_vector_type(2)));
constexpr int64_t kProbeChunk = 8192;
constexpr int kProbeU = 8;

__global__ __launch_bounds__(256) void stream_copy_kernel(
    const dv2* __restrict__ a, dv2* __restrict__ b, int64_t n2)
{
    const int64_t lo = (int64_t)blockIdx.x * kProbeChunk;
    const int64_t hi = lo + kProbeChunk < n2 ? lo + kProbeChunk : n2;
    for (int64_t x = lo + threadIdx.x; x < hi; x += 256 * kProbeU) {
        dv2 v[kProbeU];
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) {
            const int64_t y = x + u * 256;
            v[u] = y < hi ? __builtin_nontemporal_load(&a[y]) : dv2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) {
            const int64_t y = x + u * 256;
            if (y < hi) __builtin_nontemporal_store(v[u], &b[y]);
        }
    }
}

// The paper's array-update loop a[i] += 1 (in place), same streaming form.
__global__ __launch_bounds__(256) void stream_update_kernel(dv2* __restrict__ a, int64_t n2)
{
    const int64_t lo = (int64_t)blockIdx.x * kProbeChunk;
    const int64_t hi = lo + kProbeChunk < n2 ? lo + kProbeChunk : n2;
    for (int64_t x = lo + threadIdx.x; x < hi; x += 256 * kProbeU) {
        dv2 v[kProbeU];
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) {
            const int64_t y = x + u * 256;
            v[u] = y < hi ? __builtin_nontemporal_load(&a[y]) : dv2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < kProbeU; ++u) {
            const int64_t y = x + u * 256;
            if (y < hi) __builtin_nontemporal_store(v[u] + 1.0, &a[y]);
        }
    }
}

// One Jacobi sweep (Eq. (1)) of the interior, one thread per cell, for boxes
// small enough to sit in the caches: the k-streaming trip kernel needs a
// pipeline of several dependent steps per tile, while here a sweep is one
// round of independent loads.  Same fold order, times fl(1/6).
__global__ __launch_bounds__(256) void sweep1_kernel(const double* __restrict__ a,
                                                     double* __restrict__ b, int64_t px,
                                                     int64_t py, int nx, int ny, int nz)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63) + 1;
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6) + 1;
    const int k = blockIdx.z + 1;
    if (i > nx || j > ny || k > nz) return;
    const int64_t c = (int64_t)k * py + (int64_t)j * px + i;
    double s = a[c - 1] + a[c + 1];
    s = s + a[c - px];
    s = s + a[c + px];
    s = s + a[c - py];
    s = s + a[c + py];
    b[c] = s * (1.0 / 6.0);
}

int grid_for_elems(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int residual_plan(AuxProblem* a)
{
    a->rtx = (a->nx + kRX - 1) / kRX;
    a->rty = (a->ny + kRY - 1) / kRY;
    const int64_t plane = (int64_t)a->rtx * a->rty;
    // Enough blocks to fill the chip (>= 2048) with segments of >= 16 planes.
    int64_t segs = (2048 + plane - 1) / plane;
    const int64_t max_segs = (a->nz + 15) / 16;
    if (segs > max_segs) segs = max_segs;
    if (segs < 1) segs = 1;
    a->rseg_len = (int)((a->nz + segs - 1) / segs);
    a->rsegs = (a->nz + a->rseg_len - 1) / a->rseg_len;
    a->rblocks = (int)(plane * a->rsegs);
    return a->rblocks;
}

namespace {
int grid_rows(int64_t rows, int count)
{
    int64_t g = rows < 4096 ? rows : 4096;
    if (count > 1 && g > 512) g = 512;
    return (int)(g < 1 ? 1 : g);
}
}  // namespace

hipError_t launch_residual_tab(const AuxProblem* table, int count,
                               const AuxProblem& one, const int* parity,
                               int total_blocks, double* partials, double* out,
                               hipStream_t s)
{
    hipLaunchKernelGGL(residual_pass1, dim3(total_blocks), dim3(kRedThreads), 0,
                       s, table, count, one, parity, partials);
    hipLaunchKernelGGL(residual_pass2, dim3(table ? count : 1), dim3(kRedThreads),
                       0, s, table, one, partials, out);
    return hipGetLastError();
}

hipError_t launch_make_rhs_tab(const AuxProblem* table, int count,
                               const AuxProblem& one, const int* parity,
                               const double* out, int* scale_exp, hipStream_t s)
{
    const int64_t rows = table ? (int64_t)512 : (int64_t)one.ny * one.nz;
    hipLaunchKernelGGL(make_rhs_kernel,
                       dim3(grid_rows(rows, table ? count : 1), table ? count : 1),
                       dim3(256), 0, s, table, one, parity, out, scale_exp);
    return hipGetLastError();
}

hipError_t launch_apply_correction_tab(const AuxProblem* table, int count,
                                       const AuxProblem& one,
                                       const int* parity, int which,
                                       const int* scale_exp, hipStream_t s)
{
    const int64_t rows = table ? (int64_t)512 : (int64_t)one.ny * one.nz;
    hipLaunchKernelGGL(apply_correction_kernel,
                       dim3(grid_rows(rows, table ? count : 1), table ? count : 1),
                       dim3(256), 0, s, table, one, parity, which, scale_exp);
    return hipGetLastError();
}

hipError_t launch_zero_e_tab(const AuxProblem* table, int count,
                             const AuxProblem& one, hipStream_t s)
{
    hipLaunchKernelGGL(zero_e_kernel, dim3(table ? 256 : 2048, table ? count : 1),
                       dim3(256), 0, s, table, one);
    return hipGetLastError();
}

hipError_t launch_flip_parity(int* word, int* ticket, hipStream_t s)
{
    hipLaunchKernelGGL(flip_parity_kernel, dim3(1), dim3(64), 0, s, word, ticket);
    return hipGetLastError();
}

hipError_t launch_set_int(int* word, int value, hipStream_t s)
{
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, word, value);
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
                       dim3((int)((int64_t)ny2 * nz2 < 65536 ? (int64_t)ny2 * nz2 : 65536)), dim3(256), 0, s,
                       src, spx, spy, dst, dpx, dpy, nx2, ny2, nz2);
    return hipGetLastError();
}

hipError_t launch_sweep1_f64(const double* a, double* b, int64_t px, int64_t py, int nx,
                             int ny, int nz, hipStream_t s)
{
    hipLaunchKernelGGL(sweep1_kernel, dim3((nx + 63) / 64, (ny + 3) / 4, nz), dim3(256), 0, s,
                       a, b, px, py, nx, ny, nz);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const double* a, double* b, int64_t n,
                              hipStream_t s)
{
    const int64_t n2 = n / 2;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)((n2 + kProbeChunk - 1) / kProbeChunk)),
                       dim3(256), 0, s, reinterpret_cast<const dv2*>(a),
                       reinterpret_cast<dv2*>(b), n2);
    return hipGetLastError();
}

hipError_t launch_stream_update(double* a, int64_t n, hipStream_t s)
{
    const int64_t n2 = n / 2;
    hipLaunchKernelGGL(stream_update_kernel, dim3((unsigned)((n2 + kProbeChunk - 1) / kProbeChunk)),
                       dim3(256), 0, s, reinterpret_cast<dv2*>(a), n2);
    return hipGetLastError();
}

}  // namespace jacobi_impl
