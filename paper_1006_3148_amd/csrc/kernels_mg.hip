// Grid-transfer and residual kernels of the multigrid correction solve
// (FP32), the use of the Jacobi update as a multigrid smoother that the paper
// names (Sect. 1.1; conclusions).  The smoothing sweeps themselves are the
// trip kernel's weighted FP32 sweeps with a right-hand side.
//
// Vertex-centred levels: an n^3 interior (n = 2^k - 1) in a dense (n+2)^3
// box with a zero boundary layer; coarse point I sits on fine point 2I.
// Every sum below is a left fold in the order written, with no fused
// multiply-add (-ffp-contract=off), and all weights are powers of two, so
// results are bitwise reproducible.

#include <hip/hip_runtime.h>

#include "internal.h"

namespace jacobi_impl {
namespace {

__device__ __forceinline__ int64_t cell(int i, int j, int k, int n)
{
    const int64_t p = n + 2;
    return ((int64_t)k * p + j) * p + i;
}

// r = (fold(e nbrs) + rhs) - 6 e on the interior (boundary untouched).
__global__ __launch_bounds__(256) void mg_residual_kernel(const float* __restrict__ e,
                                                          const float* __restrict__ rhs,
                                                          float* __restrict__ r, int n)
{
    const int64_t nv = (int64_t)n * n * n;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int i = (int)(v % n) + 1, j = (int)((v / n) % n) + 1, k = (int)(v / ((int64_t)n * n)) + 1;
    const int64_t c = cell(i, j, k, n), px = n + 2, py = px * px;
    float s = e[c - 1] + e[c + 1];
    s = s + e[c - px];
    s = s + e[c + px];
    s = s + e[c - py];
    s = s + e[c + py];
    s = s + rhs[c];
    r[c] = s - 6.0f * e[c];
}

// rc[I] = sum over d in {-1,0,1}^3 (dz, dy, dx nested ascending) of
// 2^-(1+|dx|+|dy|+|dz|) r[2I + d]: full weighting times 4 (the coarse
// operator's doubled spacing).
__global__ __launch_bounds__(256) void mg_restrict_kernel(const float* __restrict__ r, int n,
                                                          float* __restrict__ rc, int nc)
{
    const int64_t nv = (int64_t)nc * nc * nc;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int I = (int)(v % nc) + 1, J = (int)((v / nc) % nc) + 1,
              K = (int)(v / ((int64_t)nc * nc)) + 1;
    float acc = 0.f;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int a = (dx != 0) + (dy != 0) + (dz != 0);
                const float c = a == 0 ? 0.5f : a == 1 ? 0.25f : a == 2 ? 0.125f : 0.0625f;
                acc = acc + c * r[cell(2 * I + dx, 2 * J + dy, 2 * K + dz, n)];
            }
    rc[cell(I, J, K, nc)] = acc;
}

// e[i] += trilinear prolongation of ec: per axis an even fine index takes the
// coarse point i/2 (weight 1), an odd one the points (i-1)/2 and (i+1)/2
// (weight 1/2 each); terms are folded z, y, x nested ascending.
__global__ __launch_bounds__(256) void mg_prolong_add_kernel(const float* __restrict__ ec,
                                                             int nc, float* __restrict__ e,
                                                             int n)
{
    const int64_t nv = (int64_t)n * n * n;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int i = (int)(v % n) + 1, j = (int)((v / n) % n) + 1, k = (int)(v / ((int64_t)n * n)) + 1;
    const int nzt = (k & 1) ? 2 : 1, nyt = (j & 1) ? 2 : 1, nxt = (i & 1) ? 2 : 1;
    const int kz = (k & 1) ? (k - 1) >> 1 : k >> 1;
    const int jy = (j & 1) ? (j - 1) >> 1 : j >> 1;
    const int ix = (i & 1) ? (i - 1) >> 1 : i >> 1;
    const float wz = (k & 1) ? 0.5f : 1.f, wy = (j & 1) ? 0.5f : 1.f, wx = (i & 1) ? 0.5f : 1.f;
    const float w = (wz * wy) * wx;
    float val = 0.f;
    for (int a = 0; a < nzt; ++a)
        for (int b = 0; b < nyt; ++b)
            for (int c = 0; c < nxt; ++c) val = val + w * ec[cell(ix + c, jy + b, kz + a, nc)];
    const int64_t f = cell(i, j, k, n);
    e[f] = e[f] + val;
}

int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

hipError_t launch_mg_residual(const float* e, const float* rhs, float* r, int n, hipStream_t s)
{
    hipLaunchKernelGGL(mg_residual_kernel, dim3(blocks_for((int64_t)n * n * n)), dim3(256), 0,
                       s, e, rhs, r, n);
    return hipGetLastError();
}

hipError_t launch_mg_restrict(const float* r, int n, float* rc, hipStream_t s)
{
    const int nc = (n - 1) / 2;
    hipLaunchKernelGGL(mg_restrict_kernel, dim3(blocks_for((int64_t)nc * nc * nc)), dim3(256),
                       0, s, r, n, rc, nc);
    return hipGetLastError();
}

hipError_t launch_mg_prolong_add(const float* ec, float* e, int n, hipStream_t s)
{
    const int nc = (n - 1) / 2;
    hipLaunchKernelGGL(mg_prolong_add_kernel, dim3(blocks_for((int64_t)n * n * n)), dim3(256),
                       0, s, ec, nc, e, n);
    return hipGetLastError();
}

}  // namespace jacobi_impl
