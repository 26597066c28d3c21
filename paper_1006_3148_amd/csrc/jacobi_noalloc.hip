// jacobi_residual_noalloc: the residual norm of jacobi_residual for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  It needs no handle and
// no workspace: the per-block reduction partials live in `scratch`, a static
// device array of this library, one copy per GPU, held until the process
// ends.
//
// Host code never passes `scratch` itself to a kernel: on the host the name
// is a stand-in, not a device address.  The device address of each GPU's
// copy is looked up once per device with hipGetSymbolAddress (with that
// device current) and cached; kernels get that pointer.
//
// Every call on a GPU shares that GPU's copy, so calls that overlap on one
// GPU (different streams, different threads) race on it; calls on one
// stream are ordered and safe.  Nothing in the array needs to start at zero:
// pass 1 of the reduction writes every partial that pass 2 reads.

#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"
#include "jacobi.h"
#include "runtime_common.h"

using namespace jacobi_impl;

namespace {

// Two doubles (sum of r^2, max |r|) per residual block.
constexpr int64_t kScratchBytes = JACOBI_NOALLOC_SCRATCH_BYTES;
constexpr int64_t kMaxBlocks = kScratchBytes / (2 * (int64_t)sizeof(double));

__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on
// the first call on each device).
int scratch_ptr(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(JACOBI_EUNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_ptr[dev];
    return JACOBI_OK;
}

}  // namespace

extern "C" int jacobi_residual_noalloc(const double* origin, int64_t px, int64_t py,
                                       int64_t nx, int64_t ny, int64_t nz, double* out,
                                       void* stream)
{
    if (!origin || !out) return fail(JACOBI_EINVAL, "null argument");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 65536 || ny > 65536 || nz > 65536)
        return fail(JACOBI_EINVAL, "interior dims must be in 1..65536");
    if (px < nx + 2 || py < px * (ny + 2))
        return fail(JACOBI_EINVAL, "pitches must hold the box: px >= nx+2, py >= px*(ny+2)");
    AuxProblem a{};
    a.u[0] = origin;
    a.u[1] = origin;
    a.px = px;
    a.py = py;
    a.nx = (int)nx;
    a.ny = (int)ny;
    a.nz = (int)nz;
    const int blocks = residual_plan(&a);
    a.rblock_base = 0;
    if (blocks > kMaxBlocks)
        return fail(JACOBI_EINVAL,
                    "residual needs %d reduction blocks; the static scratch holds %lld "
                    "(ceil(nx/62)*ceil(ny/16) must be <= %lld)",
                    blocks, (long long)kMaxBlocks, (long long)kMaxBlocks);
    double* partials = nullptr;
    int rc = scratch_ptr(&partials);
    if (rc != JACOBI_OK) return rc;
    hipError_t e = launch_residual_tab(nullptr, 1, a, nullptr, blocks, partials, out,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "residual launch");
}
