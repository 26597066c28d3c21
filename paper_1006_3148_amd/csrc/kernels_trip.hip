// Temporally blocked 3D 7-point Jacobi trip kernel for gfx950 (CDNA4).
//
// One launch applies T sweeps of Eq. (1) of the paper (Sect. 1.1) to the whole
// box while reading the grid from HBM once and writing it once (the
// temporally blocked bandwidth model, Eq. (4) of Sect. 2.3: T updates cost
// one read and one write stream per cell).
//
// Mapping (the GPU counterpart of the paper's pipeline of threads handing a
// cache-resident block from update to update, Sect. 2.1):
//  * a workgroup owns a tile of 64 i-columns x (R*W) j-rows and one segment of
//    the k axis; lane = i, wave w holds rows [w*R, w*R+R);
//  * the tile streams along k.  Stage s (sweep s of the trip) keeps, per
//    owned cell, two registers: P = (in-plane sum of the previous stage's
//    plane q) + (its plane q-1 value), and C = its plane-q value.  When plane
//    q+1 of stage s-1 arrives, stage s completes plane q as (P + X(q+1))*c6
//    and passes it to stage s+1 in the same step.  This keeps the addition
//    order of Eq. (1) exactly: i-1, i+1, j-1, j+1, k-1, k+1;
//  * i-neighbours come from the adjacent lanes through DPP wave shifts, j
//    neighbours from the wave's own registers, and the two edge rows of each
//    wave through LDS (one barrier per stage, double-buffered);
//  * tiles overlap by T cells in i and j and by T planes between k segments
//    (ghost zones): stage s is exact on a region that shrinks by one cell per
//    stage, and only the central (64-2T) x (R*W-2T) x seg_len block is stored.
//    The paper avoids this redundancy with its one-cell block shift; here the
//    redundant work is the price of keeping every stage on-chip;
//  * boundary-layer cells pass through unchanged (Dirichlet boundary).
//
// Compressed grid (Sect. 2.1): with mode 1 src and dst are the same storage
// and dst is src shifted by (-T,-T,-T) (dir=+1) or (+T,+T,+T) (dir=-1), the
// paper's per-update shift vector times T.  A cell may only be overwritten
// after every tile that reads it has loaded it.  Tiles are taken from a ticket
// counter in an order in which every such reader has a smaller ticket, and a
// tile spins on the readers' progress words before each store: the first
// condition of Eq. (3) (Sect. 2.2) with per-tile counters instead of
// per-thread ones.  A bounded spin turns a lost tile into an error word
// instead of a hang.
//
// Compiled with -ffp-contract=off: no fused multiply-add, so results are
// bitwise equal to the plain definition.

#include <type_traits>

#include "internal.h"
#include "trip_device.h"

namespace jacobi_impl {
namespace {

template <typename Real, int T, int R, int W, int PF, bool RHS, bool FLAGS, bool EDGE>
__device__ __forceinline__ void run_tile(const TripParams& p, const Geo& g, int tile,
                                         Real (*xch)[W][2][64])
{
    constexpr int H = R * W;
    constexpr int OX = 64 - 2 * T;
    constexpr int OY = H - 2 * T;
    const Real c6 = Sixth<Real>::v;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const int tx = tile % g.tiles_x;
    const int rest = tile / g.tiles_x;
    const int ty = rest % g.tiles_y;
    const int seg = rest / g.tiles_y;

    const int i = tx * OX - T + lane;
    const int j0 = ty * OY - T + wave * R;
    const int k0 = seg * g.seg_len;
    const int k1 = min(k0 + g.seg_len, g.nz + 2);
    const int a = max(k0 - T, 0);
    const int b = min(k1 - 1 + T, g.nz + 1);
    const int nsteps = k1 - a + T;

    const Real* __restrict__ src = static_cast<const Real*>(g.src);
    Real* __restrict__ dst = static_cast<Real*>(g.dst);
    const int64_t px = g.px, py = g.py;

    bool lane_int = true, lane_box = true;
    bool row_int[R], row_box[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        row_int[r] = true;
        row_box[r] = true;
    }
    if (EDGE) {
        lane_box = (unsigned)i <= (unsigned)(g.nx + 1);
        lane_int = i >= 1 && i <= g.nx;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = j0 + r;
            row_box[r] = (unsigned)j <= (unsigned)(g.ny + 1);
            row_int[r] = j >= 1 && j <= g.ny;
        }
    }
    const bool lane_out = lane >= T && lane < 64 - T && i <= g.nx + 1;
    bool row_out[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int tr = wave * R + r;
        row_out[r] = tr >= T && tr < H - T && (j0 + r) <= g.ny + 1;
    }

    // Dependees of this tile under the compressed-grid shift: the tiles whose
    // input regions contain cells this tile overwrites.
    int dep = -1;
    if (FLAGS && lane < 7) {
        const int d = lane + 1;  // bits (dx, dy, dz) of the neighbour offset
        const int sgn = p.dir > 0 ? -1 : 1;
        const int ntx = tx + ((d & 1) ? sgn : 0);
        const int nty = ty + ((d & 2) ? sgn : 0);
        const int nsg = seg + ((d & 4) ? sgn : 0);
        if (ntx >= 0 && ntx < g.tiles_x && nty >= 0 && nty < g.tiles_y &&
            nsg >= 0 && nsg < g.segs)
            dep = (nsg * g.tiles_y + nty) * g.tiles_x + ntx;
    }
    int known = FLAGS ? 0 : kDone;

    Real P[T][R], C[T][R];
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            P[s][r] = Real(0);
            C[s][r] = Real(0);
        }
    float rq[RHS ? T : 1][R];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int s = 0; s < (RHS ? T : 1); ++s) rq[s][r] = 0.f;

    // Addressing: a scalar (per-plane) base plus a 32-bit per-row byte offset
    // that is loop invariant; src, dst and rhs frames share the pitches.
    uint32_t voff[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        voff[r] = (uint32_t)(((int64_t)(j0 + r) * px + i) * (int64_t)sizeof(Real));
    const int64_t plane_bytes = py * (int64_t)sizeof(Real);
    const char* src_b = reinterpret_cast<const char*>(src);
    const char* rhs_b = reinterpret_cast<const char*>(g.rhs);
    char* dst_b = reinterpret_cast<char*>(dst);
    const int64_t rplane_bytes = g.rpy * (int64_t)sizeof(float);

    // Register ring of the next PF input planes (and rhs planes): plane
    // loads are issued PF steps before use, so each step does not wait for a
    // full memory round trip.
    Real ring[PF][R];
    float rring[RHS ? PF : 1][R];
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        const int q = a + d;
        const char* sp = src_b + (int64_t)q * plane_bytes;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ring[d][r] = Real(0);
            if (q <= b && (!EDGE || (lane_box && row_box[r])))
                ring[d][r] = *reinterpret_cast<const Real*>(sp + voff[r]);
        }
        if (RHS) {
            const int qr = a - 1 + d;  // rhs plane stage 1 uses at step d
            const char* rp = rhs_b + (int64_t)qr * rplane_bytes;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                rring[RHS ? d : 0][r] = 0.f;
                if (qr >= 1 && qr <= g.nz && (!EDGE || (lane_box && row_box[r])))
                    rring[RHS ? d : 0][r] = *reinterpret_cast<const float*>(
                        rp + voff[r] / (sizeof(Real) / sizeof(float)));
            }
        }
    }

    int phase = 0;
#pragma unroll 2
    for (int n = 0; n < nsteps; ++n) {
        Real x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = ring[0][r];
        if (RHS) {
#pragma unroll
            for (int r = 0; r < R; ++r) rq[0][r] = rring[0][r];
        }
#pragma unroll
        for (int d = 0; d + 1 < PF; ++d)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                ring[d][r] = ring[d + 1][r];
                if (RHS) rring[RHS ? d : 0][r] = rring[RHS ? d + 1 : 0][r];
            }
        // Issue the loads of plane a+n+PF (used PF steps from now).
        const int qn = a + n + PF;
#pragma unroll
        for (int r = 0; r < R; ++r) ring[PF - 1][r] = Real(0);
        if (qn <= b) {
            const char* sp = src_b + (int64_t)qn * plane_bytes;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (!EDGE || (lane_box && row_box[r]))
                    ring[PF - 1][r] = *reinterpret_cast<const Real*>(sp + voff[r]);
        }
        if (RHS) {
            const int qr = a + n + PF - 1;  // rhs plane stage 1 uses at step n+PF
#pragma unroll
            for (int r = 0; r < R; ++r) rring[RHS ? PF - 1 : 0][r] = 0.f;
            if (qr >= 1 && qr <= g.nz) {
                const char* rp = rhs_b + (int64_t)qr * rplane_bytes;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (!EDGE || (lane_box && row_box[r]))
                        rring[RHS ? PF - 1 : 0][r] = *reinterpret_cast<const float*>(
                            rp + voff[r] / (sizeof(Real) / sizeof(float)));
            }
        }

        // The T stages of this step.  Only the first and last steps of a tile
        // see the boundary planes 0 and nz+1 (pass-through); the common steps
        // take the branch-free variant.
        auto stages = [&](auto bnd_tag) {
            constexpr bool BND = decltype(bnd_tag)::value;
#pragma unroll
            for (int s = 0; s < T; ++s) {
                const int q = a + n - s;  // plane arriving at stage s+1
                const int pe = q - 1;     // plane stage s+1 completes now
                Real(*buf)[2][64] = xch[phase & 1];
                ++phase;
                buf[wave][0][lane] = x[0];
                buf[wave][1][lane] = x[R - 1];
                __syncthreads();
                if (FLAGS && s == 0 && threadIdx.x == 0) {
                    // every wave has finished step n-1: plane a+n-1 is consumed
                    flag_store(p.flags + (int64_t)tile * kFlagStride, a + n);
                }
                const Real up = buf[wave > 0 ? wave - 1 : 0][1][lane];
                const Real dn = buf[wave < W - 1 ? wave + 1 : W - 1][0][lane];
                const bool bnd = BND && ((pe == 0) || (pe == g.nz + 1));
                // Row by row; `above` keeps the old value of row r-1.
                Real above = up;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const Real xo = x[r];
                    const Real below = (r == R - 1) ? dn : x[r < R - 1 ? r + 1 : 0];
                    const Real inpl = ((from_left(xo) + from_right(xo)) + above) + below;
                    Real e;
                    if (bnd) {
                        e = C[s][r];
                    } else {
                        Real sum = P[s][r] + xo;
                        if (RHS) sum = sum + (Real)rq[RHS ? s : 0][r];
                        e = sum * c6;
                        if (EDGE) e = (lane_int && row_int[r]) ? e : C[s][r];
                    }
                    P[s][r] = inpl + C[s][r];
                    C[s][r] = xo;
                    x[r] = e;
                    above = xo;
                }
            }
        };
        if (a + n - T <= 0 || a + n - 1 >= g.nz + 1)
            stages(std::true_type{});
        else
            stages(std::false_type{});
        if (RHS) {
#pragma unroll
            for (int s = (RHS ? T : 1) - 1; s > 0; --s)
#pragma unroll
                for (int r = 0; r < R; ++r) rq[s][r] = rq[s - 1][r];
        }

        // x now holds plane pe_T of the last stage.
        const int pe = a + n - T;
        if (pe >= k0 && pe < k1) {
            if (FLAGS) {
                // Storage plane overwritten by this store, in input-frame
                // terms; planes outside the box are shift room nobody reads.
                const int ow = p.dir > 0 ? pe - T : pe + T;
                const int need = ow + 1;
                if (ow >= 0 && ow <= g.nz + 1 && known < need) {
                    int64_t spins = 0;
                    for (;;) {
                        int v = kDone;
                        if (dep >= 0) v = flag_load(p.flags + (int64_t)dep * kFlagStride);
#pragma unroll
                        for (int o = 1; o < 8; o <<= 1) v = min(v, __shfl_xor(v, o, 64));
                        v = __builtin_amdgcn_readfirstlane(v);
                        if (v >= need) {
                            known = v;
                            break;
                        }
                        if (++spins > p.spin_limit ||
                            flag_load(p.err) != 0) {
                            if (lane == 0) atomicCAS(p.err, 0, 1);
                            known = kDone;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                }
            }
            if (lane_out) {
                char* dp = dst_b + (int64_t)pe * plane_bytes;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (row_out[r]) *reinterpret_cast<Real*>(dp + voff[r]) = x[r];
            }
        }
    }
    if (FLAGS) {
        __syncthreads();
        if (threadIdx.x == 0) flag_store(p.flags + (int64_t)tile * kFlagStride, kDone);
    }
}

// MODE 0: one problem, tile = f(blockIdx) (A/B; kernel boundary between
//         trips is the only synchronization).
// MODE 1: one problem, tiles from a ticket counter, progress flags
//         (compressed single grid).
// MODE 2: a batch of independent problems described by p.table; tiles of all
//         problems from one ticket counter; A/B parity read from *p.parity.
template <typename Real, int T, int R, int W, int PF, bool RHS, int MODE>
__global__ __launch_bounds__(64 * W) void trip_kernel(TripParams p)
{
    constexpr bool FLAGS = MODE == 1;
    constexpr int H = R * W;
    constexpr int OX = 64 - 2 * T;
    constexpr int OY = H - 2 * T;
    __shared__ Real xch[2][W][2][64];
    __shared__ int tile_sh;

    for (int iter = 0;; ++iter) {
        int tile;
        if (MODE == 0) {
            if (iter > 0) return;
            tile = xcd_tile(blockIdx.x, p.ntiles);
        } else {
            __syncthreads();  // previous tile finished with tile_sh and xch
            if (threadIdx.x == 0) tile_sh = atomicAdd(p.ticket, 1);
            __syncthreads();
            const int t = tile_sh;
            if (t >= p.ntiles) return;
            tile = (MODE == 1 && p.dir < 0) ? p.ntiles - 1 - t : t;
        }
        Geo g;
        if (MODE == 2) {
            int lo = 0, hi = p.count - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (p.table[mid].tile_base <= tile)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const BatchProblem& bp = p.table[lo];
            const int par = *p.parity & 1;
            g.src = bp.grid[par];
            g.dst = bp.grid[par ^ 1];
            g.rhs = bp.rhs;
            g.px = g.rpx = bp.px;
            g.py = g.rpy = bp.py;
            g.nx = bp.nx;
            g.ny = bp.ny;
            g.nz = bp.nz;
            g.tiles_x = bp.tiles_x;
            g.tiles_y = bp.tiles_y;
            g.segs = bp.segs;
            g.seg_len = bp.seg_len;
            tile -= bp.tile_base;
        } else {
            g.src = p.src;
            g.dst = p.dst;
            g.rhs = p.rhs;
            g.px = p.px;
            g.py = p.py;
            g.rpx = p.rpx;
            g.rpy = p.rpy;
            g.nx = p.nx;
            g.ny = p.ny;
            g.nz = p.nz;
            g.tiles_x = p.tiles_x;
            g.tiles_y = p.tiles_y;
            g.segs = p.segs;
            g.seg_len = p.seg_len;
        }
        const int tx = tile % g.tiles_x;
        const int ty = (tile / g.tiles_x) % g.tiles_y;
        const int ilo = tx * OX - T, jlo = ty * OY - T;
        const bool interior_tile = ilo >= 1 && ilo + 63 <= g.nx && jlo >= 1 &&
                                   jlo + H - 1 <= g.ny;
        if (interior_tile)
            run_tile<Real, T, R, W, PF, RHS, FLAGS, false>(p, g, tile, xch);
        else
            run_tile<Real, T, R, W, PF, RHS, FLAGS, true>(p, g, tile, xch);
    }
}

template <typename Real, int T, int R, int W, int PF, bool RHS>
hipError_t launch_cfg(const TripParams& p, hipStream_t s)
{
    dim3 block(64 * W);
    if (p.mode == 0) {
        hipLaunchKernelGGL((trip_kernel<Real, T, R, W, PF, RHS, 0>),
                           dim3(p.ntiles), block, 0, s, p);
        return hipGetLastError();
    }
    // Persistent launch: as many workgroups as can be resident.
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = p.mode == 1
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, reinterpret_cast<const void*>(
                                   &trip_kernel<Real, T, R, W, PF, RHS, 1>),
                      64 * W, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, reinterpret_cast<const void*>(
                                   &trip_kernel<Real, T, R, W, PF, RHS, 2>),
                      64 * W, 0);
    if (e != hipSuccess) return e;
    int grid = cus * (per_cu > 0 ? per_cu : 1);
    if (grid > p.ntiles) grid = p.ntiles;
    if (p.mode == 1)
        hipLaunchKernelGGL((trip_kernel<Real, T, R, W, PF, RHS, 1>), dim3(grid),
                           block, 0, s, p);
    else
        hipLaunchKernelGGL((trip_kernel<Real, T, R, W, PF, RHS, 2>), dim3(grid),
                           block, 0, s, p);
    return hipGetLastError();
}

// Compiled tile shapes: R rows per wave x W waves (tile = 64 x R*W columns)
// for T = 1..8.  Configurations whose per-stage register state spills are
// still compiled; the host picks among the ones listed by trip_config_list.
#define JACOBI_TRIP_CFGS(X) \
    X(1, 4, 16) X(2, 4, 16)                                                   \
    X(1, 4, 8) X(2, 4, 8) X(3, 4, 8) X(4, 4, 8) X(5, 4, 8) X(6, 4, 8)          \
    X(1, 2, 16) X(2, 2, 16) X(3, 2, 16) X(4, 2, 16) X(5, 2, 16) X(6, 2, 16)    \
    X(7, 2, 16) X(8, 2, 16) X(7, 4, 8) X(8, 4, 8)

template <typename Real, bool RHS>
hipError_t dispatch(const TripConfig& c, const TripParams& p, hipStream_t s)
{
#define JACOBI_CASE(T_, R_, W_) \
    if (c.T == T_ && c.R == R_ && c.W == W_) return launch_cfg<Real, T_, R_, W_, kPrefetch, RHS>(p, s);
    JACOBI_TRIP_CFGS(JACOBI_CASE)
#undef JACOBI_CASE
    return hipErrorInvalidValue;
}

}  // namespace

bool trip_config_supported(int dtype_f32, const TripConfig& c)
{
    (void)dtype_f32;
#define JACOBI_SUP(T_, R_, W_) \
    if (c.T == T_ && c.R == R_ && c.W == W_) return true;
    JACOBI_TRIP_CFGS(JACOBI_SUP)
#undef JACOBI_SUP
    return false;
}

hipError_t launch_trip_f64(const TripConfig& c, const TripParams& p,
                           hipStream_t s)
{
    return dispatch<double, false>(c, p, s);
}

hipError_t launch_trip_f32(const TripConfig& c, const TripParams& p,
                           hipStream_t s)
{
    if (p.rhs || p.rhs_in_table) return dispatch<float, true>(c, p, s);
    return dispatch<float, false>(c, p, s);
}

}  // namespace jacobi_impl
