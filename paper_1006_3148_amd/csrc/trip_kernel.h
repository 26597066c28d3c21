#pragma once
// Temporally blocked 3D 7-point Jacobi trip kernel for gfx950 (CDNA4).
//
// Kernel templates; the trip_*.hip units instantiate them per precision and
// mode (split so that the instantiations compile in parallel).
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
//    wave through LDS;
//  * stage s consumes in step n what stage s-1 produced in step n-1 (stage s
//    runs two planes behind stage s-1 instead of one).  The edge rows of all
//    T stages are then exchanged together, with one barrier per step, and
//    the T stages of a step are independent chains of arithmetic; the rows
//    that need nothing from other waves are computed while the barrier and
//    the LDS reads are pending;
//  * tiles overlap by T cells in i and j and by T planes between k segments
//    (ghost zones): stage s is exact on a region that shrinks by one cell per
//    stage, and only the central (64-2T) x (R*W-2T) x seg_len block is stored.
//    The paper avoids this redundancy with its one-cell block shift; here the
//    redundant work is the price of keeping every stage on-chip;
//  * boundary-layer cells pass through unchanged (Dirichlet boundary).
//
// Compressed grid (Sect. 2.1): with mode 1 src and dst are the same storage
// and dst is src shifted by (-T,-T,-T-E) (dir=+1) or (+T,+T,+T+E) (dir=-1):
// the paper's per-update shift vector times T, plus E extra planes along the
// streaming axis (p.zshift = T+E), which give a tile E more steps of slack
// before it overwrites planes its neighbours still read.  A cell may only be
// overwritten after every tile that reads it has loaded it.  Tiles are
// claimed in an order in which every such reader comes first (one ticket
// counter, or the per-XCD claim groups of claim_grouped, which keep
// neighbouring tiles on one XCD's L2), and a tile spins on the readers'
// progress words before each store: the first condition of Eq. (3)
// (Sect. 2.2) with per-tile counters instead of per-thread ones.  A bounded
// spin turns a lost tile into an error word instead of a hang.
//
// Compiled with -ffp-contract=off: no fused multiply-add, so results are
// bitwise equal to the plain definition.

#include <type_traits>
#include <utility>

#include "internal.h"
#include "trip_configs.h"
#include "trip_device.h"

namespace jacobi_impl {
namespace {

template <int... Is, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F&& f)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// Spin until every dependee's progress word is >= need (or the bounded spin
// runs out, which raises the error word).  Out of line, so that the rare wait
// does not split the straight-line step code of the caller.
__device__ __forceinline__ int wait_progress(int* flags, int dep, int need,
                                                      long long spin_limit, int* err)
{
    const int lane = threadIdx.x & 63;
    int64_t spins = 0;
    for (;;) {
        int v = kDone;
        if (dep >= 0) v = flag_load(flags + (int64_t)dep * kFlagStride);
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) v = min(v, __shfl_xor(v, o, 64));
        v = __builtin_amdgcn_readfirstlane(v);
        if (v >= need) return v;
        if (++spins > spin_limit || flag_load(err) != 0) {
            if (lane == 0) atomicCAS(err, 0, 1);
            return kDone;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Edge-row exchange buffers in LDS: [buffer][stage][wave][top/bottom][lane].
// Two buffers (one barrier per step) when they fit in the 160 KB of LDS of a
// CU, else one buffer and a second barrier per step before it is rewritten.
template <typename Real, int T, int W>
struct Xch {
    static constexpr size_t one = (size_t)T * W * 2 * 64 * sizeof(Real);
    static constexpr int nbuf = 2 * one <= 150 * 1024 ? 2 : 1;
};

// WT: weighted (damped) sweeps e' = e + w (v - e), v the Eq. (1) update plus
// the right-hand side, w = p.omega (the multigrid smoother).
// KREV: the tile streams a k-mirrored view of the grid (origin at the top
// plane, negative plane pitch), used by backward compressed trips so that
// their stores, like a forward trip's, land behind the stream.  Logical plane
// q+1 is then physical k-1, and the update keeps Eq. (1)'s order (k-1 before
// k+1) by holding one more plane per stage.
// S27: the 27-point Jacobi update instead of Eq. (1) (A/B sweeps only): the
// mean of the 26 neighbours weighted 7/64 (6 faces), 3/128 (12 edges) and
// 1/128 (8 corners), from per-plane partial sums of the 3x3 window of plane
// p: A(p) the centre, B(p) the four in-plane faces (i-1, i+1, j-1, j+1), C(p)
// the four in-plane corners ((i-1,j-1), (i+1,j-1), (i-1,j+1), (i+1,j+1)),
// each a left fold in that order; the update of plane q-1 is
//   (7/64 ((B(q-1) + A(q-2)) + A(q)) + 3/128 ((C(q-1) + B(q-2)) + B(q)))
//     + 1/128 (C(q-2) + C(q)).
// The window moves along k like the 7-point one: a stage keeps, per cell,
// the folds started by planes q-1 and q-2 and the three sums of plane q-1.
// KR: the tile's column over planes [kb, ke) instead of its segment.
template <typename Real, int T, int R, int W, int PF, bool RHS, bool FLAGS, bool EDGE,
          bool WT = false, bool KREV = false, bool S27 = false, bool KR = false>
__device__ __forceinline__ void run_tile(const TripParams& p, const Geo& g, int tile,
                                         Real (*xch)[T][W][2][64], int kb = 0, int ke = 0)
{
    static_assert(!S27 || (!RHS && !FLAGS && !WT && !KREV && R >= 2),
                  "the 27-point update is built for plain A/B sweeps with R >= 2");
    constexpr int H = R * W;
    constexpr int OX = 64 - 2 * T;
    constexpr int OY = H - 2 * T;
    constexpr int NB = Xch<Real, T, W>::nbuf;
    // Issuing all of a step's edge-row reads right after the barrier (so
    // that their latency is paid once per step, not once per stage) holds 2T
    // more values; shapes whose stage state already fills the register
    // budget of their occupancy (256, 168, 128 VGPRs for 8, 12, 16 waves)
    // read per stage instead.  Compressed trips carry more state (progress
    // words; the mirrored view's extra plane).
    constexpr bool HOIST =
        !KREV && (S27 ? T * R <= 9
                      : T * R <= (W <= 8 ? 24 : W <= 12 ? (FLAGS ? 12 : 15) : 10));
    constexpr int NR = RHS ? 2 * T - 1 : 1;  // rhs planes held per row
    // Steps per unrolled chunk: PF, so that the prefetch slot of every step
    // is a compile-time constant (no register copies of loads in flight).
    constexpr int U = PF;
    const Real c6 = Sixth<Real>::v;
    const Real omega = (Real)p.omega;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const int tx = tile % g.tiles_x;
    const int rest = tile / g.tiles_x;
    const int ty = rest % g.tiles_y;
    const int seg = rest / g.tiles_y;

    const int i = tx * OX - T + lane;
    const int j0 = ty * OY - T + wave * R;
    const int k0 = KR ? kb : seg * g.seg_len;
    const int k1 = KR ? ke : min(k0 + g.seg_len, g.nz + 2);
    const int a = max(k0 - T, 0);
    const int b = min(k1 - 1 + T, g.nz + 1);
    // Stage s (1-based) completes plane a+n-2s+1 in step n; the last output
    // plane k1-1 of stage T is completed in step k1-a+2T-2.
    const int nsteps = k1 - a + 2 * T - 1;

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
        const int zsgn = KREV ? -1 : sgn;
        const int ntx = tx + ((d & 1) ? sgn : 0);
        const int nty = ty + ((d & 2) ? sgn : 0);
        const int nsg = seg + ((d & 4) ? zsgn : 0);
        if (ntx >= 0 && ntx < g.tiles_x && nty >= 0 && nty < g.tiles_y &&
            nsg >= 0 && nsg < g.segs)
            dep = (nsg * g.tiles_y + nty) * g.tiles_x + ntx;
    }
    int known = FLAGS ? 0 : kDone;
    // Dependee progress word loaded one step ahead (before that step's plane
    // loads), so reading it does not wait for the plane prefetch.
    int fl_ahead = 0;

    // X[s]: the plane stage s+1 consumes in this step (a plane of stage s,
    // produced by stage s in the previous step); X[T]: the plane stage T
    // completed.  P, C: per-stage k-streaming state (partial sum, and the
    // plane consumed in the previous step).
    // KREV: P holds the in-plane sum alone and D the plane before C.
    // S27: P holds the face fold B(q-1) + A(q-2) and C the centre A(q-1);
    // EP the edge fold C(q-1) + B(q-2), KP the corner sum C(q-2), BP and CP
    // the sums B(q-1) and C(q-1).
    constexpr int S27N = S27 ? T : 1;
    Real X[T + 1][R], P[T][R], C[T][R], D[KREV ? T : 1][R];
    Real EP[S27N][R], KP[S27N][R], BP[S27N][R], CP[S27N][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int s = 0; s <= T; ++s) X[s][r] = Real(0);
#pragma unroll
        for (int s = 0; s < T; ++s) {
            P[s][r] = Real(0);
            C[s][r] = Real(0);
            if (KREV) D[KREV ? s : 0][r] = Real(0);
        }
#pragma unroll
        for (int s = 0; s < S27N; ++s) {
            EP[s][r] = Real(0);
            KP[s][r] = Real(0);
            BP[s][r] = Real(0);
            CP[s][r] = Real(0);
        }
    }
    // rr[m]: rhs plane a+n-1-m; stage s+1 completes plane a+n-2s-1 and takes
    // rr[2s].
    float rr[NR][R];
#pragma unroll
    for (int m = 0; m < NR; ++m)
#pragma unroll
        for (int r = 0; r < R; ++r) rr[m][r] = 0.f;

    // Addressing: a per-plane buffer descriptor (scalar) plus a 32-bit
    // per-row byte offset that is loop invariant; src, dst and rhs frames
    // share the pitches.  Cells outside the box (edge tiles) load as 0 and
    // cells this tile does not own are not stored, through out-of-range
    // offsets.
    uint32_t voff[R], soff[R], roff[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t o =
            (uint32_t)(((int64_t)(j0 + r) * px + i) * (int64_t)sizeof(Real));
        voff[r] = (!EDGE || (lane_box && row_box[r])) ? o : kOob;
        soff[r] = (lane_out && row_out[r]) ? o : kOob;
        roff[r] = RHS ? voff[r] / (uint32_t)(sizeof(Real) / sizeof(float)) : 0u;
    }
    const int64_t plane_bytes = py * (int64_t)sizeof(Real);  // < 0 with KREV
    const uint32_t plane_b32 = (uint32_t)(plane_bytes < 0 ? -plane_bytes : plane_bytes);
    const char* src_b = reinterpret_cast<const char*>(src);
    const char* rhs_b = reinterpret_cast<const char*>(g.rhs);
    char* dst_b = reinterpret_cast<char*>(dst);
    const int64_t rplane_bytes = g.rpy * (int64_t)sizeof(float);

    // Register ring of the next PF input planes (and rhs planes): slot
    // n % PF holds plane a+n; its load is issued PF steps before use, so a
    // step does not wait for a full memory round trip.  Planes past b load
    // as 0.
    Real ring[PF][R];
    float rring[RHS ? PF : 1][R];
    auto load_plane = [&](const int q, Real(&dstv)[R]) {
        const Rsrc rs = make_rsrc(src_b + (int64_t)min(q, b) * plane_bytes,
                                  q <= b ? plane_b32 : 0u);
#pragma unroll
        for (int r = 0; r < R; ++r) dstv[r] = buf_load<Real>(rs, voff[r]);
    };
    auto load_rhs = [&](const int qr, float(&dstv)[R]) {
        const bool in = qr >= 1 && qr <= g.nz;
        const Rsrc rs = make_rsrc(rhs_b + (int64_t)(in ? qr : 1) * rplane_bytes,
                                  in ? (uint32_t)rplane_bytes : 0u);
#pragma unroll
        for (int r = 0; r < R; ++r) dstv[r] = buf_load<float>(rs, roff[r]);
    };
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        load_plane(a + d, ring[d]);
        if (RHS) load_rhs(a - 1 + d, rring[RHS ? d : 0]);  // stage 1, step d
    }

    // Store plane pe of the last stage (held in X[T]).  Called at the start
    // of the next step, so that a step's stage arithmetic is not split by the
    // conditional store.
    auto store_out = [&](const int pe) {
        const bool in = pe >= k0 && pe < k1;
        const Rsrc rd = make_rsrc(dst_b + (int64_t)(in ? pe : k0) * plane_bytes,
                                  in ? plane_b32 : 0u);
#pragma unroll
        for (int r = 0; r < R; ++r) buf_store(X[T][r], rd, soff[r]);
    };

    // One step: plane a+n enters stage 1, stage T completes plane a+n-2T+1.
    // BND: some stage may complete the boundary plane 0 or nz+1
    // (pass-through); only the first and last steps of a tile are such steps.
    auto step = [&](const int n, auto slot_tag, auto bnd_tag) {
        constexpr int sl = decltype(slot_tag)::value;
        constexpr bool BND = decltype(bnd_tag)::value;
        store_out(a + n - 2 * T);  // the plane the previous step completed
#pragma unroll
        for (int r = 0; r < R; ++r) X[0][r] = ring[sl][r];
        if (RHS) {
#pragma unroll
            for (int m = NR - 1; m > 0; --m)
#pragma unroll
                for (int r = 0; r < R; ++r) rr[m][r] = rr[m - 1][r];
#pragma unroll
            for (int r = 0; r < R; ++r) rr[0][r] = rring[RHS ? sl : 0][r];
        }
        load_plane(a + n + PF, ring[sl]);
        if (RHS) load_rhs(a + n + PF - 1, rring[RHS ? sl : 0]);

        // One exchange of the edge rows of every stage's input per step: a
        // stage consumes what the stage before it produced in the previous
        // step, so the T stages of a step are independent of each other.
        Real(*buf)[W][2][64] = xch[NB == 2 ? (n & 1) : 0];
        if (NB == 1) __syncthreads();  // previous step's reads are done
#pragma unroll
        for (int s = 0; s < T; ++s) {
            buf[s][wave][0][lane] = X[s][0];
            buf[s][wave][1][lane] = X[s][R - 1];
        }

        // Stage s+1 receives plane q = a+n-2s of stage s and completes plane
        // q-1 of row r from rows r-1, r, r+1 of X[s]: one update of Eq. (1)
        // in its fold order, with the k-streaming state of the row.
        auto update = [&](const int s, const int r, const Real above, const Real below) {
            const int pe = a + n - 2 * s - 1;
            const bool bnd = BND && ((pe == 0) || (pe == g.nz + 1));
            const Real xo = X[s][r];
            const Real inpl = ((from_left(xo) + from_right(xo)) + above) + below;
            Real e;
            if (bnd) {
                e = C[s][r];
            } else {
                Real sum = KREV ? (P[s][r] + xo) + D[KREV ? s : 0][r] : P[s][r] + xo;
                if (RHS) sum = sum + (Real)rr[RHS ? 2 * s : 0][r];
                e = sum * c6;
                if (WT) e = C[s][r] + omega * (e - C[s][r]);
                if (EDGE) e = (lane_int && row_int[r]) ? e : C[s][r];
            }
            if (KREV) {
                P[s][r] = inpl;
                D[KREV ? s : 0][r] = C[s][r];
            } else {
                P[s][r] = inpl + C[s][r];
            }
            C[s][r] = xo;
            return e;
        };

        // The outer neighbours of the edge rows: the last row of the wave
        // above and the first row of the wave below (after the barrier).
        // With HOIST all of the step's reads are issued at once, in the
        // order of use, by read_edges; edge_above / edge_below then return
        // them, else they read LDS per stage.
        Real upv[HOIST ? T : 1], dnv[HOIST ? T : 1];
        auto read_edges = [&]() {
            if constexpr (HOIST) {
#pragma unroll
                for (int s = T - 1; s >= 0; --s) {
                    upv[s] = buf[s][wave > 0 ? wave - 1 : 0][1][lane];
                    dnv[s] = buf[s][wave < W - 1 ? wave + 1 : W - 1][0][lane];
                }
            }
        };
        auto edge_above = [&](const int s) -> Real {
            if constexpr (HOIST) return upv[s];
            else return buf[s][wave > 0 ? wave - 1 : 0][1][lane];
        };
        auto edge_below = [&](const int s) -> Real {
            if constexpr (HOIST) return dnv[s];
            else return buf[s][wave < W - 1 ? wave + 1 : W - 1][0][lane];
        };

        // 27-point update of row r from the row above (j-1: its value and
        // the sum of its i-neighbours) and the row below (j+1: its i-1 and
        // i+1 neighbours), with hs the sum of row r's own i-neighbours.
        auto update27 = [&](const int s, const int r, const Real above, const Real habove,
                            const Real below, const Real lbelow, const Real rbelow,
                            const Real hs) {
            const int pe = a + n - 2 * s - 1;
            const bool bnd = BND && ((pe == 0) || (pe == g.nz + 1));
            const int s2 = S27 ? s : 0;
            const Real xo = X[s][r];
            const Real bq = (hs + above) + below;
            const Real cq = (habove + lbelow) + rbelow;
            Real e;
            if (bnd) {
                e = C[s][r];
            } else {
                const Real wf = Real(7) / Real(64), we = Real(3) / Real(128),
                           wc = Real(1) / Real(128);
                e = (wf * (P[s][r] + xo) + we * (EP[s2][r] + bq)) + wc * (KP[s2][r] + cq);
                if (EDGE) e = (lane_int && row_int[r]) ? e : C[s][r];
            }
            P[s][r] = bq + C[s][r];
            EP[s2][r] = cq + BP[s2][r];
            KP[s2][r] = CP[s2][r];
            C[s][r] = xo;
            BP[s2][r] = bq;
            CP[s2][r] = cq;
            return e;
        };

        if constexpr (S27) {
            // i-neighbours of every row of every stage's input (lane shifts),
            // then rows 1..R-2 before the barrier as below.
            Real LX[T][R], RX[T][R], HX[T][R];
            Real Y[T][R > 2 ? R - 2 : 1];
#pragma unroll
            for (int s = T - 1; s >= 0; --s) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    LX[s][r] = from_left(X[s][r]);
                    RX[s][r] = from_right(X[s][r]);
                    HX[s][r] = LX[s][r] + RX[s][r];
                }
#pragma unroll
                for (int r = 1; r + 1 < R; ++r)
                    Y[s][r - 1] = update27(s, r, X[s][r - 1], HX[s][r - 1], X[s][r + 1],
                                           LX[s][r + 1], RX[s][r + 1], HX[s][r]);
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
            read_edges();
#pragma unroll
            for (int s = T - 1; s >= 0; --s) {
                const Real up = edge_above(s);
                const Real dn = edge_below(s);
                const Real hup = from_left(up) + from_right(up);
                const Real e0 = update27(s, 0, up, hup, X[s][1], LX[s][1], RX[s][1], HX[s][0]);
                const Real e1 = update27(s, R - 1, X[s][R - 2], HX[s][R - 2], dn,
                                         from_left(dn), from_right(dn), HX[s][R - 1]);
                X[s + 1][0] = e0;
                X[s + 1][R - 1] = e1;
#pragma unroll
                for (int r = 1; r + 1 < R; ++r) X[s + 1][r] = Y[s][r - 1];
                __builtin_amdgcn_sched_barrier(0);
            }
            return;
        }

        // Rows 1..R-2 of every stage need nothing from the other waves:
        // computed before the barrier (into Y, since X[s] rows are still read
        // by the edge rows after it).  Descending s, so that X[s+1] is
        // overwritten only after stage s+2 has read it.
        Real Y[T][R > 2 ? R - 2 : 1];
#pragma unroll
        for (int s = T - 1; s >= 0; --s) {
#pragma unroll
            for (int r = 1; r + 1 < R; ++r)
                Y[s][r - 1] = update(s, r, X[s][r - 1], X[s][r + 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
        // Rows 0 and R-1 take their outer neighbours from the waves above
        // and below.
        read_edges();
#pragma unroll
        for (int s = T - 1; s >= 0; --s) {
            const Real up = edge_above(s);
            const Real dn = edge_below(s);
            const Real e0 = update(s, 0, up, R > 1 ? X[s][R > 1 ? 1 : 0] : dn);
            const Real e1 = R > 1 ? update(s, R - 1, X[s][R > 1 ? R - 2 : 0], dn) : e0;
            X[s + 1][0] = e0;
            X[s + 1][R - 1] = e1;
#pragma unroll
            for (int r = 1; r + 1 < R; ++r) X[s + 1][r] = Y[s][r - 1];
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // Compressed grid: before a chunk of U steps, publish this tile's
    // progress and wait until the dependees have consumed every storage plane
    // the chunk's stores overwrite.  Done once per chunk, so that the steps
    // themselves stay straight-line code.  The dependees' words are read one
    // chunk ahead, and only while what the tile knows does not already cover
    // the next chunk's stores (each read goes past the L2 to memory shared by
    // all XCDs).  Publishing less often measured slower: dependents wait.
    auto need_of = [&](const int n0) {
        // Stores of the chunk from n0 (and the one after its last step):
        // planes up to a+n0+U-2T of the output, i.e. this storage plane in
        // input-frame terms (planes outside the box are shift room nobody
        // reads).  <= 0: nothing to wait for.
        const int pe_hi = min(a + n0 + U - 2 * T, k1 - 1);
        if (pe_hi < k0) return 0;
        return min(p.dir > 0 || KREV ? pe_hi - p.zshift : pe_hi + p.zshift, g.nz + 1) + 1;
    };
    auto sync_chunk = [&](const int n0) {
        if (n0 > 0 && threadIdx.x == 0) {
            // all waves passed the barrier of step n0-1: planes up to
            // a+n0-2 are consumed
            flag_store(p.flags + (int64_t)tile * kFlagStride, a + n0 - 1);
        }
        const int need = need_of(n0);
        if (need > 0 && known < need) {
            int v0 = fl_ahead;
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) v0 = min(v0, __shfl_xor(v0, o, 64));
            known = max(known, __builtin_amdgcn_readfirstlane(v0));
        }
        if (__builtin_expect(need > 0 && known < need, 0))
            known = wait_progress(p.flags, dep, need, p.spin_limit, p.err);
        // Read ahead, before the chunk's plane loads.  A skipped read leaves
        // `known` (never more than the dependees' true progress).
        if (known < need_of(n0 + U))
            fl_ahead = dep >= 0 ? flag_load(p.flags + (int64_t)dep * kFlagStride) : kDone;
        else
            fl_ahead = dep >= 0 ? known : kDone;
        // The chunk's stores must follow the reads of the progress words.
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };

    // U consecutive steps from n0 (a multiple of U).
    auto chunk = [&](const int n0, auto bnd_tag) {
        if (FLAGS) {
            sync_chunk(n0);
        } else {
            // A fence at every chunk boundary (no instruction at workgroup
            // scope) keeps the compiler from moving memory operations between
            // chunks; without it the unrolled steps are interleaved and the
            // stage state spills.
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        static_for<U>([&](auto u) {
            constexpr int k = decltype(u)::value;
            step(n0 + k, std::integral_constant<int, (k % PF)>{}, bnd_tag);
        });
    };
    // Steps before `head` and from `tail` on may touch a boundary plane.  The
    // last chunk may run up to U-1 steps past nsteps: they load and store
    // nothing.
    const int head = min(nsteps, max(0, 2 * T - a));
    const int tail = max(head, min(nsteps, g.nz + 2 - a));
    int n = 0;
    for (; n < head; n += U) chunk(n, std::true_type{});
    for (; n + U <= tail; n += U) chunk(n, std::false_type{});
    for (; n < nsteps; n += U) chunk(n, std::true_type{});
    store_out(a + n - 2 * T);
    if (FLAGS) {
        __syncthreads();
        if (threadIdx.x == 0) flag_store(p.flags + (int64_t)tile * kFlagStride, kDone);
    }
}

// Teams (MODE 3): team r applies trip r of the launch.  Before tile `tile`
// of team r starts, the tiles whose outputs its input region reads (its
// neighbours within one tile in i, j and k, itself included) must have
// finished team r-1 -- the safety half of Eq. (3), on per-tile counters of
// completed teams -- and, with looseness d_u >= 0, every tile must have
// finished team r-d_u-1 (a team runs at most d_u trips ahead of the slowest
// tile; d_u = 0 is lockstep, a barrier between trips inside the kernel).
// Every wave waits itself and then acquires at agent scope, so the planes
// other workgroups wrote (possibly on another XCD) are read from memory.
// The bounded spin raises the error word instead of hanging.
__device__ __attribute__((noinline)) void wait_team(const int* flags, const int* done,
                                                    int* err, int tiles_x, int tiles_y,
                                                    int segs, int ntiles, int looseness,
                                                    long long spin_limit, int tile, int team)
{
    const int lane = threadIdx.x & 63;
    const int tx = tile % tiles_x;
    const int ty = (tile / tiles_x) % tiles_y;
    const int sg = tile / (tiles_x * tiles_y);
    const int* word = nullptr;
    int need = 0;
    if (lane < 27) {
        const int nx = tx + lane % 3 - 1, ny = ty + (lane / 3) % 3 - 1,
                  ns = sg + lane / 9 - 1;
        if (nx >= 0 && nx < tiles_x && ny >= 0 && ny < tiles_y && ns >= 0 && ns < segs) {
            word = flags + (int64_t)((ns * tiles_y + ny) * tiles_x + nx) * kFlagStride;
            need = team;
        }
    } else if (lane == 27 && looseness >= 0 && team - looseness - 1 >= 0) {
        word = done + (int64_t)(team - looseness - 1) * kFlagStride;
        need = ntiles;
    }
    int64_t spins = 0;
    for (;;) {
        const bool ok = !word || flag_load(word) >= need;
        if (__all(ok)) break;
        if (++spins > spin_limit || flag_load(err) != 0) {
            if (lane == 0) atomicCAS(err, 0, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Publishes "tile finished team": every wave releases its stores at agent
// scope, then one thread raises the tile's counter and the team's count.
__device__ __forceinline__ void finish_team(const TripParams& p, int tile, int team)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        flag_store(p.flags + (int64_t)tile * kFlagStride, team + 1);
        __hip_atomic_fetch_add(p.done + (int64_t)team * kFlagStride, 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// MODE 0: one problem, tile = f(blockIdx) (A/B; kernel boundary between
//         trips is the only synchronization).
// MODE 1: one problem, tiles from a ticket counter or per-XCD claim groups,
//         progress flags (compressed single grid); KREV: a backward trip in
//         the k-mirrored view.
// MODE 2: a batch of independent problems described by p.table; tiles of all
//         problems from one ticket counter; A/B parity read from *p.parity.
// MODE 3: one problem, p.teams trips in one persistent launch (A/B): work
//         items (team, tile) from one ticket counter in team-major order,
//         so every item an item waits for has a smaller ticket (no
//         deadlock, whatever number of workgroups is resident).
// MODE 4: one problem (A/B), the tail of a trip whose first columns ran
//         whole in a MODE 0 launch: p.groups columns from column p.chunk on,
//         in segments of p.seg_len planes, one tile per workgroup.
template <typename Real, int T, int R, int W, int PF, bool RHS, int MODE, bool WT = false,
          bool KREV = false, bool S27 = false>
__global__ __launch_bounds__(64 * W) void trip_kernel(TripParams p)
{
    constexpr bool FLAGS = MODE == 1;
    constexpr int H = R * W;
    constexpr int OX = 64 - 2 * T;
    constexpr int OY = H - 2 * T;
    __shared__ Real xch[Xch<Real, T, W>::nbuf][T][W][2][64];
    __shared__ int tile_sh;

    for (int iter = 0;; ++iter) {
        int tile;
        int team = 0;
        int kb = 0, ke = 0;  // MODE 4: the tile's planes
        if (MODE == 0) {
            if (iter > 0) return;
            tile = p.chunk > 0 ? band_tile(blockIdx.x, p.ntiles) : xcd_tile(blockIdx.x, p.ntiles);
        } else if (MODE == 4) {
            if (iter > 0) return;
            const int local = xcd_tile(blockIdx.x, p.ntiles);
            const int sg = local / p.groups;
            tile = p.chunk + (local - sg * p.groups);
            kb = sg * p.seg_len;
            ke = min(kb + p.seg_len, p.nz + 2);
        } else {
            __syncthreads();  // previous tile finished with tile_sh and xch
            if (threadIdx.x == 0)
                tile_sh = MODE == 1 && p.groups > 1
                              ? claim_grouped(p.gcnt, blockIdx.x & 7, p.chunk, p.ntiles)
                              : atomicAdd(p.ticket, 1);
            __syncthreads();
            // Uniform across the workgroup: read it into a scalar register,
            // so that the per-plane buffer descriptors built from it stay
            // scalar (otherwise every buffer access becomes a waterfall loop
            // over the lanes).
            const int t = __builtin_amdgcn_readfirstlane(tile_sh);
            if (MODE == 3) {
                if (t >= p.ntiles * p.teams) return;
                team = t / p.ntiles;
                tile = t - team * p.ntiles;
            } else {
                if (t >= p.ntiles) return;
                tile = t;
                if (MODE == 1 && p.dir < 0) {
                    // mirrored order: all axes, or i and j only in the
                    // k-mirrored view (whose k already runs backwards)
                    const int pl = p.tiles_x * p.tiles_y;
                    tile = KREV ? (t / pl) * pl + (pl - 1 - t % pl) : p.ntiles - 1 - t;
                }
            }
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
            const int par = __builtin_amdgcn_readfirstlane(*p.parity) & 1;
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
            // MODE 3: odd teams read the grid even teams write
            const bool swap = MODE == 3 && (team & 1);
            g.src = swap ? p.dst : p.src;
            g.dst = swap ? const_cast<void*>(p.src) : p.dst;
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
        if (MODE == 3 && team > 0)
            wait_team(p.flags, p.done, p.err, p.tiles_x, p.tiles_y, p.segs, p.ntiles,
                      p.looseness, p.spin_limit, tile, team);
        if constexpr (MODE == 4) {
            if (interior_tile)
                run_tile<Real, T, R, W, PF, RHS, FLAGS, false, WT, KREV, S27, true>(p, g, tile,
                                                                                     xch, kb, ke);
            else
                run_tile<Real, T, R, W, PF, RHS, FLAGS, true, WT, KREV, S27, true>(p, g, tile,
                                                                                    xch, kb, ke);
        } else if (interior_tile) {
            run_tile<Real, T, R, W, PF, RHS, FLAGS, false, WT, KREV, S27>(p, g, tile, xch);
        } else {
            run_tile<Real, T, R, W, PF, RHS, FLAGS, true, WT, KREV, S27>(p, g, tile, xch);
        }
        if (MODE == 3) finish_team(p, tile, team);
    }
}

// Launches one trip in MODE with tile shape (T, R, W).
template <typename Real, int T, int R, int W, int PF, bool RHS, int MODE, bool WT = false,
          bool KREV = false, bool S27 = false>
hipError_t launch_mode(const TripParams& p, hipStream_t s)
{
    const dim3 block(64 * W);
    if constexpr (MODE == 0 || MODE == 4) {
        hipLaunchKernelGGL((trip_kernel<Real, T, R, W, PF, RHS, MODE, WT, false, S27>),
                           dim3(p.ntiles), block, 0, s, p);
        return hipGetLastError();
    }
    // Persistent launch: as many workgroups as can be resident.
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu,
            reinterpret_cast<const void*>(&trip_kernel<Real, T, R, W, PF, RHS, MODE, WT, KREV, S27>),
            64 * W, 0);
    if (e != hipSuccess) return e;
    int grid = cus * (per_cu > 0 ? per_cu : 1);
    const int64_t items = MODE == 3 ? (int64_t)p.ntiles * p.teams : p.ntiles;
    if (grid > items) grid = (int)items;
    TripParams q = p;
    // Per-XCD claim groups need a workgroup in every group; a chunk is the
    // tiles one XCD holds at a time (0: one workgroup per tile).
    if (MODE == 1 && q.groups > 1) {
        if (grid < kClaimGroups)
            q.groups = 1;
        else
            q.chunk = grid >= items ? 0 : grid / kClaimGroups;
    }
    hipLaunchKernelGGL((trip_kernel<Real, T, R, W, PF, RHS, MODE, WT, KREV, S27>), dim3(grid),
                       block, 0, s, q);
    return hipGetLastError();
}

// Launches the compiled tile shape `c` of one precision, rhs flag and mode.
template <typename Real, bool RHS, int MODE, bool WT = false, bool KREV = false>
hipError_t dispatch_unit(const TripConfig& c, const TripParams& p, hipStream_t s)
{
#define JACOBI_CASE(T_, R_, W_)                     \
    if (c.T == T_ && c.R == R_ && c.W == W_)        \
        return launch_mode<Real, T_, R_, W_, kPrefetch, RHS, MODE, WT, KREV>(p, s);
    JACOBI_TRIP_CFGS(JACOBI_CASE)
#undef JACOBI_CASE
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace jacobi_impl
