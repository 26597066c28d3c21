// Host runtime of libjacobi: descriptor validation, trip planning (how many
// sweeps each launch fuses, tile shape, k segments), the compressed-grid
// shift bookkeeping and the C-ABI entry points declared in include/jacobi.h.
//
// The paper's team sweep (Sect. 2.1) becomes one "trip": a launch that applies
// t sweeps to the whole box with one read and one write of the grid.  n sweeps
// are split into floor(n/t) trips of t plus one shorter trip; since every trip
// computes exactly the plain sweeps, the split does not change a single bit.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "jacobi.h"
#include "internal.h"
#include "runtime_common.h"

using namespace jacobi_impl;

namespace jacobi_impl {

namespace {
thread_local std::string g_err;
}

const char* last_error_text() { return g_err.c_str(); }

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(JACOBI_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Tile shape (rows per wave, waves) per T: the fastest shape measured on a
// 512^3 FP64 box.  The compressed grid's persistent tiles are fastest with 4
// rows x 8 waves at every T.
TripConfig default_cfg(int T, bool compressed, bool s27)
{
    if (s27) {
        switch (T) {
        case 1: return TripConfig{1, 4, 8};
        case 2: return TripConfig{2, 3, 12};
        case 3: return TripConfig{3, 3, 8};
        default: return TripConfig{T, 3, 8};
        }
    }
    if (compressed) return TripConfig{T, 4, 8};
    switch (T) {
    case 1:
    case 2: return TripConfig{T, 4, 16};
    case 3: return TripConfig{T, 4, 12};
    case 4:
    case 6: return TripConfig{T, 3, 12};
    default: return TripConfig{T, 4, 8};
    }
}

bool make_plan(int64_t nx, int64_t ny, int64_t nz, const TripConfig& cfg,
               int seg_req, bool compressed, int target_tiles, Plan* out, int min_seg)
{
    const int T = cfg.T;
    const int OX = 64 - 2 * T;
    const int OY = cfg.R * cfg.W - 2 * T;
    const int need = compressed ? 2 * T : 1;
    if (OX < need || OY < need) return false;
    Plan p;
    p.cfg = cfg;
    p.tiles_x = (int)((nx + 2 + OX - 1) / OX);
    p.tiles_y = (int)((ny + 2 + OY - 1) / OY);
    const int64_t nz2 = nz + 2;
    const int64_t plane_tiles = (int64_t)p.tiles_x * p.tiles_y;
    if (seg_req > 0) {
        if (compressed && seg_req < std::max(2 * T, min_seg)) return false;
        p.seg_len = (int)std::min<int64_t>(seg_req, nz2);
    } else {
        // Minimise (rounds of concurrent tiles) x (steps of one tile): a tile
        // of a segment of len planes takes len + 3T - 1 steps (T ghost planes
        // on each side, and stage T runs 2T-1 steps behind stage 1).
        const int conc = target_tiles > 0 ? target_tiles : kCUs;
        double best = 1e300;
        int best_len = (int)nz2;
        const int min_len = std::max(compressed ? std::max(2 * T, min_seg) : 1, 4 * T);
        for (int64_t segs = 1; segs <= 256; ++segs) {
            const int64_t len = (nz2 + segs - 1) / segs;
            if (len < min_len && segs > 1) break;
            const int64_t real_segs = (nz2 + len - 1) / len;
            const int64_t tiles = plane_tiles * real_segs;
            const int64_t rounds = (tiles + conc - 1) / conc;
            const double cost = (double)rounds * (double)(len + 3 * T);
            if (cost < best * 0.999) {
                best = cost;
                best_len = (int)len;
            }
        }
        p.seg_len = best_len;
    }
    p.segs = (int)((nz2 + p.seg_len - 1) / p.seg_len);
    const int64_t nt = plane_tiles * p.segs;
    if (nt > (1 << 30)) return false;
    p.ntiles = (int)nt;
    *out = p;
    return true;
}

}  // namespace jacobi_impl

struct jacobi_s {
    jacobi_desc d{};
    int t = 4;
    int64_t px = 0, py = 0;  // storage pitches of the FP64 grid(s)
    int room = 0;            // compressed: shift room in i and j (2t)
    int off = 0;             // compressed: current origin offset in i and j
    int zextra = 0;          // compressed: extra k shift per trip (E)
    int roomz = 0;           // compressed: shift room in k (2t + 2E)
    int offz = 0;            // compressed: current origin offset in k
    int cur = 0;             // AB: grid holding the current iterate
    hipStream_t stream = nullptr;
    int tile_rows = 0, rpw = 0, seg_req = 0;
    int inner = 32;
    int64_t sweeps = 0;
    int64_t spin_limit = 1 << 25;
    Plan plans[9];           // plans[T] for T = 1..t
    // t = 0 (A/B FP64): candidates are timed on the first jacobi_sweep call
    // with enough sweeps; until then trips use the default t.
    bool tune_pending = false;
    double tune_ms = 0;
    struct TuneEntry {
        TripConfig cfg;
        double glups;
    };
    std::vector<TuneEntry> tune_log;
    // workspace carve-up
    char* ws = nullptr;
    int* ticket = nullptr;
    int* err = nullptr;
    int* scale_exp = nullptr;
    double* red_out = nullptr;
    double* partials = nullptr;
    int* gcnt = nullptr;     // claim-group counters (compressed trips)
    int* flags = nullptr;
    int64_t flag_ints = 0;
    // compressed trips claim tiles in per-XCD groups; JACOBI_XCD_ORDER=0
    // falls back to one ticket counter
    bool xcd_order = true;
    bool krev = false;  // backward compressed trips use the k-mirrored view
    // A/B trips of several generations of workgroups take tiles in band
    // order (each generation one band of 256 consecutive tiles, 32 per XCD);
    // JACOBI_AB_BANDS=0 gives every XCD one contiguous range instead
    bool ab_bands = true;
    int* done = nullptr;     // per-team finished-tile counts (teams >= 2)
    float* e[2] = {nullptr, nullptr};
    float* rhs = nullptr;
    // multigrid levels (level 0 = e, rhs above)
    struct MgLevel {
        int n;
        float* e[2];
        float* rhs;
        Plan plan;  // FP32 trips of kMgT sweeps on this level
    };
    std::vector<MgLevel> mg;
    AuxProblem aux{};         // residual / refinement view of this problem
    // A/B FP64 graph replay (use_graph): trips are captured on `cap` once per
    // (sweep count, starting grid) and replayed on `stream`.
    hipStream_t run = nullptr;  // stream trip launches go to (stream or cap)
    hipStream_t cap = nullptr;
    struct Replay {
        int64_t n;
        int cur0, cur1;
        hipGraphExec_t exec;
    };
    std::vector<Replay> replays;
    ~jacobi_s()
    {
        for (Replay& r : replays) hipGraphExecDestroy(r.exec);
        if (cap) hipStreamDestroy(cap);
    }
};

namespace {

struct Layout {
    size_t partials_off, flags_off, done_off, e0_off, e1_off, rhs_off, total;
    int64_t flag_ints;
    std::vector<size_t> mg_off;  // multigrid levels 1.. : e0, e1, rhs
};

// Multigrid correction solve (JACOBI_F32_MULTIGRID): V(kMgNu, kMgNu) cycles
// of weighted FP32 sweeps (weight 6/7) down to an interior of at most
// kMgCoarsest cells per axis, where kMgCoarse sweeps are made.
constexpr int kMgT = 2;
constexpr int kMgNu = 2;
constexpr int kMgCoarse = 32;
constexpr int kMgCoarsest = 3;
constexpr float kMgOmega = 6.0f / 7.0f;

bool mg_levels_ok(int64_t n) { return n >= 1 && ((n + 1) & n) == 0; }

// Autotuner of single A/B FP64 handles created with t = 0: (T, rows per
// wave, waves) candidates, each timed on one warm-up and two timed trips of
// real sweeps; the default until the tuning has run is kTuneDefaultT.
const TripConfig kTuneCandidates[] = {
    {3, 4, 12}, {4, 3, 12}, {4, 4, 8}, {5, 4, 8}, {5, 3, 12}, {6, 3, 12},
};
constexpr int kTuneMaxT = 6;
constexpr int64_t kTuneSweeps = 96;  // >= 3 trips of every candidate
constexpr int kTuneDefaultT = 5;

constexpr int kMaxTeams = 1024;
// 27-point handles: the largest t compiled, the autotuner's candidates and
// the t used until the tuning has run.
constexpr int kS27MaxT = 4;
const TripConfig kS27TuneCandidates[] = {{2, 3, 12}, {2, 4, 8}, {3, 3, 8}, {4, 3, 8}};
constexpr int kS27DefaultT = 2;

struct Candidates {
    const TripConfig* c;
    int n;
};
Candidates tune_candidates(bool s27)
{
    if (s27)
        return {kS27TuneCandidates, (int)(sizeof kS27TuneCandidates / sizeof(TripConfig))};
    return {kTuneCandidates, (int)(sizeof kTuneCandidates / sizeof(TripConfig))};
}
bool config_supported(bool s27, const TripConfig& c)
{
    return s27 ? trip_config_supported_s27(c) : trip_config_supported(0, c);
}

// Extra shift along k of a compressed trip (planes).  A forward trip of L
// sweeps stores its result shifted by (-L, -L, -L-E) (a backward trip by
// (+L, +L, +L+E)): a tile then overwrites a storage plane 3L+E steps after
// the tiles it shares it with started reading it, instead of 3L, which lets
// tiles that started a little later than their neighbours run without
// waiting.  A segment of the k split must hold 2L+E planes, so an explicit
// segment length caps E.
// Backward compressed trips stream k downwards (a k-mirrored view of the
// grid) for t <= kKrevMaxT; the mirrored kernel holds one more plane per
// stage, which no longer fits in registers for larger t.  JACOBI_KREV=0
// streams them upwards like forward trips.
constexpr int kKrevMaxT = 5;
bool compressed_krev(int t)
{
    if (const char* s = std::getenv("JACOBI_KREV"))
        if (std::atoi(s) == 0) return false;
    return t <= kKrevMaxT;
}

int compressed_zextra(const jacobi_desc* d, int t)
{
    // a trip streaming upwards with a +k shift stores ahead of its stream:
    // no extra shift unless every backward trip is mirrored
    if (!compressed_krev(t)) return 0;
    int E = 2 * t;
    if (const char* s = std::getenv("JACOBI_ZEXTRA")) E = std::max(0, std::atoi(s));
    if (d->seg_len > 0) E = std::max(0, std::min(E, d->seg_len - 2 * t));
    return E;
}

// Alternative A/B FP64 tile shape for T = 5, and the planning cost of a trip:
// rounds of concurrent tiles (one workgroup per CU) x steps of one tile x
// tile rows.
constexpr TripConfig kAltCfg5{5, 3, 12};
double plan_cost(const Plan& p)
{
    const int T = p.cfg.T;
    const int64_t rounds = (p.ntiles + kCUs - 1) / kCUs;
    return (double)rounds * (p.seg_len + 3 * T) * (p.cfg.R * p.cfg.W);
}

// Split trips for the 27-point update (A/B).  A box whose tile columns are a
// few more than a multiple of the CU count leaves most CUs idle in the last
// round of equal segments (512^3, T = 3: 261 columns x 7 segments, 7.1
// rounds that take 8).  Instead the first multiple-of-kCUs columns run whole
// (all tiles of a round at the same k, so neighbouring columns share their
// ghost cells in L2), and the few columns left run in one more launch, cut
// into short segments that make about one round.  The step model below
// overstates the gain (whole columns run a little slower per step than short
// segments): measured, 512^3 T = 3 (model -18 %) ran 6.6 % faster, 1024^3
// T = 3 (-7.6 %) 1.2 % slower and 512^3 T = 4 (-3.5 %) 5.6 % slower, so it
// is taken only below 0.85 of the segments' cost.  JACOBI_KSPLIT=0 turns it
// off; JACOBI_KSPLIT=n > 0 forces it with rounds of n columns (tests).
void split_tail(Plan* p, int64_t nz)
{
    p->tail_cols = p->tail_len = p->tail_tiles = 0;
    int round = kCUs;
    bool force = false;
    if (const char* e = std::getenv("JACOBI_KSPLIT")) {
        round = std::atoi(e);
        if (round <= 0) return;
        force = true;
    }
    const int T = p->cfg.T;
    const int64_t nz2 = nz + 2;
    const int64_t cols = (int64_t)p->tiles_x * p->tiles_y;
    const int64_t full = cols / round * round, tail = cols - full;
    if (full == 0 || tail == 0) return;
    const int64_t per_col = std::max<int64_t>(1, round / tail);  // segments per tail column
    const int64_t len = std::max<int64_t>((nz2 + per_col - 1) / per_col, 2 * T);
    const int64_t tsegs = (nz2 + len - 1) / len;
    const double cost_split = (double)(full / round) * (nz2 + 3 * T) +
                              (double)((tail * tsegs + round - 1) / round) * (len + 3 * T);
    const double cost_seg = (double)((p->ntiles + kCUs - 1) / kCUs) * (p->seg_len + 3 * T);
    if (!force && !(cost_split < 0.85 * cost_seg)) return;
    p->seg_len = (int)nz2;
    p->segs = 1;
    p->ntiles = (int)full;
    p->tail_cols = (int)tail;
    p->tail_len = (int)len;
    p->tail_tiles = (int)(tail * tsegs);
}

int validate_and_plan(const jacobi_desc* d, Plan* plans, int* t_out,
                      Layout* lay)
{
    if (!d) return fail(JACOBI_EINVAL, "null descriptor");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(JACOBI_EINVAL, "interior dims must be >= 1 (got %lld %lld %lld)",
                    (long long)d->nx, (long long)d->ny, (long long)d->nz);
    if (d->nx > 65536 || d->ny > 65536 || d->nz > 65536)
        return fail(JACOBI_EINVAL, "interior dims must be <= 65536");
    if (d->dtype != JACOBI_F64 && d->dtype != JACOBI_F32_REFINED &&
        d->dtype != JACOBI_F32_MULTIGRID)
        return fail(JACOBI_EINVAL, "unknown dtype %d", d->dtype);
    const bool mg = d->dtype == JACOBI_F32_MULTIGRID;
    if (mg && (d->layout != JACOBI_LAYOUT_AB || d->nx != d->ny || d->nx != d->nz ||
               !mg_levels_ok(d->nx) || d->teams > 1))
        return fail(JACOBI_EUNSUPPORTED,
                    "the multigrid correction needs the AB layout and an n^3 interior with "
                    "n = 2^k - 1 (got %lld x %lld x %lld)",
                    (long long)d->nx, (long long)d->ny, (long long)d->nz);
    if (d->layout != JACOBI_LAYOUT_AB && d->layout != JACOBI_LAYOUT_COMPRESSED)
        return fail(JACOBI_EINVAL, "unknown layout %d", d->layout);
    if (d->stencil != 0 && d->stencil != 7 && d->stencil != 27)
        return fail(JACOBI_EINVAL, "stencil must be 0, 7 or 27 (got %d)", d->stencil);
    const bool s27 = d->stencil == 27;
    if (s27 && (d->dtype != JACOBI_F64 || d->layout != JACOBI_LAYOUT_AB || d->teams > 1))
        return fail(JACOBI_EUNSUPPORTED,
                    "the 27-point update needs FP64, the AB layout and teams <= 1");
    const bool tune = d->t == 0 && d->layout == JACOBI_LAYOUT_AB && d->dtype == JACOBI_F64 &&
                      d->tile_rows == 0 && d->rows_per_wave == 0 && d->seg_len == 0;
    const int t = mg                ? kMgT
                  : d->t != 0       ? d->t
                  : tune            ? (s27 ? kS27MaxT : kTuneMaxT)
                  : s27             ? kS27DefaultT
                                    : 4;
    if (t < 1 || t > (s27 ? kS27MaxT : 8))
        return fail(JACOBI_EUNSUPPORTED, "sweeps per trip t=%d not supported (1..%d)", t,
                    s27 ? kS27MaxT : 8);
    if (d->inner_sweeps < 0) return fail(JACOBI_EINVAL, "inner_sweeps < 0");
    if (d->teams < 0 || d->teams > kMaxTeams)
        return fail(JACOBI_EINVAL, "teams must be in 0..%d", kMaxTeams);
    if (d->teams > 1 && (d->layout != JACOBI_LAYOUT_AB || d->dtype != JACOBI_F64))
        return fail(JACOBI_EUNSUPPORTED,
                    "several trips per launch (teams >= 2) need the AB layout and FP64");
    if (d->seg_len < 0) return fail(JACOBI_EINVAL, "seg_len < 0");
    const bool comp = d->layout == JACOBI_LAYOUT_COMPRESSED;
    const int room = comp ? 2 * t : 0;
    const int zextra = comp ? compressed_zextra(d, t) : 0;
    const int64_t plane_bytes = (d->nx + 2 + room) * (d->ny + 2 + room) * 8;
    if (plane_bytes >= ((int64_t)1 << 31))
        return fail(JACOBI_EINVAL, "one k-plane must be < 2 GiB");
    int64_t max_tiles = 0;
    for (int T = 1; T <= t; ++T) {
        TripConfig cfg = default_cfg(T, comp, s27);
        const bool shape_given = T == t && !mg && (d->tile_rows > 0 || d->rows_per_wave > 0);
        if (shape_given) {
            const int R = d->rows_per_wave > 0 ? d->rows_per_wave : 4;
            const int rows = d->tile_rows > 0 ? d->tile_rows : cfg.R * cfg.W;
            if (rows % R != 0)
                return fail(JACOBI_EINVAL, "tile_rows must be a multiple of rows_per_wave");
            cfg = TripConfig{T, R, rows / R};
        }
        if (s27 ? !trip_config_supported_s27(cfg)
                : !trip_config_supported(d->dtype != JACOBI_F64, cfg))
            return fail(JACOBI_EUNSUPPORTED,
                        "tile shape t=%d rows=%d rows_per_wave=%d is not compiled",
                        T, cfg.R * cfg.W, cfg.R);
        if (!make_plan(d->nx, d->ny, d->nz, cfg, T == t ? d->seg_len : 0, comp,
                       kCUs, &plans[T], comp ? 2 * T + zextra : 0))
            return fail(JACOBI_EUNSUPPORTED,
                        "tile shape t=%d rows=%d cannot cover this box%s", T,
                        cfg.R * cfg.W,
                        comp ? " (compressed needs tiles and segments >= 2t)" : "");
        // Dense trips of T = 5 (A/B FP64, and the FP32 correction trips,
        // which run on dense grids whatever the FP64 layout): the 3x12 tile
        // (three waves per SIMD) costs per row and step what the 4x8 tile
        // (two waves) does, so the shape with fewer rounds x steps x rows
        // wins (4x8 at 512^3: one generation of 240 tiles; 3x12 at 1024^3:
        // 3 rounds of one 1026-plane segment against 7 of two).
        const bool dense_trips = (d->dtype == JACOBI_F64 && !comp) ||
                                 d->dtype == JACOBI_F32_REFINED;
        if (T == 5 && !shape_given && !s27 && !mg && dense_trips) {
            Plan alt;
            if (make_plan(d->nx, d->ny, d->nz, kAltCfg5, T == t ? d->seg_len : 0, comp, kCUs,
                          &alt, comp ? 2 * T + zextra : 0) &&
                plan_cost(alt) < plan_cost(plans[T]))
                plans[T] = alt;
        }
        if (s27 && (T == t ? d->seg_len : 0) == 0) split_tail(&plans[T], d->nz);
        max_tiles = std::max<int64_t>(max_tiles, plans[T].ntiles);
    }
    if (tune) {
        const Candidates cs = tune_candidates(s27);
        for (int q = 0; q < cs.n; ++q) {
            const TripConfig& c = cs.c[q];
            Plan pl;
            if (config_supported(s27, c) &&
                make_plan(d->nx, d->ny, d->nz, c, 0, false, kCUs, &pl))
                max_tiles = std::max<int64_t>(max_tiles, pl.ntiles);
        }
    }
    *t_out = t;
    Layout L{};
    AuxProblem ap{};
    ap.nx = (int)d->nx;
    ap.ny = (int)d->ny;
    ap.nz = (int)d->nz;
    const int nb = residual_plan(&ap);
    L.partials_off = 256;
    L.flags_off = (size_t)round_up(L.partials_off + 2 * (int64_t)nb * sizeof(double), 256);
    const bool teams = d->teams > 1;
    // claim-group counters, then one progress word per tile
    L.flag_ints = (comp || teams) ? (max_tiles + kClaimGroups) * kFlagStride : 0;
    L.done_off = (size_t)round_up(L.flags_off + L.flag_ints * sizeof(int), 256);
    size_t end = L.done_off + (teams ? (size_t)d->teams * kFlagStride * sizeof(int) : 0);
    L.e0_off = L.e1_off = L.rhs_off = 0;
    L.mg_off.clear();
    if (d->dtype != JACOBI_F64) {
        const int64_t box = (d->nx + 2) * (d->ny + 2) * (d->nz + 2);
        const size_t fb = (size_t)round_up(box * (int64_t)sizeof(float), 256);
        L.e0_off = end;
        L.e1_off = end + fb;
        L.rhs_off = end + 2 * fb;
        end += 3 * fb;
    }
    if (mg) {
        // coarser levels: e0, e1, rhs boxes each
        for (int64_t n = (d->nx - 1) / 2; n >= 1; n = (n - 1) / 2) {
            const size_t fb = (size_t)round_up((n + 2) * (n + 2) * (n + 2) * 4, 256);
            L.mg_off.push_back(end);
            end += 3 * fb;
            if (n <= kMgCoarsest) break;
        }
    }
    L.total = end;
    *lay = L;
    return JACOBI_OK;
}

hipError_t launch_trip(jacobi_t* h, int T, bool f32, const void* src, void* dst,
                       const float* rhs, int64_t px, int64_t py, int mode,
                       int dir, int teams = 1, int zshift = 0, bool krev = false)
{
    const Plan& pl = h->plans[T];
    TripParams p{};
    p.src = src;
    p.dst = dst;
    p.rhs = rhs;
    p.px = px;
    p.py = py;
    p.rpx = px;
    p.rpy = py;
    p.nx = (int)h->d.nx;
    p.ny = (int)h->d.ny;
    p.nz = (int)h->d.nz;
    p.tiles_x = pl.tiles_x;
    p.tiles_y = pl.tiles_y;
    p.segs = pl.segs;
    p.seg_len = pl.seg_len;
    p.ntiles = pl.ntiles;
    p.mode = mode;
    p.dir = dir;
    p.flags = h->flags;
    p.ticket = h->ticket;
    // Claim groups start a tile's dependees at about the same time as the
    // tile rather than before it; that needs the slack of T >= 4 (5T steps).
    p.groups = h->xcd_order && T >= 4 ? kClaimGroups : 1;
    p.gcnt = h->gcnt;
    if (mode == 0 && h->ab_bands && pl.ntiles > kCUs) p.chunk = 1;  // band order (band_tile)
    p.zshift = zshift > 0 ? zshift : T;
    p.krev = krev ? 1 : 0;
    p.s27 = h->d.stencil == 27 ? 1 : 0;
    p.err = h->err;
    p.spin_limit = h->spin_limit;
    p.teams = teams;
    p.looseness = h->d.looseness;
    p.done = h->done;
    if (mode == 1 || mode == 3) {
        hipError_t e = launch_fill_i32(h->gcnt, 0,
                                       (int64_t)(kClaimGroups + pl.ntiles) * kFlagStride, h->run);
        if (e == hipSuccess && mode == 3)
            e = launch_fill_i32(h->done, 0, (int64_t)teams * kFlagStride, h->run);
        if (e == hipSuccess) e = launch_fill_i32(h->ticket, 0, 1, h->run);
        if (e != hipSuccess) return e;
    }
    if (mode == 0 && pl.tail_cols > 0) {  // split trip (split_tail): whole columns, then the tail
        hipError_t e = launch_trip_f64(pl.cfg, p, h->run);
        if (e != hipSuccess) return e;
        p.mode = 4;
        p.ntiles = pl.tail_tiles;
        p.chunk = pl.ntiles;
        p.groups = pl.tail_cols;
        p.seg_len = pl.tail_len;
        p.segs = (int)((h->d.nz + 2 + pl.tail_len - 1) / pl.tail_len);
        return launch_trip_f64(pl.cfg, p, h->run);
    }
    return f32 ? launch_trip_f32(pl.cfg, p, h->run)
               : launch_trip_f64(pl.cfg, p, h->run);
}

// A/B: cell (0,0,0) of grid `which`.
double* grid_origin(jacobi_t* h, int which)
{
    return static_cast<double*>(which == 0 ? h->d.grid0 : h->d.grid1);
}

// Compressed: cell (0,0,0) of the frame at offsets (off, off, offz).
double* comp_origin(jacobi_t* h, int off, int offz)
{
    return static_cast<double*>(h->d.grid0) + off * (1 + h->px) + (int64_t)offz * h->py;
}

double* current_origin(jacobi_t* h)
{
    if (h->d.layout == JACOBI_LAYOUT_AB) return grid_origin(h, h->cur);
    return comp_origin(h, h->off, h->offz);
}

// Direction (+1 forward: offsets decrease) and length of the next compressed
// trip of at most L sweeps.  A trip must keep both offsets in range: i and j
// move by L in [0, room], k by L+E in [0, roomz].  Forward trips lower
// offz - off by E and backward trips raise it, so the direction that moves it
// back towards E is tried first; if neither fits L, the trip is shortened
// (results do not depend on how sweeps are split into trips).
int comp_next_trip(const jacobi_t* h, int* L)
{
    const int E = h->zextra;
    auto fits = [&](int dir, int len) {
        return dir > 0 ? h->off >= len && h->offz >= len + E
                       : h->room - h->off >= len && h->roomz - h->offz >= len + E;
    };
    const int first = h->offz - h->off < E ? -1 : 1;
    if (fits(first, *L)) return first;
    if (fits(-first, *L)) return -first;
    for (int dir : {first, -first}) {
        const int len = dir > 0 ? std::min(h->off, h->offz - E)
                                : std::min(h->room - h->off, h->roomz - h->offz - E);
        if (len >= 1) {
            *L = std::min(*L, len);
            return dir;
        }
    }
    return 0;  // unreachable: room = 2t keeps one direction open
}

// n FP64 sweeps of the u grid(s).
int run_f64(jacobi_t* h, int64_t n)
{
    while (n > 0) {
        int L = (int)std::min<int64_t>(h->t, n);
        hipError_t e;
        if (h->d.layout == JACOBI_LAYOUT_AB && h->d.teams > 1 && n >= 2 * (int64_t)h->t) {
            // several full trips in one persistent launch
            const int k = (int)std::min<int64_t>(n / h->t, h->d.teams);
            L = k * h->t;
            e = launch_trip(h, h->t, false, grid_origin(h, h->cur),
                            grid_origin(h, 1 - h->cur), nullptr, h->px, h->py, 3, 1, k);
            h->cur ^= (k & 1);
        } else if (h->d.layout == JACOBI_LAYOUT_AB && L == 1 && h->d.stencil != 27 &&
                   h->d.nx * h->d.ny * h->d.nz <= kSmallBoxCells) {
            e = launch_sweep1_f64(grid_origin(h, h->cur), grid_origin(h, 1 - h->cur), h->px,
                                  h->py, (int)h->d.nx, (int)h->d.ny, (int)h->d.nz, h->run);
            h->cur ^= 1;
        } else if (h->d.layout == JACOBI_LAYOUT_AB) {
            e = launch_trip(h, L, false, grid_origin(h, h->cur),
                            grid_origin(h, 1 - h->cur), nullptr, h->px, h->py,
                            0, 1);
            h->cur ^= 1;
        } else {
            const int dir = comp_next_trip(h, &L);
            if (dir == 0) return fail(JACOBI_ESTATE, "no room for a compressed trip");
            const int noff = h->off - dir * L;
            const int noffz = h->offz - dir * (L + h->zextra);
            if (dir < 0 && h->krev) {
                // k-mirrored view: origin at plane nz+1, negative pitch
                const int64_t top = (h->d.nz + 1) * h->py;
                e = launch_trip(h, L, false, comp_origin(h, h->off, h->offz) + top,
                                comp_origin(h, noff, noffz) + top, nullptr, h->px, -h->py, 1,
                                dir, 1, L + h->zextra, true);
            } else {
                e = launch_trip(h, L, false, comp_origin(h, h->off, h->offz),
                                comp_origin(h, noff, noffz), nullptr, h->px, h->py, 1, dir,
                                1, L + h->zextra);
            }
            h->off = noff;
            h->offz = noffz;
        }
        if (e != hipSuccess) return hip_fail(e, "trip launch");
        n -= L;
        h->sweeps += L;
    }
    return JACOBI_OK;
}

// Residual / refinement view of the current iterate.
const AuxProblem& aux_view(jacobi_t* h)
{
    h->aux.u[0] = current_origin(h);
    h->aux.u[1] = h->aux.u[0];
    return h->aux;
}

// One outer step of the FP32-refined iteration with m inner sweeps.
int outer_f32(jacobi_t* h, int64_t m)
{
    const int nx = (int)h->d.nx, ny = (int)h->d.ny, nz = (int)h->d.nz;
    const int64_t epx = nx + 2, epy = (int64_t)(nx + 2) * (ny + 2);
    (void)nz;
    const AuxProblem& a = aux_view(h);
    hipError_t e = launch_residual_tab(nullptr, 1, a, nullptr, a.rblocks,
                                       h->partials, h->red_out, h->stream);
    if (e == hipSuccess)
        e = launch_make_rhs_tab(nullptr, 1, a, nullptr, h->red_out, h->scale_exp,
                                h->stream);
    if (e == hipSuccess) e = launch_zero_e_tab(nullptr, 1, a, h->stream);
    if (e != hipSuccess) return hip_fail(e, "refinement set-up");
    int ce = 0;
    int64_t left = m;
    while (left > 0) {
        const int L = (int)std::min<int64_t>(h->t, left);
        e = launch_trip(h, L, true, h->e[ce], h->e[1 - ce], h->rhs, epx, epy, 0, 1);
        if (e != hipSuccess) return hip_fail(e, "FP32 trip launch");
        ce ^= 1;
        left -= L;
    }
    e = launch_apply_correction_tab(nullptr, 1, a, nullptr, ce, h->scale_exp,
                                    h->stream);
    if (e != hipSuccess) return hip_fail(e, "correction launch");
    h->sweeps += m;
    return JACOBI_OK;
}

// A/B FP64 sweeps through a captured graph: capture run_f64's trips once per
// (n, starting grid) on the internal stream, then launch the executable graph
// on the caller's stream.  At most kMaxReplays graphs are kept; beyond that
// the sweeps run eagerly.
constexpr size_t kMaxReplays = 8;

int replay_f64(jacobi_t* h, int64_t n)
{
    jacobi_s::Replay* hit = nullptr;
    for (jacobi_s::Replay& r : h->replays)
        if (r.n == n && r.cur0 == h->cur) hit = &r;
    if (!hit) {
        if (h->replays.size() >= kMaxReplays) return run_f64(h, n);
        hipError_t e = hipSuccess;
        if (!h->cap) e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "capture stream");
        const int cur0 = h->cur;
        const int64_t sweeps0 = h->sweeps;
        e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "begin capture");
        h->run = h->cap;
        const int rc = run_f64(h, n);
        h->run = h->stream;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(h->cap, &g);
        jacobi_s::Replay r{n, cur0, h->cur, nullptr};
        h->cur = cur0;  // captured, not yet run
        h->sweeps = sweeps0;
        if (rc != JACOBI_OK) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        e = hipGraphInstantiate(&r.exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
        h->replays.push_back(r);
        hit = &h->replays.back();
    }
    hipError_t e = hipGraphLaunch(hit->exec, h->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    h->cur = hit->cur1;
    h->sweeps += n;
    return JACOBI_OK;
}

// `sweeps` weighted FP32 sweeps on multigrid level l (trips of kMgT); the
// current buffer index is updated.
hipError_t mg_smooth(jacobi_t* h, int l, int* cur, int sweeps)
{
    const jacobi_s::MgLevel& L = h->mg[l];
    hipError_t e = hipSuccess;
    for (int done = 0; done < sweeps && e == hipSuccess; done += kMgT) {
        TripParams p{};
        p.src = L.e[*cur];
        p.dst = L.e[1 - *cur];
        p.rhs = L.rhs;
        p.px = p.rpx = L.n + 2;
        p.py = p.rpy = (int64_t)(L.n + 2) * (L.n + 2);
        p.nx = p.ny = p.nz = L.n;
        p.tiles_x = L.plan.tiles_x;
        p.tiles_y = L.plan.tiles_y;
        p.segs = L.plan.segs;
        p.seg_len = L.plan.seg_len;
        p.ntiles = L.plan.ntiles;
        p.mode = 0;
        p.dir = 1;
        p.weighted = 1;
        p.omega = kMgOmega;
        e = launch_trip_f32(L.plan.cfg, p, h->stream);
        *cur ^= 1;
    }
    return e;
}

// One V-cycle on level l from a zero correction e[0]; returns the buffer
// holding the result in *out.
hipError_t mg_vcycle(jacobi_t* h, int l, int* out)
{
    const jacobi_s::MgLevel& L = h->mg[l];
    int cur = 0;
    if (L.n <= kMgCoarsest || l + 1 >= (int)h->mg.size()) {
        hipError_t e = mg_smooth(h, l, &cur, kMgCoarse);
        *out = cur;
        return e;
    }
    hipError_t e = mg_smooth(h, l, &cur, kMgNu);
    if (e == hipSuccess) e = launch_mg_residual(L.e[cur], L.rhs, L.e[1 - cur], L.n, h->stream);
    const jacobi_s::MgLevel& C = h->mg[l + 1];
    if (e == hipSuccess) e = launch_mg_restrict(L.e[1 - cur], L.n, C.rhs, h->stream);
    if (e == hipSuccess)
        e = launch_fill_f32(C.e[0], 0.f, (int64_t)(C.n + 2) * (C.n + 2) * (C.n + 2), h->stream);
    int cc = 0;
    if (e == hipSuccess) e = mg_vcycle(h, l + 1, &cc);
    if (e == hipSuccess) e = launch_mg_prolong_add(C.e[cc], L.e[cur], L.n, h->stream);
    if (e == hipSuccess) e = mg_smooth(h, l, &cur, kMgNu);
    *out = cur;
    return e;
}

// One outer step of the multigrid-corrected refinement: FP64 residual,
// rhs = fl32(r 2^-s), one V-cycle from zero, u += fl64(e) 2^s.
int outer_mg(jacobi_t* h)
{
    const AuxProblem& a = aux_view(h);
    hipError_t e = launch_residual_tab(nullptr, 1, a, nullptr, a.rblocks, h->partials,
                                       h->red_out, h->stream);
    if (e == hipSuccess)
        e = launch_make_rhs_tab(nullptr, 1, a, nullptr, h->red_out, h->scale_exp, h->stream);
    if (e == hipSuccess) e = launch_zero_e_tab(nullptr, 1, a, h->stream);
    int cur = 0;
    if (e == hipSuccess) e = mg_vcycle(h, 0, &cur);
    if (e == hipSuccess)
        e = launch_apply_correction_tab(nullptr, 1, a, nullptr, cur, h->scale_exp, h->stream);
    if (e != hipSuccess) return hip_fail(e, "multigrid step");
    h->sweeps += 1;
    return JACOBI_OK;
}

// Times every candidate on real sweeps of the iterate (A/B FP64 sweeps are
// bitwise the same for every configuration) and keeps the fastest.
int autotune_single(jacobi_t* h, int64_t* n)
{
    hipEvent_t a = nullptr, b = nullptr, t0 = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventRecord(t0, h->stream);
    const double cells = (double)h->d.nx * h->d.ny * h->d.nz;
    double best = -1;
    Plan best_plan = h->plans[h->t];
    const bool s27 = h->d.stencil == 27;
    const Candidates cs = tune_candidates(s27);
    for (int q = 0; q < cs.n; ++q) {
        const TripConfig& c = cs.c[q];
        if (e != hipSuccess) break;
        Plan pl;
        if (!config_supported(s27, c) ||
            !make_plan(h->d.nx, h->d.ny, h->d.nz, c, 0, false, kCUs, &pl))
            continue;
        if (s27) split_tail(&pl, h->d.nz);
        const Plan saved = h->plans[c.T];
        h->plans[c.T] = pl;
        float ms = 0;
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
            if (r == 1) e = hipEventRecord(a, h->stream);
            if (e == hipSuccess)
                e = launch_trip(h, c.T, false, grid_origin(h, h->cur),
                                grid_origin(h, 1 - h->cur), nullptr, h->px, h->py, 0, 1);
            h->cur ^= 1;
        }
        if (e == hipSuccess) e = hipEventRecord(b, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        h->plans[c.T] = saved;
        h->sweeps += 3 * c.T;
        *n -= 3 * c.T;
        if (e != hipSuccess) break;
        const double glups = cells * 2 * c.T / (ms * 1e-3) / 1e9;
        h->tune_log.push_back({c, glups});
        if (glups > best) {
            best = glups;
            best_plan = pl;
        }
    }
    float total = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&total, t0, b);
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    if (t0) hipEventDestroy(t0);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    h->tune_ms = total;
    h->t = best_plan.cfg.T;
    h->plans[h->t] = best_plan;
    h->tune_pending = false;
    return JACOBI_OK;
}

int check_pending(jacobi_t* h)
{
    int errw = 0;
    hipError_t e = hipMemcpyAsync(&errw, h->err, sizeof(int),
                                  hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    if (errw != 0) {
        e = launch_fill_i32(h->err, 0, 1, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "error word reset");
        return fail(JACOBI_ETIMEOUT,
                    "a tile progress wait exceeded its spin bound; results of "
                    "the affected sweeps are undefined");
    }
    return JACOBI_OK;
}

}  // namespace

extern "C" {

const char* jacobi_last_error(void) { return last_error_text(); }

int jacobi_tile_supported(int32_t dtype, int32_t t, int32_t tile_rows,
                          int32_t rows_per_wave)
{
    if (rows_per_wave <= 0 || tile_rows <= 0 || tile_rows % rows_per_wave) return 0;
    return trip_config_supported(dtype == JACOBI_F32_REFINED,
                                 TripConfig{t, rows_per_wave, tile_rows / rows_per_wave})
               ? 1
               : 0;
}

int jacobi_grid_bytes(const jacobi_desc* d, size_t* bytes)
{
    if (!d || !bytes) return fail(JACOBI_EINVAL, "null argument");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(JACOBI_EINVAL, "interior dims must be >= 1");
    const int t = d->t == 0 ? 4 : d->t;
    // Compressed: 2t planes of shift room in i and j, so that a trip of any
    // length <= t fits in one direction from every offset (no split trips
    // when sweep counts are not multiples of t), and 2t + 2E in k.
    const bool comp = d->layout == JACOBI_LAYOUT_COMPRESSED;
    const int room = comp ? 2 * t : 0;
    const int roomz = comp ? room + 2 * compressed_zextra(d, t) : 0;
    *bytes = (size_t)((d->nx + 2 + room) * (d->ny + 2 + room) * (d->nz + 2 + roomz) * 8);
    return JACOBI_OK;
}

int jacobi_workspace_size(const jacobi_desc* d, size_t* bytes)
{
    if (!bytes) return fail(JACOBI_EINVAL, "null argument");
    Plan plans[9];
    int t = 0;
    Layout L{};
    int rc = validate_and_plan(d, plans, &t, &L);
    if (rc != JACOBI_OK) return rc;
    *bytes = L.total;
    return JACOBI_OK;
}

int jacobi_create(const jacobi_desc* d, jacobi_t** out)
{
    if (!out) return fail(JACOBI_EINVAL, "null output handle pointer");
    *out = nullptr;
    Plan plans[9];
    int t = 0;
    Layout L{};
    int rc = validate_and_plan(d, plans, &t, &L);
    if (rc != JACOBI_OK) return rc;
    if (!d->grid0) return fail(JACOBI_EINVAL, "grid0 is null");
    if (reinterpret_cast<uintptr_t>(d->grid0) % 16)
        return fail(JACOBI_EINVAL, "grid0 must be 16-byte aligned");
    if (d->layout == JACOBI_LAYOUT_AB) {
        if (!d->grid1) return fail(JACOBI_EINVAL, "grid1 is null (AB layout)");
        if (reinterpret_cast<uintptr_t>(d->grid1) % 16)
            return fail(JACOBI_EINVAL, "grid1 must be 16-byte aligned");
        if (d->grid1 == d->grid0) return fail(JACOBI_EINVAL, "grid1 == grid0");
    }
    if (!d->workspace || d->workspace_bytes < L.total)
        return fail(JACOBI_EWORKSPACE, "workspace of %zu bytes needed, %zu given",
                    L.total, d->workspace ? d->workspace_bytes : (size_t)0);
    if (reinterpret_cast<uintptr_t>(d->workspace) % 256)
        return fail(JACOBI_EINVAL, "workspace must be 256-byte aligned");

    jacobi_t* h = new (std::nothrow) jacobi_s();
    if (!h) return fail(JACOBI_EINVAL, "out of host memory");
    h->d = *d;
    h->t = t;
    const bool s27 = d->stencil == 27;
    if (d->t == 0 && t == (s27 ? kS27MaxT : kTuneMaxT)) {
        h->tune_pending = true;
        h->t = s27 ? kS27DefaultT : kTuneDefaultT;
    }
    for (int T = 1; T <= t; ++T) h->plans[T] = plans[T];
    const bool comp = d->layout == JACOBI_LAYOUT_COMPRESSED;
    h->room = comp ? 2 * t : 0;
    h->off = h->room;
    h->zextra = comp ? compressed_zextra(d, t) : 0;
    h->roomz = h->room + 2 * h->zextra;
    h->offz = h->roomz;
    h->px = d->nx + 2 + h->room;
    h->py = h->px * (d->ny + 2 + h->room);
    h->stream = static_cast<hipStream_t>(d->stream);
    h->run = h->stream;
    h->inner = d->inner_sweeps > 0 ? d->inner_sweeps : 32;
    if (const char* s = std::getenv("JACOBI_SPIN_LIMIT")) {
        long long v = std::atoll(s);
        if (v > 0) h->spin_limit = v;
    }
    h->ws = static_cast<char*>(d->workspace);
    h->ticket = reinterpret_cast<int*>(h->ws);
    h->err = h->ticket + 1;
    h->scale_exp = h->ticket + 2;
    h->red_out = reinterpret_cast<double*>(h->ws + 64);
    h->partials = reinterpret_cast<double*>(h->ws + L.partials_off);
    h->gcnt = reinterpret_cast<int*>(h->ws + L.flags_off);
    h->flags = h->gcnt + kClaimGroups * kFlagStride;
    if (const char* s = std::getenv("JACOBI_XCD_ORDER")) h->xcd_order = std::atoi(s) != 0;
    h->krev = compressed_krev(t);
    if (const char* s = std::getenv("JACOBI_AB_BANDS")) h->ab_bands = std::atoi(s) != 0;
    h->flag_ints = L.flag_ints;
    h->done = reinterpret_cast<int*>(h->ws + L.done_off);
    if (d->dtype != JACOBI_F64) {
        h->e[0] = reinterpret_cast<float*>(h->ws + L.e0_off);
        h->e[1] = reinterpret_cast<float*>(h->ws + L.e1_off);
        h->rhs = reinterpret_cast<float*>(h->ws + L.rhs_off);
    }
    if (d->dtype == JACOBI_F32_MULTIGRID) {
        int64_t n = d->nx;
        jacobi_s::MgLevel lv0{(int)n, {h->e[0], h->e[1]}, h->rhs, h->plans[kMgT]};
        h->mg.push_back(lv0);
        for (size_t q = 0; q < L.mg_off.size(); ++q) {
            n = (n - 1) / 2;
            const size_t fb = (size_t)round_up((n + 2) * (n + 2) * (n + 2) * 4, 256);
            jacobi_s::MgLevel lv{};
            lv.n = (int)n;
            lv.e[0] = reinterpret_cast<float*>(h->ws + L.mg_off[q]);
            lv.e[1] = reinterpret_cast<float*>(h->ws + L.mg_off[q] + fb);
            lv.rhs = reinterpret_cast<float*>(h->ws + L.mg_off[q] + 2 * fb);
            if (!make_plan(n, n, n, default_cfg(kMgT), 0, false, kCUs, &lv.plan)) {
                delete h;
                return fail(JACOBI_EUNSUPPORTED, "no trip plan for multigrid level n=%lld",
                            (long long)n);
            }
            h->mg.push_back(lv);
        }
    }
    h->aux.nx = (int)d->nx;
    h->aux.ny = (int)d->ny;
    h->aux.nz = (int)d->nz;
    h->aux.px = h->px;
    h->aux.py = h->py;
    h->aux.epx = d->nx + 2;
    h->aux.epy = (d->nx + 2) * (d->ny + 2);
    h->aux.e[0] = h->e[0];
    h->aux.e[1] = h->e[1];
    h->aux.rhs = h->rhs;
    residual_plan(&h->aux);
    h->aux.rblock_base = 0;
    hipError_t e = launch_fill_i32(h->ticket, 0, 16, h->stream);
    if (e == hipSuccess && d->layout == JACOBI_LAYOUT_AB) {
        const int nx2 = (int)d->nx + 2, ny2 = (int)d->ny + 2, nz2 = (int)d->nz + 2;
        e = launch_copy_box_f64(static_cast<const double*>(d->grid0), h->px, h->py,
                                static_cast<double*>(d->grid1), h->px, h->py, nx2,
                                ny2, nz2, h->stream);
    }
    if (e == hipSuccess && d->dtype != JACOBI_F64) {
        const int64_t box = (d->nx + 2) * (d->ny + 2) * (d->nz + 2);
        e = launch_fill_f32(h->e[0], 0.f, box, h->stream);
        if (e == hipSuccess) e = launch_fill_f32(h->e[1], 0.f, box, h->stream);
        if (e == hipSuccess) e = launch_fill_f32(h->rhs, 0.f, box, h->stream);
        // coarse levels: zero boxes (the boundary layers stay zero for good)
        for (size_t q = 1; q < h->mg.size() && e == hipSuccess; ++q) {
            const int64_t nb = (int64_t)(h->mg[q].n + 2) * (h->mg[q].n + 2) * (h->mg[q].n + 2);
            e = launch_fill_f32(h->mg[q].e[0], 0.f, nb, h->stream);
            if (e == hipSuccess) e = launch_fill_f32(h->mg[q].e[1], 0.f, nb, h->stream);
            if (e == hipSuccess) e = launch_fill_f32(h->mg[q].rhs, 0.f, nb, h->stream);
        }
    }
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "set-up launch");
    }
    *out = h;
    return JACOBI_OK;
}

int jacobi_sweep(jacobi_t* h, int64_t n_steps)
{
    if (!h) return fail(JACOBI_EINVAL, "null handle");
    if (n_steps < 0) return fail(JACOBI_EINVAL, "n_steps < 0");
    if (h->tune_pending && n_steps >= kTuneSweeps) {
        int rc = autotune_single(h, &n_steps);
        if (rc != JACOBI_OK) return rc;
    }
    if (h->d.dtype == JACOBI_F64 && h->d.use_graph && h->d.layout == JACOBI_LAYOUT_AB &&
        n_steps > 0)
        return replay_f64(h, n_steps);
    if (h->d.dtype == JACOBI_F64) return run_f64(h, n_steps);
    if (h->d.dtype == JACOBI_F32_MULTIGRID) {
        for (int64_t q = 0; q < n_steps; ++q) {
            int rc = outer_mg(h);
            if (rc != JACOBI_OK) return rc;
        }
        return JACOBI_OK;
    }
    while (n_steps > 0) {
        const int64_t m = std::min<int64_t>(h->inner, n_steps);
        int rc = outer_f32(h, m);
        if (rc != JACOBI_OK) return rc;
        n_steps -= m;
    }
    return JACOBI_OK;
}

int jacobi_residual(jacobi_t* h, double* l2, double* maxabs)
{
    if (!h || !l2) return fail(JACOBI_EINVAL, "null argument");
    if (h->d.stencil == 27)
        return fail(JACOBI_EUNSUPPORTED, "the residual is that of the 7-point equation");
    const AuxProblem& a = aux_view(h);
    hipError_t e = launch_residual_tab(nullptr, 1, a, nullptr, a.rblocks,
                                       h->partials, h->red_out, h->stream);
    if (e != hipSuccess) return hip_fail(e, "residual launch");
    double out[2] = {0, 0};
    e = hipMemcpyAsync(out, h->red_out, sizeof out, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "residual copy");
    int rc = check_pending(h);
    if (rc != JACOBI_OK) return rc;
    *l2 = out[0];
    if (maxabs) *maxabs = out[1];
    return JACOBI_OK;
}

int jacobi_solve(jacobi_t* h, double rel_tol, double r0, int64_t max_sweeps,
                 int64_t check_every, int64_t* sweeps_done, double* final_l2)
{
    if (!h) return fail(JACOBI_EINVAL, "null handle");
    if (!(rel_tol > 0) || max_sweeps < 0 || check_every < 1)
        return fail(JACOBI_EINVAL, "need rel_tol > 0, max_sweeps >= 0, check_every >= 1");
    double r = 0;
    int rc = jacobi_residual(h, &r, nullptr);
    if (rc != JACOBI_OK) return rc;
    if (!(r0 > 0)) r0 = r;
    int64_t done = 0;
    while (r > rel_tol * r0 && done < max_sweeps) {
        const int64_t m = std::min(check_every, max_sweeps - done);
        rc = jacobi_sweep(h, m);
        if (rc != JACOBI_OK) return rc;
        done += m;
        rc = jacobi_residual(h, &r, nullptr);
        if (rc != JACOBI_OK) return rc;
    }
    if (sweeps_done) *sweeps_done = done;
    if (final_l2) *final_l2 = r;
    return JACOBI_OK;
}

int jacobi_sync(jacobi_t* h)
{
    if (!h) return fail(JACOBI_EINVAL, "null handle");
    return check_pending(h);
}

int jacobi_current(jacobi_t* h, void** origin, int64_t strides[3])
{
    if (!h || !origin || !strides) return fail(JACOBI_EINVAL, "null argument");
    *origin = current_origin(h);
    strides[0] = 1;
    strides[1] = h->px;
    strides[2] = h->py;
    return JACOBI_OK;
}

int jacobi_info(jacobi_t* h, int64_t* sweeps_done, int32_t* t,
                int32_t* tile_rows, int32_t* seg_len)
{
    if (!h) return fail(JACOBI_EINVAL, "null handle");
    if (sweeps_done) *sweeps_done = h->sweeps;
    if (t) *t = h->t;
    if (tile_rows) *tile_rows = h->plans[h->t].cfg.R * h->plans[h->t].cfg.W;
    if (seg_len) *seg_len = h->plans[h->t].seg_len;
    return JACOBI_OK;
}

int jacobi_tune_log(jacobi_t* h, int32_t cap, int32_t* t, int32_t* tile_rows,
                    int32_t* rows_per_wave, double* glups, int32_t* n, double* tune_ms)
{
    if (!h || !n || cap < 0) return fail(JACOBI_EINVAL, "null argument");
    const int m = (int)std::min<size_t>((size_t)cap, h->tune_log.size());
    for (int q = 0; q < m; ++q) {
        const auto& e = h->tune_log[q];
        if (t) t[q] = e.cfg.T;
        if (tile_rows) tile_rows[q] = e.cfg.R * e.cfg.W;
        if (rows_per_wave) rows_per_wave[q] = e.cfg.R;
        if (glups) glups[q] = e.glups;
    }
    *n = (int32_t)h->tune_log.size();
    if (tune_ms) *tune_ms = h->tune_ms;
    return JACOBI_OK;
}

int jacobi_destroy(jacobi_t* h)
{
    if (!h) return JACOBI_OK;
    // replayed graphs may still be running on the caller's stream
    if (!h->replays.empty()) (void)hipStreamSynchronize(h->stream);
    delete h;
    return JACOBI_OK;
}

int jacobi_probe_copy(const double* src, double* dst, int64_t n, void* stream)
{
    if (!src || !dst || n < 2 || (n & 1) ||
        (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
        return fail(JACOBI_EINVAL, "probe needs even n >= 2 and 16-byte aligned buffers");
    hipError_t e = launch_stream_copy(src, dst, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "copy probe");
}

int jacobi_probe_update(double* a, int64_t n, void* stream)
{
    if (!a || n < 2 || (n & 1) || reinterpret_cast<uintptr_t>(a) % 16)
        return fail(JACOBI_EINVAL, "probe needs even n >= 2 and a 16-byte aligned buffer");
    hipError_t e = launch_stream_update(a, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "update probe");
}

}  // extern "C"
