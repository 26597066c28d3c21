// Batched runtime of libjacobi: many independent Laplace problems of uneven
// sizes swept together.
//
// * One persistent launch per trip covers every (problem, tile) pair of the
//   batch (trip kernel MODE 2): workgroups take tiles from one ticket counter
//   in largest-problem-first order, so small and large problems load-balance
//   on the whole chip.  The A/B parity lives in device memory and is flipped
//   (with the ticket reset) by a one-thread kernel after every trip, so the
//   same launch sequence is valid from either parity.
// * The whole schedule of a jacobi_batch_sweep(n) call is captured once into a
//   hipGraph and replayed (one graph launch per call).  No memset nodes: flags
//   and counters are reset by kernels.
// * Autotuner: with t == 0 the first sweeps of the batch are spent timing
//   candidate (t, tile shape) configurations with HIP events on the real
//   problems.  Every configuration computes exactly the plain sweeps, so the
//   tuning sweeps are real work, not a detour; the fastest configuration (by
//   measured GLUP/s) is used for the rest.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <vector>

#include "internal.h"
#include "jacobi.h"
#include "runtime_common.h"

using namespace jacobi_impl;

namespace {

struct TripSet {
    bool ready = false;
    TripConfig cfg{0, 0, 0};
    int ntiles = 0;
    std::vector<BatchProblem> host64, host32;
};

// Candidate shapes of the autotuner (all compiled; see the trip kernel).
const TripConfig kCandidates[] = {
    {2, 4, 16}, {3, 4, 12}, {3, 2, 16}, {4, 3, 12}, {4, 4, 8}, {5, 4, 8}, {5, 3, 12},
    {6, 3, 12},
};

struct WsLayout {
    size_t aux_off, tab_off, partials_off, out_off, scale_off, f32_off, total;
    std::vector<size_t> e0, e1, rhs;  // per problem, bytes from ws start
    int total_rblocks;
};

}  // namespace

struct jacobi_batch_s {
    int count = 0;
    std::vector<int64_t> dims;
    std::vector<void*> g0, g1;
    std::vector<int> order;  // table order (largest problem first)
    int dtype = JACOBI_F64;
    int t_req = 0;
    int t = 4;
    bool tuned = false;
    int inner = 32;
    bool use_graph = true;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    char* ws = nullptr;
    int* ticket = nullptr;
    int* err = nullptr;
    int* parity = nullptr;
    int* eparity = nullptr;
    AuxProblem* d_aux = nullptr;
    BatchProblem* d_tab = nullptr;  // [9][2][count]
    double* partials = nullptr;
    double* red_out = nullptr;
    int* scale_exp = nullptr;
    int total_rblocks = 0;
    std::vector<AuxProblem> aux;
    TripSet sets[9];
    int64_t sweeps = 0;
    int host_parity = 0;
    double cells = 0;
    double tune_ms = 0;
    std::vector<std::pair<TripConfig, double>> tune_log;
    std::map<int64_t, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_objs;
};

namespace {

int64_t box_elems(const int64_t* d) { return (d[0] + 2) * (d[1] + 2) * (d[2] + 2); }

int validate_batch(const jacobi_batch_desc* d, WsLayout* L)
{
    if (!d) return fail(JACOBI_EINVAL, "null batch descriptor");
    if (d->count < 1 || d->count > (1 << 20))
        return fail(JACOBI_EINVAL, "count must be 1..2^20 (got %d)", d->count);
    if (!d->dims) return fail(JACOBI_EINVAL, "dims is null");
    if (d->dtype != JACOBI_F64 && d->dtype != JACOBI_F32_REFINED)
        return fail(JACOBI_EINVAL, "unknown dtype %d", d->dtype);
    if (d->t < 0 || d->t > 8)
        return fail(JACOBI_EUNSUPPORTED, "t=%d not supported (0 = autotune, 1..8)", d->t);
    if (d->inner_sweeps < 0) return fail(JACOBI_EINVAL, "inner_sweeps < 0");
    if (d->tile_rows || d->rows_per_wave) {
        const int R = d->rows_per_wave > 0 ? d->rows_per_wave : 4;
        const int rows = d->tile_rows > 0 ? d->tile_rows : 32;
        if (d->t == 0)
            return fail(JACOBI_EINVAL, "a tile shape needs an explicit t");
        if (rows % R || !trip_config_supported(d->dtype, TripConfig{d->t, R, rows / R}))
            return fail(JACOBI_EUNSUPPORTED, "tile shape rows=%d rows_per_wave=%d not compiled",
                        rows, R);
    }
    int64_t rb = 0;
    for (int q = 0; q < d->count; ++q) {
        const int64_t* x = d->dims + 3 * q;
        if (x[0] < 1 || x[1] < 1 || x[2] < 1 || x[0] > 65536 || x[1] > 65536 ||
            x[2] > 65536)
            return fail(JACOBI_EINVAL, "problem %d: dims must be 1..65536", q);
        if ((x[0] + 2) * (x[1] + 2) * 8 >= ((int64_t)1 << 31))
            return fail(JACOBI_EINVAL, "problem %d: one k-plane must be < 2 GiB", q);
        AuxProblem a{};
        a.nx = (int)x[0];
        a.ny = (int)x[1];
        a.nz = (int)x[2];
        rb += residual_plan(&a);
    }
    if (rb > (1 << 30)) return fail(JACOBI_EINVAL, "batch too large");
    WsLayout l;
    size_t off = 256;
    l.aux_off = off;
    off = (size_t)round_up(off + (size_t)d->count * sizeof(AuxProblem), 256);
    l.tab_off = off;
    off = (size_t)round_up(off + (size_t)9 * 2 * d->count * sizeof(BatchProblem), 256);
    l.partials_off = off;
    off = (size_t)round_up(off + (size_t)rb * 2 * sizeof(double), 256);
    l.out_off = off;
    off = (size_t)round_up(off + (size_t)d->count * 2 * sizeof(double), 256);
    l.scale_off = off;
    off = (size_t)round_up(off + (size_t)d->count * sizeof(int), 256);
    l.f32_off = off;
    if (d->dtype == JACOBI_F32_REFINED) {
        for (int q = 0; q < d->count; ++q) {
            const size_t fb = (size_t)round_up(box_elems(d->dims + 3 * q) * 4, 256);
            l.e0.push_back(off);
            l.e1.push_back(off + fb);
            l.rhs.push_back(off + 2 * fb);
            off += 3 * fb;
        }
    }
    l.total = off;
    l.total_rblocks = (int)rb;
    *L = l;
    return JACOBI_OK;
}

BatchProblem* tab_ptr(jacobi_batch_t* h, int T, int f32)
{
    return h->d_tab + ((size_t)T * 2 + f32) * h->count;
}

// Tables of the trip kernel for `cfg` (uploaded into slot cfg.T).
int ensure_set(jacobi_batch_t* h, const TripConfig& cfg)
{
    TripSet& s = h->sets[cfg.T];
    if (s.ready && s.cfg.R == cfg.R && s.cfg.W == cfg.W) return JACOBI_OK;
    s.host64.assign(h->count, BatchProblem{});
    s.host32.assign(h->count, BatchProblem{});
    // A batch with plenty of tile columns streams each column's whole k
    // range in one tile; one with fewer tiles than two per CU splits k into
    // segments the way a single problem does, so the launch fills the GPU.
    std::vector<Plan> plans(h->count);
    int64_t whole = 0;
    for (int pos = 0; pos < h->count; ++pos) {
        const int64_t* x = &h->dims[3 * h->order[pos]];
        if (!make_plan(x[0], x[1], x[2], cfg, 0, false, 1, &plans[pos]))
            return fail(JACOBI_EUNSUPPORTED, "tile shape t=%d rows=%d cannot cover problem %d",
                        cfg.T, cfg.R * cfg.W, h->order[pos]);
        whole += plans[pos].ntiles;
    }
    if (whole < 2 * kCUs) {
        for (int pos = 0; pos < h->count; ++pos) {
            const int64_t* x = &h->dims[3 * h->order[pos]];
            if (!make_plan(x[0], x[1], x[2], cfg, 0, false, kCUs, &plans[pos]))
                return fail(JACOBI_EUNSUPPORTED, "tile shape t=%d rows=%d cannot cover problem %d",
                            cfg.T, cfg.R * cfg.W, h->order[pos]);
        }
    }
    int base = 0;
    for (int pos = 0; pos < h->count; ++pos) {
        const int q = h->order[pos];
        const int64_t* x = &h->dims[3 * q];
        const Plan& pl = plans[pos];
        BatchProblem b{};
        b.px = x[0] + 2;
        b.py = (x[0] + 2) * (x[1] + 2);
        b.nx = (int)x[0];
        b.ny = (int)x[1];
        b.nz = (int)x[2];
        b.tiles_x = pl.tiles_x;
        b.tiles_y = pl.tiles_y;
        b.segs = pl.segs;
        b.seg_len = pl.seg_len;
        b.tile_base = base;
        base += pl.ntiles;
        b.grid[0] = h->g0[q];
        b.grid[1] = h->g1[q];
        b.rhs = nullptr;
        s.host64[pos] = b;
        if (h->dtype == JACOBI_F32_REFINED) {
            b.grid[0] = h->aux[q].e[0];
            b.grid[1] = h->aux[q].e[1];
            b.rhs = h->aux[q].rhs;
            s.host32[pos] = b;
        }
    }
    s.ntiles = base;
    s.cfg = cfg;
    hipError_t e = hipMemcpyAsync(tab_ptr(h, cfg.T, 0), s.host64.data(),
                                  sizeof(BatchProblem) * h->count,
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && h->dtype == JACOBI_F32_REFINED)
        e = hipMemcpyAsync(tab_ptr(h, cfg.T, 1), s.host32.data(),
                           sizeof(BatchProblem) * h->count, hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    s.ready = true;
    return JACOBI_OK;
}

hipError_t trip(jacobi_batch_t* h, int T, bool f32, hipStream_t s)
{
    const TripSet& ts = h->sets[T];
    TripParams p{};
    p.mode = 2;
    p.ntiles = ts.ntiles;
    p.table = tab_ptr(h, T, f32 ? 1 : 0);
    p.count = h->count;
    p.parity = f32 ? h->eparity : h->parity;
    p.rhs_in_table = f32 ? 1 : 0;
    p.ticket = h->ticket;
    p.err = h->err;
    p.dir = 1;
    hipError_t e = f32 ? launch_trip_f32(ts.cfg, p, s) : launch_trip_f64(ts.cfg, p, s);
    if (e != hipSuccess) return e;
    return launch_flip_parity(f32 ? h->eparity : h->parity, h->ticket, s);
}

int prepare_sets(jacobi_batch_t* h, int T)
{
    for (int x = 1; x <= T; ++x) {
        if (h->sets[x].ready) continue;
        int rc = ensure_set(h, default_cfg(x));
        if (rc != JACOBI_OK) return rc;
    }
    return JACOBI_OK;
}

// Enqueue n sweeps (no host synchronization).  Host parity is tracked.
int enqueue(jacobi_batch_t* h, int64_t n, hipStream_t s, int* parity_flips)
{
    int flips = 0;
    hipError_t e = hipSuccess;
    if (h->dtype == JACOBI_F64) {
        while (n > 0 && e == hipSuccess) {
            const int L = (int)std::min<int64_t>(h->t, n);
            e = trip(h, L, false, s);
            ++flips;
            n -= L;
        }
    } else {
        while (n > 0 && e == hipSuccess) {
            const int64_t m = std::min<int64_t>(h->inner, n);
            AuxProblem none{};
            e = launch_residual_tab(h->d_aux, h->count, none, h->parity,
                                    h->total_rblocks, h->partials, h->red_out, s);
            if (e == hipSuccess)
                e = launch_make_rhs_tab(h->d_aux, h->count, none, h->parity,
                                        h->red_out, h->scale_exp, s);
            if (e == hipSuccess) e = launch_zero_e_tab(h->d_aux, h->count, none, s);
            if (e == hipSuccess) e = launch_set_int(h->eparity, 0, s);
            int ce = 0;
            int64_t left = m;
            while (left > 0 && e == hipSuccess) {
                const int L = (int)std::min<int64_t>(h->t, left);
                e = trip(h, L, true, s);
                ce ^= 1;
                left -= L;
            }
            if (e == hipSuccess)
                e = launch_apply_correction_tab(h->d_aux, h->count, none, h->parity,
                                                ce, h->scale_exp, s);
            n -= m;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    *parity_flips = flips;
    return JACOBI_OK;
}

int autotune(jacobi_batch_t* h, int64_t* n)
{
    hipEvent_t a = nullptr, b = nullptr, t0 = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
        hipEventCreate(&t0) != hipSuccess || hipEventRecord(t0, h->stream) != hipSuccess) {
        if (a) hipEventDestroy(a);
        if (b) hipEventDestroy(b);
        if (t0) hipEventDestroy(t0);
        return fail(JACOBI_EHIP, "event create");
    }
    double best = -1;
    TripConfig best_cfg = default_cfg(4);
    const bool f32 = h->dtype == JACOBI_F32_REFINED;
    for (const TripConfig& c : kCandidates) {
        if (!f32 && *n < 3 * c.T) break;
        if (!trip_config_supported(h->dtype, c)) continue;
        int rc = ensure_set(h, c);
        if (rc != JACOBI_OK) continue;
        // FP64 batches are tuned on real sweeps of the iterate.  FP32-refined
        // batches are tuned on FP32 trips of the correction grids, which are
        // reset before every outer step, so the iterate is not touched.
        hipError_t e = trip(h, c.T, f32, h->stream);
        if (!f32) h->host_parity ^= 1;
        if (e == hipSuccess) e = hipEventRecord(a, h->stream);
        for (int r = 0; r < 2 && e == hipSuccess; ++r) {
            e = trip(h, c.T, f32, h->stream);
            if (!f32) h->host_parity ^= 1;
        }
        if (e == hipSuccess) e = hipEventRecord(b, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) {
            hipEventDestroy(a);
            hipEventDestroy(b);
            hipEventDestroy(t0);
            return hip_fail(e, "autotune");
        }
        if (!f32) {
            h->sweeps += 3 * c.T;
            *n -= 3 * c.T;
        }
        const double glups = h->cells * 2 * c.T / (ms * 1e-3) / 1e9;
        h->tune_log.push_back({c, glups});
        if (glups > best) {
            best = glups;
            best_cfg = c;
        }
    }
    // tune_ms: the whole tuning on the stream, warm-up trips included
    float total = 0;
    hipError_t e = hipEventElapsedTime(&total, t0, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipEventDestroy(t0);
    if (e == hipSuccess) h->tune_ms = total;
    h->t = best_cfg.T;
    int rc = ensure_set(h, best_cfg);
    if (rc != JACOBI_OK) return rc;
    h->tuned = true;
    return JACOBI_OK;
}

int check_err(jacobi_batch_t* h)
{
    int w = 0;
    hipError_t e = hipMemcpyAsync(&w, h->err, sizeof(int), hipMemcpyDeviceToHost,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "batch synchronize");
    if (w) return fail(JACOBI_ETIMEOUT, "progress wait exceeded its bound");
    return JACOBI_OK;
}

}  // namespace

extern "C" {

int jacobi_batch_workspace_size(const jacobi_batch_desc* d, size_t* bytes)
{
    if (!bytes) return fail(JACOBI_EINVAL, "null argument");
    WsLayout L;
    int rc = validate_batch(d, &L);
    if (rc != JACOBI_OK) return rc;
    *bytes = L.total;
    return JACOBI_OK;
}

int jacobi_batch_create(const jacobi_batch_desc* d, jacobi_batch_t** out)
{
    if (!out) return fail(JACOBI_EINVAL, "null output handle pointer");
    *out = nullptr;
    WsLayout L;
    int rc = validate_batch(d, &L);
    if (rc != JACOBI_OK) return rc;
    if (!d->grid0 || !d->grid1) return fail(JACOBI_EINVAL, "grid arrays are null");
    for (int q = 0; q < d->count; ++q) {
        if (!d->grid0[q] || !d->grid1[q] || d->grid0[q] == d->grid1[q])
            return fail(JACOBI_EINVAL, "problem %d: grid pointers null or equal", q);
        if ((reinterpret_cast<uintptr_t>(d->grid0[q]) |
             reinterpret_cast<uintptr_t>(d->grid1[q])) % 16)
            return fail(JACOBI_EINVAL, "problem %d: grids must be 16-byte aligned", q);
    }
    if (!d->workspace || d->workspace_bytes < L.total)
        return fail(JACOBI_EWORKSPACE, "workspace of %zu bytes needed", L.total);
    if (reinterpret_cast<uintptr_t>(d->workspace) % 256)
        return fail(JACOBI_EINVAL, "workspace must be 256-byte aligned");

    jacobi_batch_t* h = new (std::nothrow) jacobi_batch_s();
    if (!h) return fail(JACOBI_EINVAL, "out of host memory");
    h->count = d->count;
    h->dims.assign(d->dims, d->dims + 3 * d->count);
    h->g0.assign(d->grid0, d->grid0 + d->count);
    h->g1.assign(d->grid1, d->grid1 + d->count);
    h->dtype = d->dtype;
    h->t_req = d->t;
    h->t = d->t > 0 ? d->t : 4;
    h->inner = d->inner_sweeps > 0 ? d->inner_sweeps : 32;
    h->use_graph = d->use_graph != 0;
    h->stream = static_cast<hipStream_t>(d->stream);
    h->ws = static_cast<char*>(d->workspace);
    h->ticket = reinterpret_cast<int*>(h->ws);
    h->err = h->ticket + 1;
    h->parity = h->ticket + 2;
    h->eparity = h->ticket + 3;
    h->d_aux = reinterpret_cast<AuxProblem*>(h->ws + L.aux_off);
    h->d_tab = reinterpret_cast<BatchProblem*>(h->ws + L.tab_off);
    h->partials = reinterpret_cast<double*>(h->ws + L.partials_off);
    h->red_out = reinterpret_cast<double*>(h->ws + L.out_off);
    h->scale_exp = reinterpret_cast<int*>(h->ws + L.scale_off);
    h->total_rblocks = L.total_rblocks;
    h->order.resize(h->count);
    std::iota(h->order.begin(), h->order.end(), 0);
    std::stable_sort(h->order.begin(), h->order.end(), [&](int x, int y) {
        return box_elems(&h->dims[3 * x]) > box_elems(&h->dims[3 * y]);
    });
    h->aux.assign(h->count, AuxProblem{});
    int base = 0;
    for (int q = 0; q < h->count; ++q) {
        const int64_t* x = &h->dims[3 * q];
        AuxProblem& a = h->aux[q];
        a.u[0] = static_cast<const double*>(h->g0[q]);
        a.u[1] = static_cast<const double*>(h->g1[q]);
        a.px = a.epx = x[0] + 2;
        a.py = a.epy = (x[0] + 2) * (x[1] + 2);
        a.nx = (int)x[0];
        a.ny = (int)x[1];
        a.nz = (int)x[2];
        residual_plan(&a);
        a.rblock_base = base;
        base += a.rblocks;
        if (h->dtype == JACOBI_F32_REFINED) {
            a.e[0] = reinterpret_cast<float*>(h->ws + L.e0[q]);
            a.e[1] = reinterpret_cast<float*>(h->ws + L.e1[q]);
            a.rhs = reinterpret_cast<float*>(h->ws + L.rhs[q]);
        }
        h->cells += (double)x[0] * x[1] * x[2];
    }
    hipError_t e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = launch_fill_i32(h->ticket, 0, 64, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->d_aux, h->aux.data(), sizeof(AuxProblem) * h->count,
                           hipMemcpyHostToDevice, h->stream);
    // Both grids carry the boundary layer; the second starts as a copy.
    for (int q = 0; q < h->count && e == hipSuccess; ++q) {
        const int64_t* x = &h->dims[3 * q];
        e = launch_copy_box_f64(static_cast<const double*>(h->g0[q]), x[0] + 2,
                                (x[0] + 2) * (x[1] + 2), static_cast<double*>(h->g1[q]),
                                x[0] + 2, (x[0] + 2) * (x[1] + 2), (int)x[0] + 2,
                                (int)x[1] + 2, (int)x[2] + 2, h->stream);
        if (e == hipSuccess && h->dtype == JACOBI_F32_REFINED) {
            const int64_t n = box_elems(x);
            e = launch_fill_f32(h->aux[q].e[0], 0.f, n, h->stream);
            if (e == hipSuccess) e = launch_fill_f32(h->aux[q].e[1], 0.f, n, h->stream);
            if (e == hipSuccess) e = launch_fill_f32(h->aux[q].rhs, 0.f, n, h->stream);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        if (h->cap) hipStreamDestroy(h->cap);
        delete h;
        return hip_fail(e, "batch set-up");
    }
    if (d->t > 0 && (d->tile_rows || d->rows_per_wave)) {
        const int R = d->rows_per_wave > 0 ? d->rows_per_wave : 4;
        const int rows = d->tile_rows > 0 ? d->tile_rows : 32;
        rc = ensure_set(h, TripConfig{d->t, R, rows / R});
        if (rc != JACOBI_OK) {
            hipStreamDestroy(h->cap);
            delete h;
            return rc;
        }
    }
    h->tuned = d->t > 0;
    *out = h;
    return JACOBI_OK;
}

int jacobi_batch_sweep(jacobi_batch_t* h, int64_t n_steps)
{
    if (!h) return fail(JACOBI_EINVAL, "null handle");
    if (n_steps < 0) return fail(JACOBI_EINVAL, "n_steps < 0");
    if (n_steps == 0) return JACOBI_OK;
    if (!h->tuned) {
        int rc = autotune(h, &n_steps);
        if (rc != JACOBI_OK) return rc;
    }
    int rc = prepare_sets(h, h->t);
    if (rc != JACOBI_OK) return rc;
    if (n_steps == 0) return JACOBI_OK;
    int flips = 0;
    if (!h->use_graph) {
        rc = enqueue(h, n_steps, h->stream, &flips);
        if (rc != JACOBI_OK) return rc;
    } else {
        auto it = h->graphs.find(n_steps);
        if (it == h->graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t x = nullptr;
            hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "begin capture");
            rc = enqueue(h, n_steps, h->cap, &flips);
            e = hipStreamEndCapture(h->cap, &g);
            if (rc != JACOBI_OK || e != hipSuccess) {
                if (g) hipGraphDestroy(g);
                return rc != JACOBI_OK ? rc : hip_fail(e, "end capture");
            }
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                hipGraphDestroy(g);
                return hip_fail(e, "graph instantiate");
            }
            h->graph_objs.push_back(g);
            it = h->graphs.emplace(n_steps, x).first;
        } else {
            // the same schedule: same number of parity flips
            int64_t n = n_steps;
            if (h->dtype == JACOBI_F64)
                while (n > 0) {
                    n -= std::min<int64_t>(h->t, n);
                    ++flips;
                }
        }
        hipError_t e = hipGraphLaunch(it->second, h->stream);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
    }
    h->host_parity ^= (flips & 1);
    h->sweeps += n_steps;
    return JACOBI_OK;
}

int jacobi_batch_residual(jacobi_batch_t* h, double* l2, double* maxabs)
{
    if (!h || !l2) return fail(JACOBI_EINVAL, "null argument");
    AuxProblem none{};
    hipError_t e = launch_residual_tab(h->d_aux, h->count, none, h->parity,
                                       h->total_rblocks, h->partials, h->red_out,
                                       h->stream);
    if (e != hipSuccess) return hip_fail(e, "batch residual");
    std::vector<double> out(2 * (size_t)h->count);
    e = hipMemcpyAsync(out.data(), h->red_out, out.size() * sizeof(double),
                       hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "batch residual copy");
    int rc = check_err(h);
    if (rc != JACOBI_OK) return rc;
    for (int q = 0; q < h->count; ++q) {
        l2[q] = out[2 * q];
        if (maxabs) maxabs[q] = out[2 * q + 1];
    }
    return JACOBI_OK;
}

int jacobi_batch_solve(jacobi_batch_t* h, double rel_tol, const double* r0,
                       int64_t max_sweeps, int64_t check_every, int64_t* sweeps_done,
                       double* final_l2)
{
    if (!h || !sweeps_done || !final_l2) return fail(JACOBI_EINVAL, "null argument");
    if (!(rel_tol > 0) || max_sweeps < 0 || check_every < 1)
        return fail(JACOBI_EINVAL, "need rel_tol > 0, max_sweeps >= 0, check_every >= 1");
    std::vector<double> r(h->count), ref(h->count);
    std::vector<char> done(h->count, 0);
    int rc = jacobi_batch_residual(h, r.data(), nullptr);
    if (rc != JACOBI_OK) return rc;
    for (int q = 0; q < h->count; ++q) {
        ref[q] = (r0 && r0[q] > 0) ? r0[q] : r[q];
        sweeps_done[q] = -1;
        final_l2[q] = r[q];
    }
    int64_t swept = 0;
    int left = h->count;
    for (;;) {
        for (int q = 0; q < h->count; ++q) {
            if (!done[q] && r[q] <= rel_tol * ref[q]) {
                done[q] = 1;
                --left;
                sweeps_done[q] = swept;
                final_l2[q] = r[q];
            }
        }
        if (left == 0 || swept >= max_sweeps) break;
        const int64_t m = std::min(check_every, max_sweeps - swept);
        rc = jacobi_batch_sweep(h, m);
        if (rc != JACOBI_OK) return rc;
        swept += m;
        rc = jacobi_batch_residual(h, r.data(), nullptr);
        if (rc != JACOBI_OK) return rc;
    }
    for (int q = 0; q < h->count; ++q)
        if (!done[q]) final_l2[q] = r[q];
    return JACOBI_OK;
}

int jacobi_batch_current(jacobi_batch_t* h, int32_t i, void** origin,
                         int64_t strides[3])
{
    if (!h || !origin || !strides) return fail(JACOBI_EINVAL, "null argument");
    if (i < 0 || i >= h->count) return fail(JACOBI_EINVAL, "problem index out of range");
    *origin = h->host_parity ? h->g1[i] : h->g0[i];
    strides[0] = 1;
    strides[1] = h->dims[3 * i] + 2;
    strides[2] = (h->dims[3 * i] + 2) * (h->dims[3 * i + 1] + 2);
    return JACOBI_OK;
}

int jacobi_batch_info(jacobi_batch_t* h, int64_t* sweeps_done, int32_t* t,
                      int32_t* tile_rows, int32_t* rows_per_wave,
                      double* tune_ms)
{
    if (!h) return fail(JACOBI_EINVAL, "null handle");
    if (sweeps_done) *sweeps_done = h->sweeps;
    const TripConfig& c = h->sets[h->t].ready ? h->sets[h->t].cfg : default_cfg(h->t);
    if (t) *t = h->t;
    if (tile_rows) *tile_rows = c.R * c.W;
    if (rows_per_wave) *rows_per_wave = c.R;
    if (tune_ms) *tune_ms = h->tune_ms;
    return JACOBI_OK;
}

int jacobi_batch_tune_log(jacobi_batch_t* h, int32_t cap, int32_t* t,
                          int32_t* tile_rows, int32_t* rows_per_wave,
                          double* glups, int32_t* n)
{
    if (!h || !n) return fail(JACOBI_EINVAL, "null argument");
    const int m = (int)h->tune_log.size();
    *n = m;
    for (int x = 0; x < m && x < cap; ++x) {
        if (t) t[x] = h->tune_log[x].first.T;
        if (tile_rows) tile_rows[x] = h->tune_log[x].first.R * h->tune_log[x].first.W;
        if (rows_per_wave) rows_per_wave[x] = h->tune_log[x].first.R;
        if (glups) glups[x] = h->tune_log[x].second;
    }
    return JACOBI_OK;
}

int jacobi_batch_sync(jacobi_batch_t* h)
{
    if (!h) return fail(JACOBI_EINVAL, "null handle");
    return check_err(h);
}

int jacobi_batch_destroy(jacobi_batch_t* h)
{
    if (!h) return JACOBI_OK;
    // work, graphs included, may still be running on the caller's stream
    if (h->stream || !h->graphs.empty()) (void)hipStreamSynchronize(h->stream);
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t g : h->graph_objs) (void)hipGraphDestroy(g);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
    return JACOBI_OK;
}

}  // extern "C"
