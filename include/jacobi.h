/*
 * jacobi.h -- C-ABI of libjacobi: temporally blocked 3D 7-point Jacobi on
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Wittmann, Hager, Treibig, Wellein, "Leveraging shared caches for
 * parallel temporal blocking of stencil codes on multicore processors and
 * clusters", 2010):
 *   - Sect. 1.1, Eq. (1): one sweep updates every interior cell of an
 *     (nx+2) x (ny+2) x (nz+2) box as
 *         B[i,j,k] = (A[i-1,j,k] + A[i+1,j,k] + A[i,j-1,k] + A[i,j+1,k]
 *                     + A[i,j,k-1] + A[i,j,k+1]) / 6,
 *     successive sweeps writing grids A and B in turn; the outer layer of the
 *     box is a fixed Dirichlet boundary (the boundary value problem).
 *   - Sect. 2.1: temporal blocking -- t sweeps are applied per trip through
 *     memory; the optional "compressed grid" keeps a single grid and stores
 *     each trip's result shifted by (-t,-t,-t) or (+t,+t,+t) (here with E
 *     extra planes along k, see jacobi_grid_bytes).
 *   - Sect. 2.2, Eq. (3): relaxed synchronization through per-worker progress
 *     counters instead of global barriers.
 *
 * Arithmetic: the six neighbours are summed as a left fold in the order above
 * (i-1, i+1, j-1, j+1, k-1, k+1), then multiplied by the rounded constant
 * fl(1/6); IEEE round-to-nearest, no fused multiply-add.  FP64 results are
 * bitwise identical for every t, layout and tile shape.
 *
 * 27-point update (jacobi_desc.stencil = 27; not in the paper, another
 * stencil on the same k-streaming pipeline): the weighted mean of the 26
 * neighbours, 7/64 for each of the 6 faces, 3/128 for each of the 12 edges
 * and 1/128 for each of the 8 corners (the weights sum to 1).  With, for
 * plane p of the 3x3 window of A around (i,j), a(p) the centre, b(p) the left
 * fold of (i-1,j), (i+1,j), (i,j-1), (i,j+1) and c(p) that of (i-1,j-1),
 * (i+1,j-1), (i-1,j+1), (i+1,j+1):
 *     B[i,j,k] = (7/64 ((b(k) + a(k-1)) + a(k+1))
 *                 + 3/128 ((c(k) + b(k-1)) + b(k+1)))
 *                + 1/128 (c(k-1) + c(k+1)),
 * bitwise identical for every t and tile shape.
 *
 * Memory: every device buffer is owned by the caller (e.g. allocated with
 * PyTorch); the library allocates no device memory and owns only the host
 * handle (and the static reduction array of jacobi_residual_noalloc).  Box layout: element (i,j,k) of a frame with origin O and strides
 * (1, px, py) is O[k*py + j*px + i]; i is contiguous.
 *
 * Errors: every function returns 0 (JACOBI_OK) or a negative jacobi_status and
 * never aborts; jacobi_last_error() gives a message for the calling thread.
 * Kernel launches are asynchronous on the descriptor's stream; faults of a
 * launched kernel and watchdog time-outs surface at the next call that
 * synchronizes (jacobi_residual, jacobi_solve, jacobi_sync).
 *
 * A handle is not thread-safe; use one handle per stream.
 */
#ifndef JACOBI_H
#define JACOBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    JACOBI_OK = 0,
    JACOBI_EINVAL = -1,       /* bad argument (null, size, range, alignment) */
    JACOBI_EUNSUPPORTED = -2, /* valid request the library does not support */
    JACOBI_EWORKSPACE = -3,   /* workspace missing or too small */
    JACOBI_EHIP = -4,         /* HIP runtime error (launch or kernel fault) */
    JACOBI_ETIMEOUT = -5,     /* a progress-flag wait exceeded its spin bound */
    JACOBI_ESTATE = -6        /* call not valid in the handle's state */
} jacobi_status;

typedef enum {
    JACOBI_F64 = 0,         /* FP64 sweeps */
    JACOBI_F32_REFINED = 1, /* FP32 sweeps of the correction equation, FP64
                               residual and FP64 defect-correction update */
    JACOBI_F32_MULTIGRID = 2 /* as JACOBI_F32_REFINED, but the correction
                               equation is solved by one FP32 multigrid
                               V(2,2)-cycle whose smoother is the weighted
                               Jacobi sweep e' = e + (6/7)(v - e), v the
                               Eq. (1) update plus the right-hand side (the
                               Jacobi update as multigrid smoother,
                               Sect. 1.1); AB layout, n^3 interior with
                               n = 2^k - 1; jacobi_sweep(h, n) makes n outer
                               steps and t is ignored */
} jacobi_dtype;

typedef enum {
    JACOBI_LAYOUT_AB = 0,        /* two grids, written in turn (Sect. 1.1) */
    JACOBI_LAYOUT_COMPRESSED = 1 /* one grid, shifted stores (Sect. 2.1) */
} jacobi_layout;

typedef struct {
    int64_t nx, ny, nz;  /* interior dims, each >= 1; box is (n+2) per axis */
    int32_t dtype;       /* jacobi_dtype */
    int32_t layout;      /* jacobi_layout */
    int32_t t;           /* sweeps per trip, 1..8; 0 = autotune for A/B FP64
                            handles with default tile and segments (the first
                            jacobi_sweep of >= 96 sweeps times the candidate
                            (t, tile) configurations on real sweeps, keeps the
                            fastest; t = 5 until then), else 4 */
    int32_t tile_rows;   /* j-rows per tile: 0 = default for t (for A/B FP64
                            trips of t = 5 the planner picks the 4x8 or the
                            3x12 shape by box size), else one of the
                            compiled shapes (jacobi_tile_supported) */
    int32_t rows_per_wave; /* 0 = default; with tile_rows selects the shape */
    int32_t seg_len;     /* k planes per tile segment, 0 = automatic;
                            COMPRESSED needs >= 2t, and caps E (below) at
                            seg_len - 2t */
    int32_t inner_sweeps;/* JACOBI_F32_REFINED: FP32 sweeps per outer
                            correction step (0 = 32) */
    int32_t use_graph;   /* 1: A/B FP64 jacobi_sweep calls are captured once
                            per (n_steps, current grid) into a hipGraph on an
                            internal stream (up to 8 kept) and replayed on
                            `stream`; 0: every trip is launched eagerly */
    int32_t teams;       /* A/B FP64: 0 or 1 = one launch per trip (kernel
                            boundaries are the only synchronization); k >= 2
                            = up to k trips ("teams", Sect. 2.1) in one
                            persistent launch, tiles synchronized by per-tile
                            progress counters (Sect. 2.2, Eq. (3)); 1..1024 */
    int32_t looseness;   /* with teams >= 2, the upper looseness d_u of
                            Eq. (3): a tile starts trip r only once every
                            tile has finished trip r-d_u-1 (0 = lockstep, a
                            barrier between trips inside the launch); < 0 =
                            no such bound (neighbour counters only) */
    void *grid0;         /* FP64 grid buffer (device); see jacobi_grid_bytes */
    void *grid1;         /* second FP64 grid for JACOBI_LAYOUT_AB, else NULL */
    void *workspace;     /* device scratch owned by the caller */
    size_t workspace_bytes;
    void *stream;        /* hipStream_t (NULL = default stream) */
    int32_t stencil;     /* 0 or 7: Eq. (1); 27: the 27-point Jacobi update
                            (below), FP64 and the AB layout only, teams <= 1,
                            t in 1..4; t = 0 autotunes as above among the
                            27-point candidates (t = 2 until then);
                            jacobi_residual and jacobi_solve return
                            JACOBI_EUNSUPPORTED.  Its compiled tile shapes
                            (t, tile_rows, rows_per_wave): (1,32,4),
                            (2,32,4), (2,36,3), (2,32,2), (3,24,3),
                            (3,32,4), (4,24,3); the defaults for t = 1..4
                            are (1,32,4), (2,36,3), (3,24,3), (4,24,3)
                            (jacobi_tile_supported answers for Eq. (1)) */
} jacobi_desc;

typedef struct jacobi_s jacobi_t;

/* Bytes each grid buffer must hold for `d` (dims, layout, t and seg_len are
 * read).  AB: (nx+2)(ny+2)(nz+2) doubles.  COMPRESSED: the box plus 2t shift
 * planes in i and j and 2t+2E in k, (nx+2+2t)(ny+2+2t)(nz+2+2t+2E) doubles
 * (2t, not t, so that a trip of any length <= t fits from every shift
 * offset).  A trip of L sweeps shifts by L in i and j and by L+E in k, with
 * E = 2t for t <= 5 (at most seg_len - 2t when seg_len is set) and E = 0 for
 * t > 5: the extra k shift lets a tile run up to E steps behind its
 * neighbours before they wait for it.  JACOBI_KREV and JACOBI_ZEXTRA (see
 * jacobi_create) change E and must be the same here and there.
 * Errors: JACOBI_EINVAL. */
int jacobi_grid_bytes(const jacobi_desc *d, size_t *bytes);

/* Bytes of device workspace `d` needs (flags, reduction partials, and for
 * JACOBI_F32_REFINED two FP32 correction grids and an FP32 right-hand side).
 * The workspace must be 256-byte aligned.  Errors: JACOBI_EINVAL. */
int jacobi_workspace_size(const jacobi_desc *d, size_t *bytes);

/* Validates `d` and creates a handle.  The caller must have written the
 * initial box (boundary values and initial interior) into the frame that
 * jacobi_current() reports for the new handle (for AB: grid0 with strides
 * (1, nx+2, (nx+2)(ny+2)); for COMPRESSED: grid0 at the offset reported).
 * May launch set-up kernels on the stream (AB: copies the box into grid1 so
 * both grids carry the boundary).  Errors: JACOBI_EINVAL (null pointers,
 * dims < 1 or > 2^20, misaligned buffers), JACOBI_EUNSUPPORTED (t or tile
 * shape not compiled), JACOBI_EWORKSPACE, JACOBI_EHIP.
 * Environment, read here (diagnostics; results are the same bits):
 *   JACOBI_SPIN_LIMIT=n   bound on a compressed tile's waits (then
 *                         JACOBI_ETIMEOUT);
 *   JACOBI_XCD_ORDER=0    compressed trips take tiles from one ticket counter
 *                         instead of per-XCD claim groups (used for trips of
 *                         4 or more sweeps);
 *   JACOBI_AB_BANDS=0     A/B trips of several workgroup generations give each
 *                         XCD one contiguous range of tiles instead of bands;
 *   JACOBI_KREV=0         backward compressed trips stream k upwards (E = 0);
 *   JACOBI_ZEXTRA=planes  the extra k shift E of compressed trips. */
int jacobi_create(const jacobi_desc *d, jacobi_t **out);

/* Applies n_steps Jacobi sweeps (JACOBI_F32_REFINED: n_steps FP32 inner
 * sweeps, grouped into outer correction steps of inner_sweeps) to the
 * current iterate.  Asynchronous on the stream.  n_steps >= 0. */
int jacobi_sweep(jacobi_t *h, int64_t n_steps);

/* ||fold(u nbrs) - 6u||_2 over the interior of the current iterate, FP64,
 * deterministic fixed-order reduction (7-point handles only).  Synchronizes the stream; reports a
 * pending kernel fault (JACOBI_EHIP) or watchdog time-out (JACOBI_ETIMEOUT).
 * Optional `maxabs` receives max |r|. */
int jacobi_residual(jacobi_t *h, double *l2, double *maxabs);

/* Runs sweeps until ||r||_2 <= rel_tol * r0, checking every `check_every`
 * sweeps, at most max_sweeps.  r0 <= 0 means: the residual of the current
 * iterate.  Outputs the sweeps done and the final residual norm. */
int jacobi_solve(jacobi_t *h, double rel_tol, double r0, int64_t max_sweeps,
                 int64_t check_every, int64_t *sweeps_done, double *final_l2);

/* Waits for the stream and reports pending errors as jacobi_residual does. */
int jacobi_sync(jacobi_t *h);

/* Pointer to logical cell (0,0,0) of the current iterate and its strides in
 * elements {1, px, py}.  Valid until the next jacobi_sweep. */
int jacobi_current(jacobi_t *h, void **origin, int64_t strides[3]);

/* Sweeps applied so far and the trip configuration in use. */
int jacobi_info(jacobi_t *h, int64_t *sweeps_done, int32_t *t,
                int32_t *tile_rows, int32_t *seg_len);

/* The autotuner's measurements of a t = 0 handle: up to `cap` entries of
 * (t, tile_rows, rows_per_wave, GLUP/s); *n = entries made (0 before the
 * tuning has run); optional *tune_ms = the tuning's duration on the stream. */
int jacobi_tune_log(jacobi_t *h, int32_t cap, int32_t *t, int32_t *tile_rows,
                    int32_t *rows_per_wave, double *glups, int32_t *n,
                    double *tune_ms);

/* Releases the handle; never frees caller buffers. */
int jacobi_destroy(jacobi_t *h);

/* Message of the last error of the calling thread ("" if none). */
const char *jacobi_last_error(void);

/* 1 if the trip kernel is compiled for sweeps-per-trip t with tiles of
 * `tile_rows` j-rows made of `rows_per_wave`-row waves, else 0. */
int jacobi_tile_supported(int32_t dtype, int32_t t, int32_t tile_rows,
                          int32_t rows_per_wave);

/* ---- batched problems ---------------------------------------------------
 * Many independent problems of uneven sizes swept together: one persistent
 * launch per trip covers every tile of every problem (largest problems first,
 * one ticket counter), and the schedule of each distinct n_steps is captured
 * once into a hipGraph and replayed.  Both grids of problem q are dense boxes
 * (nx+2)(ny+2)(nz+2) doubles, caller-owned; grid0[q] holds the initial box
 * before jacobi_batch_create (which copies it into grid1[q]).
 * With t == 0 the library's autotuner times its candidate (t, tile shape)
 * configurations on the first sweeps of the batch (HIP events; FP64: these
 * are real sweeps and count toward n_steps; FP32-refined: FP32 trips of the
 * correction grids, the iterate is untouched) and keeps the fastest. */
typedef struct {
    int32_t count;            /* number of problems, >= 1 */
    int32_t dtype;            /* JACOBI_F64 or JACOBI_F32_REFINED */
    const int64_t *dims;      /* host array [count][3]: nx, ny, nz */
    void *const *grid0;       /* host array [count] of device pointers */
    void *const *grid1;       /* host array [count] of device pointers */
    int32_t t;                /* sweeps per trip 1..8; 0 = autotune */
    int32_t tile_rows;        /* with t > 0: tile shape (0 = default) */
    int32_t rows_per_wave;
    int32_t inner_sweeps;     /* JACOBI_F32_REFINED: FP32 sweeps per outer step */
    int32_t use_graph;        /* nonzero: capture/replay hipGraphs */
    int32_t reserved;
    void *workspace;          /* device, 256-byte aligned */
    size_t workspace_bytes;
    void *stream;
} jacobi_batch_desc;

typedef struct jacobi_batch_s jacobi_batch_t;

int jacobi_batch_workspace_size(const jacobi_batch_desc *d, size_t *bytes);
int jacobi_batch_create(const jacobi_batch_desc *d, jacobi_batch_t **out);
/* n_steps sweeps of every problem (F32_REFINED: FP32 inner sweeps grouped in
 * outer steps of inner_sweeps).  Asynchronous apart from the first call of
 * an autotuned batch (which synchronizes to read its timers). */
int jacobi_batch_sweep(jacobi_batch_t *h, int64_t n_steps);
/* Per-problem residual norms (and optional max |r|), host arrays [count];
 * synchronizes. */
int jacobi_batch_residual(jacobi_batch_t *h, double *l2, double *maxabs);
/* Sweeps every problem until each has ||r_q|| <= rel_tol * r0[q] (r0 NULL or
 * r0[q] <= 0: the problem's current residual), checking every check_every
 * sweeps, at most max_sweeps.  sweeps_done[q] = sweeps at the first check
 * where problem q met its tolerance (-1 if it never did); final_l2[q] = its
 * residual then (or at the end).  Problems that converged keep being swept
 * until all have (their reported counts are not affected). */
int jacobi_batch_solve(jacobi_batch_t *h, double rel_tol, const double *r0,
                       int64_t max_sweeps, int64_t check_every,
                       int64_t *sweeps_done, double *final_l2);
int jacobi_batch_current(jacobi_batch_t *h, int32_t i, void **origin,
                         int64_t strides[3]);
/* Sweeps done, chosen configuration, and the time spent tuning (ms). */
int jacobi_batch_info(jacobi_batch_t *h, int64_t *sweeps_done, int32_t *t,
                      int32_t *tile_rows, int32_t *rows_per_wave,
                      double *tune_ms);
/* The autotuner's measurements: up to `cap` entries; *n = entries made. */
int jacobi_batch_tune_log(jacobi_batch_t *h, int32_t cap, int32_t *t,
                          int32_t *tile_rows, int32_t *rows_per_wave,
                          double *glups, int32_t *n);
int jacobi_batch_sync(jacobi_batch_t *h);
int jacobi_batch_destroy(jacobi_batch_t *h);

/* ---- no-allocation residual ----------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual of jacobi_residual, ||fold(u nbrs) - 6u||_2 and max |r| over the
 * interior of the FP64 field whose logical cell (0,0,0) is at `origin`
 * (strides {1, px, py} elements; boundary layer included, so px >= nx+2,
 * py >= px*(ny+2)), written to the device array out[0] (norm), out[1]
 * (max |r|).  No handle, no workspace, no allocation: the reduction partials
 * live in a static device array of the library, JACOBI_NOALLOC_SCRATCH_BYTES
 * per GPU, held until the process ends; the field may need up to
 * JACOBI_NOALLOC_SCRATCH_BYTES / 16 reduction blocks, i.e.
 * ceil(nx/62) * ceil(ny/16) <= 65536 (larger fields: JACOBI_EINVAL).
 * Asynchronous on `stream`; the result is bitwise that of jacobi_residual.
 * All calls on one GPU share its array: calls that overlap on one GPU
 * (different streams or threads) race; calls on one stream are ordered.
 * Errors: JACOBI_EINVAL, JACOBI_EHIP. */
#define JACOBI_NOALLOC_SCRATCH_BYTES (1 << 20)
int jacobi_residual_noalloc(const double *origin, int64_t px, int64_t py,
                            int64_t nx, int64_t ny, int64_t nz, double *out,
                            void *stream);

/* ---- bandwidth probes (Table 1 of the paper: STREAM copy and the
 *      array-update loop a[i] += 1 of Sect. 2.3) ---------------------------
 * n doubles, n even, 16-byte aligned device buffers; asynchronous. */
int jacobi_probe_copy(const double *src, double *dst, int64_t n, void *stream);
int jacobi_probe_update(double *a, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* JACOBI_H */
