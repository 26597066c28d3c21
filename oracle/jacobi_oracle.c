/*
 * CPU oracle for the 3D 7-point Jacobi method -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU library shares no code with it.
 *
 * Plain, slow, obviously correct: every function is the textbook definition
 * written out with triple loops, no blocking, no fusion, no reordering.
 *
 * Grid layout ("box"): (nz+2) x (ny+2) x (nx+2) values, i contiguous:
 *     index(i, j, k) = (k*(ny+2) + j)*(nx+2) + i.
 * The outer layer is the Dirichlet boundary; interior is 1..nx, 1..ny, 1..nz.
 *
 * Arithmetic (readings of the paper, Sect. 1.1, Eq. (1)):
 *   - the six neighbours are summed as a left fold in the order Eq. (1) lists
 *     them: i-1, i+1, j-1, j+1, k-1, k+1;
 *   - the sum is multiplied by the rounded constant fl(1/6) (the paper counts
 *     one multiplication and five additions per update, Sect. 2.3);
 *   - IEEE round-to-nearest, no fused multiply-add (built -ffp-contract=off).
 * Successive sweeps write grids A and B in turn (Sect. 1.1).
 *
 * Built with:  gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, k) ((((int64_t)(k)) * (ny + 2) + (j)) * (nx + 2) + (i))

static const double C6 = 1.0 / 6.0;       /* fl64(1/6) = 0x3FC5555555555555 */
static const float C6F = 1.0f / 6.0f;     /* fl32(1/6) = 0x3E2AAAAB */

/* One Jacobi sweep, Eq. (1): dst(interior) = C6 * fold(src neighbours);
 * dst(boundary layer) = src(boundary layer). */
static void sweep_f64(const double *src, double *dst, int64_t nx, int64_t ny,
                      int64_t nz, int nthreads)
{
    int64_t k;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (k = 0; k < nz + 2; ++k) {
        for (int64_t j = 0; j < ny + 2; ++j) {
            for (int64_t i = 0; i < nx + 2; ++i) {
                int interior = (i >= 1 && i <= nx && j >= 1 && j <= ny &&
                                k >= 1 && k <= nz);
                if (!interior) {
                    dst[IDX(i, j, k)] = src[IDX(i, j, k)];
                    continue;
                }
                double s = src[IDX(i - 1, j, k)];
                s = s + src[IDX(i + 1, j, k)];
                s = s + src[IDX(i, j - 1, k)];
                s = s + src[IDX(i, j + 1, k)];
                s = s + src[IDX(i, j, k - 1)];
                s = s + src[IDX(i, j, k + 1)];
                dst[IDX(i, j, k)] = s * C6;
            }
        }
    }
}

/* nsweeps successive sweeps starting from `a`; `b` is a second box used as
 * the other grid.  On return the result is in `a` (copied back if nsweeps is
 * odd).  Returns 0, or -1 on bad arguments. */
int oracle_sweeps_f64(double *a, double *b, int64_t nx, int64_t ny,
                      int64_t nz, int64_t nsweeps, int nthreads)
{
    if (!a || !b || nx < 1 || ny < 1 || nz < 1 || nsweeps < 0)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    double *cur = a, *nxt = b;
    for (int64_t s = 0; s < nsweeps; ++s) {
        sweep_f64(cur, nxt, nx, ny, nz, nthreads);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != a)
        memcpy(a, cur, sizeof(double) * (size_t)((nx + 2) * (ny + 2) * (nz + 2)));
    return 0;
}

/* One single-precision sweep of the correction equation
 *     e(interior) = (fold(e neighbours) + rhs) * fl32(1/6),
 * the Jacobi iteration for 6e - sum6(e) = rhs.  `rhs` is a box of the same
 * shape (only interior entries are read); NULL means rhs = 0.  The boundary
 * layer of dst is copied from src. */
static void sweep_f32(const float *src, float *dst, const float *rhs,
                      int64_t nx, int64_t ny, int64_t nz, int nthreads)
{
    int64_t k;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (k = 0; k < nz + 2; ++k) {
        for (int64_t j = 0; j < ny + 2; ++j) {
            for (int64_t i = 0; i < nx + 2; ++i) {
                int interior = (i >= 1 && i <= nx && j >= 1 && j <= ny &&
                                k >= 1 && k <= nz);
                if (!interior) {
                    dst[IDX(i, j, k)] = src[IDX(i, j, k)];
                    continue;
                }
                float s = src[IDX(i - 1, j, k)];
                s = s + src[IDX(i + 1, j, k)];
                s = s + src[IDX(i, j - 1, k)];
                s = s + src[IDX(i, j + 1, k)];
                s = s + src[IDX(i, j, k - 1)];
                s = s + src[IDX(i, j, k + 1)];
                if (rhs)
                    s = s + rhs[IDX(i, j, k)];
                dst[IDX(i, j, k)] = s * C6F;
            }
        }
    }
}

int oracle_sweeps_f32(float *a, float *b, const float *rhs, int64_t nx,
                      int64_t ny, int64_t nz, int64_t nsweeps, int nthreads)
{
    if (!a || !b || nx < 1 || ny < 1 || nz < 1 || nsweeps < 0)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    float *cur = a, *nxt = b;
    for (int64_t s = 0; s < nsweeps; ++s) {
        sweep_f32(cur, nxt, rhs, nx, ny, nz, nthreads);
        float *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != a)
        memcpy(a, cur, sizeof(float) * (size_t)((nx + 2) * (ny + 2) * (nz + 2)));
    return 0;
}

/* Residual of the discrete Laplace equation at every interior cell:
 *     r = fold(u neighbours) - fl(6 * u)
 * (the same neighbour fold as the sweep).  r is a box; its boundary layer is
 * set to zero. */
int oracle_residual_f64(const double *u, double *r, int64_t nx, int64_t ny,
                        int64_t nz, int nthreads)
{
    if (!u || !r || nx < 1 || ny < 1 || nz < 1)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    int64_t k;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (k = 0; k < nz + 2; ++k) {
        for (int64_t j = 0; j < ny + 2; ++j) {
            for (int64_t i = 0; i < nx + 2; ++i) {
                int interior = (i >= 1 && i <= nx && j >= 1 && j <= ny &&
                                k >= 1 && k <= nz);
                if (!interior) {
                    r[IDX(i, j, k)] = 0.0;
                    continue;
                }
                double s = u[IDX(i - 1, j, k)];
                s = s + u[IDX(i + 1, j, k)];
                s = s + u[IDX(i, j - 1, k)];
                s = s + u[IDX(i, j + 1, k)];
                s = s + u[IDX(i, j, k - 1)];
                s = s + u[IDX(i, j, k + 1)];
                r[IDX(i, j, k)] = s - 6.0 * u[IDX(i, j, k)];
            }
        }
    }
    return 0;
}

/* 2-norm of the residual over the interior, sum of squares accumulated in
 * long double in storage order (single thread). */
double oracle_residual_norm_f64(const double *u, int64_t nx, int64_t ny,
                                int64_t nz)
{
    if (!u || nx < 1 || ny < 1 || nz < 1)
        return -1.0;
    long double acc = 0.0L;
    for (int64_t k = 1; k <= nz; ++k) {
        for (int64_t j = 1; j <= ny; ++j) {
            for (int64_t i = 1; i <= nx; ++i) {
                double s = u[IDX(i - 1, j, k)];
                s = s + u[IDX(i + 1, j, k)];
                s = s + u[IDX(i, j - 1, k)];
                s = s + u[IDX(i, j + 1, k)];
                s = s + u[IDX(i, j, k - 1)];
                s = s + u[IDX(i, j, k + 1)];
                double r = s - 6.0 * u[IDX(i, j, k)];
                acc += (long double)r * (long double)r;
            }
        }
    }
    return (double)sqrtl(acc);
}

/* Number of threads an OpenMP parallel region gets by default. */
/* ------------------------------------------------------------------------
 * 27-point Jacobi (not in the paper; one of the "other stencils" the k-
 * streaming pipeline can carry).  The Jacobi update for the 27-point
 * Laplacian with face, edge and corner weights 14, 3 and 1 over 128 (they
 * sum to 1), with this fold order: per plane p at the cell's (i, j),
 *   A(p) = x(i, j, p),
 *   B(p) = ((x(i-1,j) + x(i+1,j)) + x(i,j-1)) + x(i,j+1),
 *   C(p) = ((x(i-1,j-1) + x(i+1,j-1)) + x(i-1,j+1)) + x(i+1,j+1);
 * then F = (B(k) + A(k-1)) + A(k+1)      (the 6 faces),
 *      E = (C(k) + B(k-1)) + B(k+1)      (the 12 edges),
 *      K = C(k-1) + C(k+1)               (the 8 corners),
 *      u' = (W_F F + W_E E) + W_C K,  W_F = 7/64, W_E = 3/128, W_C = 1/128
 * (dyadic, so the weights are exact).  The whole boundary layer (faces,
 * edges and corners of the box) is read and passed through unchanged.
 * ---------------------------------------------------------------------- */
static const double W27_F = 7.0 / 64.0;
static const double W27_E = 3.0 / 128.0;
static const double W27_C = 1.0 / 128.0;

static void sweep27_f64(const double *src, double *dst, int64_t nx, int64_t ny,
                        int64_t nz, int nthreads)
{
    int64_t k;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (k = 0; k < nz + 2; ++k) {
        for (int64_t j = 0; j < ny + 2; ++j) {
            for (int64_t i = 0; i < nx + 2; ++i) {
                int interior = (i >= 1 && i <= nx && j >= 1 && j <= ny &&
                                k >= 1 && k <= nz);
                if (!interior) {
                    dst[IDX(i, j, k)] = src[IDX(i, j, k)];
                    continue;
                }
                double a[3], b[3], c[3];
                for (int d = 0; d < 3; ++d) {
                    const int64_t p = k - 1 + d;
                    a[d] = src[IDX(i, j, p)];
                    double bs = src[IDX(i - 1, j, p)];
                    bs = bs + src[IDX(i + 1, j, p)];
                    bs = bs + src[IDX(i, j - 1, p)];
                    bs = bs + src[IDX(i, j + 1, p)];
                    b[d] = bs;
                    double cs = src[IDX(i - 1, j - 1, p)];
                    cs = cs + src[IDX(i + 1, j - 1, p)];
                    cs = cs + src[IDX(i - 1, j + 1, p)];
                    cs = cs + src[IDX(i + 1, j + 1, p)];
                    c[d] = cs;
                }
                const double f = (b[1] + a[0]) + a[2];
                const double e = (c[1] + b[0]) + b[2];
                const double kk = c[0] + c[2];
                dst[IDX(i, j, k)] = (W27_F * f + W27_E * e) + W27_C * kk;
            }
        }
    }
}

int oracle_sweeps27_f64(double *a, double *b, int64_t nx, int64_t ny,
                        int64_t nz, int64_t nsweeps, int nthreads)
{
    if (!a || !b || nx < 1 || ny < 1 || nz < 1 || nsweeps < 0)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    double *cur = a, *nxt = b;
    for (int64_t s = 0; s < nsweeps; ++s) {
        sweep27_f64(cur, nxt, nx, ny, nz, nthreads);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != a)
        memcpy(a, cur, sizeof(double) * (size_t)((nx + 2) * (ny + 2) * (nz + 2)));
    return 0;
}

int oracle_max_threads(void)
{
    return omp_get_max_threads();
}
