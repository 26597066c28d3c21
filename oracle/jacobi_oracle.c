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
int oracle_max_threads(void)
{
    return omp_get_max_threads();
}
