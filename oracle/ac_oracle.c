/*
 * Allen-Cahn explicit finite-difference stepper: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU path is compared against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links, calls or falls back to it, and the two share no code.
 *
 * What is computed (Kim, "Fast Numerical Simulation of Allen-Cahn Equation"):
 *   PDE      phi_t = -F'(phi)/eps^2 + Lap phi,  F(phi) = (phi^2 - 1)^2 / 4
 *                                                     (section 1, Eq. oriACeq)
 *   grid     cell centres x_i = a + (i - 1/2) h, row-major, x fastest
 *                                                     (section 2, grid definition)
 *   BC       zero Neumann: each ghost cell equals the interior cell next to it
 *            along the face normal, so a neighbour that lies outside the grid
 *            is replaced by the cell itself        (section 2, boundary condition)
 *   scheme   phi^{n+1} = phi^n + dt * ( (phi^n - (phi^n)^3)/eps^2 + Lap_h phi^n )
 *            with the 5-point Laplacian in 2D       (section 2.1, Eq. pytorchACeq)
 *            and its 7-point extension in 3D        (section 2: "easily extended")
 *
 * Readings where the paper is silent:
 *   - the 3D operator is the 7-point Laplacian with the same face rule;
 *   - the neighbour sum is written per axis, (x- + x+) + (y- + y+) [+ (z- + z+)],
 *     so that reflecting an axis leaves every sum bitwise unchanged;
 *   - the update keeps the literal form phi + dt*(-(phi^3 - phi)/eps^2 + Lap),
 *     not the (1+alpha)phi - alpha phi^3 rearrangement, which does not keep
 *     phi = +-1 bitwise fixed.
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off so no FMA contraction or
 * reassociation changes the rounding of the expressions as written.  OpenMP
 * (over rows / planes / instances) is used for timing only: every cell is
 * computed by the same expression from the previous time level, so the result
 * does not depend on the thread count.
 */
#define _GNU_SOURCE
#include <sched.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* One explicit step on a 2D grid (section 2.1, Eq. pytorchACeq). */
static void step2d_once(const double *p, double *q, int64_t nx, int64_t ny,
                        double h, double dt, double eps, int nthreads)
{
#pragma omp parallel for num_threads(nthreads) schedule(static) if (nthreads > 1)
    for (int64_t j = 0; j < ny; ++j) {
        for (int64_t i = 0; i < nx; ++i) {
            const int64_t c = j * nx + i;
            const double v = p[c];
            /* zero-Neumann ghost: a missing neighbour reads the cell itself */
            const double xm = (i > 0) ? p[c - 1] : v;
            const double xp = (i < nx - 1) ? p[c + 1] : v;
            const double ym = (j > 0) ? p[c - nx] : v;
            const double yp = (j < ny - 1) ? p[c + nx] : v;
            const double lap = ((xm + xp) + (ym + yp) - 4.0 * v) / (h * h);
            const double reaction = -(v * v * v - v) / (eps * eps);
            q[c] = v + dt * (reaction + lap);
        }
    }
}

/* One explicit step on a 3D grid: the 7-point extension of the 2D scheme. */
static void step3d_once(const double *p, double *q, int64_t nx, int64_t ny,
                        int64_t nz, double h, double dt, double eps, int nthreads)
{
    const int64_t plane = nx * ny;
#pragma omp parallel for num_threads(nthreads) schedule(static) if (nthreads > 1)
    for (int64_t k = 0; k < nz; ++k) {
        for (int64_t j = 0; j < ny; ++j) {
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t c = k * plane + j * nx + i;
                const double v = p[c];
                const double xm = (i > 0) ? p[c - 1] : v;
                const double xp = (i < nx - 1) ? p[c + 1] : v;
                const double ym = (j > 0) ? p[c - nx] : v;
                const double yp = (j < ny - 1) ? p[c + nx] : v;
                const double zm = (k > 0) ? p[c - plane] : v;
                const double zp = (k < nz - 1) ? p[c + plane] : v;
                const double lap =
                    ((xm + xp) + (ym + yp) + (zm + zp) - 6.0 * v) / (h * h);
                const double reaction = -(v * v * v - v) / (eps * eps);
                q[c] = v + dt * (reaction + lap);
            }
        }
    }
}

/* Number of CPUs this process may run on (sched_getaffinity). */
int ora_cpus_available(void)
{
    cpu_set_t set;
    CPU_ZERO(&set);
    if (sched_getaffinity(0, sizeof(set), &set) != 0)
        return 1;
    int n = CPU_COUNT(&set);
    return n > 0 ? n : 1;
}

/* Advance phi (nx*ny doubles, row-major, x fastest) by nsteps explicit steps.
 * Returns 0 on success, -1 on bad arguments, -2 if scratch allocation fails. */
int ora_step2d(double *phi, int64_t nx, int64_t ny, double h, double dt,
               double eps, int64_t nsteps, int nthreads)
{
    if (!phi || nx < 1 || ny < 1 || nsteps < 0 || nthreads < 1)
        return -1;
    const size_t n = (size_t)nx * (size_t)ny;
    double *tmp = (double *)malloc(n * sizeof(double));
    if (!tmp)
        return -2;
    double *src = phi, *dst = tmp;
    for (int64_t s = 0; s < nsteps; ++s) {
        step2d_once(src, dst, nx, ny, h, dt, eps, nthreads);
        double *t = src; src = dst; dst = t;
    }
    if (src != phi)
        memcpy(phi, src, n * sizeof(double));
    free(tmp);
    return 0;
}

/* Advance phi (nx*ny*nz doubles, index (k*ny + j)*nx + i) by nsteps steps. */
int ora_step3d(double *phi, int64_t nx, int64_t ny, int64_t nz, double h,
               double dt, double eps, int64_t nsteps, int nthreads)
{
    if (!phi || nx < 1 || ny < 1 || nz < 1 || nsteps < 0 || nthreads < 1)
        return -1;
    const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    double *tmp = (double *)malloc(n * sizeof(double));
    if (!tmp)
        return -2;
    double *src = phi, *dst = tmp;
    for (int64_t s = 0; s < nsteps; ++s) {
        step3d_once(src, dst, nx, ny, nz, h, dt, eps, nthreads);
        double *t = src; src = dst; dst = t;
    }
    if (src != phi)
        memcpy(phi, src, n * sizeof(double));
    free(tmp);
    return 0;
}

/* Independent 2D instances, each with its own size and (h, dt, eps); the same
 * loop as ora_step2d per instance.  Threads split the instance list. */
int ora_step_batched2d(int32_t n_inst, double *const *phis, const int64_t *nx,
                       const int64_t *ny, const double *h, const double *dt,
                       const double *eps, int64_t nsteps, int nthreads)
{
    if (n_inst < 0 || (n_inst > 0 && (!phis || !nx || !ny || !h || !dt || !eps)))
        return -1;
    int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) if (nthreads > 1) reduction(| : bad)
    for (int32_t b = 0; b < n_inst; ++b) {
        if (ora_step2d(phis[b], nx[b], ny[b], h[b], dt[b], eps[b], nsteps, 1) != 0)
            bad |= 1;
    }
    return bad ? -1 : 0;
}
