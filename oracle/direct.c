/*
 * Direct-summation oracle for the voxel gravity forward model.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; it is the plain definition
 * that the fast multipole path approximates.
 *
 * What it computes (May & Knepley, "Optimal, scalable forward models for
 * computing gravity anomalies"):
 *   - Eq. (1) (Sec. 1.1): g(r) = G * integral of rho(x) (r - x) / |r - x|^3 dV,
 *     with the sign convention of Eq. (1): g points from the mass towards r.
 *   - The potential of Eqs. (2)-(4): phi(r) = G * integral of rho(x)/|r - x| dV,
 *     which satisfies lap(phi) = -4 pi G rho, phi -> 0 at infinity and
 *     g = -grad(phi).
 *   - Sec. 2.1: the density is constant on each cell of an
 *     Mx x My x Mz brick mesh, and the integral over a cell is taken with a
 *     one-point (cell centroid, weight = cell volume) or a two-point-per-axis
 *     tensor Gauss-Legendre rule (points at centre +- h/(2 sqrt 3) on each
 *     axis, weight = volume / 8).  The quadrature turns every cell into point
 *     masses, so the discrete sum is the N-body sum of Eq. (11) (Sec. 2.3)
 *     times G.
 *   - A point pair at zero separation contributes nothing (the exact field of
 *     a uniform cell at its own centroid vanishes by symmetry; the paper is
 *     silent on the coincident term).
 *
 * Floating point: IEEE binary64, every per-target (or per-cell) sum
 * accumulated with Neumaier's compensated summation.  Built with
 * -ffp-contract=off so that no FMA contraction changes the rounding.
 *
 * Layouts (all row-major, C order):
 *   rho     [batch][nz][ny][nx]   x index fastest
 *   targets [m][3]                (x, y, z)
 *   out     [batch][m][comps]     comps = 1: (gz); 3: (gx, gy, gz);
 *                                 4: (phi, gx, gy, gz)
 *   resid   [batch][m][comps]     same layout as out (input of the transpose)
 *   drho    [batch][nz][ny][nx]   output of the transpose
 *
 * Return value: 0 on success, -1 on invalid arguments, -2 on allocation
 * failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double s;
    double c;
} nsum_t;

/* Neumaier's improvement of Kahan summation. */
static inline void nsum_add(nsum_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double nsum_value(const nsum_t *a) { return a->s + a->c; }

/* Gauss-Legendre rule on [-1/2, 1/2] (units of the cell edge).
 * Returns the number of points per axis; fills abscissae and weights. */
static int gauss_rule(int q, double x[2], double w[2])
{
    if (q == 1) {
        x[0] = 0.0;
        w[0] = 1.0;
        return 1;
    }
    if (q == 2) {
        double a = 0.5 / sqrt(3.0);
        x[0] = -a;
        x[1] = a;
        w[0] = 0.5;
        w[1] = 0.5;
        return 2;
    }
    return 0;
}

static int valid_comps(int comps) { return comps == 1 || comps == 3 || comps == 4; }

/* Field of all cells at each target: Eq. (1) under the cell quadrature. */
int oracle_forward(int nx, int ny, int nz, const double *origin, const double *h,
                   int q, int batch, const double *rho, int64_t m,
                   const double *targets, int comps, double G, double *out)
{
    double gx[2], gw[2];
    int nq = gauss_rule(q, gx, gw);
    if (nq == 0 || nx < 0 || ny < 0 || nz < 0 || batch < 1 || m < 0 ||
        !valid_comps(comps))
        return -1;
    const int64_t ncell = (int64_t)nx * ny * nz;
    const double vol = h[0] * h[1] * h[2];
    int err = 0;

#pragma omp parallel
    {
        nsum_t *acc = (nsum_t *)malloc(sizeof(nsum_t) * (size_t)batch * 4);
        if (!acc) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t j = 0; j < m; ++j) {
            if (!acc)
                continue;
            const double tx = targets[3 * j + 0];
            const double ty = targets[3 * j + 1];
            const double tz = targets[3 * j + 2];
            memset(acc, 0, sizeof(nsum_t) * (size_t)batch * 4);
            for (int k = 0; k < nz; ++k)
                for (int jj = 0; jj < ny; ++jj)
                    for (int i = 0; i < nx; ++i) {
                        const int64_t cell = ((int64_t)k * ny + jj) * nx + i;
                        int any = 0;
                        for (int b = 0; b < batch; ++b)
                            any |= rho[b * ncell + cell] != 0.0;
                        if (!any)
                            continue; /* every term of this cell is zero */
                        const double cx = origin[0] + (i + 0.5) * h[0];
                        const double cy = origin[1] + (jj + 0.5) * h[1];
                        const double cz = origin[2] + (k + 0.5) * h[2];
                        for (int a = 0; a < nq; ++a)
                            for (int bq = 0; bq < nq; ++bq)
                                for (int c = 0; c < nq; ++c) {
                                    const double px = cx + gx[c] * h[0];
                                    const double py = cy + gx[bq] * h[1];
                                    const double pz = cz + gx[a] * h[2];
                                    const double w = vol * gw[a] * gw[bq] * gw[c];
                                    const double dx = tx - px;
                                    const double dy = ty - py;
                                    const double dz = tz - pz;
                                    const double r2 = dx * dx + dy * dy + dz * dz;
                                    if (r2 == 0.0)
                                        continue; /* coincident pair */
                                    const double r = sqrt(r2);
                                    const double inv_r = 1.0 / r;
                                    const double inv_r3 = 1.0 / (r2 * r);
                                    for (int b = 0; b < batch; ++b) {
                                        const double mm = rho[b * ncell + cell] * w;
                                        if (mm == 0.0)
                                            continue;
                                        nsum_t *ab = acc + 4 * b;
                                        if (comps == 4)
                                            nsum_add(&ab[0], mm * inv_r);
                                        if (comps != 1) {
                                            nsum_add(&ab[1], mm * dx * inv_r3);
                                            nsum_add(&ab[2], mm * dy * inv_r3);
                                        }
                                        nsum_add(&ab[3], mm * dz * inv_r3);
                                    }
                                }
                    }
            for (int b = 0; b < batch; ++b) {
                double *o = out + ((int64_t)b * m + j) * comps;
                const nsum_t *ab = acc + 4 * b;
                if (comps == 1) {
                    o[0] = G * nsum_value(&ab[3]);
                } else if (comps == 3) {
                    o[0] = G * nsum_value(&ab[1]);
                    o[1] = G * nsum_value(&ab[2]);
                    o[2] = G * nsum_value(&ab[3]);
                } else {
                    o[0] = G * nsum_value(&ab[0]);
                    o[1] = G * nsum_value(&ab[1]);
                    o[2] = G * nsum_value(&ab[2]);
                    o[3] = G * nsum_value(&ab[3]);
                }
            }
        }
        free(acc);
    }
    return err;
}

/* Transpose of oracle_forward: drho[b][cell] = sum over targets j and output
 * components c of resid[b][j][c] * d out[b][j][c] / d rho[b][cell].
 * Each cell is an independent sum over the same pair set as the forward
 * (coincident pairs excluded), so the two are exact transposes up to
 * rounding. */
int oracle_adjoint(int nx, int ny, int nz, const double *origin, const double *h,
                   int q, int batch, const double *resid, int64_t m,
                   const double *targets, int comps, double G, double *drho)
{
    double gx[2], gw[2];
    int nq = gauss_rule(q, gx, gw);
    if (nq == 0 || nx < 0 || ny < 0 || nz < 0 || batch < 1 || m < 0 ||
        !valid_comps(comps))
        return -1;
    const int64_t ncell = (int64_t)nx * ny * nz;
    const double vol = h[0] * h[1] * h[2];
    int err = 0;

#pragma omp parallel
    {
        nsum_t *acc = (nsum_t *)malloc(sizeof(nsum_t) * (size_t)batch);
        if (!acc) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t cell = 0; cell < ncell; ++cell) {
            if (!acc)
                continue;
            const int i = (int)(cell % nx);
            const int jj = (int)((cell / nx) % ny);
            const int k = (int)(cell / ((int64_t)nx * ny));
            const double cx = origin[0] + (i + 0.5) * h[0];
            const double cy = origin[1] + (jj + 0.5) * h[1];
            const double cz = origin[2] + (k + 0.5) * h[2];
            memset(acc, 0, sizeof(nsum_t) * (size_t)batch);
            for (int a = 0; a < nq; ++a)
                for (int bq = 0; bq < nq; ++bq)
                    for (int c = 0; c < nq; ++c) {
                        const double px = cx + gx[c] * h[0];
                        const double py = cy + gx[bq] * h[1];
                        const double pz = cz + gx[a] * h[2];
                        const double w = vol * gw[a] * gw[bq] * gw[c];
                        for (int64_t j = 0; j < m; ++j) {
                            const double dx = targets[3 * j + 0] - px;
                            const double dy = targets[3 * j + 1] - py;
                            const double dz = targets[3 * j + 2] - pz;
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 == 0.0)
                                continue;
                            const double r = sqrt(r2);
                            const double inv_r = 1.0 / r;
                            const double inv_r3 = 1.0 / (r2 * r);
                            for (int b = 0; b < batch; ++b) {
                                const double *rr = resid + ((int64_t)b * m + j) * comps;
                                double s;
                                if (comps == 1)
                                    s = rr[0] * dz * inv_r3;
                                else if (comps == 3)
                                    s = (rr[0] * dx + rr[1] * dy + rr[2] * dz) * inv_r3;
                                else
                                    s = rr[0] * inv_r +
                                        (rr[1] * dx + rr[2] * dy + rr[3] * dz) * inv_r3;
                                nsum_add(&acc[b], w * s);
                            }
                        }
                    }
            for (int b = 0; b < batch; ++b)
                drho[b * ncell + cell] = G * nsum_value(&acc[b]);
        }
        free(acc);
    }
    return err;
}

/* Transpose restricted to a list of cells: drho[b][k] for cell index
 * cells[k] (flat index into [nz][ny][nx]); same pair set and arithmetic as
 * oracle_adjoint, for sampled checks on large meshes. */
int oracle_adjoint_cells(int nx, int ny, int nz, const double *origin, const double *h, int q,
                         int batch, const double *resid, int64_t m, const double *targets,
                         int comps, double G, int64_t ncells, const int64_t *cells, double *drho)
{
    double gx[2], gw[2];
    int nq = gauss_rule(q, gx, gw);
    if (nq == 0 || nx < 0 || ny < 0 || nz < 0 || batch < 1 || m < 0 || ncells < 0 ||
        !valid_comps(comps))
        return -1;
    const int64_t ncell = (int64_t)nx * ny * nz;
    const double vol = h[0] * h[1] * h[2];
    int err = 0;
#pragma omp parallel
    {
        nsum_t *acc = (nsum_t *)malloc(sizeof(nsum_t) * (size_t)batch);
        if (!acc) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t kk = 0; kk < ncells; ++kk) {
            const int64_t cell = cells[kk];
            if (!acc || cell < 0 || cell >= ncell)
                continue;
            const int i = (int)(cell % nx);
            const int jj = (int)((cell / nx) % ny);
            const int k = (int)(cell / ((int64_t)nx * ny));
            const double cx = origin[0] + (i + 0.5) * h[0];
            const double cy = origin[1] + (jj + 0.5) * h[1];
            const double cz = origin[2] + (k + 0.5) * h[2];
            memset(acc, 0, sizeof(nsum_t) * (size_t)batch);
            for (int a = 0; a < nq; ++a)
                for (int bq = 0; bq < nq; ++bq)
                    for (int c = 0; c < nq; ++c) {
                        const double px = cx + gx[c] * h[0];
                        const double py = cy + gx[bq] * h[1];
                        const double pz = cz + gx[a] * h[2];
                        const double w = vol * gw[a] * gw[bq] * gw[c];
                        for (int64_t j = 0; j < m; ++j) {
                            const double dx = targets[3 * j + 0] - px;
                            const double dy = targets[3 * j + 1] - py;
                            const double dz = targets[3 * j + 2] - pz;
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 == 0.0)
                                continue;
                            const double r = sqrt(r2);
                            const double inv_r = 1.0 / r;
                            const double inv_r3 = 1.0 / (r2 * r);
                            for (int b = 0; b < batch; ++b) {
                                const double *rr = resid + ((int64_t)b * m + j) * comps;
                                double sv;
                                if (comps == 1)
                                    sv = rr[0] * dz * inv_r3;
                                else if (comps == 3)
                                    sv = (rr[0] * dx + rr[1] * dy + rr[2] * dz) * inv_r3;
                                else
                                    sv = rr[0] * inv_r +
                                         (rr[1] * dx + rr[2] * dy + rr[3] * dz) * inv_r3;
                                nsum_add(&acc[b], w * sv);
                            }
                        }
                    }
            for (int b = 0; b < batch; ++b)
                drho[b * ncells + kk] = G * nsum_value(&acc[b]);
        }
        free(acc);
    }
    return err;
}

/* Direct sum over an explicit list of point masses (no lattice): used by the
 * tests that pin the voxel path to plain point-mass physics. */
int oracle_points(int64_t n, const double *src, const double *mass, int64_t m,
                  const double *targets, int comps, double G, double *out)
{
    if (n < 0 || m < 0 || !valid_comps(comps))
        return -1;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < m; ++j) {
        nsum_t acc[4];
        memset(acc, 0, sizeof(acc));
        for (int64_t i = 0; i < n; ++i) {
            const double dx = targets[3 * j + 0] - src[3 * i + 0];
            const double dy = targets[3 * j + 1] - src[3 * i + 1];
            const double dz = targets[3 * j + 2] - src[3 * i + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0)
                continue;
            const double r = sqrt(r2);
            const double inv_r3 = 1.0 / (r2 * r);
            nsum_add(&acc[0], mass[i] / r);
            nsum_add(&acc[1], mass[i] * dx * inv_r3);
            nsum_add(&acc[2], mass[i] * dy * inv_r3);
            nsum_add(&acc[3], mass[i] * dz * inv_r3);
        }
        double *o = out + j * comps;
        if (comps == 1) {
            o[0] = G * nsum_value(&acc[3]);
        } else if (comps == 3) {
            o[0] = G * nsum_value(&acc[1]);
            o[1] = G * nsum_value(&acc[2]);
            o[2] = G * nsum_value(&acc[3]);
        } else {
            for (int c = 0; c < 4; ++c)
                o[c] = G * nsum_value(&acc[c]);
        }
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads later calls use (n >= 1); returns the
 * number now in effect.  Lets the benchmark time the oracle on one core and
 * on all cores in one process. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
