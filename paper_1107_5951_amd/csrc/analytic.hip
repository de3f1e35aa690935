// grav_analytic: the closed-form summation method of Sec. 2.1 (SUM-AN).  gz
// at the plan's evaluation points is the sum over all cells of the exact
// attraction of a uniform rectangular prism (the closed form the paper takes
// from Li & Chouteau): with u, v, w the offsets from the evaluation point to a
// corner and r their length,
//   F(u, v, w) = u ln(v + r) + v ln(u + r) - w atan(u v / (w r)),
// and a cell's gz is G rho times the alternating sum of F over its eight
// corners (sign (-1)^(i+j+k), index 1 = lower corner), which makes gz > 0
// above a positive anomaly as in Eq. (1).  No quadrature: the result is exact
// for a cell-wise constant density, up to rounding.
//
// Vertex form.  Every grid vertex is a corner of up to eight cells, so the
// sum over cells and corners regroups into one evaluation of F per vertex V
// with the weight W_V = sum over the cells c having V as a corner of
// -(-1)^(di+dj+dk) rho_c, (di, dj, dk) in {0, 1}^3 the corner's position in c
// (1 = upper).  Same terms, eight times fewer transcendental evaluations; the
// weights are formed while the vertices are staged in LDS.
// Positions are in the lattice frame (cell units), where F scales so that
// the physical gz is G h times the lattice sum.  FP64 throughout: the
// alternating corner sum cancels to O(h^3) of its terms.
//
// Work is split over targets (256 per workgroup) and chunks of vertices, the
// chunk partials added in a fixed order, as in grav_direct.
#include <algorithm>

#include "resolve.hpp"

namespace grav {

// Weight of vertex (A, B, C) (vertices (nx+1) x (ny+1) x (nz+1)) for model bm.
__device__ inline double an_weight(const DevGeom &g, const double *rho, int bm, int A, int Bv, int C)
{
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    double w = 0.0;
    for (int d = 0; d < 8; ++d) {
        const int di = d & 1, dj = (d >> 1) & 1, dk = (d >> 2) & 1;
        const int ix = A - di, iy = Bv - dj, iz = C - dk;
        if (ix < 0 || iy < 0 || iz < 0 || ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2])
            continue;
        const double r = rho[bm * ncell + ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix];
        w += ((di + dj + dk) & 1) ? r : -r;
    }
    return w;
}

__device__ inline double an_F(double u, double v, double w)
{
    const double r = sqrt(u * u + v * v + w * w);
    const double t1 = u == 0.0 ? 0.0 : u * log(v + r > 0.0 ? v + r : 1.0);
    const double t2 = v == 0.0 ? 0.0 : v * log(u + r > 0.0 ? u + r : 1.0);
    const double t3 = w == 0.0 ? 0.0 : w * atan(u * v / (w * r));
    return t1 + t2 - t3;
}

// Partial sums: grid (target tiles of 256) x (vertex chunks); chunk c writes
// part[c][target][model] (or, with one chunk, the output directly).
__global__ void __launch_bounds__(256)
k_analytic(DevGeom g, const double *rho, const double *tpos, int64_t chunk, double *part, const uint32_t *perm,
           double *out)
{
    __shared__ double sv[256][4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < g.M;
    const int64_t vx = g.n[0] + 1, vy = g.n[1] + 1, vz = g.n[2] + 1;
    const int64_t nv = vx * vy * vz;
    const int64_t cb = (int64_t)blockIdx.y * chunk, ce = min(nv, cb + chunk);
    double tp[3] = {0, 0, 0};
    if (valid)
        for (int a = 0; a < 3; ++a)
            tp[a] = tpos[3 * i + a];
    for (int bm = 0; bm < g.B; ++bm) {
        double acc = 0.0;
        for (int64_t c0 = cb; c0 < ce; c0 += 256) {
            __syncthreads();
            const int64_t c = c0 + threadIdx.x;
            if (c < ce) {
                const int A = (int)(c % vx), Bv = (int)((c / vx) % vy), C = (int)(c / (vx * vy));
                sv[threadIdx.x][0] = (double)A;
                sv[threadIdx.x][1] = (double)Bv;
                sv[threadIdx.x][2] = (double)C;
                sv[threadIdx.x][3] = an_weight(g, rho, bm, A, Bv, C);
            } else {
                sv[threadIdx.x][0] = sv[threadIdx.x][1] = sv[threadIdx.x][2] = 0.0;
                sv[threadIdx.x][3] = 0.0;
            }
            __syncthreads();
            if (!valid)
                continue;
            const int nc = (int)min((int64_t)256, ce - c0);
            for (int k = 0; k < nc; ++k) {
                const double wv = sv[k][3];
                if (wv == 0.0)
                    continue;  // the same vertex for every thread: no divergence
                acc += wv * an_F(sv[k][0] - tp[0], sv[k][1] - tp[1], sv[k][2] - tp[2]);
            }
        }
        if (!valid)
            continue;
        if (gridDim.y > 1)
            part[((int64_t)blockIdx.y * g.M + i) * g.B + bm] = acc;
        else
            out[(int64_t)bm * g.M + perm[i]] = g.G * g.h * acc;
    }
}

__global__ void __launch_bounds__(256)
k_analytic_finish(DevGeom g, const double *part, int nchunk, const uint32_t *perm, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.M * g.B)
        return;
    const int64_t i = t / g.B;
    const int bm = (int)(t % g.B);
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c)
        v += part[((int64_t)c * g.M + i) * g.B + bm];
    out[(int64_t)bm * g.M + perm[i]] = g.G * g.h * v;
}

}  // namespace grav

using namespace grav;

extern "C" grav_status grav_analytic(grav_plan_t plan, const double *rho, double *gz_out, void *stream)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (p->d.components != 1 || p->n_spts > 0)
        return GRAV_EUNSUPPORTED;
    if (p->M == 0)
        return GRAV_OK;
    if (!rho || !gz_out)
        return GRAV_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    GRAV_HIP(hipGetDevice(&cur));
    if (cur != p->device)
        GRAV_HIP(hipSetDevice(p->device));
    grav_status st = begin_call(p, s);
    if (st == GRAV_OK) {
        const DevGeom g = make_geom(p);
        const int64_t nv = (int64_t)(p->d.nx + 1) * (p->d.ny + 1) * (p->d.nz + 1);
        // the direct sum's chunking and partial buffer (4 values per target
        // and model there, 1 here)
        const int nchunk = p->direct_chunks;
        const int64_t chunk = (nv + nchunk - 1) / nchunk;
        const dim3 grid((unsigned)((p->M + 255) / 256), (unsigned)nchunk), blk(256);
        hipLaunchKernelGGL(k_analytic, grid, blk, 0, s, g, rho, (const double *)p->d_tpos, chunk, p->d_dpart,
                           (const uint32_t *)p->d_perm, gz_out);
        st = hipGetLastError() == hipSuccess ? GRAV_OK : GRAV_EDEVICE;
        if (st == GRAV_OK && nchunk > 1) {
            hipLaunchKernelGGL(k_analytic_finish, dim3((unsigned)((p->M * p->B + 255) / 256)), dim3(256), 0, s, g,
                               (const double *)p->d_dpart, nchunk, (const uint32_t *)p->d_perm, gz_out);
            st = hipGetLastError() == hipSuccess ? GRAV_OK : GRAV_EDEVICE;
        }
    }
    if (st == GRAV_OK)
        st = end_call(p, s);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return st;
}
