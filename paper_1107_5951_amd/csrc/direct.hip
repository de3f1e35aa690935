// grav_direct: the summation method of Sec. 2.1 (SUM-G1 / SUM-G2) on the
// GPU, over a plan's evaluation points.  Every target takes the direct sum
// over every quadrature point of every cell, Eq. (1) discretised with the
// 1- or 2-point Gauss rule, with the same pair set and coincidence rule as
// the FMM's near field.  It is the paper's baseline against which the FMM's
// cost is compared, and an independent check of the FMM at medium sizes.
//
// One thread per sorted target (256 per workgroup); the densities of the
// mesh are streamed through LDS in slabs of 256 cells shared by the
// workgroup.  Positions are in the lattice frame (cell units), so source
// coordinates are exact small integers plus the Gauss offsets.
#include <algorithm>

#include "resolve.hpp"

namespace grav {

template <typename T>
__global__ void __launch_bounds__(256)
k_direct(DevGeom g, const double *rho, const double *tpos, const uint32_t *perm, double *out)
{
    __shared__ double srho[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < g.M;
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const T go = (T)(0.5 / 1.7320508075688772);  // Gauss point offset, cell units
    // target relative to the mesh origin, in cell units; FP32 runs keep the
    // whole-cell part exact by splitting it off
    double tp[3] = {0, 0, 0};
    if (valid)
        for (int a = 0; a < 3; ++a)
            tp[a] = tpos[3 * i + a];
    for (int bm = 0; bm < g.B; ++bm) {
        T acc[4] = {0, 0, 0, 0};
        for (int64_t c0 = 0; c0 < ncell; c0 += 256) {
            __syncthreads();
            const int64_t c = c0 + threadIdx.x;
            srho[threadIdx.x] = c < ncell ? rho[(int64_t)bm * ncell + c] : 0.0;
            __syncthreads();
            if (!valid)
                continue;
            const int nc = (int)min((int64_t)256, ncell - c0);
            int ix = (int)(c0 % g.n[0]), iy = (int)((c0 / g.n[0]) % g.n[1]), iz = (int)(c0 / ((int64_t)g.n[0] * g.n[1]));
            for (int k = 0; k < nc; ++k) {
                const T rv = (T)srho[k];
                if (rv != (T)0) {
                    const T cx = (T)(tp[0] - (double)ix - 0.5), cy = (T)(tp[1] - (double)iy - 0.5),
                            cz = (T)(tp[2] - (double)iz - 0.5);
                    if (g.q == 1) {
                        const T r2 = cx * cx + cy * cy + cz * cz;
                        if (r2 > coincident2<T>()) {
                            const T ri = rsqrt_t(r2);
                            const T m = rv * ri;
                            const T m3 = m * ri * ri;
                            acc[0] += m;
                            acc[1] += m3 * cx;
                            acc[2] += m3 * cy;
                            acc[3] += m3 * cz;
                        }
                    } else {
                        const T mw = rv * (T)0.125;
#pragma unroll
                        for (int gp = 0; gp < 8; ++gp) {
                            const T ux = cx - ((gp & 1) ? go : -go);
                            const T uy = cy - ((gp & 2) ? go : -go);
                            const T uz = cz - ((gp & 4) ? go : -go);
                            const T r2 = ux * ux + uy * uy + uz * uz;
                            if (r2 > coincident2<T>()) {
                                const T ri = rsqrt_t(r2);
                                const T m = mw * ri;
                                const T m3 = m * ri * ri;
                                acc[0] += m;
                                acc[1] += m3 * ux;
                                acc[2] += m3 * uy;
                                acc[3] += m3 * uz;
                            }
                        }
                    }
                }
                if (++ix == g.n[0]) {
                    ix = 0;
                    if (++iy == g.n[1]) {
                        iy = 0;
                        ++iz;
                    }
                }
            }
        }
        if (!valid)
            continue;
        double *o = out + ((int64_t)bm * g.M + perm[i]) * g.C;
        const double sg = g.G * g.h, sp = g.G * g.h * g.h;
        if (g.C == 1) {
            o[0] = sg * (double)acc[3];
        } else if (g.C == 3) {
            o[0] = sg * (double)acc[1];
            o[1] = sg * (double)acc[2];
            o[2] = sg * (double)acc[3];
        } else {
            o[0] = sp * (double)acc[0];
            o[1] = sg * (double)acc[1];
            o[2] = sg * (double)acc[2];
            o[3] = sg * (double)acc[3];
        }
    }
}

}  // namespace grav

using namespace grav;

extern "C" grav_status grav_direct(grav_plan_t plan, const double *rho, double *g_out, void *stream)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (p->M == 0)
        return GRAV_OK;
    if (!rho || !g_out)
        return GRAV_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    GRAV_HIP(hipGetDevice(&cur));
    if (cur != p->device)
        GRAV_HIP(hipSetDevice(p->device));
    grav_status st = begin_call(p, s);
    if (st == GRAV_OK) {
        const DevGeom g = make_geom(p);
        const dim3 grid((unsigned)((p->M + 255) / 256)), blk(256);
        if (p->d.precision == GRAV_FP64)
            hipLaunchKernelGGL(k_direct<double>, grid, blk, 0, s, g, rho, (const double *)p->d_tpos,
                               (const uint32_t *)p->d_perm, g_out);
        else
            hipLaunchKernelGGL(k_direct<float>, grid, blk, 0, s, g, rho, (const double *)p->d_tpos,
                               (const uint32_t *)p->d_perm, g_out);
        st = hipGetLastError() == hipSuccess ? GRAV_OK : GRAV_EDEVICE;
    }
    if (st == GRAV_OK)
        st = end_call(p, s);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return st;
}
