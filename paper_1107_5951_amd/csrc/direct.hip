// grav_direct: the summation method of Sec. 2.1 (SUM-G1 / SUM-G2) on the
// GPU, over a plan's evaluation points.  Every target takes the direct sum
// over every quadrature point of every cell, Eq. (1) discretised with the
// 1- or 2-point Gauss rule, with the same pair set and coincidence rule as
// the FMM's near field.  It is the paper's baseline against which the FMM's
// cost is compared, and an independent check of the FMM at medium sizes.
//
// Work is split over targets (256 per workgroup, one per thread) and over
// chunks of source cells, so that small target sets still fill the device;
// a second kernel adds the chunk partials in a fixed order.  Positions are in
// the lattice frame (cell units), so source coordinates are exact small
// integers plus the Gauss offsets.
#include <algorithm>
#include <mutex>

#include "resolve.hpp"

namespace grav {

// Partial sums: grid (target tiles of 256) x (source chunks); chunk c of CH
// cells writes part[c][target][model][4] (or, with one chunk, the output
// directly).  Within a workgroup the chunk is staged through LDS 256 cells at
// a time as (x, y, z, rho) relative to the chunk's first cell, so the pair
// arithmetic needs no index bookkeeping.  The pair terms of one staged batch
// (at most 256 cells, 2,048 quadrature points) are summed in T and each
// batch's sum is added to an FP64 accumulator, so in FP32 the rounding error
// grows with the batch length, not with the number of cells.
template <typename T>
__global__ void __launch_bounds__(256)
k_direct(DevGeom g, const double *rho, const double *tpos, int64_t chunk, double *part,
         const uint32_t *perm, double *out)
{
    __shared__ T scell[256][4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < g.M;
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t cb = (int64_t)blockIdx.y * chunk, ce = min(ncell, cb + chunk);
    const int bx = (int)(cb % g.n[0]), by = (int)((cb / g.n[0]) % g.n[1]), bz = (int)(cb / ((int64_t)g.n[0] * g.n[1]));
    const T go = (T)(0.5 / 1.7320508075688772);  // Gauss point offset, cell units
    // target relative to the centre of the chunk's first cell (exact in FP64,
    // then rounded once)
    T tp[3] = {0, 0, 0};
    if (valid) {
        tp[0] = (T)(tpos[3 * i + 0] - (double)bx - 0.5);
        tp[1] = (T)(tpos[3 * i + 1] - (double)by - 0.5);
        tp[2] = (T)(tpos[3 * i + 2] - (double)bz - 0.5);
    }
    for (int bm = 0; bm < g.B; ++bm) {
        double acc64[4] = {0, 0, 0, 0};
        for (int64_t c0 = cb; c0 < ce; c0 += 256) {
            __syncthreads();
            const int64_t c = c0 + threadIdx.x;
            if (c < ce) {
                const int ix = (int)(c % g.n[0]), iy = (int)((c / g.n[0]) % g.n[1]),
                          iz = (int)(c / ((int64_t)g.n[0] * g.n[1]));
                scell[threadIdx.x][0] = (T)(ix - bx);
                scell[threadIdx.x][1] = (T)(iy - by);
                scell[threadIdx.x][2] = (T)(iz - bz);
                scell[threadIdx.x][3] = (T)rho[(int64_t)bm * ncell + c];
            } else {
                scell[threadIdx.x][0] = scell[threadIdx.x][1] = scell[threadIdx.x][2] = 0;
                scell[threadIdx.x][3] = 0;
            }
            __syncthreads();
            if (!valid)
                continue;
            const int nc = (int)min((int64_t)256, ce - c0);
            T acc[4] = {0, 0, 0, 0};
            for (int k = 0; k < nc; ++k) {
                const T rv = scell[k][3];
                if (rv == (T)0)
                    continue;
                const T cx = tp[0] - scell[k][0], cy = tp[1] - scell[k][1], cz = tp[2] - scell[k][2];
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
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc64[c] += (double)acc[c];
        }
        if (!valid)
            continue;
        if (gridDim.y > 1) {
            double *o = part + (((int64_t)blockIdx.y * g.M + i) * g.B + bm) * 4;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                o[c] = acc64[c];
            continue;
        }
        // one chunk: write the output (descriptor order, G applied)
        double *o = out + ((int64_t)bm * g.M + perm[i]) * g.C;
        const double sg = g.G * g.h, sp = g.G * g.h * g.h;
        if (g.C == 1) {
            o[0] = sg * acc64[3];
        } else if (g.C == 3) {
            o[0] = sg * acc64[1];
            o[1] = sg * acc64[2];
            o[2] = sg * acc64[3];
        } else {
            o[0] = sp * acc64[0];
            o[1] = sg * acc64[1];
            o[2] = sg * acc64[2];
            o[3] = sg * acc64[3];
        }
    }
}

// Sum the chunk partials in chunk order and write the output in descriptor
// order, G applied.  One thread per (sorted target, model).
__global__ void __launch_bounds__(256)
k_direct_finish(DevGeom g, const double *part, int nchunk, const uint32_t *perm, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.M * g.B)
        return;
    const int64_t i = t / g.B;
    const int bm = (int)(t % g.B);
    double v[4] = {0, 0, 0, 0};
    for (int c = 0; c < nchunk; ++c)
        for (int k = 0; k < 4; ++k)
            v[k] += part[(((int64_t)c * g.M + i) * g.B + bm) * 4 + k];
    double *o = out + ((int64_t)bm * g.M + perm[i]) * g.C;
    const double sg = g.G * g.h, sp = g.G * g.h * g.h;
    if (g.C == 1) {
        o[0] = sg * v[3];
    } else if (g.C == 3) {
        o[0] = sg * v[1];
        o[1] = sg * v[2];
        o[2] = sg * v[3];
    } else {
        o[0] = sp * v[0];
        o[1] = sg * v[1];
        o[2] = sg * v[2];
        o[3] = sg * v[3];
    }
}

}  // namespace grav

namespace grav {

// Enqueue the direct sum with its chunk partials in `part` (device memory of
// at least direct_chunks x M x B x 4 doubles when direct_chunks > 1).
static grav_status enqueue_direct(Plan *p, const double *rho, double *g_out, double *part, hipStream_t s)
{
    const DevGeom g = make_geom(p);
    const int64_t ncell = (int64_t)p->d.nx * p->d.ny * p->d.nz;
    const int nchunk = p->direct_chunks;
    const int64_t chunk = (ncell + nchunk - 1) / nchunk;
    const dim3 grid((unsigned)((p->M + 255) / 256), (unsigned)nchunk), blk(256);
    if (p->d.precision == GRAV_FP64)
        hipLaunchKernelGGL(k_direct<double>, grid, blk, 0, s, g, rho, (const double *)p->d_tpos, chunk, part,
                           (const uint32_t *)p->d_perm, g_out);
    else
        hipLaunchKernelGGL(k_direct<float>, grid, blk, 0, s, g, rho, (const double *)p->d_tpos, chunk, part,
                           (const uint32_t *)p->d_perm, g_out);
    GRAV_HIP(hipGetLastError());
    if (nchunk > 1) {
        hipLaunchKernelGGL(k_direct_finish, dim3((unsigned)((p->M * p->B + 255) / 256)), dim3(256), 0, s, g,
                           (const double *)part, nchunk, (const uint32_t *)p->d_perm, g_out);
        GRAV_HIP(hipGetLastError());
    }
    return GRAV_OK;
}

// Chunk partials of grav_direct_noalloc: a fixed device array (one copy per
// GPU, alive until the process ends) in place of the plan's buffer.  Host
// code must not use the name: it stands for a host-side shadow, so kernels
// get the device address from hipGetSymbolAddress (scratch_ptr below).
constexpr size_t kScratchDoubles = (size_t)1 << 20;  // 8 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kScratchDevices = 64;
static std::once_flag g_scratch_once[kScratchDevices];
static double *g_scratch_ptr[kScratchDevices];
static hipError_t g_scratch_err[kScratchDevices];

// Device address of `scratch` on device dev, which must be current: looked up
// once per device, on that device's first call.
static grav_status scratch_ptr(int dev, double **out)
{
    if (dev < 0 || dev >= kScratchDevices)
        return GRAV_EUNSUPPORTED;
    std::call_once(g_scratch_once[dev], [dev]() {
        void *ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? (double *)ptr : nullptr;
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
        return GRAV_EDEVICE;
    *out = g_scratch_ptr[dev];
    return GRAV_OK;
}

}  // namespace grav

using namespace grav;

extern "C" grav_status grav_direct(grav_plan_t plan, const double *rho, double *g_out, void *stream)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (p->n_spts > 0)
        return GRAV_EUNSUPPORTED;  // the summation sums over the cells' quadrature points
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
    if (st == GRAV_OK)
        st = enqueue_direct(p, rho, g_out, p->d_dpart, s);
    if (st == GRAV_OK)
        st = end_call(p, s);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return st;
}

extern "C" grav_status grav_direct_noalloc(grav_plan_t plan, const double *rho, double *g_out, void *stream)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (p->n_spts > 0)
        return GRAV_EUNSUPPORTED;
    if (p->M == 0)
        return GRAV_OK;
    if (!rho || !g_out)
        return GRAV_EINVAL;
    const size_t need = p->direct_chunks > 1 ? (size_t)p->direct_chunks * p->M * p->B * 4 : 0;
    if (need > kScratchDoubles)
        return GRAV_EUNSUPPORTED;  // partials larger than the 8 MiB device array
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    GRAV_HIP(hipGetDevice(&cur));
    if (cur != p->device)
        GRAV_HIP(hipSetDevice(p->device));
    double *part = nullptr;
    grav_status st = scratch_ptr(p->device, &part);
    if (st == GRAV_OK)
        st = begin_call(p, s);
    if (st == GRAV_OK)
        st = enqueue_direct(p, rho, g_out, part, s);
    if (st == GRAV_OK)
        st = end_call(p, s);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return st;
}
