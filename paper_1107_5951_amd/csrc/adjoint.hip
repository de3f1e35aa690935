// Adjoint evaluation: the exact transpose of grav_eval's linear map rho -> g.
//
// Eq. (1) is linear in the density (Sec. 1.1), and so is every FMM stage of
// Sec. 2.3 (lattice P2M, M2M, M2L, L2L, L2P, the near-field sum of Eq. (13)
// and the combine), so the transpose of the forward map applies the
// transposed stages in reverse order:
//
//   w      = C^T r                      combine^T (scaling, descriptor order)
//   LE_L   = L2P^T w                    per target leaf
//   LE_l   = sum_children L2L_c^T LE_l+1    l = L-1 .. 2
//   ME_l   = sum_d K_d^T LE_l[S - d]    M2L^T, every source box S, levels 2 .. L
//   ME_l  += M2M_c^T ME_l-1[parent]     l = 3 .. L
//   drho   = P2M^T ME_L + NEAR^T w      per cell
//
// with the same operators (the FP32-rounded M2L matrices in mixed
// precision), the same interaction lists and the same point pairs and
// coincidence rule as the forward pass, so <A rho, r> = <rho, A^T r> holds to
// rounding.  Every kernel computes one output element per thread by a plain
// loop over its inputs, read from global memory: no atomics, no LDS, no
// cross-lane operations, and a fixed summation order, so results are
// deterministic.  Every index that comes from a plan table is checked against
// the size of the array it addresses before it is used.
#include <algorithm>

#include "resolve.hpp"

namespace grav {

namespace {

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// combine^T: the weights that multiply (phi, gx, gy, gz) of each sorted
// target in the lattice frame (G and the lattice-to-physical scale of the
// combine folded in).  One thread per (sorted target, model).
__global__ void __launch_bounds__(256)
k_t_weights(DevGeom g, const double *resid, const uint32_t *perm, double *w)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.M * g.B)
        return;
    const int64_t i = t / g.B;
    const int bm = (int)(t - i * g.B);
    const int64_t u = perm[i];
    double *o = w + t * 4;
    if (u < 0 || u >= g.M) {
        o[0] = o[1] = o[2] = o[3] = 0.0;
        return;
    }
    const double *r = resid + ((int64_t)bm * g.M + u) * g.C;
    const double sg = g.G * g.h, sp = g.G * g.h * g.h;
    if (g.C == 1) {
        o[0] = o[1] = o[2] = 0.0;
        o[3] = sg * r[0];
    } else if (g.C == 3) {
        o[0] = 0.0;
        o[1] = sg * r[0];
        o[2] = sg * r[1];
        o[3] = sg * r[2];
    } else {
        o[0] = sp * r[0];
        o[1] = sg * r[1];
        o[2] = sg * r[2];
        o[3] = sg * r[3];
    }
}

// The matrix stages below give each thread up to MT density models (a
// group), so that every operator entry or pair geometry it loads serves MT
// models; groups are ceil(B / MT).

// L2P^T: the adjoint of leaf expansion coefficient k is the sum over the
// leaf's targets of the weights times the derivatives of (phi, grad phi) of
// the local expansion with respect to that coefficient, scaled as the
// combine scales the far field (phi / w, -grad phi / w^2).  One thread per
// (target leaf, model group, coefficient).
template <int MT>
__global__ void __launch_bounds__(256)
k_t_l2p(DevGeom g, const double *tpos, const int64_t *leaf_start, const uint32_t *tkey, int64_t n_leaf,
        const double *w, double *le)
{
    const int NG = (g.B + MT - 1) / MT;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_leaf * NG * g.PS)
        return;
    const int k = (int)(t % g.PS);
    const int64_t rest = t / g.PS;
    const int grp = (int)(rest % NG);
    const int64_t leaf = rest / NG;
    const DevLev &lv = g.lev[g.L];
    double acc[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
        acc[u] = 0.0;
    if (k < g.P2) {
        const uint32_t key = tkey[lv.tbox_off + leaf];
        const int lc[3] = {(int)compact3(key), (int)compact3(key >> 1), (int)compact3(key >> 2)};
        double centre[3];
        for (int a = 0; a < 3; ++a)
            centre[a] = ((double)(lc[a] - g.shift[a]) + 0.5) * g.b;
        const double inv_w = 1.0 / (double)g.b, inv_w2 = inv_w * inv_w;
        const int64_t ts = max(leaf_start[leaf], (int64_t)0), te = min(leaf_start[leaf + 1], g.M);
        for (int64_t j = ts; j < te; ++j) {
            double d[4];
            l2p_coef(g.P, k, (tpos[3 * j + 0] - centre[0]) * inv_w, (tpos[3 * j + 1] - centre[1]) * inv_w,
                     (tpos[3 * j + 2] - centre[2]) * inv_w, d);
            const double d0 = d[0] * inv_w, d1 = d[1] * inv_w2, d2 = d[2] * inv_w2, d3 = d[3] * inv_w2;
#pragma unroll
            for (int u = 0; u < MT; ++u) {
                const int bm = grp * MT + u;
                if (bm < g.B) {
                    const double *wj = w + (j * g.B + bm) * 4;
                    acc[u] += wj[0] * d0 - (wj[1] * d1 + wj[2] * d2 + wj[3] * d3);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < MT; ++u) {
        const int bm = grp * MT + u;
        if (bm < g.B)
            le[((lv.tgt_off + leaf) * g.B + bm) * g.PS + k] = acc[u];  // padding k >= p^2 gets 0
    }
}

// L2L^T (upward over the target boxes): LE_l[box] = sum over the box's
// children c of L2L_c^T LE_l+1[c], L2L row-major [octant][out t][in s], so
// the thread of coefficient s reads column s.  One thread per (box of level
// l, model group, coefficient s).
template <int MT>
__global__ void __launch_bounds__(256)
k_t_l2l(DevGeom g, int l, const uint32_t *tkey, const int32_t *tchild, const double *l2l, double *le)
{
    const int NG = (g.B + MT - 1) / MT;
    const DevLev &lv = g.lev[l];
    const DevLev &lc = g.lev[l + 1];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= lv.n_tgt * NG * g.PS)
        return;
    const int s = (int)(t % g.PS);
    const int64_t rest = t / g.PS;
    const int grp = (int)(rest % NG);
    const int64_t box = rest / NG;
    double acc[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
        acc[u] = 0.0;
    if (s < g.P2) {
        const int64_t a = tchild[lv.tchild_off + box], e = tchild[lv.tchild_off + box + 1];
        for (int64_t ch = max(a, (int64_t)0); ch < min(e, lc.n_tgt); ++ch) {
            const int oct = (int)(tkey[lc.tbox_off + ch] & 7u);
            const double *col = l2l + (int64_t)oct * g.PS * g.PS + s;
            const double *y = le + ((lc.tgt_off + ch) * g.B + grp * MT) * g.PS;
            for (int q = 0; q < g.P2; ++q) {
                const double m = col[(int64_t)q * g.PS];
#pragma unroll
                for (int u = 0; u < MT; ++u)
                    if (grp * MT + u < g.B)
                        acc[u] += m * y[(int64_t)u * g.PS + q];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < MT; ++u) {
        const int bm = grp * MT + u;
        if (bm < g.B)
            le[((lv.tgt_off + box) * g.B + bm) * g.PS + s] = acc[u];
    }
}

// M2L^T: ME_l[S] = sum over the offsets d of the reverse list of S's parity
// class, for which T = S - d is a target box, of K_d^T LE_l[T] (the forward
// M2L adds K_d ME[T + d] into LE[T] for exactly these pairs).  K is stored
// plain, [offset][row i (LE)][column j (ME)], p^2 x p^2.  One workgroup per
// source box of any level >= 2: its threads first look up the box's 189
// reverse offsets in the level's target-box map (an LDS list, invalid
// entries -1, kept in list order), then each thread accumulates
// coefficients j of a model group over the valid entries.
template <int MT>
__global__ void __launch_bounds__(256)
k_t_m2l(DevGeom g, int64_t n_tbox, const int32_t *tmap, int64_t n_tmap, const int32_t *roffs, const double *K,
        const double *le, double *me)
{
    __shared__ int32_t pt[kClassOffsets], pid[kClassOffsets];
    __shared__ int32_t nvalid;
    const int NG = (g.B + MT - 1) / MT;
    const int64_t sbox = blockIdx.x;  // over all levels' source blocks
    int l = 2;
    while (l < g.L && sbox >= g.lev[l + 1].me_off)
        ++l;
    const DevLev &lv = g.lev[l];
    const int64_t r = sbox - lv.me_off;
    const int x = lv.s0[0] + (int)(r % lv.ns[0]);
    const int y = lv.s0[1] + (int)((r / lv.ns[0]) % lv.ns[1]);
    const int z = lv.s0[2] + (int)(r / ((int64_t)lv.ns[0] * lv.ns[1]));
    const int cls = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
    if (threadIdx.x == 0)
        nvalid = 0;
    __syncthreads();
    for (int o = threadIdx.x; o < kClassOffsets; o += blockDim.x) {
        const int32_t *e = roffs + (cls * kClassOffsets + o) * 4;
        int32_t tb = -1;
        const int id = e[3];
        const int mx = x - e[0] - lv.s0[0] + 3, my = y - e[1] - lv.s0[1] + 3, mz = z - e[2] - lv.s0[2] + 3;
        if (id >= 0 && id < kNumOffsets && mx >= 0 && my >= 0 && mz >= 0 && mx < lv.ns[0] + 6 &&
            my < lv.ns[1] + 6 && mz < lv.ns[2] + 6) {
            const int64_t mi = lv.tmap_off + ((int64_t)mz * (lv.ns[1] + 6) + my) * (lv.ns[0] + 6) + mx;
            if (mi < n_tmap) {
                const int64_t v = tmap[mi];
                if (v >= 0 && v < lv.n_tgt && lv.tgt_off + v < n_tbox)
                    tb = (int32_t)v;
            }
        }
        pt[o] = tb;
        pid[o] = id;
        if (tb >= 0)
            atomicAdd(&nvalid, 1);  // only the count: the entries keep list order
    }
    __syncthreads();
    const bool any = nvalid > 0;
    for (int64_t oi = threadIdx.x; oi < (int64_t)NG * g.PS; oi += blockDim.x) {
        const int j = (int)(oi % g.PS);
        const int grp = (int)(oi / g.PS);
        double acc[MT];
#pragma unroll
        for (int u = 0; u < MT; ++u)
            acc[u] = 0.0;
        if (any && j < g.P2) {
            for (int o = 0; o < kClassOffsets; ++o) {
                const int32_t tb = pt[o];
                if (tb < 0)
                    continue;
                const double *kc = K + (int64_t)pid[o] * g.P2 * g.P2 + j;
                const double *yv = le + ((lv.tgt_off + tb) * g.B + grp * MT) * g.PS;
                for (int i = 0; i < g.P2; ++i) {
                    const double kv = kc[(int64_t)i * g.P2];
#pragma unroll
                    for (int u = 0; u < MT; ++u)
                        if (grp * MT + u < g.B)
                            acc[u] += kv * yv[(int64_t)u * g.PS + i];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < MT; ++u) {
            const int bm = grp * MT + u;
            if (bm < g.B)
                me[(sbox * g.B + bm) * g.PS + j] = acc[u];
        }
    }
}

// M2M^T (downward over the source blocks): ME_l[child] += M2M_c^T
// ME_l-1[parent], M2M row-major [octant][out i][in j], so the thread of
// coefficient j reads column j.  One thread per (source box of level l,
// model group, coefficient j).
template <int MT>
__global__ void __launch_bounds__(256) k_t_m2m(DevGeom g, int l, const double *m2m, double *me)
{
    const int NG = (g.B + MT - 1) / MT;
    const DevLev &lv = g.lev[l];
    const DevLev &lp = g.lev[l - 1];
    const int64_t n_box = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_box * NG * g.PS)
        return;
    const int j = (int)(t % g.PS);
    if (j >= g.P2)
        return;  // padding stays zero (written by M2L^T)
    const int64_t rest = t / g.PS;
    const int grp = (int)(rest % NG);
    const int64_t box = rest / NG;
    const int x = lv.s0[0] + (int)(box % lv.ns[0]);
    const int y = lv.s0[1] + (int)((box / lv.ns[0]) % lv.ns[1]);
    const int z = lv.s0[2] + (int)(box / ((int64_t)lv.ns[0] * lv.ns[1]));
    const int64_t par = dense_index(lp, x >> 1, y >> 1, z >> 1);
    if (par < 0)
        return;
    const int oct = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
    const double *col = m2m + (int64_t)oct * g.PS * g.PS + j;
    const double *mp = me + ((lp.me_off + par) * g.B + grp * MT) * g.PS;
    double acc[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
        acc[u] = 0.0;
    for (int i = 0; i < g.P2; ++i) {
        const double m = col[(int64_t)i * g.PS];
#pragma unroll
        for (int u = 0; u < MT; ++u)
            if (grp * MT + u < g.B)
                acc[u] += m * mp[(int64_t)u * g.PS + i];
    }
#pragma unroll
    for (int u = 0; u < MT; ++u) {
        const int bm = grp * MT + u;
        if (bm < g.B)
            me[((lv.me_off + box) * g.B + bm) * g.PS + j] += acc[u];
    }
}

// P2M^T and the near-field transpose, per cell: drho[cell] = sum_k Pm[v][k]
// ME_L[leaf][k] (v = the cell's place in its leaf), plus, over the targets j
// of the 27 leaves around the cell's leaf (the forward near field pairs every
// target of a leaf with every quadrature point of its 27 neighbours), the
// weights times the pair terms (1/r, (t - x)/r^3) of each of the cell's
// quadrature points, with the forward's coincidence rule and arithmetic type
// T.  One thread per (cell, model group): the pair geometry is computed once
// for the group's models.
template <typename T, int MT>
__global__ void __launch_bounds__(256)
k_t_cells(DevGeom g, const double *tpos, const int64_t *leaf_start, int64_t n_leaf, const int32_t *tmap,
          int64_t n_tmap, const double *w, const double *me, const double *pm, double *drho)
{
    const int NG = (g.B + MT - 1) / MT;
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell * NG)
        return;
    const int grp = (int)(t / ncell);
    const int64_t cell = t - (int64_t)grp * ncell;
    const int ix = (int)(cell % g.n[0]), iy = (int)((cell / g.n[0]) % g.n[1]),
              iz = (int)(cell / ((int64_t)g.n[0] * g.n[1]));
    const int b = g.b;
    const DevLev &lv = g.lev[g.L];
    // the cell's leaf (root-relative) and place in it
    const int lx = ix / b + g.shift[0], ly = iy / b + g.shift[1], lz = iz / b + g.shift[2];
    const int v = (ix % b) + b * ((iy % b) + b * (iz % b));
    double acc[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
        acc[u] = 0.0;
    if (g.L >= 2) {
        const int64_t sl = dense_index(lv, lx, ly, lz);
        if (sl >= 0) {
            const double *mp = me + ((lv.me_off + sl) * g.B + grp * MT) * g.PS;
            const double *pr = pm + (int64_t)v * g.PS;
            for (int k = 0; k < g.P2; ++k) {
                const double pv = pr[k];
#pragma unroll
                for (int u = 0; u < MT; ++u)
                    if (grp * MT + u < g.B)
                        acc[u] += pv * mp[(int64_t)u * g.PS + k];
            }
        }
    }
    // near field: quadrature points of this cell relative to its centre
    const T go = (T)(0.5 / 1.7320508075688772);
    const int mxl = lv.ns[0] + 6, myl = lv.ns[1] + 6, mzl = lv.ns[2] + 6;
    for (int nb = 0; nb < 27; ++nb) {
        const int tx = lx + nb % 3 - 1, ty = ly + (nb / 3) % 3 - 1, tz = lz + nb / 9 - 1;
        const int mx = tx - lv.s0[0] + 3, my = ty - lv.s0[1] + 3, mz = tz - lv.s0[2] + 3;
        if (mx < 0 || my < 0 || mz < 0 || mx >= mxl || my >= myl || mz >= mzl)
            continue;
        const int64_t mi = lv.tmap_off + ((int64_t)mz * myl + my) * mxl + mx;
        if (mi >= n_tmap)
            continue;
        const int64_t tl = tmap[mi];
        if (tl < 0 || tl >= n_leaf)
            continue;
        // target positions relative to the corner of the target leaf, as the
        // forward near field forms them, and the cell centre in that frame
        const int cx = (tx - g.shift[0]) * b, cy = (ty - g.shift[1]) * b, cz = (tz - g.shift[2]) * b;
        const T sx = (T)(ix - cx) + (T)0.5, sy = (T)(iy - cy) + (T)0.5, sz = (T)(iz - cz) + (T)0.5;
        const int64_t ts = max(leaf_start[tl], (int64_t)0), te = min(leaf_start[tl + 1], g.M);
        T part[MT];
#pragma unroll
        for (int u = 0; u < MT; ++u)
            part[u] = 0;
        for (int64_t j = ts; j < te; ++j) {
            const T ux = (T)(tpos[3 * j + 0] - (double)cx) - sx;
            const T uy = (T)(tpos[3 * j + 1] - (double)cy) - sy;
            const T uz = (T)(tpos[3 * j + 2] - (double)cz) - sz;
            // the pair geometry of the cell's quadrature points: (1/r, d/r^3)
            T f[8][4];
            const int np = g.q == 1 ? 1 : 8;
#pragma unroll
            for (int gp = 0; gp < 8; ++gp) {
                if (gp >= np) {
                    f[gp][0] = f[gp][1] = f[gp][2] = f[gp][3] = 0;
                    continue;
                }
                const T px = g.q == 1 ? ux : ux - ((gp & 1) ? go : -go);
                const T py = g.q == 1 ? uy : uy - ((gp & 2) ? go : -go);
                const T pz = g.q == 1 ? uz : uz - ((gp & 4) ? go : -go);
                const T r2 = px * px + py * py + pz * pz;
                const T wq = g.q == 1 ? (T)1 : (T)0.125;
                if (r2 > coincident2<T>()) {
                    const T ri = rsqrt_t(r2);
                    const T ri3 = ri * ri * ri;
                    f[gp][0] = wq * ri;
                    f[gp][1] = wq * px * ri3;
                    f[gp][2] = wq * py * ri3;
                    f[gp][3] = wq * pz * ri3;
                } else {
                    f[gp][0] = f[gp][1] = f[gp][2] = f[gp][3] = 0;
                }
            }
#pragma unroll
            for (int u = 0; u < MT; ++u) {
                const int bm = grp * MT + u;
                if (bm >= g.B)
                    continue;
                const double *wj = w + (j * g.B + bm) * 4;
                const T w0 = (T)wj[0], w1 = (T)wj[1], w2 = (T)wj[2], w3 = (T)wj[3];
                T sum = 0;
#pragma unroll
                for (int gp = 0; gp < 8; ++gp)
                    if (gp < np)
                        sum += w0 * f[gp][0] + (w1 * f[gp][1] + w2 * f[gp][2] + w3 * f[gp][3]);
                part[u] += sum;
            }
        }
#pragma unroll
        for (int u = 0; u < MT; ++u)
            acc[u] += (double)part[u];
    }
#pragma unroll
    for (int u = 0; u < MT; ++u) {
        const int bm = grp * MT + u;
        if (bm < g.B)
            drho[(int64_t)bm * ncell + cell] = acc[u];
    }
}

__global__ void __launch_bounds__(256) k_t_zero(double *x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        x[i] = 0.0;
}

}  // namespace

template <int MT>
static grav_status enqueue_adjoint_mt(Plan *p, const double *resid, double *drho, hipStream_t s)
{
    const DevGeom g = make_geom(p);
    const int L = p->L;
    const int64_t ncell = (int64_t)p->d.nx * p->d.ny * p->d.nz;
    const int64_t NG = (p->B + MT - 1) / MT;
    const dim3 blk(256);
    auto grid = [](int64_t n) { return dim3((unsigned)ceil_div(n, 256)); };
    if (ncell * NG > 0x7fffffffll * 256 || p->n_me > 0x7fffffffll)
        return GRAV_EUNSUPPORTED;
    stage_begin(p, "weights", s);
    hipLaunchKernelGGL(k_t_weights, grid(p->M * p->B), blk, 0, s, g, resid, (const uint32_t *)p->d_perm,
                       p->d_near);
    GRAV_HIP(hipGetLastError());
    stage_end(p, s);
    if (L >= 2) {
        stage_begin(p, "l2pT", s);
        hipLaunchKernelGGL(k_t_l2p<MT>, grid(p->n_leaf * NG * p->PS), blk, 0, s, g, (const double *)p->d_tpos,
                           (const int64_t *)p->d_leaf_start, (const uint32_t *)p->d_tkey, p->n_leaf,
                           (const double *)p->d_near, p->d_le);
        GRAV_HIP(hipGetLastError());
        stage_end(p, s);
        stage_begin(p, "l2lT", s);
        for (int l = L - 1; l >= 2; --l) {
            if (p->lev[l].n_tgt == 0)
                continue;
            hipLaunchKernelGGL(k_t_l2l<MT>, grid(p->lev[l].n_tgt * NG * p->PS), blk, 0, s, g, l,
                               (const uint32_t *)p->d_tkey, (const int32_t *)p->d_tchild, (const double *)p->d_l2l,
                               p->d_le);
            GRAV_HIP(hipGetLastError());
        }
        stage_end(p, s);
        stage_begin(p, "m2lT", s);
        hipLaunchKernelGGL(k_t_m2l<MT>, dim3((unsigned)p->n_me), blk, 0, s, g, p->n_tbox,
                           (const int32_t *)p->d_tmap, p->n_tmap, (const int32_t *)p->d_rclass_off,
                           (const double *)p->d_kplain, (const double *)p->d_le, p->d_me);
        GRAV_HIP(hipGetLastError());
        stage_end(p, s);
        stage_begin(p, "m2mT", s);
        for (int l = 3; l <= L; ++l) {
            hipLaunchKernelGGL(k_t_m2m<MT>, grid(p->lev[l].n_src * NG * p->PS), blk, 0, s, g, l,
                               (const double *)p->d_m2m, p->d_me);
            GRAV_HIP(hipGetLastError());
        }
        stage_end(p, s);
    }
    stage_begin(p, "cellsT", s);
    if (p->d.precision == GRAV_FP64)
        hipLaunchKernelGGL((k_t_cells<double, MT>), grid(ncell * NG), blk, 0, s, g, (const double *)p->d_tpos,
                           (const int64_t *)p->d_leaf_start, p->n_leaf, (const int32_t *)p->d_tmap, p->n_tmap,
                           (const double *)p->d_near, (const double *)p->d_me, (const double *)p->d_pm, drho);
    else
        hipLaunchKernelGGL((k_t_cells<float, MT>), grid(ncell * NG), blk, 0, s, g, (const double *)p->d_tpos,
                           (const int64_t *)p->d_leaf_start, p->n_leaf, (const int32_t *)p->d_tmap, p->n_tmap,
                           (const double *)p->d_near, (const double *)p->d_me, (const double *)p->d_pm, drho);
    GRAV_HIP(hipGetLastError());
    stage_end(p, s);
    return GRAV_OK;
}

grav_status enqueue_adjoint(Plan *p, const double *resid, double *drho, hipStream_t s)
{
    // one model per thread for single-model plans, groups of eight otherwise
    return p->B == 1 ? enqueue_adjoint_mt<1>(p, resid, drho, s) : enqueue_adjoint_mt<8>(p, resid, drho, s);
}

}  // namespace grav

using namespace grav;

extern "C" grav_status grav_adjoint(grav_plan_t plan, const double *resid, double *drho_out, void *stream)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!drho_out || (p->M > 0 && !resid))
        return GRAV_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    GRAV_HIP(hipGetDevice(&cur));
    if (cur != p->device)
        GRAV_HIP(hipSetDevice(p->device));
    grav_status st = begin_call(p, s);
    if (st == GRAV_OK) {
        if (p->M == 0) {
            // no evaluation points: the transpose is zero (a fill kernel, not a
            // memset, so that the call can be recorded in a graph)
            const int64_t n = (int64_t)p->d.nx * p->d.ny * p->d.nz * p->B;
            hipLaunchKernelGGL(k_t_zero, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, drho_out, n);
            st = hipGetLastError() == hipSuccess ? GRAV_OK : GRAV_EDEVICE;
        } else {
            st = enqueue_adjoint(p, resid, drho_out, s);
        }
    }
    if (st == GRAV_OK)
        st = end_call(p, s);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return st;
}
