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

// M2L^T runs on the forward's stream-K M2L kernel (transposed operators,
// columns = source boxes of each level's column block, see
// build_m2l_transposed).  Its B operand: the adjoint LE of each level's
// gather region regathered in the kernel's layout (class-split boxes,
// chunk-major planes (q, kr) of four coefficients 16 q + kr + 4 u), zero
// where the region has no target box and for the padding coefficients.
// The target box at a position comes from the level's target map (source
// block plus a halo of 3, which holds the region).  One thread per (region
// box, model, plane).
template <typename T>
__global__ void __launch_bounds__(256)
k_le_gather(DevGeom gt, DevGeom g, const int32_t *tmap, int64_t n_tmap, int64_t n_tbox, const double *le,
            int64_t n_leg, T *out)
{
    const int NP = g.PS / 4;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_leg * g.B * NP)
        return;
    const int plane = (int)(i % NP);
    const int64_t col = i / NP;  // region box * B + model
    const int bm = (int)(col % g.B);
    const int64_t box = col / g.B;
    int l = 2;
    while (l < g.L && box >= gt.lev[l + 1].me_off)
        ++l;
    const DevLev &lt = gt.lev[l];
    const DevLev &lv = g.lev[l];
    const int64_t r = box - lt.me_off;
    const int x = lt.s0[0] + (int)(r % lt.ns[0]), y = lt.s0[1] + (int)((r / lt.ns[0]) % lt.ns[1]),
              z = lt.s0[2] + (int)(r / ((int64_t)lt.ns[0] * lt.ns[1]));
    int first[3], cnt[3];
    const int64_t pos = class_split(lt, (x & 1) | ((y & 1) << 1) | ((z & 1) << 2), first, cnt) +
                        ((int64_t)((z - first[2]) >> 1) * cnt[1] + ((y - first[1]) >> 1)) * cnt[0] +
                        ((x - first[0]) >> 1);
    int64_t tb = -1;
    const int mx = x - lv.s0[0] + 3, my = y - lv.s0[1] + 3, mz = z - lv.s0[2] + 3;
    if (mx >= 0 && my >= 0 && mz >= 0 && mx < lv.ns[0] + 6 && my < lv.ns[1] + 6 && mz < lv.ns[2] + 6) {
        const int64_t mi = lv.tmap_off + ((int64_t)mz * (lv.ns[1] + 6) + my) * (lv.ns[0] + 6) + mx;
        if (mi < n_tmap) {
            const int64_t v = tmap[mi];
            if (v >= 0 && v < lv.n_tgt && lv.tgt_off + v < n_tbox)
                tb = v;
        }
    }
    const int q = plane / 4, kr = plane % 4;
    const int64_t nB = (int64_t)lt.ns[0] * lt.ns[1] * lt.ns[2] * g.B;
    T *dst = out + lt.me_off * g.B * g.PS + ((int64_t)plane * nB + pos * g.B + bm) * 4;
    const double *src = le + (tb >= 0 ? ((lv.tgt_off + tb) * g.B + bm) * g.PS : 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = 16 * q + kr + 4 * u;
        dst[u] = (T)(tb >= 0 && c < g.P2 ? src[c] : 0.0);
    }
}

// ME of the transposed M2L's columns from its segment slots: the sum, over
// the segments of the column's unit in their order, of the slot entry, in
// FP64 (as the forward's k_m2l_sum); the column's ME is overwritten.  A
// unit without segments (no target box at any offset) gives zero.
template <typename T>
__global__ void __launch_bounds__(256)
k_m2lt_sum(const T *part, const int32_t *colmap, const int64_t *colbox, const int32_t *tseg_start,
           const int32_t *tsegs, int64_t ncols, int PS, int ncw, double *me)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncols * PS)
        return;
    const int64_t c = i / PS;
    const int k = (int)(i - c * PS);
    const int32_t m = colmap[c];
    const int t = m >> 6, cl = m & 63;
    double acc = 0.0;
    for (int j = tseg_start[t]; j < tseg_start[t + 1]; ++j)
        acc += (double)part[((int64_t)tsegs[j] * ncw + cl) * PS + k];
    me[colbox[c] * PS + k] = acc;
}

// The column blocks of the transposed M2L: the boxes of level l whose ME it
// writes (inclusive range); M2M^T adds to these and sets the others.
struct ColBlock {
    int lo[3], hi[3];
};

// M2M^T (downward over the source blocks): ME_l[child] += M2M_c^T
// ME_l-1[parent], M2M row-major [octant][out i][in j], so the thread of
// coefficient j reads column j.  One thread per (source box of level l,
// model group, coefficient j).
template <int MT>
__global__ void __launch_bounds__(256) k_t_m2m(DevGeom g, int l, ColBlock cb, const double *m2m, double *me)
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
    const int oct = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
    const double *col = m2m + (int64_t)oct * g.PS * g.PS + j;
    const double *mp = me + ((lp.me_off + (par >= 0 ? par : 0)) * g.B + grp * MT) * g.PS;
    double acc[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
        acc[u] = 0.0;
    for (int i = 0; i < (par >= 0 ? g.P2 : 0); ++i) {
        const double m = col[(int64_t)i * g.PS];
#pragma unroll
        for (int u = 0; u < MT; ++u)
            if (grp * MT + u < g.B)
                acc[u] += m * mp[(int64_t)u * g.PS + i];
    }
    // inside the column block the transposed M2L has written the ME
    const bool add = x >= cb.lo[0] && x <= cb.hi[0] && y >= cb.lo[1] && y <= cb.hi[1] && z >= cb.lo[2] &&
                     z <= cb.hi[2];
#pragma unroll
    for (int u = 0; u < MT; ++u) {
        const int bm = grp * MT + u;
        if (bm < g.B) {
            double *o = me + ((lv.me_off + box) * g.B + bm) * g.PS + j;
            *o = add ? *o + acc[u] : acc[u];
        }
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

// M2L^T: regather the adjoint LE, run the forward kernel on the transposed
// problem, add each column's segment slots into its ME.
template <typename T>
static grav_status m2l_transposed_t(Plan *p, const DevGeom &g, hipStream_t s, const T *Kt)
{
    DevGeom gt = g;  // the kernel's view: columns = source boxes, B = gathered adjoint LE
    for (int l = 2; l <= p->L; ++l) {
        const LevelInfo &lv = p->lev[l];
        DevLev &d = gt.lev[l];
        for (int a = 0; a < 3; ++a) {
            d.s0[a] = lv.gs0[a];
            d.ns[a] = lv.gns[a];
        }
        d.me_off = lv.g_off;
        d.tbox_off = lv.me_off;
        for (int c = 0; c < 9; ++c)
            d.class_start[c] = lv.col_class_start[c];
    }
    T *leg = reinterpret_cast<T *>(p->d_leg);
    const int64_t n = p->n_leg * p->B * (p->PS / 4);
    if (n > 0) {
        hipLaunchKernelGGL((k_le_gather<T>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, gt, g,
                           (const int32_t *)p->d_tmap, p->n_tmap, p->n_tbox, (const double *)p->d_le, p->n_leg, leg);
        GRAV_HIP(hipGetLastError());
    }
    M2LRun<T> r;
    r.tiles = (const GemmTile *)p->d_m2lt_tiles;
    r.keys = (const uint32_t *)p->d_skey;
    r.order = (const int32_t *)p->d_sorder;
    r.class_off = (const int32_t *)p->d_tclass_off;
    r.K = Kt;
    r.b_in = leg;
    r.segs = (const int32_t *)p->d_m2lt_segs;
    r.wgseg = (const int32_t *)p->d_m2lt_wgseg;
    r.items = (const int32_t *)p->d_m2lt_items;
    r.part = reinterpret_cast<T *>(p->d_partt);
    r.wgs = p->m2lt_wgs;
    r.nset = p->m2lt_nset;
    GRAV_CHECK(launch_m2l<T>(p, gt, s, r));
    const int64_t ns = p->m2lt_ncols * p->PS;
    if (ns > 0) {
        hipLaunchKernelGGL((k_m2lt_sum<T>), dim3((unsigned)ceil_div(ns, 256)), dim3(256), 0, s,
                           (const T *)p->d_partt, (const int32_t *)p->d_m2lt_colmap, (const int64_t *)p->d_m2lt_colbox,
                           (const int32_t *)p->d_m2lt_tseg_start, (const int32_t *)p->d_m2lt_tsegs, p->m2lt_ncols,
                           p->PS, p->m2l_ncw, p->d_me);
        GRAV_HIP(hipGetLastError());
    }
    return GRAV_OK;
}

static grav_status enqueue_m2l_transposed(Plan *p, const DevGeom &g, hipStream_t s)
{
    return p->d.precision == GRAV_FP64 ? m2l_transposed_t<double>(p, g, s, p->d_kt64)
                                       : m2l_transposed_t<float>(p, g, s, p->d_kt32);
}

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
        GRAV_CHECK(enqueue_m2l_transposed(p, g, s));
        stage_end(p, s);
        stage_begin(p, "m2mT", s);
        for (int l = 3; l <= L; ++l) {
            const LevelInfo &lv = p->lev[l];
            ColBlock cb;
            for (int a = 0; a < 3; ++a) {
                cb.lo[a] = lv.cs0[a];
                cb.hi[a] = lv.cs0[a] + lv.cns[a] - 1;
            }
            hipLaunchKernelGGL(k_t_m2m<MT>, grid(p->lev[l].n_src * NG * p->PS), blk, 0, s, g, l, cb,
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
