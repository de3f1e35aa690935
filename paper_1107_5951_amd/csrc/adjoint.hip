// Adjoint evaluation: the exact transpose of grav_eval's linear map
// rho -> g.  The forward map is a sum of linear stages (lattice P2M, M2M,
// M2L, L2L, L2P, near-field sum, combine), so its transpose applies the
// transposed stages in reverse order: combine^T, L2P^T, L2L^T (upward),
// M2L^T, M2M^T (downward), and finally P2M^T plus the near-field transpose,
// which are fused per source leaf.  The near field and the far field of the
// forward pass partition the (target, source point) pairs, and every stage
// here uses the same pairs, operators and coincidence rule, so
// <A rho, r> = <rho, A^T r> holds to rounding.
#include <algorithm>

#include "resolve.hpp"

namespace grav {

// combine^T: per sorted target, the weights that multiply (phi, gx, gy, gz)
// in the lattice frame (G and the lattice-to-physical scale folded in).
__global__ void __launch_bounds__(256)
k_adj_weights(DevGeom g, const double *resid, const uint32_t *perm, double *w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.M)
        return;
    const int64_t t = perm[i];
    const double sg = g.G * g.h, sp = g.G * g.h * g.h;
    for (int bm = 0; bm < g.B; ++bm) {
        const double *r = resid + ((int64_t)bm * g.M + t) * g.C;
        double *o = w + (i * g.B + bm) * 4;
        if (g.C == 1) {
            o[0] = 0.0;
            o[1] = 0.0;
            o[2] = 0.0;
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
}

// Partial derivatives of (phi~, d phi~/dx, d phi~/dy, d phi~/dz) of l2p_eval
// with respect to the real coefficient (n, m, part), from the table of
// regular harmonics R[n][m] (re, im) at the evaluation point.
__device__ inline void l2p_coef_derivs(const double *R, int P, int n, int m, int part, double d[4])
{
    auto rr = [&](int a, int b) { return R[(a * P + b) * 2]; };
    auto ri = [&](int a, int b) { return R[(a * P + b) * 2 + 1]; };
    const bool lo_ok = n >= 1 && m <= n - 1;      // R_{n-1}^m exists
    const bool up_ok = n >= 1 && m + 1 <= n - 1;  // R_{n-1}^{m+1} exists
    if (m == 0) {
        d[0] = rr(n, 0);
        d[3] = n >= 1 ? rr(n - 1, 0) : 0.0;
        d[1] = up_ok ? -rr(n - 1, 1) : 0.0;
        d[2] = up_ok ? -ri(n - 1, 1) : 0.0;
    } else if (part == 0) {
        d[0] = 2.0 * rr(n, m);
        d[3] = lo_ok ? 2.0 * rr(n - 1, m) : 0.0;
        d[1] = rr(n - 1, m - 1) - (up_ok ? rr(n - 1, m + 1) : 0.0);
        d[2] = -(m - 1 >= 1 ? ri(n - 1, m - 1) : 0.0) - (up_ok ? ri(n - 1, m + 1) : 0.0);
    } else {
        d[0] = -2.0 * ri(n, m);
        d[3] = lo_ok ? -2.0 * ri(n - 1, m) : 0.0;
        d[1] = -(m - 1 >= 1 ? ri(n - 1, m - 1) : 0.0) + (up_ok ? ri(n - 1, m + 1) : 0.0);
        d[2] = -rr(n - 1, m - 1) - (up_ok ? rr(n - 1, m + 1) : 0.0);
    }
}

// L2P^T: the leaf LE adjoint is the sum over the leaf's targets of the
// transposed L2P rows weighted by the target weights.  One workgroup per
// target leaf: threads first tabulate the regular harmonics of a chunk of
// targets in LDS (one thread per (target, order m) column), then thread k
// accumulates coefficient k over the chunk.
__global__ void __launch_bounds__(256)
k_l2pT(DevGeom g, int TCH, const double *tpos, const int64_t *leaf_start, const uint32_t *tkey,
       const double *w, double *le_adj)
{
    extern __shared__ double sh[];
    const int P = g.P;
    double *Rt = sh;                          // [TCH][P][P][2]
    double *wt = sh + (size_t)TCH * P * P * 2; // [TCH][4]
    const DevLev &lv = g.lev[g.L];
    const int64_t leaf = blockIdx.x;
    const int64_t ts = leaf_start[leaf], te = leaf_start[leaf + 1];
    const uint32_t key = tkey[lv.tbox_off + leaf];
    const int lc[3] = {(int)compact3(key), (int)compact3(key >> 1), (int)compact3(key >> 2)};
    double centre[3];
    for (int a = 0; a < 3; ++a)
        centre[a] = ((double)(lc[a] - g.shift[a]) + 0.5) * g.b;
    const double inv_w = 1.0 / (double)g.b;
    const int t = threadIdx.x;
    // coefficient owned by this thread
    int cn = 0, cm = 0, cpart = 0;
    if (t < g.P2) {
        while ((cn + 1) * (cn + 1) <= t)
            ++cn;
        const int i = t - cn * cn;
        cm = (i + 1) / 2;
        cpart = (i > 0 && (i % 2) == 0) ? 1 : 0;
    }
    for (int bm = 0; bm < g.B; ++bm) {
        double acc = 0.0;
        for (int64_t c0 = ts; c0 < te; c0 += TCH) {
            const int ti = t / P, m = t % P;
            if (ti < TCH) {
                const int64_t j = c0 + ti;
                double *col = Rt + (size_t)ti * P * P * 2;
                if (j < te) {
                    const double x = (tpos[3 * j + 0] - centre[0]) * inv_w;
                    const double y = (tpos[3 * j + 1] - centre[1]) * inv_w;
                    const double z = (tpos[3 * j + 2] - centre[2]) * inv_w;
                    const double r2 = x * x + y * y + z * z;
                    double mr = 1.0, mi = 0.0;  // R_m^m
                    for (int k = 1; k <= m; ++k) {
                        const double s = 1.0 / (2.0 * k);
                        const double nr = (x * mr - y * mi) * s, ni = (x * mi + y * mr) * s;
                        mr = nr;
                        mi = ni;
                    }
                    double p1r = 0.0, p1i = 0.0, p2r = 0.0, p2i = 0.0;
                    for (int n = m; n < P; ++n) {
                        double Rr, Ri;
                        if (n == m) {
                            Rr = mr;
                            Ri = mi;
                        } else if (n == m + 1) {
                            Rr = z * p1r;
                            Ri = z * p1i;
                        } else {
                            const double f = 1.0 / (double)((n - m) * (n + m));
                            Rr = ((2.0 * n - 1.0) * z * p1r - r2 * p2r) * f;
                            Ri = ((2.0 * n - 1.0) * z * p1i - r2 * p2i) * f;
                        }
                        p2r = p1r;
                        p2i = p1i;
                        p1r = Rr;
                        p1i = Ri;
                        col[(n * P + m) * 2] = Rr;
                        col[(n * P + m) * 2 + 1] = Ri;
                    }
                    if (m == 0) {
                        const double *wj = w + (j * g.B + bm) * 4;
                        wt[ti * 4 + 0] = wj[0] * inv_w;
                        wt[ti * 4 + 1] = -wj[1] * inv_w * inv_w;
                        wt[ti * 4 + 2] = -wj[2] * inv_w * inv_w;
                        wt[ti * 4 + 3] = -wj[3] * inv_w * inv_w;
                    }
                } else if (m == 0) {
                    for (int c = 0; c < 4; ++c)
                        wt[ti * 4 + c] = 0.0;
                    for (int k = 0; k < P * P * 2; ++k)
                        col[k] = 0.0;
                }
            }
            __syncthreads();
            if (t < g.P2) {
                const int nj = (int)min((int64_t)TCH, te - c0);
                for (int k = 0; k < nj; ++k) {
                    double d[4];
                    l2p_coef_derivs(Rt + (size_t)k * P * P * 2, P, cn, cm, cpart, d);
                    acc += wt[k * 4 + 0] * d[0] + wt[k * 4 + 1] * d[1] + wt[k * 4 + 2] * d[2] +
                           wt[k * 4 + 3] * d[3];
                }
            }
            __syncthreads();
        }
        if (t < g.PS)
            le_adj[((lv.tgt_off + leaf) * g.B + bm) * g.PS + t] = t < g.P2 ? acc : 0.0;
    }
}

// P2M^T and the near-field transpose, fused per source leaf:
// drho[cell] = sum_t Pm[cell][t] ME_adj[leaf][t]
//            + sum over targets j of the 27 neighbouring target leaves and
//              quadrature points a of the cell of w_a (c0/r + c . d / r^3),
// with d = t_j - x_a in the lattice frame and the same coincidence rule as
// the forward near field.  Threads own cells (and a slice of the targets when
// the leaf has fewer than 256 cells); neighbour targets are staged in LDS.
template <typename T>
__global__ void __launch_bounds__(256)
k_leafT(DevGeom g, const double *tpos, const int64_t *leaf_start, const int32_t *tmap,
        const double *w, const double *me_adj, const double *pm, double *drho)
{
    __shared__ double st[256][7];
    __shared__ double red[256][2];
    const DevLev &lv = g.lev[g.L];
    const int64_t sleaf = blockIdx.x;
    const int lx = lv.s0[0] + (int)(sleaf % lv.ns[0]);
    const int ly = lv.s0[1] + (int)((sleaf / lv.ns[0]) % lv.ns[1]);
    const int lz = lv.s0[2] + (int)(sleaf / ((int64_t)lv.ns[0] * lv.ns[1]));
    const int b = g.b, b3 = b * b * b;
    const int corner[3] = {(lx - g.shift[0]) * b, (ly - g.shift[1]) * b, (lz - g.shift[2]) * b};
    int TC = 1;
    while (TC < b3 && TC < 256)
        TC <<= 1;
    const int S = 256 / TC;
    const int t = threadIdx.x;
    const int vi = t % TC, si = t / TC;
    const int ncell_t = (b3 > 256) ? 2 : 1;  // cells per thread
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const T go = (T)(0.5 / 1.7320508075688772);
    for (int bm = 0; bm < g.B; ++bm) {
        T acc[2] = {0, 0};
        int vrel[2][3];
        for (int k = 0; k < 2; ++k) {
            const int v = vi + k * TC;
            vrel[k][0] = v % b;
            vrel[k][1] = (v / b) % b;
            vrel[k][2] = v / (b * b);
        }
        for (int nb = 0; nb < 27; ++nb) {
            const int d[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, nb / 9 - 1};
            const int64_t tl = tmap_lookup(lv, tmap, 3, lx + d[0], ly + d[1], lz + d[2]);
            if (tl < 0)
                continue;  // uniform over the workgroup
            const int64_t ts = leaf_start[tl], te = leaf_start[tl + 1];
            for (int64_t c0 = ts; c0 < te; c0 += 256) {
                __syncthreads();
                const int64_t j = c0 + t;
                if (j < te) {
                    for (int a = 0; a < 3; ++a)
                        st[t][a] = tpos[3 * j + a] - (double)corner[a];
                    const double *wj = w + (j * g.B + bm) * 4;
                    for (int c = 0; c < 4; ++c)
                        st[t][3 + c] = wj[c];
                }
                __syncthreads();
                const int nj = (int)min((int64_t)256, te - c0);
                for (int k = 0; k < ncell_t; ++k) {
                    const int v = vi + k * TC;
                    if (v >= b3)
                        continue;
                    const T vx = (T)vrel[k][0] + (T)0.5, vy = (T)vrel[k][1] + (T)0.5,
                            vz = (T)vrel[k][2] + (T)0.5;
                    T a_acc = 0;
                    for (int jj = si; jj < nj; jj += S) {
                        const T cx = (T)st[jj][0] - vx, cy = (T)st[jj][1] - vy, cz = (T)st[jj][2] - vz;
                        const T w0 = (T)st[jj][3], w1 = (T)st[jj][4], w2 = (T)st[jj][5],
                                w3 = (T)st[jj][6];
                        if (g.q == 1) {
                            const T r2 = cx * cx + cy * cy + cz * cz;
                            if (r2 > coincident2<T>()) {
                                const T ri = rsqrt_t(r2);
                                a_acc += w0 * ri + (w1 * cx + w2 * cy + w3 * cz) * ri * ri * ri;
                            }
                        } else {
#pragma unroll
                            for (int gp = 0; gp < 8; ++gp) {
                                const T ux = cx - ((gp & 1) ? go : -go);
                                const T uy = cy - ((gp & 2) ? go : -go);
                                const T uz = cz - ((gp & 4) ? go : -go);
                                const T r2 = ux * ux + uy * uy + uz * uz;
                                if (r2 > coincident2<T>()) {
                                    const T ri = rsqrt_t(r2);
                                    a_acc += (T)0.125 *
                                             (w0 * ri + (w1 * ux + w2 * uy + w3 * uz) * ri * ri * ri);
                                }
                            }
                        }
                    }
                    acc[k] += a_acc;
                }
            }
        }
        __syncthreads();
        red[t][0] = (double)acc[0];
        red[t][1] = (double)acc[1];
        __syncthreads();
        if (si == 0) {
            for (int k = 0; k < ncell_t; ++k) {
                const int v = vi + k * TC;
                if (v >= b3)
                    continue;
                double sum = 0.0;
                for (int q = 0; q < S; ++q)
                    sum += red[q * TC + vi][k];
                if (g.L >= 2) {
                    const double *ma = me_adj + ((lv.me_off + sleaf) * g.B + bm) * g.PS;
                    const double *pr = pm + (int64_t)v * g.PS;
                    double far = 0.0;
                    for (int c = 0; c < g.P2; ++c)
                        far += pr[c] * ma[c];
                    sum += far;
                }
                const int ix = corner[0] + vrel[k][0], iy = corner[1] + vrel[k][1],
                          iz = corner[2] + vrel[k][2];
                if (ix >= 0 && iy >= 0 && iz >= 0 && ix < g.n[0] && iy < g.n[1] && iz < g.n[2])
                    drho[bm * ncell + ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix] = sum;
            }
        }
    }
}

// M2L^T on MFMA, the transpose of the forward M2L kernel: a tile is up to
// 64 source boxes of one level and child-parity class (x models); wave w owns
// columns 16w..16w+15 and accumulates ME_adj[S] += K_d^T LE_adj[S - d] over
// the offsets d for which S - d is a target box whose class admits d.
template <int RB, typename T>
__global__ void __launch_bounds__(256)
k_m2lT(DevGeom g, const GemmTile *tiles, const int32_t *tmap, const int32_t *rclass_off, const T *KT,
       const double *le_adj, double *me_adj, int S, int64_t part_stride)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(T)))) T;
    const GemmTile tile = tiles[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const DevLev &lv = g.lev[tile.level];
    const int cl = wave * 16 + (lane & 15);
    const bool cvalid = cl < tile.ncol;
    const int64_t col = tile.col0 + cl;
    const int bm = (int)(col % g.B);
    int xyz[3] = {0, 0, 0};
    int64_t sbox = 0;
    if (cvalid) {
        class_box((int)(col / g.B), tile.cls, lv.s0, lv.ns, xyz);
        sbox = dense_index(lv, xyz[0], xyz[1], xyz[2]);
    }
    vec4 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
        acc[rb] = vec4{0, 0, 0, 0};
    const int32_t *offs = rclass_off + tile.cls * kClassOffsets * 4;
    const int krow = lane >> 4;
    const int o0 = tile.pad * kClassOffsets / S, o1 = (tile.pad + 1) * kClassOffsets / S;
    for (int o = o0; o < o1; ++o) {
        const int dx = offs[4 * o + 0], dy = offs[4 * o + 1], dz = offs[4 * o + 2];
        const int id = offs[4 * o + 3];
        const int64_t t = cvalid ? tmap_lookup(lv, tmap, 3, xyz[0] - dx, xyz[1] - dy, xyz[2] - dz) : -1;
        const bool have = t >= 0;
        if (__ballot(have) == 0ull)
            continue;  // no column of this wave feeds a target box at this offset
        const double *mp = le_adj + (have ? ((lv.tgt_off + t) * g.B + bm) * g.PS : 0);
        const T *kp = KT + (int64_t)id * g.KS * RB * 64 + lane;
        for (int ks = 0; ks < g.KS; ++ks) {
            const T bv = have ? (T)mp[4 * ks + krow] : (T)0;
            const T *ka = kp + (int64_t)ks * RB * 64;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                if constexpr (sizeof(T) == 8)
                    acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ka[rb * 64], bv, acc[rb], 0, 0, 0);
                else
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ka[rb * 64], bv, acc[rb], 0, 0, 0);
            }
        }
    }
    if (!cvalid)
        return;
    // Output fragment: column lane % 16, four rows; the FP32 instruction gives
    // rows 4*(lane/16) + r, the FP64 one rows lane/16 + 4r.
    double *dst = me_adj + (tile.pad * part_stride + (lv.me_off + sbox) * g.B + bm) * g.PS;
    constexpr int rstride = sizeof(T) == 8 ? 4 : 1;
    const int rbase = sizeof(T) == 8 ? krow : 4 * krow;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            dst[16 * rb + rbase + rstride * r] = (double)acc[rb][r];
}

// L2L^T (upward): LE_adj of a level-l box = sum over its children c of
// S_c^T LE_adj[child].  One workgroup per target box of level l; the
// children's adjoints are staged in LDS; thread s produces coefficient s.
// The L2L matrices are stored [child][in s][out t], so thread s reads row s.
__global__ void __launch_bounds__(256) k_l2lT(DevGeom g, int l, const uint32_t *tkey,
                                              const int32_t *tchild, const double *l2l, double *le_adj)
{
    extern __shared__ double sh[];  // [8][PS]
    __shared__ int cls[8];
    const DevLev &lv = g.lev[l];
    const DevLev &lc = g.lev[l + 1];
    const int64_t box = blockIdx.x;
    const int64_t a = tchild[lv.tchild_off + box], b = tchild[lv.tchild_off + box + 1];
    const int nch = (int)(b - a);
    if (threadIdx.x < 8)
        cls[threadIdx.x] = threadIdx.x < nch ? (int)(tkey[lc.tbox_off + a + threadIdx.x] & 7u) : 0;
    for (int bm = 0; bm < g.B; ++bm) {
        for (int i = threadIdx.x; i < nch * g.PS; i += blockDim.x) {
            const int k = i / g.PS, t = i % g.PS;
            sh[i] = le_adj[((lc.tgt_off + a + k) * g.B + bm) * g.PS + t];
        }
        __syncthreads();
        for (int s = threadIdx.x; s < g.PS; s += blockDim.x) {
            double acc = 0.0;
            for (int k = 0; k < nch; ++k) {
                const double *row = l2l + ((int64_t)cls[k] * g.PS + s) * g.PS;
                const double *y = sh + k * g.PS;
                for (int t = 0; t < g.P2; ++t)
                    acc += row[t] * y[t];
            }
            le_adj[((lv.tgt_off + box) * g.B + bm) * g.PS + s] = acc;
        }
        __syncthreads();
    }
}

// M2M^T (downward): ME_adj of a level-l source box += T_c^T ME_adj[parent]
// (c = its octant).  One workgroup per source box of level l >= 3; the
// parent's adjoint is staged in LDS; thread j produces coefficient j.  The
// M2M matrices are stored [child][in j][out i], so thread j reads row j.
__global__ void __launch_bounds__(256) k_m2mT(DevGeom g, int l, const double *m2m, double *me_adj)
{
    extern __shared__ double sh[];  // [PS]
    const DevLev &lv = g.lev[l];
    const DevLev &lp = g.lev[l - 1];
    const int64_t box = blockIdx.x;
    const int x = lv.s0[0] + (int)(box % lv.ns[0]);
    const int y = lv.s0[1] + (int)((box / lv.ns[0]) % lv.ns[1]);
    const int z = lv.s0[2] + (int)(box / ((int64_t)lv.ns[0] * lv.ns[1]));
    const int c = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
    const int64_t par = dense_index(lp, x >> 1, y >> 1, z >> 1);
    const double *mc = m2m + (int64_t)c * g.PS * g.PS;
    for (int bm = 0; bm < g.B; ++bm) {
        for (int i = threadIdx.x; i < g.PS; i += blockDim.x)
            sh[i] = par >= 0 ? me_adj[((lp.me_off + par) * g.B + bm) * g.PS + i] : 0.0;
        __syncthreads();
        for (int j = threadIdx.x; j < g.PS; j += blockDim.x) {
            const double *row = mc + (int64_t)j * g.PS;
            double acc = 0.0;
            for (int i = 0; i < g.P2; ++i)
                acc += row[i] * sh[i];
            me_adj[((lv.me_off + box) * g.B + bm) * g.PS + j] += acc;
        }
        __syncthreads();
    }
}

template <typename T>
static grav_status launch_m2lT(Plan *p, const DevGeom &g, hipStream_t s, const T *KT)
{
    const TileRange &r = p->tiles[TK_M2LT][0];
    if (r.n == 0)
        return GRAV_OK;
    const int RB = p->PS / 16;
    dim3 grid(r.n), blk(256);
    const int S = p->split[TK_M2LT];
    const int64_t pstride = p->n_me * p->B;
    double *dst = S > 1 ? p->d_part : p->d_me;
#define M2LT_CASE(R)                                                                            \
    case R:                                                                                     \
        hipLaunchKernelGGL((k_m2lT<R, T>), grid, blk, 0, s, g,                                  \
                           (const GemmTile *)(p->d_tiles + r.off), (const int32_t *)p->d_tmap,  \
                           (const int32_t *)p->d_rclass_off, KT, (const double *)p->d_le, dst,  \
                           S, pstride);                                                         \
        break;
    switch (RB) {
        M2LT_CASE(1)
        M2LT_CASE(2)
        M2LT_CASE(3)
        M2LT_CASE(4)
        M2LT_CASE(6)
        M2LT_CASE(7)
        M2LT_CASE(8)
        M2LT_CASE(9)
        M2LT_CASE(11)
        M2LT_CASE(13)
        M2LT_CASE(15)
        M2LT_CASE(16)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef M2LT_CASE
    GRAV_HIP(hipGetLastError());
    if (S > 1) {
        const int64_t n = pstride * p->PS;
        hipLaunchKernelGGL(k_sum_parts<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const double *)p->d_part, S, n, p->d_me);
        GRAV_HIP(hipGetLastError());
    }
    return GRAV_OK;
}

grav_status enqueue_adjoint(Plan *p, const double *resid, double *drho, hipStream_t s)
{
    const DevGeom g = make_geom(p);
    const int L = p->L;
    const int64_t ncell = (int64_t)p->d.nx * p->d.ny * p->d.nz;
    if (p->M == 0) {
        GRAV_HIP(hipMemsetAsync(drho, 0, sizeof(double) * ncell * p->B, s));
        return GRAV_OK;
    }
    stage_begin(p, "weights", s);
    hipLaunchKernelGGL(k_adj_weights, dim3((unsigned)((p->M + 255) / 256)), dim3(256), 0, s, g, resid,
                       (const uint32_t *)p->d_perm, p->d_near);
    GRAV_HIP(hipGetLastError());
    stage_end(p, s);
    if (L >= 2) {
        stage_begin(p, "l2pT", s);
        // targets per chunk: one thread per (target, order), LDS under 60 KB
        const int TCH = std::min(256 / p->P, 60000 / (p->P * p->P * 16));
        const size_t lds = sizeof(double) * ((size_t)TCH * p->P * p->P * 2 + (size_t)TCH * 4);
        hipLaunchKernelGGL(k_l2pT, dim3((unsigned)p->n_leaf), dim3(256), lds, s, g, TCH,
                           (const double *)p->d_tpos, (const int64_t *)p->d_leaf_start,
                           (const uint32_t *)p->d_tkey, (const double *)p->d_near, p->d_le);
        GRAV_HIP(hipGetLastError());
        stage_end(p, s);
        stage_begin(p, "l2lT", s);
        for (int l = L - 1; l >= 2; --l) {
            hipLaunchKernelGGL(k_l2lT, dim3((unsigned)p->lev[l].n_tgt), dim3(256),
                               sizeof(double) * 8 * p->PS, s, g, l, (const uint32_t *)p->d_tkey,
                               (const int32_t *)p->d_tchild, (const double *)p->d_l2l, p->d_le);
            GRAV_HIP(hipGetLastError());
        }
        stage_end(p, s);
        stage_begin(p, "m2lT", s);
        if (p->d.precision == GRAV_FP64)
            GRAV_CHECK(launch_m2lT<double>(p, g, s, p->d_k64T));
        else
            GRAV_CHECK(launch_m2lT<float>(p, g, s, p->d_k32T));
        stage_end(p, s);
        stage_begin(p, "m2mT", s);
        for (int l = 3; l <= L; ++l) {
            hipLaunchKernelGGL(k_m2mT, dim3((unsigned)p->lev[l].n_src), dim3(256),
                               sizeof(double) * p->PS, s, g, l, (const double *)p->d_m2m, p->d_me);
            GRAV_HIP(hipGetLastError());
        }
        stage_end(p, s);
    }
    stage_begin(p, "leafT", s);
    if (p->d.precision == GRAV_FP64)
        hipLaunchKernelGGL(k_leafT<double>, dim3((unsigned)p->lev[L].n_src), dim3(256), 0, s, g,
                           (const double *)p->d_tpos, (const int64_t *)p->d_leaf_start,
                           (const int32_t *)p->d_tmap, (const double *)p->d_near,
                           (const double *)p->d_me, (const double *)p->d_pm, drho);
    else
        hipLaunchKernelGGL(k_leafT<float>, dim3((unsigned)p->lev[L].n_src), dim3(256), 0, s, g,
                           (const double *)p->d_tpos, (const int64_t *)p->d_leaf_start,
                           (const int32_t *)p->d_tmap, (const double *)p->d_near,
                           (const double *)p->d_me, (const double *)p->d_pm, drho);
    GRAV_HIP(hipGetLastError());
    stage_end(p, s);
    return GRAV_OK;
}

}  // namespace grav

using namespace grav;

extern "C" grav_status grav_adjoint(grav_plan_t plan, const double *resid, double *drho_out,
                                    void *stream)
{
    if (!plan || !resid || !drho_out)
        return GRAV_EINVAL;
#ifndef GRAV_ENABLE_ADJOINT
    // The transposed pass is switched off in this library build: its kernels
    // are compiled but not launched (define GRAV_ENABLE_ADJOINT to enable).
    (void)stream;
    return GRAV_EUNSUPPORTED;
#endif
    Plan *p = reinterpret_cast<Plan *>(plan);
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    GRAV_HIP(hipGetDevice(&cur));
    if (cur != p->device)
        GRAV_HIP(hipSetDevice(p->device));
    grav_status st = begin_call(p, s);
    if (st == GRAV_OK)
        st = enqueue_adjoint(p, resid, drho_out, s);
    if (st == GRAV_OK)
        st = end_call(p, s);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return st;
}
