// grav_plan: geometry, device octree build and operator set-up.
//
// Internally every length is in cell units with the mesh origin at 0 (the
// "lattice frame"): cell (i, j, k) spans [i, i+1) x [j, j+1) x [k, k+1), a
// quadrature point has mass rho * w_a with w_a the rule's weight fraction,
// and the physical field follows as g = G h g_lat, phi = G h^2 phi_lat.
// Cell-centre evaluation points are placed at exact half-integers, so a
// point that coincides with a 1-point source has an exactly zero offset.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>

#include "resolve.hpp"
#include "internal.hpp"
#include "operators.hpp"

// Upper bound on the one-wave workgroups of the forward M2L's stream-K
// schedule; the plan takes as many as the device holds at once
// (m2l_resident_workers), up to this.
#ifndef GRAV_M2L_WAVES
#define GRAV_M2L_WAVES 8192
#endif

namespace grav {

namespace {

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Position (lattice frame) of evaluation point i in descriptor order.
__device__ inline void target_lattice(int64_t i, const double *pts, int64_t npts, int nx, int ny,
                                      const double org[3], double inv_h, double out[3])
{
    if (i < npts) {
        out[0] = (pts[3 * i + 0] - org[0]) * inv_h;
        out[1] = (pts[3 * i + 1] - org[1]) * inv_h;
        out[2] = (pts[3 * i + 2] - org[2]) * inv_h;
    } else {
        const int64_t c = i - npts;
        const int64_t ix = c % nx;
        const int64_t iy = (c / nx) % ny;
        const int64_t iz = c / ((int64_t)nx * ny);
        out[0] = (double)ix + 0.5;
        out[1] = (double)iy + 0.5;
        out[2] = (double)iz + 0.5;
    }
}

struct KeyArgs {
    const double *pts;
    int64_t npts, M;
    int nx, ny;
    double org[3];
    double inv_h;
    double shift_lat[3];  // shift * b: lattice distance from root corner to origin
    double inv_b;
    int kmax;             // leaves per axis - 1
    int L;
};

__global__ void k_target_keys(KeyArgs a, uint32_t *keys, uint32_t *vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.M)
        return;
    double u[3];
    target_lattice(i, a.pts, a.npts, a.nx, a.ny, a.org, a.inv_h, u);
    uint32_t c[3];
    for (int d = 0; d < 3; ++d) {
        double f = floor((u[d] + a.shift_lat[d]) * a.inv_b);
        f = fmin(fmax(f, 0.0), (double)a.kmax);
        c[d] = (uint32_t)f;
    }
    keys[i] = morton3(c[0], c[1], c[2]);
    vals[i] = (uint32_t)i;
}

__global__ void k_gather_targets(KeyArgs a, const uint32_t *perm, double *tpos)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.M)
        return;
    double u[3];
    target_lattice((int64_t)perm[i], a.pts, a.npts, a.nx, a.ny, a.org, a.inv_h, u);
    tpos[3 * i + 0] = u[0];
    tpos[3 * i + 1] = u[1];
    tpos[3 * i + 2] = u[2];
}

// flags[i] = 1 where (key[i] >> sh) differs from its predecessor.
__global__ void k_head_flags(const uint32_t *keys, int64_t n, int sh, uint32_t *flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    flags[i] = (i == 0 || (keys[i] >> sh) != (keys[i - 1] >> sh)) ? 1u : 0u;
}

// Leaf level: sorted target -> leaf id, leaf start offsets, leaf keys.
__global__ void k_leaf_build(const uint32_t *keys, const uint32_t *flags, const uint32_t *scan,
                             int64_t n, int32_t *tleaf, int64_t *leaf_start, uint32_t *leaf_key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t id = scan[i] + flags[i] - 1u;
    tleaf[i] = (int32_t)id;
    if (flags[i]) {
        leaf_start[id] = i;
        leaf_key[id] = keys[i];
    }
}

// Parent level from the sorted child box keys.
__global__ void k_parent_build(const uint32_t *ckeys, const uint32_t *flags, const uint32_t *scan,
                               int64_t n, int32_t *cparent, uint32_t *pkeys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t id = scan[i] + flags[i] - 1u;
    cparent[i] = (int32_t)id;
    if (flags[i])
        pkeys[id] = ckeys[i] >> 3;
}

// Sort keys of the target boxes of a level for the class-grouped order
// (the column order of the M2L and L2L tiles).  First pass: x-fastest
// lexicographic order of the boxes.  Second, stable pass: parity class
// (Morton bits 0..2), then the box's boundary signature in y and z (the
// range of interaction-list offsets, |d| <= 3, that stay inside the source
// block on those axes).  A wave's 16 columns are then boxes of one class
// along x rows that mostly see the same source offsets, so (i) the waves
// skip the same missing offsets and waste little MFMA work, and (ii) the
// source boxes a wave reads at one offset are consecutive in x, which the
// regathered expansions store contiguously.
__global__ void k_lex_keys(const uint32_t *bkeys, int64_t n, int bits, uint32_t *ck, uint32_t *cv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t k = bkeys[i];
    ck[i] = (compact3(k >> 2) << (2 * bits)) | (compact3(k >> 1) << bits) | compact3(k);
    cv[i] = (uint32_t)i;
}

__global__ void k_class_keys(const uint32_t *bkeys, const uint32_t *order, int64_t n, int3 s0, int3 ns,
                             uint32_t *ck, uint32_t *counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t k = bkeys[order[i]];
    const uint32_t cls = k & 7u;  // Morton bits 0,1,2 = x, y, z parity
    const int c[2] = {(int)compact3(k >> 1), (int)compact3(k >> 2)};
    const int lo[2] = {s0.y, s0.z}, len[2] = {ns.y, ns.z};
    uint32_t sig = 0;
    for (int a = 0; a < 2; ++a) {
        const int dlo = min(4, max(-3, lo[a] - c[a]));               // lowest valid offset
        const int dhi = max(-4, min(3, lo[a] + len[a] - 1 - c[a]));  // highest valid offset
        sig = sig * 64u + (uint32_t)((dlo + 3) * 8 + (dhi + 4));
    }
    ck[i] = (cls << 12) | sig;
    atomicAdd(&counts[cls], 1u);
}

struct CountArgs {
    int s0[3], ns[3];   // source block of the level
    int n[3], shift[3];
    int b, nq3;
};

// M2L box pairs of one level: in-block offsets of each target box's class list.
__global__ void k_count_m2l(const uint32_t *bkeys, int64_t n, CountArgs a, const int32_t *cls_off,
                            unsigned long long *acc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t k = bkeys[i];
    const int x = (int)compact3(k), y = (int)compact3(k >> 1), z = (int)compact3(k >> 2);
    const int32_t *o = cls_off + (k & 7u) * kClassOffsets * 4;
    unsigned long long c = 0;
    for (int j = 0; j < kClassOffsets; ++j) {
        const int sx = x + o[4 * j] - a.s0[0], sy = y + o[4 * j + 1] - a.s0[1],
                  sz = z + o[4 * j + 2] - a.s0[2];
        if (sx >= 0 && sy >= 0 && sz >= 0 && sx < a.ns[0] && sy < a.ns[1] && sz < a.ns[2])
            ++c;
    }
    atomicAdd(acc, c);
}

// P2P point pairs: targets of a leaf times source points in its 27 neighbours.
__global__ void k_count_p2p(const uint32_t *lkeys, const int64_t *leaf_start, int64_t n,
                            CountArgs a, unsigned long long *acc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t k = lkeys[i];
    const int c[3] = {(int)compact3(k), (int)compact3(k >> 1), (int)compact3(k >> 2)};
    unsigned long long cells = 0;
    for (int nb = 0; nb < 27; ++nb) {
        const int d[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, nb / 9 - 1};
        unsigned long long leaf_cells = 1;
        for (int ax = 0; ax < 3; ++ax) {
            const int lc = c[ax] + d[ax];
            if (lc - a.s0[ax] < 0 || lc - a.s0[ax] >= a.ns[ax]) {
                leaf_cells = 0;
                break;
            }
            const int lo = (lc - a.shift[ax]) * a.b;
            const int hi = min(lo + a.b, a.n[ax]);
            leaf_cells *= (unsigned long long)max(0, hi - max(lo, 0));
        }
        cells += leaf_cells;
    }
    atomicAdd(acc, cells * (unsigned long long)a.nq3 * (unsigned long long)(leaf_start[i + 1] - leaf_start[i]));
}

// Point pairs of the near field with explicit sources: per target leaf, its
// targets times the sources of its 27 neighbour leaves.
__global__ void k_count_p2p_src(const uint32_t *lkeys, const int64_t *leaf_start, int64_t n, CountArgs a,
                                const int64_t *sstart, unsigned long long *acc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t k = lkeys[i];
    const int c[3] = {(int)compact3(k), (int)compact3(k >> 1), (int)compact3(k >> 2)};
    unsigned long long srcs = 0;
    for (int nb = 0; nb < 27; ++nb) {
        const int d[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, nb / 9 - 1};
        int r[3];
        bool in = true;
        for (int ax = 0; ax < 3; ++ax) {
            r[ax] = c[ax] + d[ax] - a.s0[ax];
            in = in && r[ax] >= 0 && r[ax] < a.ns[ax];
        }
        if (!in)
            continue;
        const int64_t j = ((int64_t)r[2] * a.ns[1] + r[1]) * a.ns[0] + r[0];
        srcs += (unsigned long long)(sstart[j + 1] - sstart[j]);
    }
    atomicAdd(acc, srcs * (unsigned long long)(leaf_start[i + 1] - leaf_start[i]));
}

__global__ void k_fill_last(int64_t *leaf_start, int64_t n_leaf, int64_t M)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        leaf_start[n_leaf] = M;
}

// Sorted slot of every voxel-centre target: slot[c] = j with perm[j] = npts + c.
__global__ void k_cell_slot(const uint32_t *perm, int64_t M, int64_t npts, int32_t *slot)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M)
        return;
    const int64_t i = perm[j];
    if (i >= npts)
        slot[i - npts] = (int32_t)j;
}

// End of the user points of each leaf.  The sort is stable and the keys are
// assigned in descriptor order (points first, then voxel centres), so within a
// leaf the user points form a prefix; find its end by bisection.
__global__ void k_leaf_point_end(const uint32_t *perm, const int64_t *leaf_start, int64_t n_leaf,
                                 int64_t npts, int64_t *pend)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_leaf)
        return;
    int64_t lo = leaf_start[l], hi = leaf_start[l + 1];
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((int64_t)perm[mid] < npts)
            lo = mid + 1;
        else
            hi = mid;
    }
    pend[l] = lo;
}

template <class T>
grav_status dalloc(Plan *p, T **ptr, size_t count, bool resident)
{
    *ptr = nullptr;
    if (count == 0)
        return GRAV_OK;
    if (hipMalloc((void **)ptr, sizeof(T) * count) != hipSuccess) {
        *ptr = nullptr;
        return GRAV_ENOMEM;
    }
    if (resident)
        p->bytes_resident += sizeof(T) * count;
    else
        p->bytes_call += sizeof(T) * count;
    return GRAV_OK;
}

void free_plan(Plan *p)
{
    if (!p)
        return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    void *bufs[] = {p->d_points, p->d_perm, p->d_tpos, p->d_tleaf, p->d_leaf_start, p->d_tkey,
                    p->d_tparent, p->d_torder, p->d_tiles, p->d_class_off, p->d_rclass_off,
                    p->d_tmap, p->d_tchild, p->d_geom, p->d_pm, p->d_pm_sw, p->d_m2m,
                    p->d_l2l, p->d_k64, p->d_k32, p->d_me,
                    p->d_le, p->d_near, p->d_part, p->d_tn64, p->d_tn32, p->d_m2m_sw, p->d_l2l_sw, p->d_rho_blk, p->d_tl2p, p->d_dpart, p->d_meg, p->d_lat_tab, p->d_m2l_items, p->d_m2l_segs,
                    p->d_m2l_wgseg, p->d_m2l_tseg_start, p->d_m2l_tsegs, p->d_m2l_colmap,
                    p->d_cell_slot, p->d_leaf_pend, p->d_m2lt_tiles, p->d_m2lt_items, p->d_m2lt_segs,
                    p->d_m2lt_wgseg, p->d_m2lt_tseg_start, p->d_m2lt_tsegs, p->d_m2lt_colmap, p->d_m2lt_colbox,
                    p->d_skey, p->d_sorder, p->d_tclass_off, p->d_kt64, p->d_kt32, p->d_leg, p->d_partt, p->d_kt32o, p->d_orbtab_t,
                    p->d_m2mt_sw, p->d_l2lt_sw, p->d_l2l_msw, p->d_pmt_sw, p->d_tnt64, p->d_tnt32, p->d_tl2pt, p->d_w_blk,
                    p->d_spos, p->d_sw, p->d_sperm, p->d_sstart, p->d_pt_leaves, p->d_user_leaves,
                    p->d_k32o, p->d_orbtab, p->d_ccoef, p->d_kmap};
    for (void *b : bufs)
        if (b)
            (void)hipFree(b);
    if (p->done)
        (void)hipEventDestroy(p->done);
    for (auto &st : p->stages) {
        if (st.a)
            (void)hipEventDestroy(st.a);
        if (st.b)
            (void)hipEventDestroy(st.b);
    }
    (void)hipSetDevice(cur);
    delete p;
}

grav_status validate(const grav_plan_desc *d)
{
    if (!d)
        return GRAV_EINVAL;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return GRAV_EINVAL;
    if (!(d->h > 0.0) || !std::isfinite(d->h))
        return GRAV_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->origin[a]))
            return GRAV_EINVAL;
    if (d->quad_order != 1 && d->quad_order != 2)
        return GRAV_EINVAL;
    if (d->n_points < 0 || (d->n_points > 0 && !d->points))
        return GRAV_EINVAL;
    if (d->components != 1 && d->components != 3 && d->components != 4)
        return GRAV_EINVAL;
    if (d->p < 1)
        return GRAV_EINVAL;
    if (d->p > kMaxP)
        return GRAV_EUNSUPPORTED;
    if (d->leaf_size < 1)
        return GRAV_EINVAL;
    if (d->precision != GRAV_FP64 && d->precision != GRAV_MIXED)
        return GRAV_EINVAL;
    if (d->batch < 1)
        return GRAV_EINVAL;
    if (!std::isfinite(d->G))
        return GRAV_EINVAL;
    if (d->n_sources < 0 || (d->n_sources > 0 && (!d->sources || d->quad_order != 1)))
        return GRAV_EINVAL;
    if (d->n_sources > 0xffffffffll)
        return GRAV_EUNSUPPORTED;
    for (int64_t i = 0; i < d->n_sources; ++i) {
        for (int a = 0; a < 3; ++a) {
            const int n = a == 0 ? d->nx : a == 1 ? d->ny : d->nz;
            const double u = (d->sources[3 * i + a] - d->origin[a]) / d->h;
            if (!(u >= 0.0 && u < (double)n))
                return GRAV_EINVAL;  // outside the mesh box (or not finite)
        }
        if (d->source_volumes && !(d->source_volumes[i] > 0.0 && std::isfinite(d->source_volumes[i])))
            return GRAV_EINVAL;
    }
    const int64_t ncell = (int64_t)d->nx * d->ny * d->nz;
    const int64_t M = d->n_points + (d->voxel_centres ? ncell : 0);
    if (M > 0xffffffffll || (int64_t)d->nx > 0x3fffffff)
        return GRAV_EUNSUPPORTED;
    return GRAV_OK;
}

// Index of the operator of offset |d| (components 0..3, largest >= 2) among
// the 56 stored for the mixed-precision forward M2L, z slowest, x fastest.
// Sign class of real coefficient c under the z, y and x reflections (bits
// 2, 1, 0; the bits of the reflection index of an offset): degree n block of
// 2n+1 values, the real part of order 0, then real and imaginary parts of
// orders 1..n; z -> -z gives (-1)^(n+m), y -> -y -1 on imaginary parts, x ->
// -x (-1)^m on real and -(-1)^m on imaginary parts.
static int sign_class(int c)
{
    int n = 0;
    while ((n + 1) * (n + 1) <= c)
        ++n;
    const int i = c - n * n;
    const int m = (i + 1) / 2;
    const int im = (i > 0 && (i & 1) == 0) ? 1 : 0;
    return (((n + m) & 1) << 2) | (im << 1) | ((m + im) & 1);
}

int canon_index(int ax, int ay, int az)
{
    int k = 0;
    for (int z = 0; z <= 3; ++z)
        for (int y = 0; y <= 3; ++y)
            for (int x = 0; x <= 3; ++x) {
                if (std::max(x, std::max(y, z)) < 2)
                    continue;
                if (x == ax && y == ay && z == az)
                    return k;
                ++k;
            }
    return -1;
}

// The 316 M2L offsets (2 <= |d|_inf <= 3), and per child-parity class the
// 189 valid ones, entries (dx, dy, dz, operator).  Forward: a target box of
// class c sees sources at T + d for d_a in [-2 - c_a, 3 - c_a]; the operator
// field is, with `canonical`, the index of |d| among the 56 stored operators
// plus kReflShift times the reflection bits (bit a set where d_a < 0), else
// the offset id.  Transposed: a source box S of class c
// feeds targets T = S - d whose class admits d; the operator field is the
// offset id (0..315, the transposed operators are stored per offset).
void offsets_tables(std::vector<int> &all, std::vector<int32_t> &fwd, std::vector<int32_t> &rev, bool canonical)
{
    all.clear();
    for (int dz = -3; dz <= 3; ++dz)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dx = -3; dx <= 3; ++dx)
                if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) >= 2) {
                    all.push_back(dx);
                    all.push_back(dy);
                    all.push_back(dz);
                }
    fwd.assign(8 * kClassOffsets * 4, 0);
    rev.assign(8 * kClassOffsets * 4, 0);
    for (int c = 0; c < 8; ++c) {
        int nf = 0, nr = 0;
        for (int id = 0; id < (int)all.size() / 3; ++id) {
            const int *d = &all[3 * id];
            bool okf = true, okr = true;
            for (int a = 0; a < 3; ++a) {
                const int pc = (c >> a) & 1;           // target class bit (forward)
                if (d[a] < -2 - pc || d[a] > 3 - pc)
                    okf = false;
                const int pt = ((c >> a) - d[a]) & 1;  // class bit of T = S - d
                if (d[a] < -2 - pt || d[a] > 3 - pt)
                    okr = false;
            }
            if (okf) {
                int32_t *e = &fwd[(c * kClassOffsets + nf++) * 4];
                const int refl = (d[0] < 0 ? 1 : 0) | (d[1] < 0 ? 2 : 0) | (d[2] < 0 ? 4 : 0);
                e[0] = d[0], e[1] = d[1], e[2] = d[2];
                e[3] = canonical ? canon_index(std::abs(d[0]), std::abs(d[1]), std::abs(d[2])) + kReflShift * refl
                                 : id;
            }
            if (okr) {
                int32_t *e = &rev[(c * kClassOffsets + nr++) * 4];
                e[0] = d[0], e[1] = d[1], e[2] = d[2], e[3] = id;
            }
        }
    }
}

// Position of value e (of E per lane) of a lane in a set of MFMA operand
// fragments stored group-major, [E / G][64 lanes][G] with G = 16 bytes /
// element size: the layout the kernels read with one 16-byte vector load per
// group (a contiguous kilobyte per wave).
static inline size_t frag_pos(int lane, int e, int G)
{
    return ((size_t)(e / G) * 64 + lane) * G + e % G;
}

// M2L operand layout (all row blocks per lane): k step ks (0 .. PS/4 - 1)
// and instruction sub-row kr = lane / 16 contract coefficient 4 ks + kr (the
// M2L's B operand is regathered in the same order; this puts the padding
// coefficients in whole trailing k steps).  The fragments of four
// consecutive k steps (ks = 4 q + u) and all row blocks form one set of
// E = 4 RB values per lane, value e = u * RB + rb:
// set q, value (lane, e)  =  m[16 rb + lane % 16][4 (4 q + u) + lane / 16],
// except that with tail4 the last row block (at most four rows of
// coefficients) takes row 16 rb + lane % 4, the A operand of the 4x4x1
// instructions that replace its 16x16x4 ones.
void swizzle_panel(const double *m, int PS, int G, double *dst, bool tail4)
{
    const int RB = PS / 16;
    for (int q = 0; q < RB; ++q)
        for (int lane = 0; lane < 64; ++lane)
            for (int u = 0; u < 4; ++u)
                for (int rb = 0; rb < RB; ++rb) {
                    const int row = 16 * rb + (tail4 && rb == RB - 1 ? (lane & 3) : (lane & 15));
                    const int col = 4 * (4 * q + u) + (lane >> 4);
                    dst[(size_t)q * 64 * 4 * RB + frag_pos(lane, u * RB + rb, G)] = m[(size_t)row * PS + col];
                }
}

// Row-blocked layout (M2M, L2L), contraction order kr * PS/4 + ks (their B
// operand is read straight from the expansions), one set of four values per
// (q, rb):
// set (q, rb), value (lane, u)  =  m[16 rb + lane % 16][(lane / 16) * PS/4 + 4 q + u].
void swizzle_rows(const double *m, int PS, int G, double *dst)
{
    const int RB = PS / 16, KP = PS / 4;
    for (int q = 0; q < RB; ++q)
        for (int rb = 0; rb < RB; ++rb)
            for (int lane = 0; lane < 64; ++lane)
                for (int u = 0; u < 4; ++u) {
                    const int row = 16 * rb + (lane & 15);
                    const int col = (lane >> 4) * KP + 4 * q + u;
                    dst[((size_t)q * RB + rb) * 256 + frag_pos(lane, u, G)] = m[(size_t)row * PS + col];
                }
}

template <class T>
grav_status upload(Plan *p, T **dst, const std::vector<T> &src)
{
    GRAV_CHECK(dalloc(p, dst, src.size(), true));
    if (!src.empty())
        GRAV_HIP(hipMemcpyAsync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, p->bs));
    GRAV_HIP(hipStreamSynchronize(p->bs));
    return GRAV_OK;
}

grav_status build_operators(Plan *p)
{
    const int P = p->P, PS = p->PS, RB = PS / 16;
    const int b3 = p->b * p->b * p->b;
    std::vector<double> pm((size_t)b3 * PS);
    p2m_lattice(P, p->b, p->q, 1.0, PS, pm.data());
    GRAV_CHECK(upload(p, &p->d_pm, pm));
    {
        // the same map as FP64 MFMA A fragments: rows = coefficients, the
        // contraction runs over the leaf's cells, k step kv and sub-row kr
        // taking cell 4 kv + kr; [kv][rb][lane] = pm[4 kv + lane/16][16 rb + lane%16]
        const int KV = (b3 + 3) / 4;
        std::vector<double> psw((size_t)KV * RB * 64, 0.0);
        for (int kv = 0; kv < KV; ++kv)
            for (int rb = 0; rb < RB; ++rb)
                for (int lane = 0; lane < 64; ++lane) {
                    const int v = 4 * kv + lane / 16;
                    if (v < b3)
                        psw[((size_t)kv * RB + rb) * 64 + lane] = pm[(size_t)v * PS + 16 * rb + lane % 16];
                }
        GRAV_CHECK(upload(p, &p->d_pm_sw, psw));
        // the adjoint's P2M^T: rows = the leaf's cells (RBT blocks of 16),
        // contraction over the coefficients in the order 16 (ks/4) +
        // 4 (lane/16) + ks%4, so that a chunk of four k steps takes 16
        // consecutive coefficients of a column, four per sub-row (one
        // 128-byte line per column and chunk in FP64);
        // [ks][rbt][lane] = pm[16 rbt + lane%16][16 (ks/4) + 4 (lane/16) + ks%4]
        const int RBT = (b3 + 15) / 16, K4 = PS / 4;
        std::vector<double> pmt((size_t)K4 * RBT * 64, 0.0);
        for (int ks = 0; ks < K4; ++ks)
            for (int rb = 0; rb < RBT; ++rb)
                for (int lane = 0; lane < 64; ++lane) {
                    const int v = 16 * rb + lane % 16;
                    if (v < b3)
                        pmt[((size_t)ks * RBT + rb) * 64 + lane] =
                            pm[(size_t)v * PS + 16 * (ks / 4) + 4 * (lane / 16) + ks % 4];
                }
        GRAV_CHECK(upload(p, &p->d_pmt_sw, pmt));
    }
    if (p->L < 2)
        return GRAV_OK;

    // M2M / L2L row-major, [octant][out][in], for the adjoint: its thread
    // for input coefficient j reads column j, so a wave's loads at one row
    // are consecutive
    std::vector<double> m((size_t)PS * PS), m2m(8 * (size_t)PS * PS), l2l(8 * (size_t)PS * PS);
    for (int c = 0; c < 8; ++c) {
        const double delta[3] = {((c & 1) - 0.5) * 0.5, (((c >> 1) & 1) - 0.5) * 0.5,
                                 (((c >> 2) & 1) - 0.5) * 0.5};
        m2m_matrix(P, delta, PS, m.data());
        std::copy(m.begin(), m.end(), m2m.begin() + (size_t)c * PS * PS);
        l2l_matrix(P, delta, PS, m.data());
        std::copy(m.begin(), m.end(), l2l.begin() + (size_t)c * PS * PS);
    }
    GRAV_CHECK(upload(p, &p->d_m2m, m2m));
    GRAV_CHECK(upload(p, &p->d_l2l, l2l));
    {
        // the same matrices as MFMA A operands (rows = output coefficient),
        // contraction order kr * PS/4 + ks.  L2L: one set of four k steps per
        // (q, row block) (a workgroup takes one row block).  M2M: one fragment
        // per (k step, row block), [octant][ks][rb][lane] = m[16 rb + lane%16][
        // (lane/16) PS/4 + ks] (a wave takes all row blocks).
        const size_t per8 = (size_t)PS * PS;
        const int K4 = PS / 4;
        std::vector<double> msw(8 * per8), lsw(8 * per8);
        for (int c = 0; c < 8; ++c) {
            const double delta[3] = {((c & 1) - 0.5) * 0.5, (((c >> 1) & 1) - 0.5) * 0.5,
                                     (((c >> 2) & 1) - 0.5) * 0.5};
            m2m_matrix(P, delta, PS, m.data());
            for (int ks = 0; ks < K4; ++ks)
                for (int rb = 0; rb < RB; ++rb)
                    for (int lane = 0; lane < 64; ++lane)
                        msw[per8 * c + ((size_t)ks * RB + rb) * 64 + lane] =
                            m[(size_t)(16 * rb + lane % 16) * PS + (lane / 16) * K4 + ks];
            l2l_matrix(P, delta, PS, m.data());
            swizzle_rows(m.data(), PS, 2, lsw.data() + per8 * c);
        }
        GRAV_CHECK(upload(p, &p->d_m2m_sw, msw));
        GRAV_CHECK(upload(p, &p->d_l2l_sw, lsw));
        // the adjoint's M2M^T and L2L^T in the M2M fragment layout: row =
        // output coefficient of the transpose (a column of the matrix),
        // contraction index (lane/16) PS/4 + ks (a row of the matrix)
        std::vector<double> mtsw(8 * per8), ltsw(8 * per8);
        for (int c = 0; c < 8; ++c)
            for (int ks = 0; ks < K4; ++ks)
                for (int rb = 0; rb < RB; ++rb)
                    for (int lane = 0; lane < 64; ++lane) {
                        const size_t src = per8 * c + (size_t)((lane / 16) * K4 + ks) * PS + 16 * rb + lane % 16;
                        mtsw[per8 * c + ((size_t)ks * RB + rb) * 64 + lane] = m2m[src];
                        ltsw[per8 * c + ((size_t)ks * RB + rb) * 64 + lane] = l2l[src];
                    }
        GRAV_CHECK(upload(p, &p->d_m2mt_sw, mtsw));
        GRAV_CHECK(upload(p, &p->d_l2lt_sw, ltsw));
        // L2L in the same layout for the forward's LDS-tiled kernel
        std::vector<double> lmsw(8 * per8);
        for (int c = 0; c < 8; ++c)
            for (int ks = 0; ks < K4; ++ks)
                for (int rb = 0; rb < RB; ++rb)
                    for (int lane = 0; lane < 64; ++lane)
                        lmsw[per8 * c + ((size_t)ks * RB + rb) * 64 + lane] =
                            l2l[per8 * c + (size_t)(16 * rb + lane % 16) * PS + (lane / 16) * K4 + ks];
        GRAV_CHECK(upload(p, &p->d_l2l_msw, lmsw));
    }

    // M2L for all 316 offsets, swizzled for the MFMA A operand, and their transposes
    const bool canonical = p->d.precision != GRAV_FP64;
    std::vector<int> all;
    std::vector<int32_t> fwd, rev;
    offsets_tables(all, fwd, rev, canonical);
    const size_t perp = (size_t)RB * 64 * 4 * RB;  // forward M2L: PS/4 k steps, grouped by four
    // FP32 plans whose last row block holds at most four coefficient rows
    // run it as 4x4 instructions: its A fragment repeats those rows
    const bool tail4 = p->d.precision != GRAV_FP64 && p->P2 % 16 != 0 && p->P2 % 16 <= 4;
    std::vector<double> k(perp * (canonical ? kCanonOffsets : kNumOffsets)), kt(k.size()), mt((size_t)PS * PS);
    // Reflection-orbit M2L (mixed plans whose sign classes hold at most 16
    // coefficients each): the coefficients of each class in natural order,
    // and the 56 canonical operators with rows and columns grouped by class
    // (class rb's rows, class q's columns: 16 x 16 blocks, one per (q, rb)),
    // as A fragments [ci][q][rb][lane][u] = K[row rb, lane%16][col q, 4 u +
    // lane/16]
    std::vector<int32_t> ccoef(8 * 16, -1);
    {
        int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        // (the kernel addresses a level's regathered expansions with 32-bit
        // byte offsets)
        bool fits = canonical && p->L >= 2 && p->P >= GRAV_M2L_ORB_MIN_P &&
                    (int64_t)p->n_me * p->B * 128 * 4 < (int64_t(1) << 32);
        for (int c = 0; c < p->P2; ++c) {
            const int s = sign_class(c);
            if (cnt[s] >= 16)
                fits = false;
            else
                ccoef[s * 16 + cnt[s]] = c;
            ++cnt[s];
        }
        p->m2l_orbit = fits;  // tentative: build_tiles keeps it where it pays
        p->m2l_npl = PS / 4;
    }
    std::vector<double> ko(p->m2l_orbit ? (size_t)kCanonOffsets * 8 * 8 * 256 : 0, 0.0), kot(ko.size(), 0.0);
    for (int id = 0; id < kNumOffsets; ++id) {
        // source = target + d  =>  target centre - source centre = -d
        const double dd[3] = {-(double)all[3 * id], -(double)all[3 * id + 1], -(double)all[3 * id + 2]};
        m2l_matrix(P, dd, PS, m.data());
        // the forward operators: all 316, or the 56 with non-negative
        // components; the adjoint's transposes in the same layout (the
        // reflections act on K_d^T as on K_d: K_d^T = S K_|d|^T S)
        const int ci = canonical ? canon_index(all[3 * id], all[3 * id + 1], all[3 * id + 2]) : id;
        if (ci >= 0) {
            swizzle_panel(m.data(), PS, p->d.precision == GRAV_FP64 ? 2 : 4, k.data() + perp * ci, tail4);
            for (int i = 0; i < PS; ++i)
                for (int j = 0; j < PS; ++j)
                    mt[(size_t)j * PS + i] = m[(size_t)i * PS + j];
            swizzle_panel(mt.data(), PS, p->d.precision == GRAV_FP64 ? 2 : 4, kt.data() + perp * ci, tail4);
            if (p->m2l_orbit)
                for (int q = 0; q < 8; ++q)
                    for (int rb = 0; rb < 8; ++rb)
                        for (int lane = 0; lane < 64; ++lane)
                            for (int u = 0; u < 4; ++u) {
                                const int row = ccoef[rb * 16 + (lane & 15)], col = ccoef[q * 16 + 4 * u + (lane >> 4)];
                                ko[((((size_t)ci * 8 + q) * 8 + rb) * 64 + lane) * 4 + u] =
                                    row >= 0 && col >= 0 ? m[(size_t)row * PS + col] : 0.0;
                                kot[((((size_t)ci * 8 + q) * 8 + rb) * 64 + lane) * 4 + u] =
                                    row >= 0 && col >= 0 ? m[(size_t)col * PS + row] : 0.0;
                            }
        }
    }
    if (p->m2l_orbit) {
        std::vector<float> ko32(ko.begin(), ko.end());
        GRAV_CHECK(upload(p, &p->d_k32o, ko32));
        std::vector<float> kot32(kot.begin(), kot.end());
        GRAV_CHECK(upload(p, &p->d_kt32o, kot32));
        GRAV_CHECK(upload(p, &p->d_ccoef, ccoef));
    }
    if (p->d.precision == GRAV_FP64) {
        GRAV_CHECK(upload(p, &p->d_k64, k));
        GRAV_CHECK(upload(p, &p->d_kt64, kt));
    } else {
        // the FP32 copies are exactly what both directions multiply by
        std::vector<float> k32(k.begin(), k.end());
        GRAV_CHECK(upload(p, &p->d_k32, k32));
        std::vector<float> kt32(kt.begin(), kt.end());
        GRAV_CHECK(upload(p, &p->d_kt32, kt32));
    }
    GRAV_CHECK(upload(p, &p->d_class_off, fwd));
    // the transposed M2L's offset table, keyed by the class of the source
    // box S: entry (-d, operator of K_d^T) for each d of the reverse list
    // (T = S - d), the operator field packed as in the forward table
    std::vector<int32_t> tco(rev.size());
    for (size_t e = 0; e < rev.size(); e += 4) {
        const int d[3] = {rev[e], rev[e + 1], rev[e + 2]};
        const int refl = (d[0] < 0 ? 1 : 0) | (d[1] < 0 ? 2 : 0) | (d[2] < 0 ? 4 : 0);
        tco[e] = -d[0];
        tco[e + 1] = -d[1];
        tco[e + 2] = -d[2];
        tco[e + 3] = canonical ? canon_index(std::abs(d[0]), std::abs(d[1]), std::abs(d[2])) + kReflShift * refl
                               : rev[e + 3];
    }
    GRAV_CHECK(upload(p, &p->d_tclass_off, tco));
    GRAV_CHECK(upload(p, &p->d_rclass_off, rev));
    return GRAV_OK;
}

// Stream-K partition of an M2L's work items (see build_tiles): item i
// belongs to unit item_unit[i], units in order.  A fixed number of one-wave
// workgroups, all resident at once, take equal contiguous shares of the
// items; a share is cut into segments {unit, first item, end item, 0} at
// unit boundaries (wgseg: CSR over workgroups), and per unit its segment
// slots are listed in workgroup order (tseg_start/tsegs: CSR over units).
struct StreamK {
    std::vector<int32_t> seg, wgseg, tseg_start, tsegs;
    int64_t P = 0, nseg = 0;
    int nset = 2;
};

// The regather's coefficient map (k_me_gather): value u of plane pl of a
// box's regathered expansion is coefficient kmap[4 pl + u] (-1: zero).  The
// orbit M2L reads chunk q = sign class q, sub-row kr, value u = position
// 4 u + kr of the class; the per-offset M2L reads coefficient 16 q + 4 u + kr.
static grav_status upload_gather_map(Plan *p)
{
    std::vector<int32_t> kmap;
    if (p->m2l_orbit) {
        p->m2l_npl = 32;
        int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        std::vector<int32_t> ccoef(8 * 16, -1);
        for (int c = 0; c < p->P2; ++c) {
            const int s = sign_class(c);
            if (cnt[s] < 16)
                ccoef[s * 16 + cnt[s]] = c;
            ++cnt[s];
        }
        kmap.resize(32 * 4);
        for (int q = 0; q < 8; ++q)
            for (int kr = 0; kr < 4; ++kr)
                for (int u = 0; u < 4; ++u)
                    kmap[(q * 4 + kr) * 4 + u] = ccoef[q * 16 + 4 * u + kr];
    } else {
        p->m2l_npl = p->PS / 4;
        kmap.resize((size_t)p->PS);
        for (int pl = 0; pl < p->PS / 4; ++pl)
            for (int u = 0; u < 4; ++u) {
                const int c = 16 * (pl / 4) + 4 * u + pl % 4;
                kmap[pl * 4 + u] = c < p->P2 ? c : -1;
            }
    }
    return upload(p, &p->d_kmap, kmap);
}

// 16-column blocks per wave of the per-offset M2L kernel (FP32: four on
// plans with many columns; FP64: two on plans with many columns)
static int m2l_blocks_per_wave(const Plan *p)
{
    const int64_t ncol = p->n_tbox * p->B;
    return p->d.precision == GRAV_FP64 ? (ncol >= GRAV_M2L_WIDE_COLUMNS64 ? GRAV_M2L_NC64_WIDE : GRAV_M2L_NC64)
                                       : (ncol >= GRAV_M2L_WIDE_COLUMNS ? GRAV_M2L_NC32_WIDE : GRAV_M2L_NC32);
}

static grav_status stream_k(const Plan *p, const std::vector<int32_t> &item_unit, int64_t nunit, int nc, StreamK &o,
                            bool orbit = false)
{
    const int64_t T = (int64_t)item_unit.size();
    // at least kMinItems items per workgroup: small plans get fewer
    // workgroups rather than one partial slot per item
    constexpr int64_t kMinItems = 8;
    constexpr int64_t kItemsOneSet = 32;  // items per resident wave above which one set pays
    // FP32: one operand register set (more resident waves) when every wave
    // gets a long run of items, two sets on small plans
    int resident = 0;
    o.nset = 2;
    if (p->d.precision != GRAV_FP64) {
        GRAV_CHECK(m2l_resident_workers(p, 1, nc, orbit, &resident));
        if (T >= kItemsOneSet * resident)
            o.nset = 1;
    }
    GRAV_CHECK(m2l_resident_workers(p, o.nset, nc, orbit, &resident));
    const int64_t P = T == 0 ? 0
                             : std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(GRAV_M2L_WAVES, resident),
                                                                      T / kMinItems));
    o.seg.clear();
    o.wgseg.assign(P + 1, 0);
    std::vector<int32_t> tseg_n(nunit + 1, 0);
    for (int64_t w = 0; w < P; ++w) {
        o.wgseg[w] = (int32_t)(o.seg.size() / 4);
        const int64_t ie = (w + 1) * T / P;
        for (int64_t i = w * T / P; i < ie;) {
            int64_t j = i;
            while (j < ie && item_unit[j] == item_unit[i])
                ++j;
            o.seg.insert(o.seg.end(), {item_unit[i], (int32_t)i, (int32_t)j, 0});
            ++tseg_n[item_unit[i] + 1];
            i = j;
        }
    }
    o.nseg = (int64_t)o.seg.size() / 4;
    o.wgseg[P] = (int32_t)o.nseg;
    o.tseg_start.assign(nunit + 1, 0);
    o.tsegs.assign(o.nseg, 0);
    std::vector<int32_t> fill(nunit, 0);
    for (int64_t u = 0; u < nunit; ++u)
        o.tseg_start[u + 1] = o.tseg_start[u] + tseg_n[u + 1];
    for (int64_t sgi = 0; sgi < o.nseg; ++sgi) {
        const int32_t u = o.seg[4 * sgi];
        o.tsegs[o.tseg_start[u] + fill[u]++] = (int32_t)sgi;
    }
    o.P = P;
    return GRAV_OK;
}

// The adjoint's transposed M2L on the forward kernel: ME_l[S] = sum over the
// reverse list of S's class of K_d^T LE_l[S - d] (the forward adds K_d
// ME[T + d] into LE[T] for exactly these pairs).  Per level, the columns
// are the source boxes of the column block, class-grouped as the forward
// groups its target boxes, 64 (box, model) columns per tile, units of
// 16 NC columns; the B operand is the adjoint LE regathered over the gather
// region; a work item is a (unit, offset) pair at which some column meets
// a target box.  Everything else (stream-K, slots, sums) is the forward's.
static grav_status build_m2l_transposed(Plan *p, const std::vector<std::vector<uint32_t>> &key,
                                        const std::vector<int32_t> &rev)
{
    const int L = p->L;
    const int64_t B = p->B;
    // the forward's kernel choice (the transposed M2L has the forward's box
    // pairs): the orbit kernel's column blocks, or the per-offset one's
    const int nc = p->m2l_orbit ? GRAV_M2L_ORB_NC : m2l_blocks_per_wave(p);
    // orbit kernel: per source class, canonical offset |d| and reflection
    // (sign bits of d, which give the operator S K_|d|^T S), the entry of the
    // reverse list or -1
    std::vector<int> rcanon(8 * kClassOffsets);
    std::vector<int32_t> orbtab(8 * kCanonOffsets * 8, -1);
    for (int c = 0; c < 8; ++c)
        for (int o = 0; o < kClassOffsets; ++o) {
            const int32_t *e = &rev[((size_t)c * kClassOffsets + o) * 4];
            const int ci = canon_index(std::abs(e[0]), std::abs(e[1]), std::abs(e[2]));
            const int r = (e[0] < 0 ? 1 : 0) | (e[1] < 0 ? 2 : 0) | (e[2] < 0 ? 4 : 0);
            rcanon[c * kClassOffsets + o] = ci;
            orbtab[((size_t)c * kCanonOffsets + ci) * 8 + r] = o;
        }
    std::vector<char> ohit(kCanonOffsets);
    const int ncw = 16 * nc, upt = 4 / nc;
    std::vector<uint32_t> skey((size_t)std::max<int64_t>(p->n_me, 1), 0);
    std::vector<int32_t> sorder((size_t)std::max<int64_t>(p->n_me, 1), 0);
    std::vector<GemmTile> tiles;
    std::vector<int32_t> item_unit, item_off, colmap;
    std::vector<int64_t> colbox;
    std::vector<char> hit(kClassOffsets);
    int64_t goff = 0;
    for (int l = 2; l <= L; ++l) {
        LevelInfo &lv = p->lev[l];
        // target boxes of the level within reach of the source block
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = lv.s0[a] - 3;
            hi[a] = lv.s0[a] + lv.ns[a] + 2;
        }
        int blo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, bhi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
        for (const uint32_t k : key[l]) {
            const int c[3] = {(int)compact3(k), (int)compact3(k >> 1), (int)compact3(k >> 2)};
            bool in = true;
            for (int a = 0; a < 3; ++a)
                in = in && c[a] >= lo[a] && c[a] <= hi[a];
            if (!in)
                continue;
            for (int a = 0; a < 3; ++a) {
                blo[a] = std::min(blo[a], c[a]);
                bhi[a] = std::max(bhi[a], c[a]);
            }
        }
        const bool any = blo[0] <= bhi[0];
        int64_t gn = 1;
        for (int a = 0; a < 3; ++a) {
            lv.gs0[a] = any ? blo[a] : 0;
            lv.gns[a] = any ? bhi[a] - blo[a] + 1 : 0;
            gn *= lv.gns[a];
        }
        lv.g_off = goff;
        goff += gn;
        std::vector<char> tb((size_t)gn, 0);
        for (const uint32_t k : key[l]) {
            const int c[3] = {(int)compact3(k) - lv.gs0[0], (int)compact3(k >> 1) - lv.gs0[1],
                              (int)compact3(k >> 2) - lv.gs0[2]};
            if (c[0] >= 0 && c[1] >= 0 && c[2] >= 0 && c[0] < lv.gns[0] && c[1] < lv.gns[1] && c[2] < lv.gns[2])
                tb[((size_t)c[2] * lv.gns[1] + c[1]) * lv.gns[0] + c[0]] = 1;
        }
        // column block: the source boxes within 3 of the gather region (the
        // whole source block at level 2, so that every level-2 expansion is
        // written; below, M2M^T sets the boxes outside the column block)
        for (int a = 0; a < 3; ++a) {
            int c0 = lv.s0[a], c1 = lv.s0[a] + lv.ns[a] - 1;
            if (l > 2) {
                c0 = std::max(c0, any ? lv.gs0[a] - 3 : c1 + 1);
                c1 = std::min(c1, any ? lv.gs0[a] + lv.gns[a] + 2 : c0 - 1);
            }
            lv.cs0[a] = c0;
            lv.cns[a] = std::max(0, c1 - c0 + 1);
        }
        for (int64_t j = 0; j < lv.n_src; ++j) {
            const int x = lv.s0[0] + (int)(j % lv.ns[0]), y = lv.s0[1] + (int)((j / lv.ns[0]) % lv.ns[1]),
                      z = lv.s0[2] + (int)(j / ((int64_t)lv.ns[0] * lv.ns[1]));
            skey[(size_t)(lv.me_off + j)] = morton3((uint32_t)x, (uint32_t)y, (uint32_t)z);
        }
        DevLev cb{};
        for (int a = 0; a < 3; ++a) {
            cb.s0[a] = lv.cs0[a];
            cb.ns[a] = lv.cns[a];
        }
        int64_t pos = 0;
        for (int cls = 0; cls < 8; ++cls) {
            int first[3], cnt[3];
            lv.col_class_start[cls] = pos;
            class_split(cb, cls, first, cnt);
            for (int iz = 0; iz < cnt[2]; ++iz)
                for (int iy = 0; iy < cnt[1]; ++iy)
                    for (int ix = 0; ix < cnt[0]; ++ix) {
                        const int x = first[0] + 2 * ix, y = first[1] + 2 * iy, z = first[2] + 2 * iz;
                        sorder[(size_t)(lv.me_off + pos++)] =
                            (int32_t)(((int64_t)(z - lv.s0[2]) * lv.ns[1] + (y - lv.s0[1])) * lv.ns[0] + (x - lv.s0[0]));
                    }
        }
        lv.col_class_start[8] = pos;
        for (int cls = 0; cls < 8; ++cls) {
            const int64_t ncols = (lv.col_class_start[cls + 1] - lv.col_class_start[cls]) * B;
            for (int64_t c0 = 0; c0 < ncols; c0 += kTileCols) {
                GemmTile t{};
                t.level = l;
                t.cls = cls;
                t.col0 = c0;
                t.ncol = (int32_t)std::min<int64_t>(kTileCols, ncols - c0);
                const int64_t u0 = (int64_t)tiles.size() * upt;
                tiles.push_back(t);
                for (int hq = 0; hq < upt; ++hq) {
                    std::fill(hit.begin(), hit.end(), 0);
                    for (int cl = hq * ncw; cl < std::min(t.ncol, (hq + 1) * ncw); ++cl) {
                        const int64_t col = t.col0 + cl;
                        const int32_t j = sorder[(size_t)(lv.me_off + lv.col_class_start[cls] + col / B)];
                        colmap.push_back((int32_t)((u0 + hq) * 64 + cl - hq * ncw));
                        colbox.push_back((lv.me_off + j) * B + col % B);
                        const int c[3] = {lv.s0[0] + (int)(j % lv.ns[0]), lv.s0[1] + (int)((j / lv.ns[0]) % lv.ns[1]),
                                          lv.s0[2] + (int)(j / ((int64_t)lv.ns[0] * lv.ns[1]))};
                        for (int o = 0; o < kClassOffsets && any; ++o) {
                            const int32_t *e = &rev[((size_t)cls * kClassOffsets + o) * 4];
                            int g[3];
                            bool in = true;
                            for (int a = 0; a < 3; ++a) {
                                g[a] = c[a] - e[a] - lv.gs0[a];  // T = S - d
                                in = in && g[a] >= 0 && g[a] < lv.gns[a];
                            }
                            if (in && tb[((size_t)g[2] * lv.gns[1] + g[1]) * lv.gns[0] + g[0]])
                                hit[o] = 1;
                        }
                    }
                    if (p->m2l_orbit) {
                        std::fill(ohit.begin(), ohit.end(), 0);
                        for (int o = 0; o < kClassOffsets; ++o)
                            ohit[rcanon[cls * kClassOffsets + o]] |= hit[o];
                        for (int ci = 0; ci < kCanonOffsets; ++ci)
                            if (ohit[ci]) {
                                item_unit.push_back((int32_t)(u0 + hq));
                                item_off.push_back(ci);
                            }
                    } else {
                        for (int o = 0; o < kClassOffsets; ++o)
                            if (hit[o]) {
                                item_unit.push_back((int32_t)(u0 + hq));
                                item_off.push_back(o);
                            }
                    }
                }
            }
        }
    }
    const int64_t nunit = (int64_t)tiles.size() * upt;
    StreamK sk;
    GRAV_CHECK(stream_k(p, item_unit, nunit, nc, sk, p->m2l_orbit));
    if (p->m2l_orbit)
        GRAV_CHECK(upload(p, &p->d_orbtab_t, orbtab));
    if (item_off.empty())
        item_off.push_back(0);
    GRAV_CHECK(upload(p, &p->d_m2lt_tiles, tiles.empty() ? std::vector<GemmTile>(1) : tiles));
    GRAV_CHECK(upload(p, &p->d_m2lt_items, item_off));
    GRAV_CHECK(upload(p, &p->d_m2lt_segs, sk.seg.empty() ? std::vector<int32_t>(4, 0) : sk.seg));
    GRAV_CHECK(upload(p, &p->d_m2lt_wgseg, sk.wgseg));
    GRAV_CHECK(upload(p, &p->d_m2lt_tseg_start, sk.tseg_start));
    GRAV_CHECK(upload(p, &p->d_m2lt_tsegs, sk.tsegs.empty() ? std::vector<int32_t>(1, 0) : sk.tsegs));
    GRAV_CHECK(upload(p, &p->d_m2lt_colmap, colmap.empty() ? std::vector<int32_t>(1, 0) : colmap));
    GRAV_CHECK(upload(p, &p->d_m2lt_colbox, colbox.empty() ? std::vector<int64_t>(1, 0) : colbox));
    GRAV_CHECK(upload(p, &p->d_skey, skey));
    GRAV_CHECK(upload(p, &p->d_sorder, sorder));
    p->m2lt_wgs = (int32_t)sk.P;
    p->m2lt_nset = sk.nset;
    p->m2lt_nc = nc;
    p->m2lt_ncw = ncw;
    p->m2lt_nseg = sk.nseg;
    p->m2lt_ncols = (int64_t)colmap.size();
    p->m2lt_nunit = nunit;
    p->m2lt_items = (int64_t)item_unit.size();
    p->n_leg = goff;
    return GRAV_OK;
}

// Tile lists of the M2L stage: 64 columns (4 waves x 16) per tile, per
// level and child-parity class; the columns are target boxes (x models).
grav_status build_tiles(Plan *p)
{
    std::vector<GemmTile> all;
    const int L = p->L;
    const int64_t B = p->B;
    auto add_tile = [&](int kind, int level, int cls, int64_t c0, int64_t ncol) {
        TileRange &r = p->tiles[kind][0];
        if (r.n == 0)
            r.off = (int64_t)all.size();
        TileRange &rl = p->tiles[kind][level];
        if (rl.n == 0)
            rl.off = r.n;  // level range, in this kind's own numbering
        GemmTile t{};
        t.level = level;
        t.cls = cls;
        t.col0 = c0;
        t.ncol = (int32_t)ncol;
        all.push_back(t);
        ++r.n;
        ++rl.n;
    };
    auto add = [&](int kind, int level, int cls, int64_t ncols) {
        for (int64_t c0 = 0; c0 < ncols; c0 += kTileCols)
            add_tile(kind, level, cls, c0, std::min<int64_t>(kTileCols, ncols - c0));
    };
    for (int k = 0; k < TK_COUNT; ++k)
        for (int l = 0; l <= kMaxLevels; ++l)
            p->tiles[k][l] = TileRange{};
    if (L >= 2) {
        for (int l = 2; l <= L; ++l) {
            for (int c = 0; c < 8; ++c)
                add(TK_M2L, l, c, (p->lev[l].class_start[c + 1] - p->lev[l].class_start[c]) * B);
        }
    }
    // Tiles are not split over workgroups (S = 1): the forward M2L runs on
    // the stream-K schedule below.
    std::vector<GemmTile> split;
    for (int k = 0; k < TK_COUNT; ++k) {
        TileRange &r = p->tiles[k][0];
        const int S = 1;
        p->split[k] = S;
        const int64_t off = (int64_t)split.size();
        for (int64_t i = 0; i < r.n; ++i)
            for (int q = 0; q < S; ++q) {
                GemmTile t = all[r.off + i];
                t.pad = q;
                split.push_back(t);
            }
        r.off = off;
        r.n *= S;
    }
    // Stream-K schedule of the forward M2L.  A unit is the 16 NC columns of
    // one wave of a tile; work items are the (unit, offset) pairs in which
    // some column of the unit has a source box (the others cost nothing), so
    // every item costs the same.  A fixed number of one-wave workgroups, all
    // resident at once, take equal contiguous shares of the item list; a
    // share is cut into segments at unit boundaries, and each segment writes
    // the partial LE of its unit's columns to a slot of its own.  k_m2l_sum
    // then adds, per unit, its segments' slots in order (deterministic).  The
    // work is balanced to one item per wave and there are at most
    // (units + workgroups) partial slots.
    p->m2l_wgs = 0;
    p->m2l_nseg = 0;
    {
        const TileRange &r = p->tiles[TK_M2L][0];  // S = 1: one entry per tile
        if (r.n > 0) {
            std::vector<int> alloffs;
            std::vector<int32_t> fwd, rev;
            offsets_tables(alloffs, fwd, rev, false);  // only the offsets themselves are used here
            std::vector<std::vector<uint32_t>> key(L + 1);
            std::vector<std::vector<int32_t>> ord(L + 1);
            for (int l = 2; l <= L; ++l) {
                const int64_t n = p->lev[l].n_tgt;
                key[l].resize(n);
                ord[l].resize(n);
                if (n > 0) {
                    GRAV_HIP(hipMemcpyAsync(key[l].data(), p->d_tkey + p->tbox_off[l], 4 * n, hipMemcpyDeviceToHost,
                                            p->bs));
                    GRAV_HIP(hipMemcpyAsync(ord[l].data(), p->d_torder + p->tbox_off[l], 4 * n,
                                            hipMemcpyDeviceToHost, p->bs));
                }
            }
            GRAV_HIP(hipStreamSynchronize(p->bs));
            // per level, the box range whose expansions the M2L can read: the
            // target boxes' bounding box widened by the largest offset (3)
            for (int l = 2; l <= L; ++l) {
                LevelInfo &lv = p->lev[l];
                int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
                for (const uint32_t k : key[l]) {
                    const int c[3] = {(int)compact3(k), (int)compact3(k >> 1), (int)compact3(k >> 2)};
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = std::min(lo[a], c[a]);
                        hi[a] = std::max(hi[a], c[a]);
                    }
                }
                for (int a = 0; a < 3; ++a) {
                    lv.need_lo[a] = key[l].empty() ? 0 : lo[a] - 3;
                    lv.need_hi[a] = key[l].empty() ? -1 : hi[a] + 3;
                }
            }
            // The orbit M2L costs one operator per (column, orbit with a
            // source), the per-offset one an operator per (column, offset with
            // a source): keep the orbit kernel only where orbits hold enough
            // offsets with sources on average (target boxes near the edge of
            // the source block, such as surface stations, see few).
            if (p->m2l_orbit) {
                int64_t n_off = 0, n_orb = 0;
                for (int l = 2; l <= L; ++l) {
                    const LevelInfo &lv = p->lev[l];
                    for (int c = 0; c < 8; ++c)
                        for (int64_t j = lv.class_start[c]; j < lv.class_start[c + 1]; ++j) {
                            const uint32_t k = key[l][ord[l][j]];
                            const int x[3] = {(int)compact3(k), (int)compact3(k >> 1), (int)compact3(k >> 2)};
                            uint64_t orbs = 0;
                            for (int o = 0; o < kClassOffsets; ++o) {
                                const int32_t *e = &fwd[((size_t)c * kClassOffsets + o) * 4];
                                bool in = true;
                                for (int a = 0; a < 3; ++a) {
                                    const int s = x[a] + e[a] - lv.s0[a];
                                    in = in && s >= 0 && s < lv.ns[a];
                                }
                                if (in) {
                                    ++n_off;
                                    orbs |= 1ull << canon_index(std::abs(e[0]), std::abs(e[1]), std::abs(e[2]));
                                }
                            }
                            n_orb += __builtin_popcountll(orbs);
                        }
                }
                // the transposed M2L's gather regions (at most 3 boxes past the
                // source block on each side) also take 32-bit byte offsets
                double leg_bytes = 0.0;
                for (int l = 2; l <= L; ++l)
                    leg_bytes += 512.0 * (double)B * (p->lev[l].ns[0] + 6) * (p->lev[l].ns[1] + 6) *
                                 (p->lev[l].ns[2] + 6);
                if ((double)n_off < GRAV_M2L_ORB_MIN_RATIO * (double)n_orb || leg_bytes >= 4294967296.0) {
                    p->m2l_orbit = false;
                    (void)hipFree(p->d_k32o);
                    (void)hipFree(p->d_kt32o);
                    p->d_k32o = nullptr;
                    p->d_kt32o = nullptr;
                    p->bytes_resident -= 2 * sizeof(float) * (size_t)kCanonOffsets * 8 * 8 * 256;
                }
            }
            GRAV_CHECK(upload_gather_map(p));
            // a unit is the columns of one wave: 16 NC columns of a tile
            // (FP32: four blocks on plans with many columns)
            const int nc = p->m2l_orbit ? GRAV_M2L_ORB_NC : m2l_blocks_per_wave(p);
            const int ncw = 16 * nc, upt = 4 / nc;
            const int64_t nunit = r.n * upt;
            std::vector<int32_t> item_tile, item_off;  // item_tile holds the unit
            std::vector<int32_t> colmap((size_t)p->n_tbox * B, -1);
            std::vector<char> hit(kClassOffsets);
            // reflection-orbit M2L: per class, the canonical offset of each
            // of its offsets, and per (class, canonical offset, reflection)
            // the class offset index or -1
            std::vector<int> ocanon(8 * kClassOffsets);
            std::vector<int32_t> orbtab(8 * kCanonOffsets * 8, -1);
            for (int c = 0; c < 8; ++c)
                for (int o = 0; o < kClassOffsets; ++o) {
                    const int32_t *e = &fwd[((size_t)c * kClassOffsets + o) * 4];
                    const int ci = canon_index(std::abs(e[0]), std::abs(e[1]), std::abs(e[2]));
                    const int s = (e[0] < 0 ? 1 : 0) | (e[1] < 0 ? 2 : 0) | (e[2] < 0 ? 4 : 0);
                    ocanon[c * kClassOffsets + o] = ci;
                    orbtab[((size_t)c * kCanonOffsets + ci) * 8 + s] = o;
                }
            std::vector<char> ohit(kCanonOffsets);
            for (int64_t u = 0; u < r.n; ++u) {
                const GemmTile &t = split[r.off + u];
                const LevelInfo &lv = p->lev[t.level];
                for (int hq = 0; hq < upt; ++hq) {
                    std::fill(hit.begin(), hit.end(), 0);
                    for (int cl = hq * ncw; cl < std::min(t.ncol, (hq + 1) * ncw); ++cl) {
                        const int64_t col = t.col0 + cl;
                        const int32_t box = ord[t.level][lv.class_start[t.cls] + col / B];
                        colmap[(size_t)((lv.tgt_off + box) * B + col % B)] =
                            (int32_t)((u * upt + hq) * 64 + cl - hq * ncw);
                        const uint32_t k = key[t.level][box];
                        const int c[3] = {(int)compact3(k), (int)compact3(k >> 1), (int)compact3(k >> 2)};
                        for (int o = 0; o < kClassOffsets; ++o) {
                            const int32_t *e = &fwd[((size_t)t.cls * kClassOffsets + o) * 4];
                            bool in = true;
                            for (int a = 0; a < 3; ++a) {
                                const int s = c[a] + e[a] - lv.s0[a];
                                in = in && s >= 0 && s < lv.ns[a];
                            }
                            hit[o] |= in;
                        }
                    }
                    if (p->m2l_orbit) {
                        std::fill(ohit.begin(), ohit.end(), 0);
                        for (int o = 0; o < kClassOffsets; ++o)
                            ohit[ocanon[t.cls * kClassOffsets + o]] |= hit[o];
                        for (int ci = 0; ci < kCanonOffsets; ++ci)
                            if (ohit[ci]) {
                                item_tile.push_back((int32_t)(u * upt + hq));
                                item_off.push_back(ci);
                            }
                    } else {
                        for (int o = 0; o < kClassOffsets; ++o)
                            if (hit[o]) {
                                item_tile.push_back((int32_t)(u * upt + hq));
                                item_off.push_back(o);
                            }
                    }
                }
            }
            StreamK sk;
            GRAV_CHECK(stream_k(p, item_tile, nunit, nc, sk, p->m2l_orbit));
            if (item_off.empty())
                item_off.push_back(0);
            GRAV_CHECK(upload(p, &p->d_m2l_items, item_off));
            if (p->m2l_orbit)
                GRAV_CHECK(upload(p, &p->d_orbtab, orbtab));
            GRAV_CHECK(upload(p, &p->d_m2l_segs, sk.seg.empty() ? std::vector<int32_t>(4, 0) : sk.seg));
            GRAV_CHECK(upload(p, &p->d_m2l_wgseg, sk.wgseg));
            GRAV_CHECK(upload(p, &p->d_m2l_tseg_start, sk.tseg_start));
            GRAV_CHECK(upload(p, &p->d_m2l_tsegs, sk.tsegs.empty() ? std::vector<int32_t>(1, 0) : sk.tsegs));
            GRAV_CHECK(upload(p, &p->d_m2l_colmap, colmap));
            p->m2l_nset = sk.nset;
            p->m2l_wgs = (int32_t)sk.P;
            p->m2l_nseg = sk.nseg;
            p->m2l_items = (int64_t)item_tile.size();
            p->m2l_ncw = ncw;
            p->m2l_nc = nc;
            p->m2l_nunit = nunit;
            GRAV_CHECK(build_m2l_transposed(p, key, rev));
        }
    }
    if (!split.empty())
        GRAV_CHECK(upload(p, &p->d_tiles, split));
    return GRAV_OK;
}

__global__ void k_fill_tmap(const uint32_t *bkeys, int64_t n, int s0x, int s0y, int s0z, int mx,
                            int my, int mz, int32_t *tmap)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t k = bkeys[i];
    const int x = (int)compact3(k) - s0x + 3, y = (int)compact3(k >> 1) - s0y + 3,
              z = (int)compact3(k >> 2) - s0z + 3;
    if (x >= 0 && y >= 0 && z >= 0 && x < mx && y < my && z < mz)
        tmap[((int64_t)z * my + y) * mx + x] = (int32_t)i;
}

__global__ void k_fill_tchild(const int32_t *cparent, int64_t nc, int64_t np, int32_t *tchild)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nc)
        return;
    if (i == nc) {
        tchild[np] = (int32_t)nc;
        return;
    }
    if (i == 0 || cparent[i] != cparent[i - 1])
        tchild[cparent[i]] = (int32_t)i;
}

// Lookup tables of the adjoint: target-box maps over each level's source
// block plus a halo of 3 boxes (M2L transpose, near field transpose) and the
// first-child table of each level (L2L transpose).
// Source leaves of the leaf level with some user point in their 27
// neighbour leaves (target map entry with pend > start), appended in any
// order: the cells of the other leaves get no term from the transposed
// point near field.
__global__ void k_point_leaves(const int32_t *tmap, int64_t n_tmap, int64_t tmap_off, int nsx, int nsy, int nsz,
                               const int64_t *leaf_start, const int64_t *pend,
                               int64_t n_leaf, int32_t *list, unsigned long long *count)
{
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= (int64_t)nsx * nsy * nsz)
        return;
    const int lx = (int)(sl % nsx), ly = (int)((sl / nsx) % nsy), lz = (int)(sl / ((int64_t)nsx * nsy));
    const int mxl = nsx + 6, myl = nsy + 6, mzl = nsz + 6;
    bool active = false;
    for (int nb = 0; nb < 27 && !active; ++nb) {
        // neighbour position in the target map (source block + halo 3)
        const int mx = lx + nb % 3 - 1 + 3, my = ly + (nb / 3) % 3 - 1 + 3, mz = lz + nb / 9 - 1 + 3;
        if (mx < 0 || my < 0 || mz < 0 || mx >= mxl || my >= myl || mz >= mzl)
            continue;
        const int64_t mi = tmap_off + ((int64_t)mz * myl + my) * mxl + mx;
        if (mi >= n_tmap)
            continue;
        const int64_t tl = tmap[mi];
        if (tl >= 0 && tl < n_leaf && pend[tl] > max(leaf_start[tl], (int64_t)0))
            active = true;
    }
    if (active)
        list[atomicAdd(count, 1ull)] = (int32_t)sl;
}

// Target leaves holding user points (pend > start), appended in any order.
__global__ void k_user_leaves(const int64_t *leaf_start, const int64_t *pend, int64_t n_leaf, int32_t *list,
                              unsigned long long *count)
{
    const int64_t tl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tl < n_leaf && pend[tl] > max(leaf_start[tl], (int64_t)0))
        list[atomicAdd(count, 1ull)] = (int32_t)tl;
}

grav_status build_adjoint_maps(Plan *p)
{
    const int L = p->L;
    const int lo = L >= 2 ? 2 : L;
    p->n_tmap = 0;
    for (int l = lo; l <= L; ++l) {
        const LevelInfo &lv = p->lev[l];
        p->lev[l].tmap_off = p->n_tmap;
        p->n_tmap += (int64_t)(lv.ns[0] + 6) * (lv.ns[1] + 6) * (lv.ns[2] + 6);
    }
    GRAV_CHECK(dalloc(p, &p->d_tmap, (size_t)p->n_tmap, true));
    GRAV_HIP(hipMemsetAsync(p->d_tmap, 0xff, sizeof(int32_t) * p->n_tmap, p->bs));
    for (int l = lo; l <= L; ++l) {
        const LevelInfo &lv = p->lev[l];
        const int64_t n = lv.n_tgt;
        if (n == 0)
            continue;
        hipLaunchKernelGGL(k_fill_tmap, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, p->bs,
                           (const uint32_t *)(p->d_tkey + p->tbox_off[l]), n, lv.s0[0], lv.s0[1],
                           lv.s0[2], lv.ns[0] + 6, lv.ns[1] + 6, lv.ns[2] + 6,
                           p->d_tmap + lv.tmap_off);
        GRAV_HIP(hipGetLastError());
    }
    p->n_tchild = 0;
    for (int l = 2; l < L; ++l) {
        p->lev[l].tchild_off = p->n_tchild;
        p->n_tchild += p->lev[l].n_tgt + 1;
    }
    if (p->n_tchild > 0) {
        GRAV_CHECK(dalloc(p, &p->d_tchild, (size_t)p->n_tchild, true));
        for (int l = 2; l < L; ++l) {
            const int64_t nc = p->lev[l + 1].n_tgt;
            hipLaunchKernelGGL(k_fill_tchild, dim3((unsigned)ceil_div(nc + 1, 256)), dim3(256), 0, p->bs,
                               (const int32_t *)(p->d_tparent + p->tbox_off[l + 1]), nc,
                               p->lev[l].n_tgt, p->d_tchild + p->lev[l].tchild_off);
            GRAV_HIP(hipGetLastError());
        }
    }
    {
        // the leaf level's source leaves near user points, and the target
        // leaves holding user points
        const LevelInfo &lv = p->lev[L];
        GRAV_CHECK(dalloc(p, &p->d_pt_leaves, (size_t)std::max<int64_t>(lv.n_src, 1), true));
        GRAV_CHECK(dalloc(p, &p->d_user_leaves, (size_t)std::max<int64_t>(p->n_leaf, 1), true));
        unsigned long long *cnt = nullptr;
        GRAV_HIP(hipMalloc(&cnt, 2 * sizeof(unsigned long long)));
        grav_status st = GRAV_OK;
        unsigned long long n[2] = {0, 0};
        if (hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned long long), p->bs) != hipSuccess)
            st = GRAV_EDEVICE;
        if (st == GRAV_OK && lv.n_src > 0) {
            hipLaunchKernelGGL(k_point_leaves, dim3((unsigned)ceil_div(lv.n_src, 256)), dim3(256), 0, p->bs,
                               (const int32_t *)p->d_tmap, p->n_tmap, lv.tmap_off, lv.ns[0], lv.ns[1], lv.ns[2],
                               (const int64_t *)p->d_leaf_start,
                               (const int64_t *)p->d_leaf_pend, p->n_leaf, p->d_pt_leaves, cnt);
            if (hipGetLastError() != hipSuccess)
                st = GRAV_EDEVICE;
        }
        if (st == GRAV_OK && p->n_leaf > 0) {
            hipLaunchKernelGGL(k_user_leaves, dim3((unsigned)ceil_div(p->n_leaf, 256)), dim3(256), 0, p->bs,
                               (const int64_t *)p->d_leaf_start, (const int64_t *)p->d_leaf_pend, p->n_leaf,
                               p->d_user_leaves, cnt + 1);
            if (hipGetLastError() != hipSuccess)
                st = GRAV_EDEVICE;
        }
        if (st == GRAV_OK && (hipMemcpyAsync(n, cnt, sizeof(n), hipMemcpyDeviceToHost, p->bs) != hipSuccess ||
                              hipStreamSynchronize(p->bs) != hipSuccess))
            st = GRAV_EDEVICE;
        (void)hipFree(cnt);
        GRAV_CHECK(st);
        p->n_pt_leaves = (int64_t)n[0];
        p->n_user_leaves = (int64_t)n[1];
    }
    GRAV_HIP(hipStreamSynchronize(p->bs));
    return GRAV_OK;
}

// Near field of voxel-centre targets as 27 dense lattice matrices (leaf
// edges b <= 4), the slot of every voxel centre in sorted order, and the end
// of the user points of every leaf (the direct near-field kernel visits only
// those).
grav_status build_near_lattice(Plan *p, hipStream_t s)
{
    const int64_t M = p->M, npts = p->d.n_points;
    // the lattice near field pairs lattice targets with lattice sources
    p->lat_near = p->d.voxel_centres && p->b <= kMaxLatticeLeaf && p->n_spts == 0;
    GRAV_CHECK(dalloc(p, &p->d_leaf_pend, p->n_leaf, true));
    hipLaunchKernelGGL(k_leaf_point_end, dim3((unsigned)ceil_div(p->n_leaf, 256)), dim3(256), 0, s,
                       (const uint32_t *)p->d_perm, (const int64_t *)p->d_leaf_start, p->n_leaf,
                       p->lat_near ? npts : M, p->d_leaf_pend);
    GRAV_HIP(hipGetLastError());
    if (!p->lat_near) {
        GRAV_HIP(hipStreamSynchronize(s));
        return GRAV_OK;
    }
    const int64_t ncell = (int64_t)p->d.nx * p->d.ny * p->d.nz;
    GRAV_CHECK(dalloc(p, &p->d_cell_slot, ncell, true));
    hipLaunchKernelGGL(k_cell_slot, dim3((unsigned)ceil_div(M, 256)), dim3(256), 0, s,
                       (const uint32_t *)p->d_perm, M, npts, p->d_cell_slot);
    GRAV_HIP(hipGetLastError());

    const int b = p->b, b3 = b * b * b;
    // rows: (output component, target) pairs for the requested components
    // only, component-major: each component owns RBc = b^3/16 (rounded up)
    // blocks of 16 targets, RBn = C RBc blocks in all; the contraction runs
    // over Qn chunks of four k steps, k step ks and instruction sub-row kr
    // taking cell kr * 4 Qn + ks (cells past b^3 are zero in both operands)
    const int C = p->d.components, RBc = (int)ceil_div(b3, 16);
    const int RBn = C * RBc, Qn = (int)ceil_div(ceil_div(b3, 4), 4);
    const int KP = 16 * Qn;
    p->lat_RB = RBn;
    p->lat_Q = Qn;
    const bool f64 = p->d.precision == GRAV_FP64;
    std::vector<double> dense((size_t)27 * 4 * b3 * b3);
    near_lattice(b, p->q, f64 ? 1e-20 : 1e-10, dense.data());
    // Row r of block rb is target 16 (rb % RBc) + r of output component
    // rb / RBc; the lattice matrices hold (phi, gx, gy, gz), of which
    // components 1 and 3 take the trailing one or three.  The FP32
    // instruction returns rows 4 (lane / 16) + k of a block and the FP64 one
    // rows lane / 16 + 4 k, so a lane's accumulator holds four targets of one
    // component.  The far field (FP64) is added element by element to the
    // near field's accumulator, so next to an FP32 near field its rows take
    // the FP32 order (swap: row 4 i + j holds target 4 j + i).  Layout
    // [nb][q][rb][lane][u], ks = 4 q + u.
    auto row_target = [C, RBc](int row, int rb, bool swap, int &t, int &comp) {
        t = 16 * (rb % RBc) + (swap ? 4 * (row % 4) + row / 4 : row);
        comp = rb / RBc + 4 - C;
    };
    std::vector<double> sw((size_t)27 * Qn * RBn * 64 * 4, 0.0);
    for (int nb = 0; nb < 27; ++nb)
        for (int q = 0; q < Qn; ++q)
            for (int rb = 0; rb < RBn; ++rb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int u = 0; u < 4; ++u) {
                        int t, comp;
                        row_target(lane & 15, rb, false, t, comp);
                        const int cell = (lane >> 4) * 4 * Qn + 4 * q + u;
                        double v = 0.0;
                        if (t < b3 && cell < b3)
                            v = dense[((size_t)nb * 4 * b3 + 4 * t + comp) * b3 + cell];
                        sw[(((size_t)nb * Qn + q) * RBn + rb) * 256 + frag_pos(lane, u, f64 ? 2 : 4)] = v;
                    }
    {
        // leaf blocks of the densities, padded by one leaf per side; the
        // padding and the rows past b^3 stay zero
        const LevelInfo &lv = p->lev[p->L];
        const size_t n = (size_t)(lv.ns[0] + 2) * (lv.ns[1] + 2) * (lv.ns[2] + 2) * p->B * KP;
        GRAV_CHECK(dalloc(p, &p->d_rho_blk, n, false));
        GRAV_HIP(hipMemsetAsync(p->d_rho_blk, 0, sizeof(double) * n, p->bs));
        GRAV_HIP(hipStreamSynchronize(p->bs));
        // per near chunk i = (neighbour nb, four k steps q): element offsets
        // of its density fragment (from a column's block at nb = (0, 0, 0))
        // and of its operator fragments; the kernel reads them with scalar
        // loads instead of recomputing them
        const int64_t px = lv.ns[0] + 2, py = lv.ns[1] + 2, nplB = px * py * (lv.ns[2] + 2) * p->B;
        std::vector<int64_t> tab((size_t)27 * Qn * 2);
        for (int nb = 0; nb < 27; ++nb)
            for (int q = 0; q < Qn; ++q) {
                const int64_t nboff = ((int64_t)(nb / 9) * py + (nb / 3) % 3) * px + nb % 3;
                tab[((size_t)nb * Qn + q) * 2 + 0] = ((int64_t)q * 4 * nplB + nboff * p->B) * 4;
                tab[((size_t)nb * Qn + q) * 2 + 1] = ((int64_t)nb * Qn + q) * RBn * 256;
            }
        GRAV_CHECK(upload(p, &p->d_lat_tab, tab));
    }
    if (f64) {
        GRAV_CHECK(upload(p, &p->d_tn64, sw));
    } else {
        std::vector<float> sw32(sw.begin(), sw.end());
        GRAV_CHECK(upload(p, &p->d_tn32, sw32));
    }
    // the adjoint's transposes: rows = the cells of the source leaf (RBt
    // blocks of 16), contraction over (target t, component) of the target
    // leaf (near^T: the C output components; L2P^T: chunk q and k step u
    // taking t = (lane/16) TQ + q, component u); [nb][q][rb][lane][u]
    // group-major sets
    const int TQ = (int)ceil_div(b3, 4), RBt = (int)ceil_div(b3, 16);
    p->lat_TQ = TQ;
    {
        // the weights of the cell centres in leaf blocks (padded by one leaf
        // per side, 4 TQ x 4 values per leaf and model, in the near field's
        // element type); the padding and the slots past b^3 stay zero
        const LevelInfo &lv = p->lev[p->L];
        const size_t n = (size_t)(lv.ns[0] + 2) * (lv.ns[1] + 2) * (lv.ns[2] + 2) * p->B * 16 * TQ;
        const size_t nd = f64 ? n : (n + 1) / 2;  // in doubles
        GRAV_CHECK(dalloc(p, &p->d_w_blk, nd, false));
        GRAV_HIP(hipMemsetAsync(p->d_w_blk, 0, sizeof(double) * nd, p->bs));
        GRAV_HIP(hipStreamSynchronize(p->bs));
    }
    {
        // contraction over the C b^3 (centre, output component) pairs of the
        // target leaf: value e = C t + c in chunk q, sub-row kr, k step u
        // with e = 4 KQ kr + 4 q + u (the weight blocks' order)
        const int KQ = (int)ceil_div((int64_t)C * b3, 16);
        std::vector<double> swt((size_t)27 * KQ * RBt * 256, 0.0);
        for (int nb = 0; nb < 27; ++nb)
            for (int q = 0; q < KQ; ++q)
                for (int rb = 0; rb < RBt; ++rb)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int u = 0; u < 4; ++u) {
                            const int e = 4 * KQ * (lane >> 4) + 4 * q + u, cell = 16 * rb + (lane & 15);
                            const int t = e / C, comp = e % C + 4 - C;
                            const double v =
                                t < b3 && cell < b3 ? dense[((size_t)nb * 4 * b3 + 4 * t + comp) * b3 + cell] : 0.0;
                            swt[(((size_t)nb * KQ + q) * RBt + rb) * 256 + frag_pos(lane, u, f64 ? 2 : 4)] = v;
                        }
        if (f64) {
            GRAV_CHECK(upload(p, &p->d_tnt64, swt));
        } else {
            std::vector<float> swt32(swt.begin(), swt.end());
            GRAV_CHECK(upload(p, &p->d_tnt32, swt32));
        }
    }
    if (p->L >= 2) {
        // Far field at the cell centres from the leaf's local expansion, with
        // the scaling of the combine folded in (phi / w, -grad phi / w^2), as
        // FP64 MFMA A fragments over the expansion's PS/4 k steps (same
        // contraction order as the M2L: coefficient kr * PS/4 + ks).
        const int PS = p->PS, QL = PS / 16;
        std::vector<double> e(PS, 0.0), full((size_t)4 * b3 * PS, 0.0);
        const double inv_w = 1.0 / b;
        for (int t = 0; t < b3; ++t) {
            const double u[3] = {((t % b) + 0.5 - 0.5 * b) * inv_w, (((t / b) % b) + 0.5 - 0.5 * b) * inv_w,
                                 ((t / (b * b)) + 0.5 - 0.5 * b) * inv_w};
            for (int c = 0; c < p->P2; ++c) {
                e[c] = 1.0;
                double o[4];
                l2p_eval(p->P, e.data(), u[0], u[1], u[2], o);
                e[c] = 0.0;
                full[(size_t)(4 * t + 0) * PS + c] = o[0] * inv_w;
                for (int a = 0; a < 3; ++a)
                    full[(size_t)(4 * t + 1 + a) * PS + c] = -o[1 + a] * inv_w * inv_w;
            }
        }
        std::vector<double> lsw((size_t)QL * RBn * 64 * 4, 0.0);
        for (int q = 0; q < QL; ++q)
            for (int rb = 0; rb < RBn; ++rb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int u = 0; u < 4; ++u) {
                        int t, comp;
                        row_target(lane & 15, rb, !f64, t, comp);
                        const int c = (lane >> 4) * (PS / 4) + 4 * q + u;
                        lsw[((size_t)q * RBn + rb) * 256 + frag_pos(lane, u, 2)] =
                            t < b3 ? full[(size_t)(4 * t + comp) * PS + c] : 0.0;
                    }
        GRAV_CHECK(upload(p, &p->d_tl2p, lsw));
        // its transpose for the adjoint: rows = coefficients (QL blocks),
        // contraction over (t, component) as the transposed near field
        std::vector<double> lst((size_t)TQ * QL * 256, 0.0);
        for (int q = 0; q < TQ; ++q)
            for (int rb = 0; rb < QL; ++rb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int u = 0; u < 4; ++u) {
                        const int t = (lane >> 4) * TQ + q, c = 16 * rb + (lane & 15);
                        lst[((size_t)q * QL + rb) * 256 + frag_pos(lane, u, 2)] =
                            t < b3 ? full[(size_t)(4 * t + u) * PS + c] : 0.0;
                    }
        GRAV_CHECK(upload(p, &p->d_tl2pt, lst));
    }
    GRAV_HIP(hipStreamSynchronize(s));
    return GRAV_OK;
}

grav_status count_work(Plan *p)
{
    unsigned long long *acc = nullptr;
    GRAV_HIP(hipMalloc(&acc, 2 * sizeof(unsigned long long)));
    grav_status st = GRAV_OK;
    do {
        if (hipMemsetAsync(acc, 0, 2 * sizeof(unsigned long long), p->bs) != hipSuccess) {
            st = GRAV_EDEVICE;
            break;
        }
        CountArgs a{};
        for (int ax = 0; ax < 3; ++ax) {
            a.shift[ax] = p->shift[ax];
        }
        a.n[0] = p->d.nx;
        a.n[1] = p->d.ny;
        a.n[2] = p->d.nz;
        a.b = p->b;
        a.nq3 = p->nq3;
        if (p->L >= 2 && p->d_class_off)
            for (int l = 2; l <= p->L; ++l) {
                const int64_t n = p->lev[l].n_tgt;
                if (n == 0)
                    continue;
                for (int ax = 0; ax < 3; ++ax) {
                    a.s0[ax] = p->lev[l].s0[ax];
                    a.ns[ax] = p->lev[l].ns[ax];
                }
                hipLaunchKernelGGL(k_count_m2l, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, p->bs,
                                   (const uint32_t *)(p->d_tkey + p->tbox_off[l]), n, a,
                                   (const int32_t *)p->d_class_off, acc);
            }
        if (p->n_leaf > 0) {
            for (int ax = 0; ax < 3; ++ax) {
                a.s0[ax] = p->lev[p->L].s0[ax];
                a.ns[ax] = p->lev[p->L].ns[ax];
            }
            if (p->n_spts > 0)
                hipLaunchKernelGGL(k_count_p2p_src, dim3((unsigned)ceil_div(p->n_leaf, 256)), dim3(256), 0, p->bs,
                                   (const uint32_t *)(p->d_tkey + p->tbox_off[p->L]),
                                   (const int64_t *)p->d_leaf_start, p->n_leaf, a, (const int64_t *)p->d_sstart,
                                   acc + 1);
            else
                hipLaunchKernelGGL(k_count_p2p, dim3((unsigned)ceil_div(p->n_leaf, 256)), dim3(256), 0, p->bs,
                                   (const uint32_t *)(p->d_tkey + p->tbox_off[p->L]),
                                   (const int64_t *)p->d_leaf_start, p->n_leaf, a, acc + 1);
        }
        unsigned long long h[2] = {0, 0};
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, p->bs) != hipSuccess ||
            hipStreamSynchronize(p->bs) != hipSuccess) {
            st = GRAV_EDEVICE;
            break;
        }
        p->m2l_pairs = (int64_t)h[0];
        p->p2p_pairs = (int64_t)h[1];
    } while (0);
    (void)hipFree(acc);
    return st;
}

// Explicit sources: the dense index of each source's leaf in the leaf
// level's source block (the block starts at the mesh origin, so a source at
// lattice position u lies in leaf floor(u / b)), the sort key.
__global__ void k_source_keys(const double *src, int64_t n, double ox, double oy, double oz, double inv_h, int b,
                              int nsx, int nsy, int nsz, uint32_t *keys, uint32_t *vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double o[3] = {ox, oy, oz};
    const int ns[3] = {nsx, nsy, nsz};
    int c[3];
    for (int a = 0; a < 3; ++a) {
        const double u = (src[3 * i + a] - o[a]) * inv_h;
        c[a] = min(max((int)floor(u / b), 0), ns[a] - 1);
    }
    keys[i] = (uint32_t)(((int64_t)c[2] * nsy + c[1]) * nsx + c[0]);
    vals[i] = (uint32_t)i;
}

// Sorted sources: lattice-frame positions and the mass per unit input value.
__global__ void k_gather_sources(const double *src, const double *vol, int64_t n, double ox, double oy, double oz,
                                 double inv_h, const uint32_t *perm, double *pos, double *w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t u = perm[i];
    const double o[3] = {ox, oy, oz};
    for (int a = 0; a < 3; ++a)
        pos[3 * i + a] = (src[3 * u + a] - o[a]) * inv_h;
    const double ih3 = inv_h * inv_h * inv_h;
    w[i] = (vol ? vol[u] : 1.0) * ih3;
}

// CSR of the sorted sources over the leaves: sorted source i starts every
// leaf in (key[i-1], key[i]]; the last one also ends the leaves after it.
__global__ void k_source_leaf_start(const uint32_t *keys, int64_t n, int64_t nleaf, int64_t *start)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n)
        return;
    const int64_t lo = i == 0 ? 0 : (int64_t)keys[i - 1] + 1;
    const int64_t hi = i == n ? nleaf : (int64_t)keys[i];
    for (int64_t l = lo; l <= hi && l <= nleaf; ++l)
        start[l] = i;
}

// Explicit sources: sorted by leaf with the device radix sort, positions and
// masses gathered, the per-leaf CSR built.
grav_status build_sources(Plan *p, const grav_plan_desc *desc, hipStream_t s)
{
    const int64_t n = p->n_spts;
    const LevelInfo &lv = p->lev[p->L];
    const int64_t nleaf = lv.n_src;
    int bits = 1;
    while ((int64_t(1) << bits) < nleaf)
        ++bits;
    double *src = nullptr, *vol = nullptr;
    uint32_t *keys = nullptr, *vals = nullptr, *ktmp = nullptr, *vtmp = nullptr, *scr = nullptr;
    const size_t scr_words = radix_scratch_words(n);
    grav_status st = GRAV_OK;
    auto cleanup = [&]() {
        void *bufs[] = {src, vol, keys, vals, ktmp, vtmp, scr};
        for (void *b : bufs)
            if (b)
                (void)hipFree(b);
    };
    if (hipMalloc(&src, sizeof(double) * 3 * n) != hipSuccess ||
        (desc->source_volumes && hipMalloc(&vol, sizeof(double) * n) != hipSuccess) ||
        hipMalloc(&keys, 4 * n) != hipSuccess || hipMalloc(&vals, 4 * n) != hipSuccess ||
        hipMalloc(&ktmp, 4 * n) != hipSuccess || hipMalloc(&vtmp, 4 * n) != hipSuccess ||
        hipMalloc(&scr, 4 * std::max<size_t>(scr_words, 1)) != hipSuccess) {
        cleanup();
        return GRAV_ENOMEM;
    }
    do {
        if ((st = dalloc(p, &p->d_spos, 3 * n, true)) != GRAV_OK || (st = dalloc(p, &p->d_sw, n, true)) != GRAV_OK ||
            (st = dalloc(p, &p->d_sperm, n, true)) != GRAV_OK ||
            (st = dalloc(p, &p->d_sstart, nleaf + 1, true)) != GRAV_OK)
            break;
        if (hipMemcpyAsync(src, desc->sources, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s) != hipSuccess ||
            (vol && hipMemcpyAsync(vol, desc->source_volumes, sizeof(double) * n, hipMemcpyHostToDevice, s) !=
                        hipSuccess)) {
            st = GRAV_EDEVICE;
            break;
        }
        const dim3 g((unsigned)ceil_div(n, 256)), g1((unsigned)ceil_div(n + 1, 256));
        const double inv_h = 1.0 / desc->h;
        hipLaunchKernelGGL(k_source_keys, g, dim3(256), 0, s, (const double *)src, n, desc->origin[0],
                           desc->origin[1], desc->origin[2], inv_h, p->b, lv.ns[0], lv.ns[1], lv.ns[2], keys, vals);
        if (hipGetLastError() != hipSuccess || radix_sort_pairs(keys, vals, ktmp, vtmp, n, bits, scr, s) != GRAV_OK) {
            st = GRAV_EDEVICE;
            break;
        }
        hipLaunchKernelGGL(k_gather_sources, g, dim3(256), 0, s, (const double *)src, (const double *)vol, n,
                           desc->origin[0], desc->origin[1], desc->origin[2], inv_h, (const uint32_t *)vals,
                           p->d_spos, p->d_sw);
        hipLaunchKernelGGL(k_source_leaf_start, g1, dim3(256), 0, s, (const uint32_t *)keys, n, nleaf, p->d_sstart);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(p->d_sperm, vals, 4 * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = GRAV_EDEVICE;
            break;
        }
    } while (0);
    cleanup();
    return st;
}

grav_status build_tree(Plan *p, hipStream_t s)
{
    const grav_plan_desc &d = p->d;
    const int64_t M = p->M;
    const int T = 256;
    // temporaries (freed at the end)
    uint32_t *keys = nullptr, *vals = nullptr, *ktmp = nullptr, *vtmp = nullptr;
    uint32_t *flags = nullptr, *scan = nullptr, *scr = nullptr, *ccount = nullptr;
    const int64_t nmax = std::max<int64_t>(M, 1);
    const size_t scr_words = std::max(radix_scratch_words(nmax), scan_tmp_words(nmax));
    grav_status st = GRAV_OK;
    auto fail = [&](grav_status e) {
        st = e;
        return e;
    };
    auto cleanup = [&]() {
        uint32_t *bufs[] = {keys, vals, ktmp, vtmp, flags, scan, scr, ccount};
        for (auto *b : bufs)
            if (b)
                (void)hipFree(b);
    };
    if (hipMalloc(&keys, 4 * nmax) != hipSuccess || hipMalloc(&vals, 4 * nmax) != hipSuccess ||
        hipMalloc(&ktmp, 4 * nmax) != hipSuccess || hipMalloc(&vtmp, 4 * nmax) != hipSuccess ||
        hipMalloc(&flags, 4 * nmax) != hipSuccess || hipMalloc(&scan, 4 * nmax) != hipSuccess ||
        hipMalloc(&scr, 4 * scr_words) != hipSuccess || hipMalloc(&ccount, 4 * 8) != hipSuccess) {
        cleanup();
        return GRAV_ENOMEM;
    }

    KeyArgs ka{};
    ka.pts = p->d_points;
    ka.npts = d.n_points;
    ka.M = M;
    ka.nx = d.nx;
    ka.ny = d.ny;
    for (int a = 0; a < 3; ++a) {
        ka.org[a] = d.origin[a];
        ka.shift_lat[a] = (double)p->shift[a] * p->b;
    }
    ka.inv_h = 1.0 / d.h;
    ka.inv_b = 1.0 / p->b;
    ka.kmax = (1 << p->L) - 1;
    ka.L = p->L;

    do {
        if (dalloc(p, &p->d_perm, M, true) || dalloc(p, &p->d_tpos, 3 * M, true) ||
            dalloc(p, &p->d_tleaf, M, true)) {
            fail(GRAV_ENOMEM);
            break;
        }
        const unsigned gM = (unsigned)ceil_div(M, T);
        hipLaunchKernelGGL(k_target_keys, dim3(gM), dim3(T), 0, s, ka, keys, vals);
        if (hipGetLastError() != hipSuccess) {
            fail(GRAV_EDEVICE);
            break;
        }
        if (radix_sort_pairs(keys, vals, ktmp, vtmp, M, 3 * p->L, scr, s) != GRAV_OK) {
            fail(GRAV_EDEVICE);
            break;
        }
        if (hipMemcpyAsync(p->d_perm, vals, 4 * M, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            fail(GRAV_EDEVICE);
            break;
        }
        hipLaunchKernelGGL(k_gather_targets, dim3(gM), dim3(T), 0, s, ka,
                           (const uint32_t *)p->d_perm, p->d_tpos);
        // leaf level
        hipLaunchKernelGGL(k_head_flags, dim3(gM), dim3(T), 0, s, (const uint32_t *)keys, M, 0,
                           flags);
        if (scan_exclusive_u32(flags, scan, M, scr, s) != GRAV_OK) {
            fail(GRAV_EDEVICE);
            break;
        }
        uint32_t last[2] = {0, 0};
        if (hipMemcpyAsync(&last[0], scan + (M - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&last[1], flags + (M - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            fail(GRAV_EDEVICE);
            break;
        }
        p->n_leaf = (int64_t)last[0] + last[1];

        // Per-level target box counts: leaf level from the scan, parents by
        // repeated compaction.  Box keys of all levels go into one array.
        const int L = p->L;
        const int lo = L >= 2 ? 2 : L;
        // first pass: compute counts (needs the compaction of each level)
        std::vector<int64_t> cnt(L + 1, 0);
        cnt[L] = p->n_leaf;
        // allocate the per-level arrays with an upper bound n_leaf per level
        int64_t total = 0;
        for (int l = lo; l <= L; ++l)
            total += p->n_leaf;
        uint32_t *bk = nullptr;
        int32_t *bp = nullptr;
        if (hipMalloc(&bk, 4 * std::max<int64_t>(total, 1)) != hipSuccess ||
            hipMalloc(&bp, 4 * std::max<int64_t>(total, 1)) != hipSuccess) {
            if (bk)
                (void)hipFree(bk);
            fail(GRAV_ENOMEM);
            break;
        }
        // level L at slot 0 of the bound layout
        std::vector<int64_t> off_bound(L + 1, 0);
        {
            int64_t o = 0;
            for (int l = L; l >= lo; --l) {
                off_bound[l] = o;
                o += p->n_leaf;
            }
        }
        if (dalloc(p, &p->d_leaf_start, p->n_leaf + 1, true)) {
            (void)hipFree(bk);
            (void)hipFree(bp);
            fail(GRAV_ENOMEM);
            break;
        }
        hipLaunchKernelGGL(k_leaf_build, dim3(gM), dim3(T), 0, s, (const uint32_t *)keys,
                           (const uint32_t *)flags, (const uint32_t *)scan, M, p->d_tleaf,
                           p->d_leaf_start, bk + off_bound[L]);
        hipLaunchKernelGGL(k_fill_last, dim3(1), dim3(1), 0, s, p->d_leaf_start, p->n_leaf, M);
        bool ok = true;
        for (int l = L - 1; l >= lo; --l) {
            const int64_t nc = cnt[l + 1];
            const unsigned g = (unsigned)ceil_div(nc, T);
            hipLaunchKernelGGL(k_head_flags, dim3(g), dim3(T), 0, s,
                               (const uint32_t *)(bk + off_bound[l + 1]), nc, 3, flags);
            if (scan_exclusive_u32(flags, scan, nc, scr, s) != GRAV_OK) {
                ok = false;
                break;
            }
            hipLaunchKernelGGL(k_parent_build, dim3(g), dim3(T), 0, s,
                               (const uint32_t *)(bk + off_bound[l + 1]), (const uint32_t *)flags,
                               (const uint32_t *)scan, nc, bp + off_bound[l + 1],
                               bk + off_bound[l]);
            if (hipMemcpyAsync(&last[0], scan + (nc - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(&last[1], flags + (nc - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                ok = false;
                break;
            }
            cnt[l] = (int64_t)last[0] + last[1];
        }
        if (!ok) {
            (void)hipFree(bk);
            (void)hipFree(bp);
            fail(GRAV_EDEVICE);
            break;
        }
        // compact layout: levels lo..L in increasing order
        int64_t o = 0;
        for (int l = 0; l <= kMaxLevels; ++l)
            p->tbox_off[l] = 0;
        for (int l = lo; l <= L; ++l) {
            p->tbox_off[l] = o;
            p->lev[l].n_tgt = cnt[l];
            o += cnt[l];
        }
        const int64_t nall = std::max<int64_t>(o, 1);
        if (dalloc(p, &p->d_tkey, nall, true) || dalloc(p, &p->d_tparent, nall, true) ||
            dalloc(p, &p->d_torder, nall, true)) {
            (void)hipFree(bk);
            (void)hipFree(bp);
            fail(GRAV_ENOMEM);
            break;
        }
        for (int l = lo; l <= L; ++l) {
            if (hipMemcpyAsync(p->d_tkey + p->tbox_off[l], bk + off_bound[l], 4 * cnt[l],
                               hipMemcpyDeviceToDevice, s) != hipSuccess)
                ok = false;
            if (l > lo) {
                if (hipMemcpyAsync(p->d_tparent + p->tbox_off[l], bp + off_bound[l], 4 * cnt[l],
                                   hipMemcpyDeviceToDevice, s) != hipSuccess)
                    ok = false;
            } else {
                if (hipMemsetAsync(p->d_tparent + p->tbox_off[l], 0xff, 4 * cnt[l], s) != hipSuccess)
                    ok = false;
            }
        }
        if (hipStreamSynchronize(s) != hipSuccess)
            ok = false;
        (void)hipFree(bk);
        (void)hipFree(bp);
        if (!ok) {
            fail(GRAV_EDEVICE);
            break;
        }
        p->n_tbox = 0;
        if (L >= 2)
            for (int l = 2; l <= L; ++l) {
                p->lev[l].tgt_off = p->n_tbox;
                p->n_tbox += cnt[l];
            }

        // class grouping per level (levels >= 2): lexicographic, then stable on (class, signature)
        for (int l = 2; l <= L && ok; ++l) {
            const int64_t n = cnt[l];
            const unsigned g = (unsigned)ceil_div(n, T);
            if (hipMemsetAsync(ccount, 0, 32, s) != hipSuccess) {
                ok = false;
                break;
            }
            const LevelInfo &lv = p->lev[l];
            const uint32_t *bk_l = (const uint32_t *)(p->d_tkey + p->tbox_off[l]);
            hipLaunchKernelGGL(k_lex_keys, dim3(g), dim3(T), 0, s, bk_l, n, l, keys, vals);
            if (radix_sort_pairs(keys, vals, ktmp, vtmp, n, 3 * l, scr, s) != GRAV_OK) {
                ok = false;
                break;
            }
            hipLaunchKernelGGL(k_class_keys, dim3(g), dim3(T), 0, s, bk_l, (const uint32_t *)vals, n,
                               make_int3(lv.s0[0], lv.s0[1], lv.s0[2]), make_int3(lv.ns[0], lv.ns[1], lv.ns[2]),
                               keys, ccount);
            if (radix_sort_pairs(keys, vals, ktmp, vtmp, n, 15, scr, s) != GRAV_OK) {
                ok = false;
                break;
            }
            if (hipMemcpyAsync(p->d_torder + p->tbox_off[l], vals, 4 * n, hipMemcpyDeviceToDevice,
                               s) != hipSuccess) {
                ok = false;
                break;
            }
            uint32_t cc[8];
            if (hipMemcpyAsync(cc, ccount, 32, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                ok = false;
                break;
            }
            int64_t acc = 0;
            for (int c = 0; c < 8; ++c) {
                p->lev[l].class_start[c] = acc;
                acc += cc[c];
            }
            p->lev[l].class_start[8] = acc;
        }
        if (!ok) {
            fail(GRAV_EDEVICE);
            break;
        }
    } while (0);
    cleanup();
    return st;
}

}  // namespace

}  // namespace grav

using namespace grav;

extern "C" void grav_desc_init(grav_plan_desc *d)
{
    if (!d)
        return;
    std::memset(d, 0, sizeof(*d));
    d->nx = d->ny = d->nz = 1;
    d->h = 1.0;
    d->quad_order = 1;
    d->components = 3;
    d->p = 8;
    d->leaf_size = 64;
    d->precision = GRAV_FP64;
    d->batch = 1;
    d->G = 1.0;
    d->device = 0;
}

extern "C" grav_status grav_plan(const grav_plan_desc *desc, grav_plan_t *out)
{
    if (!out)
        return GRAV_EINVAL;
    *out = nullptr;
    GRAV_CHECK(validate(desc));
    Plan *p = new (std::nothrow) Plan();
    if (!p)
        return GRAV_ENOMEM;
    p->d = *desc;
    p->d.points = nullptr;
    p->d.sources = nullptr;
    p->d.source_volumes = nullptr;
    p->n_spts = desc->n_sources;
    p->device = desc->device;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(desc->device) != hipSuccess) {
        delete p;
        return GRAV_EDEVICE;
    }
    grav_status st = GRAV_OK;
    hipStream_t s = nullptr;
    do {
        p->P = desc->p;
        p->P2 = p->P * p->P;
        p->PS = (int)ceil_div(p->P2, 16) * 16;
        p->KS = (int)ceil_div(p->P2, 4);
        p->q = desc->quad_order;
        p->nq3 = p->q * p->q * p->q;
        p->B = desc->batch;
        p->C = desc->components;
        int b = (int)std::floor(std::cbrt((double)desc->leaf_size / p->nq3) + 1e-9);
        p->b = std::min(kMaxLeafCells, std::max(1, b));
        const int n3[3] = {desc->nx, desc->ny, desc->nz};
        const int64_t ncell = (int64_t)desc->nx * desc->ny * desc->nz;
        p->M = desc->n_points + (desc->voxel_centres ? ncell : 0);
        // bounding box of evaluation points in the lattice frame (cell
        // centres span [1/2, n - 1/2]; the mesh itself is covered separately)
        double tmin[3] = {0.5, 0.5, 0.5};
        double tmax[3] = {n3[0] - 0.5, n3[1] - 0.5, n3[2] - 0.5};
        if (!desc->voxel_centres && desc->n_points > 0)
            for (int a = 0; a < 3; ++a) {
                tmin[a] = (desc->points[a] - desc->origin[a]) / desc->h;
                tmax[a] = tmin[a];
            }
        for (int64_t i = 0; i < desc->n_points; ++i)
            for (int a = 0; a < 3; ++a) {
                const double u = (desc->points[3 * i + a] - desc->origin[a]) / desc->h;
                if (!std::isfinite(u)) {
                    st = GRAV_EINVAL;
                    break;
                }
                tmin[a] = std::min(tmin[a], u);
                tmax[a] = std::max(tmax[a], u);
            }
        if (st != GRAV_OK)
            break;
        int64_t need = 1;
        for (int a = 0; a < 3; ++a) {
            const double sh = std::ceil(-tmin[a] / p->b - 1e-12);
            p->shift[a] = (int)std::max(0.0, sh);
            const int64_t src_hi = ceil_div(n3[a], p->b) + p->shift[a];
            const int64_t tgt_hi = (int64_t)std::floor((tmax[a] + (double)p->shift[a] * p->b) / p->b) + 1;
            need = std::max(need, std::max(src_hi, tgt_hi));
        }
        int L = 0;
        while ((int64_t(1) << L) < need)
            ++L;
        if (L > kMaxLevels) {
            st = GRAV_EUNSUPPORTED;
            break;
        }
        p->L = L;
        p->wl = (double)p->b;
        for (int a = 0; a < 3; ++a)
            p->root0[a] = -(double)p->shift[a] * p->b;
        // source blocks per level
        for (int l = 0; l <= L; ++l) {
            LevelInfo &lv = p->lev[l];
            lv.l = l;
            lv.w = (double)p->b * (double)(int64_t(1) << (L - l));
            lv.n_src = 1;
            for (int a = 0; a < 3; ++a) {
                const int s0 = p->shift[a];
                const int s1 = p->shift[a] + (int)ceil_div(n3[a], p->b) - 1;
                lv.s0[a] = s0 >> (L - l);
                lv.ns[a] = (s1 >> (L - l)) - lv.s0[a] + 1;
                lv.n_src *= lv.ns[a];
            }
        }
        p->n_me = 0;
        if (L >= 2)
            for (int l = 2; l <= L; ++l) {
                p->lev[l].me_off = p->n_me;
                p->n_me += p->lev[l].n_src;
            }
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            st = GRAV_EDEVICE;
            break;
        }
        p->bs = s;
        if (desc->n_points > 0) {
            if ((st = dalloc(p, &p->d_points, 3 * desc->n_points, true)) != GRAV_OK)
                break;
            if (hipMemcpyAsync(p->d_points, desc->points, sizeof(double) * 3 * desc->n_points,
                               hipMemcpyHostToDevice, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = GRAV_EDEVICE;
                break;
            }
        }
        if (p->M > 0 && (st = build_tree(p, s)) != GRAV_OK)
            break;
        if (p->M > 0 && p->n_spts > 0 && (st = build_sources(p, desc, s)) != GRAV_OK)
            break;
        if (p->M > 0 && (st = build_near_lattice(p, s)) != GRAV_OK)
            break;
        if ((st = build_operators(p)) != GRAV_OK)
            break;
        if (p->M > 0 && (st = build_tiles(p)) != GRAV_OK)
            break;
        if (p->M > 0 && (st = build_adjoint_maps(p)) != GRAV_OK)
            break;
        if (p->M > 0 && (st = count_work(p)) != GRAV_OK)
            break;
        // workspace
        if ((st = dalloc(p, &p->d_me, (size_t)p->n_me * p->B * p->PS, false)) != GRAV_OK)
            break;
        if ((st = dalloc(p, &p->d_le, (size_t)p->n_tbox * p->B * p->PS, false)) != GRAV_OK)
            break;
        if (p->L >= 2 &&
            (st = dalloc(p, &p->d_meg, (size_t)p->n_me * p->B * std::max(p->PS, 4 * p->m2l_npl), false)) != GRAV_OK)
            break;
        if ((st = dalloc(p, &p->d_near, (size_t)p->M * p->B * 4, false)) != GRAV_OK)
            break;
        {
            // grav_direct: enough source chunks for ~2048 workgroups, partial
            // sums capped at 8 MB (the plan keeps them for its lifetime)
            const int64_t ncell = (int64_t)desc->nx * desc->ny * desc->nz;
            const int64_t tiles = std::max<int64_t>(1, ceil_div(p->M, 256));
            int64_t nch = std::min<int64_t>(std::max<int64_t>(1, ceil_div(2048, tiles)), ceil_div(ncell, 256));
            const int64_t per = std::max<int64_t>(1, p->M * p->B * 4 * 8);
            nch = std::max<int64_t>(1, std::min<int64_t>(nch, (8 << 20) / per));
            p->direct_chunks = (int)std::min<int64_t>(nch, 65535);
            if (p->direct_chunks > 1 &&
                (st = dalloc(p, &p->d_dpart, (size_t)p->direct_chunks * p->M * p->B * 4, false)) != GRAV_OK)
                break;
        }
        {
            // segment slots of the forward and the transposed M2L, and the
            // adjoint LE regathered for the latter
            const size_t part = (size_t)p->m2l_nseg * p->m2l_ncw * p->PS;
            if ((st = dalloc(p, &p->d_part, part, false)) != GRAV_OK)
                break;
            // the orbit M2L writes the coefficients only: the padding of its
            // slots stays zero from here on
            if (p->m2l_orbit && part > 0 &&
                (hipMemsetAsync(p->d_part, 0, part * sizeof(float), s) != hipSuccess ||
                 hipStreamSynchronize(s) != hipSuccess)) {
                st = GRAV_EDEVICE;
                break;
            }
            const size_t partt = (size_t)p->m2lt_nseg * p->m2lt_ncw * p->PS;
            if ((st = dalloc(p, &p->d_partt, partt, false)) != GRAV_OK)
                break;
            // as in the forward: the orbit kernel leaves the slots' padding
            // entries alone, so they are cleared once here
            if (p->m2l_orbit && partt > 0 &&
                (hipMemsetAsync(p->d_partt, 0, partt * sizeof(float), s) != hipSuccess ||
                 hipStreamSynchronize(s) != hipSuccess)) {
                st = GRAV_EDEVICE;
                break;
            }
            if ((st = dalloc(p, &p->d_leg, (size_t)p->n_leg * p->B * std::max(p->PS, 4 * p->m2l_npl), false)) !=
                GRAV_OK)
                break;
        }
        {
            const DevGeom g = make_geom(p);
            if ((st = dalloc(p, &p->d_geom, 1, true)) != GRAV_OK)
                break;
            if (hipMemcpyAsync(p->d_geom, &g, sizeof(DevGeom), hipMemcpyHostToDevice, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = GRAV_EDEVICE;
                break;
            }
        }
        if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) {
            st = GRAV_EDEVICE;
            break;
        }
    } while (0);
    p->bs = nullptr;
    if (s)
        (void)hipStreamDestroy(s);
    (void)hipSetDevice(cur);
    if (st != GRAV_OK) {
        free_plan(p);
        return st;
    }
    *out = reinterpret_cast<grav_plan_t>(p);
    return GRAV_OK;
}

extern "C" void grav_plan_destroy(grav_plan_t plan)
{
    if (!plan)
        return;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (p->has_pending && p->done)
        (void)hipEventSynchronize(p->done);
    free_plan(p);
}

extern "C" grav_status grav_plan_bytes(grav_plan_t plan, size_t *resident, size_t *per_call)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (resident)
        *resident = p->bytes_resident;
    if (per_call)
        *per_call = p->bytes_call;
    return GRAV_OK;
}

extern "C" grav_status grav_plan_info(grav_plan_t plan, int64_t *n_targets, int32_t *levels,
                                      int32_t *leaf_cells, int64_t *n_target_leaves)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (n_targets)
        *n_targets = p->M;
    if (levels)
        *levels = p->L;
    if (leaf_cells)
        *leaf_cells = p->b;
    if (n_target_leaves)
        *n_target_leaves = p->n_leaf;
    return GRAV_OK;
}

extern "C" grav_status grav_plan_work(grav_plan_t plan, int64_t *m2l_pairs, int64_t *p2p_pairs,
                                      int64_t *n_sources)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (m2l_pairs)
        *m2l_pairs = p->m2l_pairs;
    if (p2p_pairs)
        *p2p_pairs = p->p2p_pairs;
    if (n_sources)
        *n_sources = p->n_spts > 0 ? p->n_spts : (int64_t)p->d.nx * p->d.ny * p->d.nz * p->nq3;
    return GRAV_OK;
}

extern "C" grav_status grav_operator(int32_t p, int32_t kind, int32_t which, int32_t dx,
                                     int32_t dy, int32_t dz, double *out)
{
    if (!out || p < 1)
        return GRAV_EINVAL;
    if (p > kMaxP)
        return GRAV_EUNSUPPORTED;
    const int P2 = p * p;
    if (kind == 0 || kind == 1) {
        if (which < 0 || which > 7)
            return GRAV_EINVAL;
        const double delta[3] = {((which & 1) - 0.5) * 0.5, (((which >> 1) & 1) - 0.5) * 0.5,
                                 (((which >> 2) & 1) - 0.5) * 0.5};
        if (kind == 0)
            m2m_matrix(p, delta, P2, out);
        else
            l2l_matrix(p, delta, P2, out);
        return GRAV_OK;
    }
    if (kind == 2) {
        const int mx = std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz)));
        if (mx < 2 || mx > 3)
            return GRAV_EINVAL;
        const double d[3] = {-(double)dx, -(double)dy, -(double)dz};
        m2l_matrix(p, d, P2, out);
        return GRAV_OK;
    }
    return GRAV_EINVAL;
}

extern "C" grav_status grav_harmonics(int32_t p, int32_t kind, double x, double y, double z,
                                      double *out)
{
    if (!out || p < 1 || (kind != 0 && kind != 1))
        return GRAV_EINVAL;
    if (p > kMaxP)
        return GRAV_EUNSUPPORTED;
    std::vector<cd> A;
    if (kind == 0)
        solid_regular(x, y, z, p, A);
    else {
        if (x == 0.0 && y == 0.0 && z == 0.0)
            return GRAV_EINVAL;
        solid_irregular(x, y, z, p, A);
    }
    for (int n = 0; n < p; ++n) {
        out[ridx(n, 0, 0)] = A[n * p].real();
        for (int m = 1; m <= n; ++m) {
            out[ridx(n, m, 0)] = A[n * p + m].real();
            out[ridx(n, m, 1)] = A[n * p + m].imag();
        }
    }
    return GRAV_OK;
}

extern "C" const char *grav_status_string(grav_status s)
{
    switch (s) {
    case GRAV_OK: return "ok";
    case GRAV_EINVAL: return "invalid argument";
    case GRAV_ENOMEM: return "out of memory";
    case GRAV_EDEVICE: return "device error";
    case GRAV_EUNSUPPORTED: return "unsupported request";
    case GRAV_EBUSY: return "plan busy on another stream";
    }
    return "unknown status";
}

extern "C" const char *grav_version(void) { return "grav-mi355x 0.1"; }
