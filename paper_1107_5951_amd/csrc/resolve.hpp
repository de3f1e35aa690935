// Index helpers of the M2L stage: tile/column/term resolution for the
// forward M2L (columns are target boxes of one child-parity class, terms the
// class's 189 interaction-list offsets).  The functions compile for host and
// device: the M2L kernels use them, and grav_plan_check runs them on the
// host to validate a plan's tables.
#pragma once

#include "eval_common.hpp"

namespace grav {

// A tile of columns: one level, one class (or none), columns [col0, col0 + ncol).
struct GemmTile {
    int32_t level;
    int32_t cls;
    int64_t col0;
    int32_t ncol;
    int32_t pad;
};

struct GemmCol {
    bool valid;
    int bm;             // density model
    int x, y, z;        // root-relative box coordinates
    int64_t box;        // index of the box in its list (meaning depends on the resolver)
};

struct GemmTerm {
    int kid;            // offset id: index of the translation matrix
    int dx, dy, dz;
};

// Enumerate the k-th box with parity class c in a dense block [s0, s0 + ns).
__host__ __device__ inline void class_box(int k, int c, const int s0[3], const int ns[3], int out[3])
{
    int first[3], cnt[3];
    for (int a = 0; a < 3; ++a) {
        const int par = (c >> a) & 1;
        first[a] = s0[a] + ((par - s0[a]) & 1);
        cnt[a] = (ns[a] - (first[a] - s0[a]) + 1) / 2;
    }
    const int kx = k % cnt[0];
    const int ky = (k / cnt[0]) % cnt[1];
    const int kz = k / (cnt[0] * cnt[1]);
    out[0] = first[0] + 2 * kx;
    out[1] = first[1] + 2 * ky;
    out[2] = first[2] + 2 * kz;
}

__host__ __device__ inline int64_t dense_index(const DevLev &lv, int x, int y, int z)
{
    const int sx = x - lv.s0[0], sy = y - lv.s0[1], sz = z - lv.s0[2];
    if (sx < 0 || sy < 0 || sz < 0 || sx >= lv.ns[0] || sy >= lv.ns[1] || sz >= lv.ns[2])
        return -1;
    return ((int64_t)sz * lv.ns[1] + sy) * lv.ns[0] + sx;
}

// Target-box map around a level's source block (halo H): index or -1.
__host__ __device__ inline int64_t tmap_lookup(const DevLev &lv, const int32_t *tmap, int H, int x, int y, int z)
{
    const int mx = lv.ns[0] + 2 * H, my = lv.ns[1] + 2 * H, mz = lv.ns[2] + 2 * H;
    const int sx = x - lv.s0[0] + H, sy = y - lv.s0[1] + H, sz = z - lv.s0[2] + H;
    if (sx < 0 || sy < 0 || sz < 0 || sx >= mx || sy >= my || sz >= mz)
        return -1;
    return tmap[lv.tmap_off + ((int64_t)sz * my + sy) * mx + sx];
}

// ---------------------------------------------------------------- resolvers
// Forward M2L: columns = target boxes of one class (class-grouped order);
// terms = the class's 189 interaction-list offsets; X = ME, Y = LE (store).
struct ResM2L {
    const DevGeom *g;
    const GemmTile *tiles;
    const uint32_t *tkey;
    const int32_t *torder;
    const int32_t *offs;  // [8][189][4]: dx, dy, dz, operator index + kReflShift x reflection bits
    __host__ __device__ int nterms(const GemmTile &) const { return kClassOffsets; }
    __host__ __device__ GemmCol column(const GemmTile &t, int cl) const
    {
        GemmCol c{};
        c.valid = cl < t.ncol;
        if (!c.valid)
            return c;
        const DevLev &lv = g->lev[t.level];
        const int64_t col = t.col0 + cl;
        c.bm = (int)(col % g->B);
        c.box = torder[lv.tbox_off + lv.class_start[t.cls] + col / g->B];
        const uint32_t key = tkey[lv.tbox_off + c.box];
        c.x = (int)compact3(key);
        c.y = (int)compact3(key >> 1);
        c.z = (int)compact3(key >> 2);
        return c;
    }
    __host__ __device__ GemmTerm term(const GemmTile &t, int i) const
    {
        const int32_t *e = offs + (t.cls * kClassOffsets + i) * 4;
        return GemmTerm{e[3] % kReflShift, e[0], e[1], e[2]};  // canonical operator index
    }
    // position of the source expansion in the regathered (class-split) array
    // the M2L reads, computed as the kernel does; a position that does not
    // enumerate back to the same box is returned out of range
    __host__ __device__ int64_t src(const GemmTile &t, const GemmCol &c, const GemmTerm &m) const
    {
        const DevLev &lv = g->lev[t.level];
        const int ax = c.x + m.dx, ay = c.y + m.dy, az = c.z + m.dz;
        if (dense_index(lv, ax, ay, az) < 0)
            return -1;
        const int sc = t.cls ^ ((m.dx & 1) | ((m.dy & 1) << 1) | ((m.dz & 1) << 2));
        int first[3], cnt[3];
        const int64_t start = class_split(lv, sc, first, cnt);
        const int64_t k = ((int64_t)((az - first[2]) >> 1) * cnt[1] + ((ay - first[1]) >> 1)) * cnt[0] +
                          ((ax - first[0]) >> 1);
        int xyz[3];
        class_box((int)k, sc, lv.s0, lv.ns, xyz);
        if (k < 0 || xyz[0] != ax || xyz[1] != ay || xyz[2] != az)
            return INT64_MAX / 2;
        return (lv.me_off + start + k) * g->B + c.bm;
    }
    __host__ __device__ int64_t out(const GemmTile &t, const GemmCol &c) const
    {
        return (g->lev[t.level].tgt_off + c.box) * g->B + c.bm;
    }
};

}  // namespace grav
