// grav_plan_check: host-side validation of a plan's index tables.
//
// Copies the plan's device tables back and runs, on the host, the same
// column/term resolvers the M2L kernels use (they are compiled for both
// sides), plus the tree tables the other kernels index,
// checking every expansion, matrix, target-range and cell index against the
// size of the buffer it addresses, and that no two columns of one stage
// write the same expansion.  No compute kernel is launched.
#include <algorithm>
#include <cstdio>
#include <string>
#include <tuple>
#include <vector>

#include "resolve.hpp"

namespace grav {

namespace {

template <class T>
std::vector<T> fetch(const T *d, size_t n)
{
    std::vector<T> h(n);
    if (n && d && hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess)
        h.clear();
    return h;
}

struct Checker {
    bool ok = true;
    std::string msg;
    void fail(const char *stage, const char *what, long long a, long long b)
    {
        if (ok) {
            char buf[256];
            std::snprintf(buf, sizeof buf, "%s: %s (%lld vs %lld)", stage, what, a, b);
            msg = buf;
        }
        ok = false;
    }
};

// Tiles of a stage whose offsets are split S ways: tile.pad in [0, S) names
// the offset range [pad * 189 / S, (pad + 1) * 189 / S) and, for S > 1, the
// slab of the partial-sum workspace it writes ([S][ysize] expansions).
template <class Res>
void check_stage(Checker &ck, const char *name, const Res &res, const TileRange &r, int S,
                 int64_t n_ids, int64_t xsize, int64_t ysize, std::vector<char> &written)
{
    written.assign((size_t)(S > 1 ? S : 1) * ysize, 0);
    for (int64_t b = 0; b < r.n && ck.ok; ++b) {
        const GemmTile &tile = res.tiles[b];
        if (tile.ncol < 1 || tile.ncol > kTileCols)
            ck.fail(name, "tile width out of range", tile.ncol, kTileCols);
        if (tile.pad < 0 || tile.pad >= S)
            ck.fail(name, "split index out of range", tile.pad, S);
        if (!ck.ok)
            break;
        const int t0 = tile.pad * res.nterms(tile) / S, t1 = (tile.pad + 1) * res.nterms(tile) / S;
        for (int cl = 0; cl < kTileCols && ck.ok; ++cl) {
            const GemmCol col = res.column(tile, cl);
            if (!col.valid)
                continue;
            for (int it = t0; it < t1; ++it) {
                const GemmTerm tm = res.term(tile, it);
                if (tm.kid < 0 || tm.kid >= n_ids)
                    ck.fail(name, "matrix id out of range", tm.kid, n_ids);
                const int64_t s = res.src(tile, col, tm);
                if (s < -1 || s >= xsize)
                    ck.fail(name, "source expansion out of range", s, xsize);
            }
            const int64_t o = res.out(tile, col);
            if (o < 0 || o >= ysize) {
                ck.fail(name, "destination expansion out of range", o, ysize);
            } else {
                const int64_t w = (S > 1 ? tile.pad : 0) * ysize + o;
                if (written[w])
                    ck.fail(name, "two columns write one expansion", o, ysize);
                written[w] = 1;
            }
        }
    }
    for (size_t i = 0; i < written.size() && ck.ok; ++i)
        if (!written[i])
            ck.fail(name, "expansion never written", (long long)i, ysize);
}

}  // namespace

}  // namespace grav

using namespace grav;

extern "C" grav_status grav_plan_check(grav_plan_t plan, char *msg, int32_t msglen)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    Checker ck;
    auto report = [&]() {
        if (msg && msglen > 0) {
            std::snprintf(msg, (size_t)msglen, "%s", ck.ok ? "ok" : ck.msg.c_str());
        }
        return ck.ok ? GRAV_OK : GRAV_EINVAL;
    };
    if (p->M == 0)
        return report();
    int cur = 0;
    GRAV_HIP(hipGetDevice(&cur));
    GRAV_HIP(hipSetDevice(p->device));
    GRAV_HIP(hipDeviceSynchronize());
    const DevGeom g = make_geom(p);
    const int L = p->L;
    int64_t ntile = 0;
    for (int k = 0; k < TK_COUNT; ++k)
        for (int l = 0; l <= kMaxLevels; ++l)
            ntile = std::max<int64_t>(ntile, p->tiles[k][l].off + p->tiles[k][l].n);
    int64_t ntb = 0;
    const int lo = L >= 2 ? 2 : L;
    for (int l = lo; l <= L; ++l)
        ntb = std::max<int64_t>(ntb, p->tbox_off[l] + p->lev[l].n_tgt);
    const auto tiles = fetch(p->d_tiles, (size_t)ntile);
    const auto tkey = fetch(p->d_tkey, (size_t)ntb);
    const auto torder = fetch(p->d_torder, (size_t)ntb);
    const auto tparent = fetch(p->d_tparent, (size_t)ntb);
    const auto tmap = fetch(p->d_tmap, (size_t)p->n_tmap);
    const auto tchild = fetch(p->d_tchild, (size_t)p->n_tchild);
    const auto leaf_start = fetch(p->d_leaf_start, (size_t)p->n_leaf + 1);
    const auto tleaf = fetch(p->d_tleaf, (size_t)p->M);
    const auto perm = fetch(p->d_perm, (size_t)p->M);
    const auto leaf_pend = fetch(p->d_leaf_pend, (size_t)p->n_leaf);
    const int64_t ncell = (int64_t)p->d.nx * p->d.ny * p->d.nz;
    const auto cell_slot = p->lat_near ? fetch(p->d_cell_slot, (size_t)ncell) : std::vector<int32_t>();
    std::vector<int32_t> coff, roff;
    if (L >= 2) {
        coff = fetch(p->d_class_off, 8 * kClassOffsets * 4);
        roff = fetch(p->d_rclass_off, 8 * kClassOffsets * 4);
    }
    (void)hipSetDevice(cur);

    // target tables
    for (int64_t i = 0; i < p->n_leaf && ck.ok; ++i)
        if (leaf_start[i] >= leaf_start[i + 1])
            ck.fail("tree", "empty or unordered leaf range", leaf_start[i], leaf_start[i + 1]);
    if (ck.ok && leaf_start[p->n_leaf] != p->M)
        ck.fail("tree", "leaf ranges do not cover the targets", leaf_start[p->n_leaf], p->M);
    std::vector<char> seen(p->M, 0);
    for (int64_t i = 0; i < p->M && ck.ok; ++i) {
        if (tleaf[i] < 0 || tleaf[i] >= p->n_leaf)
            ck.fail("tree", "target leaf out of range", tleaf[i], p->n_leaf);
        else if (i < leaf_start[tleaf[i]] || i >= leaf_start[tleaf[i] + 1])
            ck.fail("tree", "target outside its leaf range", i, tleaf[i]);
        if (perm[i] >= (uint64_t)p->M || seen[perm[i]])
            ck.fail("tree", "permutation not a bijection", perm[i], p->M);
        else
            seen[perm[i]] = 1;
    }
    // user points first within each leaf; voxel-centre slots invert perm
    const int64_t npts = p->lat_near ? p->d.n_points : p->M;
    for (int64_t i = 0; i < p->n_leaf && ck.ok; ++i) {
        const int64_t e = leaf_pend[i];
        if (e < leaf_start[i] || e > leaf_start[i + 1])
            ck.fail("tree", "user-point end outside its leaf", e, i);
        for (int64_t j = leaf_start[i]; j < leaf_start[i + 1] && ck.ok; ++j)
            if (((int64_t)perm[j] < npts) != (j < e))
                ck.fail("tree", "user points not a prefix of their leaf", j, i);
    }
    if (p->lat_near) {
        if ((int64_t)cell_slot.size() != ncell)
            ck.fail("lattice", "cell slots not readable", (long long)cell_slot.size(), ncell);
        for (int64_t c = 0; c < ncell && ck.ok; ++c) {
            const int64_t j = cell_slot[c];
            if (j < 0 || j >= p->M || (int64_t)perm[j] != p->d.n_points + c)
                ck.fail("lattice", "cell slot does not invert the permutation", c, j);
        }
    }
    for (int l = lo; l <= L && ck.ok; ++l) {
        const DevLev &lv = g.lev[l];
        for (int64_t i = 0; i < p->lev[l].n_tgt && ck.ok; ++i) {
            const uint32_t k = tkey[lv.tbox_off + i];
            if (i > 0 && k <= tkey[lv.tbox_off + i - 1])
                ck.fail("tree", "box keys not strictly increasing", l, i);
            if (l > lo) {
                const int32_t par = tparent[lv.tbox_off + i];
                if (par < 0 || par >= p->lev[l - 1].n_tgt)
                    ck.fail("tree", "parent out of range", par, p->lev[l - 1].n_tgt);
                else if (tkey[g.lev[l - 1].tbox_off + par] != (k >> 3))
                    ck.fail("tree", "parent key mismatch", l, i);
            }
            if (l >= 2) {
                const int32_t o = torder[lv.tbox_off + i];
                if (o < 0 || o >= p->lev[l].n_tgt)
                    ck.fail("tree", "class order out of range", o, p->lev[l].n_tgt);
            }
        }
        // target map entries
        const int64_t msz = (int64_t)(lv.ns[0] + 6) * (lv.ns[1] + 6) * (lv.ns[2] + 6);
        for (int64_t i = 0; i < msz && ck.ok; ++i) {
            const int32_t v = tmap[lv.tmap_off + i];
            if (v < -1 || v >= p->lev[l].n_tgt)
                ck.fail("tmap", "entry out of range", v, p->lev[l].n_tgt);
        }
    }
    // reverse interaction lists of the adjoint's M2L: offsets of the list and
    // operator ids inside the 316 stored transposes
    for (size_t e = 0; e < roff.size() && ck.ok; e += 4) {
        const int mx = std::max(std::abs(roff[e]), std::max(std::abs(roff[e + 1]), std::abs(roff[e + 2])));
        if (mx < 2 || mx > 3 || roff[e + 3] < 0 || roff[e + 3] >= kNumOffsets)
            ck.fail("m2lT", "reverse list entry out of range", (long long)e, roff[e + 3]);
    }
    // the transposed M2L's offset table: (-d) of a reverse list entry, and
    // an operator index inside the stored transposes (56 canonical ones
    // with reflection bits in mixed plans, 316 in FP64)
    if (p->d_tclass_off) {
        const auto tco = fetch(p->d_tclass_off, (size_t)8 * kClassOffsets * 4);
        const bool f64 = p->d.precision == GRAV_FP64;
        for (size_t e = 0; e < tco.size() && ck.ok; e += 4) {
            const int id = tco[e + 3] % kReflShift, refl = tco[e + 3] / kReflShift;
            if (tco[e] != -roff[e] || tco[e + 1] != -roff[e + 1] || tco[e + 2] != -roff[e + 2] || tco[e + 3] < 0 ||
                id >= (f64 ? kNumOffsets : kCanonOffsets) || refl > (f64 ? 0 : 7))
                ck.fail("m2lT", "transposed offset entry out of range", (long long)e, tco[e + 3]);
        }
    }
    for (int l = 2; l < L && ck.ok; ++l) {
        const DevLev &lv = g.lev[l];
        for (int64_t i = 0; i < p->lev[l].n_tgt && ck.ok; ++i) {
            const int32_t a = tchild[lv.tchild_off + i], b = tchild[lv.tchild_off + i + 1];
            if (!(0 <= a && a < b && b <= p->lev[l + 1].n_tgt && b - a <= 8))
                ck.fail("tchild", "bad child range", a, b);
        }
    }
    // near field / leaf kernels: neighbour leaves within the source block or skipped
    if (ck.ok && L >= 0) {
        const DevLev &lv = g.lev[L];
        for (int64_t i = 0; i < p->n_leaf && ck.ok; ++i) {
            const uint32_t k = tkey[lv.tbox_off + i];
            const int c[3] = {(int)compact3(k), (int)compact3(k >> 1), (int)compact3(k >> 2)};
            for (int a = 0; a < 3; ++a)
                if (c[a] >= (1 << L))
                    ck.fail("leaf", "leaf coordinate outside the root", c[a], 1 << L);
        }
    }

    if (L >= 2 && ck.ok) {
        // the forward M2L's stream-K schedule: segments cover every work item
        // once, in order, one unit per segment; each unit lists its segments
        // in order; every LE column maps to one valid (unit, column)
        auto schedule = [&](const char *name, const int32_t *d_items, int64_t n_items, const int32_t *d_segs,
                            int64_t nseg, const int32_t *d_wgseg, int32_t wgs, const int32_t *d_tstart,
                            const int32_t *d_tsegs, int64_t nunit) {
            const auto items = fetch(d_items, (size_t)std::max<int64_t>(1, n_items));
            const auto segs = fetch(d_segs, (size_t)std::max<int64_t>(1, nseg) * 4);
            const auto wgseg = fetch(d_wgseg, (size_t)wgs + 1);
            const auto tstart = fetch(d_tstart, (size_t)nunit + 1);
            const auto tsegs = fetch(d_tsegs, (size_t)std::max<int64_t>(1, nseg));
            if (wgseg[0] != 0 || wgseg[wgs] != nseg)
                ck.fail(name, "segment ranges do not cover the segments", wgseg[0], nseg);
            int64_t next = 0;
            for (int64_t sg = 0; sg < nseg && ck.ok; ++sg) {
                const int32_t t = segs[4 * sg], ib = segs[4 * sg + 1], ie = segs[4 * sg + 2];
                if (t < 0 || t >= nunit || ib != next || ie <= ib || ie > n_items)
                    ck.fail(name, "segment out of order or range", sg, t);
                for (int32_t it = ib; it < ie && ck.ok; ++it)
                    if (items[it] < 0 || items[it] >= kClassOffsets)
                        ck.fail(name, "work item offset out of range", it, items[it]);
                next = ie;
            }
            if (ck.ok && next != n_items)
                ck.fail(name, "segments do not cover the work items", next, n_items);
            if (ck.ok && (tstart[0] != 0 || tstart[nunit] != nseg))
                ck.fail(name, "unit segment lists do not cover the segments", tstart[nunit], nseg);
            for (int64_t t = 0; t < nunit && ck.ok; ++t)
                for (int32_t j = tstart[t]; j < tstart[t + 1] && ck.ok; ++j)
                    if (tsegs[j] < 0 || tsegs[j] >= nseg || segs[4 * tsegs[j]] != t ||
                        (j > tstart[t] && tsegs[j] <= tsegs[j - 1]))
                        ck.fail(name, "unit segment list inconsistent", t, j);
        };
        const TileRange &r = p->tiles[TK_M2L][0];
        const int64_t upt = 64 / p->m2l_ncw;
        if (p->m2l_wgs > 0) {
            const int64_t nunit = p->m2l_nunit;
            schedule("m2l", p->d_m2l_items, p->m2l_items, p->d_m2l_segs, p->m2l_nseg, p->d_m2l_wgseg, p->m2l_wgs,
                     p->d_m2l_tseg_start, p->d_m2l_tsegs, nunit);
            const auto colmap = fetch(p->d_m2l_colmap, (size_t)(p->n_tbox * p->B));
            for (int64_t c = 0; c < p->n_tbox * p->B && ck.ok; ++c) {
                const int32_t m = colmap[c];
                const int64_t u = m >> 6;
                if (m < 0 || u >= nunit || (m & 63) >= p->m2l_ncw ||
                    (u % upt) * p->m2l_ncw + (m & 63) >= tiles[r.off + u / upt].ncol)
                    ck.fail("m2l", "LE column without a unit column", c, m);
            }
        }
        // the transposed M2L (adjoint): the same schedule checks; its tiles
        // address the column blocks, its columns map to units and to ME
        // columns, each ME column at most once; the gather regions lie in
        // the target maps (source block + halo 3)
        if (ck.ok) {
            const int64_t uptt = 64 / p->m2lt_ncw, nunit = p->m2lt_nunit, ntile = nunit / uptt;
            if (p->m2lt_wgs > 0)
                schedule("m2lT", p->d_m2lt_items, p->m2lt_items, p->d_m2lt_segs, p->m2lt_nseg, p->d_m2lt_wgseg,
                         p->m2lt_wgs, p->d_m2lt_tseg_start, p->d_m2lt_tsegs, nunit);
            const auto ttiles = fetch(p->d_m2lt_tiles, (size_t)std::max<int64_t>(1, ntile));
            const auto sorder = fetch(p->d_sorder, (size_t)std::max<int64_t>(1, p->n_me));
            for (int64_t t = 0; t < ntile && ck.ok; ++t) {
                const GemmTile &tl = ttiles[t];
                if (tl.level < 2 || tl.level > L || tl.cls < 0 || tl.cls > 7 || tl.ncol < 1 || tl.ncol > kTileCols)
                    ck.fail("m2lT", "tile out of range", t, tl.level);
                else {
                    const LevelInfo &lv = p->lev[tl.level];
                    const int64_t nb = lv.col_class_start[tl.cls + 1] - lv.col_class_start[tl.cls];
                    if (tl.col0 < 0 || tl.col0 + tl.ncol > nb * p->B)
                        ck.fail("m2lT", "tile columns outside its class", t, tl.col0);
                }
            }
            for (int l = 2; l <= L && ck.ok; ++l) {
                const LevelInfo &lv = p->lev[l];
                if (lv.col_class_start[8] > lv.n_src)
                    ck.fail("m2lT", "column block larger than the source block", l, lv.col_class_start[8]);
                for (int64_t i = 0; i < lv.col_class_start[8] && ck.ok; ++i)
                    if (sorder[lv.me_off + i] < 0 || sorder[lv.me_off + i] >= lv.n_src)
                        ck.fail("m2lT", "column box outside the source block", l, sorder[lv.me_off + i]);
                for (int a = 0; a < 3 && ck.ok; ++a)
                    if (lv.gns[a] > 0 && (lv.gs0[a] < lv.s0[a] - 3 || lv.gs0[a] + lv.gns[a] > lv.s0[a] + lv.ns[a] + 3))
                        ck.fail("m2lT", "gather region outside the target map", l, a);
            }
            const auto colmap = fetch(p->d_m2lt_colmap, (size_t)std::max<int64_t>(1, p->m2lt_ncols));
            const auto colbox = fetch(p->d_m2lt_colbox, (size_t)std::max<int64_t>(1, p->m2lt_ncols));
            std::vector<char> seen((size_t)std::max<int64_t>(1, p->n_me * p->B), 0);
            for (int64_t c = 0; c < p->m2lt_ncols && ck.ok; ++c) {
                const int32_t m = colmap[c];
                const int64_t u = m >> 6;
                if (m < 0 || u >= nunit || (m & 63) >= p->m2lt_ncw ||
                    (u % uptt) * p->m2lt_ncw + (m & 63) >= ttiles[u / uptt].ncol)
                    ck.fail("m2lT", "column without a unit column", c, m);
                else if (colbox[c] < 0 || colbox[c] >= p->n_me * p->B || seen[colbox[c]]++)
                    ck.fail("m2lT", "ME column out of range or repeated", c, colbox[c]);
            }
        }
    }
    if (L >= 2 && ck.ok) {
        const int64_t xme = p->n_me * p->B, xle = p->n_tbox * p->B;
        std::vector<char> w;
        {
            const TileRange &r = p->tiles[TK_M2L][0];
            ResM2L res{&g, tiles.data() + r.off, tkey.data(), torder.data(), coff.data()};
            check_stage(ck, "m2l", res, r, p->split[TK_M2L],
                        p->d.precision == GRAV_FP64 ? kNumOffsets : kCanonOffsets, xme, xle, w);
        }
        // M2M / M2M^T: every parent of a level >= 3 box lies in the block above
        for (int l = 3; l <= L && ck.ok; ++l) {
            const DevLev &lv = g.lev[l];
            for (int z = 0; z < lv.ns[2] && ck.ok; ++z)
                for (int y = 0; y < lv.ns[1] && ck.ok; ++y)
                    for (int x = 0; x < lv.ns[0] && ck.ok; ++x)
                        if (dense_index(g.lev[l - 1], (lv.s0[0] + x) >> 1, (lv.s0[1] + y) >> 1,
                                        (lv.s0[2] + z) >> 1) < 0)
                            ck.fail("m2mT", "parent outside the source block", l, x);
        }
    }
    // explicit sources: the per-leaf CSR is monotone and covers every
    // source; the permutation is a permutation
    if (ck.ok && p->n_spts > 0) {
        const int64_t nleaf = p->lev[L].n_src;
        const auto st = fetch(p->d_sstart, (size_t)nleaf + 1);
        const auto pm = fetch(p->d_sperm, (size_t)p->n_spts);
        if (st[0] != 0 || st[nleaf] != p->n_spts)
            ck.fail("sources", "leaf ranges do not cover the sources", st[0], st[nleaf]);
        for (int64_t j = 0; j < nleaf && ck.ok; ++j)
            if (st[j + 1] < st[j])
                ck.fail("sources", "leaf ranges out of order", j, st[j]);
        std::vector<char> seen((size_t)p->n_spts, 0);
        for (int64_t i = 0; i < p->n_spts && ck.ok; ++i)
            if (pm[i] >= (uint32_t)p->n_spts || seen[pm[i]]++)
                ck.fail("sources", "sorted order is not a permutation", i, pm[i]);
    }
    return report();
}
