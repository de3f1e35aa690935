// M2L on MFMA for the forward pass (kept in its own file: its measured HBM
// traffic is tied to this source).
#include <algorithm>
#include <type_traits>

#include "resolve.hpp"

// Operand register sets of the M2L (NS template parameter): with two sets
// the loads of the next chunk are in flight during this chunk's MFMAs; with
// one, the registers leave room for more waves per SIMD (with two column
// blocks: three at p = 10 in FP32, five at p = 8), which hide the load
// latency better on large plans (256^3 volume workload: M2L 10.5 against
// 10.9 ms at p = 10, 4.3 against 4.6 ms at p = 8) but not on small ones,
// where each wave has only a few work items (64^3: 0.20 against 0.18 ms).
// The plan picks the FP32 variant by its work per resident wave (see
// build_tiles), and the number of 16-column blocks per wave by its column
// count: four blocks (each operator fragment feeds four instructions, two
// waves per SIMD) took the 256^3 M2L from 10.5 to 10.2 ms at p = 10 and from
// 4.3 to 4.05 ms at p = 8, but slowed the 64^3 one (0.20 to 0.22 ms).  The
// FP64 kernel keeps two sets while a chunk's A values fit this many bytes
// per lane.
#ifndef GRAV_M2L_DB_BYTES64
#define GRAV_M2L_DB_BYTES64 512
#endif
// One register set: raise the wave's priority while it runs a chunk's
// matrix instructions (256^3 at p = 10: 9.45 -> 9.26 ms).
#ifndef GRAV_M2L_PRIO
#define GRAV_M2L_PRIO 1
#endif


namespace grav {

// Sign bits of real coefficient c (degree n block of 2n+1 values: the real
// part of order 0, then real and imaginary parts of orders 1..n) under the
// reflections of the z, y and x axes.
__device__ inline void coef_sign_bits(int c, uint32_t &bz, uint32_t &by, uint32_t &bx)
{
    int n = 0;
    while ((n + 1) * (n + 1) <= c)
        ++n;
    const int i = c - n * n;
    const int m = (i + 1) / 2;
    const uint32_t im = (i > 0 && (i & 1) == 0) ? 1u : 0u;
    bz = (uint32_t)((n + m) & 1);
    by = im;
    bx = (uint32_t)((m + (int)im) & 1);
}

__device__ __forceinline__ float flip_sign(float v, uint32_t s)
{
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) ^ (s << 31));
}
__device__ __forceinline__ double flip_sign(double v, uint32_t s)
{
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) ^ ((uint64_t)s << 63));
}

// --------------------------------------------------------------------------
// M2L on MFMA.  A tile is up to 64 columns (target box of one level and one
// child-parity class, model), split into 4 / NC units of 16 NC columns; a
// unit's work items are the class's interaction-list offsets d at which some
// of its columns has a source box.  A workgroup is one wave; it runs its
// segments (a unit and a contiguous run of its items, see the stream-K
// schedule in build_tiles) one after the other, holding the unit's NC blocks
// of 16 columns and all row blocks.  For each d it accumulates
// LE[:, col] += K_d * ME[box(col) + d] with 16x16x4 MFMA tiles in registers
// across the segment's offsets (no atomics), then writes the segment's
// partial to its slot; every A fragment loaded feeds NC instructions.
//
// Operators: only the 56 offsets with non-negative components have stored
// matrices.  Reflecting an axis maps the real solid harmonics into
// themselves up to a sign per coefficient (degree n, order m, real or
// imaginary part): z -> -z multiplies by (-1)^(n+m), y -> -y by -1 on
// imaginary parts, x -> -x by (-1)^m on real and -(-1)^m on imaginary
// parts.  So with S the diagonal sign matrix of the reflection r that maps
// |d| to d, K_d = S K_|d| S: the kernel negates the A rows and the B entries
// whose sign bit is set, which reproduces K_d exactly (a sign flip is exact),
// and the operator set read by a launch shrinks from 316 to 56 matrices.
// The FP64 kernel reads all 316 operators (reflection bits zero).
//
// Contraction order: k step ks and sub-row kr = lane / 16 of the 16x16x4
// instruction take coefficient c = 4 ks + kr, so the coefficients c >= p^2
// of the padding fill whole trailing k steps, which are skipped (KSV = the
// k steps that hold coefficients).  A lane's B values for four consecutive
// k steps are one aligned vector load from the regathered, class-split
// expansions (the 16 source boxes of a wave at one offset are one class,
// consecutive in x, so the load covers a few contiguous runs), and the A
// fragments of four k steps and all row blocks form one group-major set
// per (d, q) (value u * RB + rb, ks = 4q + u), read with 4 RB / G 16-byte
// loads that each cover a contiguous kilobyte.  Padding coefficients
// (c >= p^2) are zero in the expansions.
// --------------------------------------------------------------------------
#ifdef GRAV_M2L_WAVES_PER_EU
#define GRAV_M2L_OCC __attribute__((amdgpu_waves_per_eu(GRAV_M2L_WAVES_PER_EU, 8)))
#else
#define GRAV_M2L_OCC
#endif

template <int RB, int KSV, int NC, typename T, int NS>
__global__ void __launch_bounds__(64) GRAV_M2L_OCC
k_m2l(DevGeom g, const GemmTile *tiles, const uint32_t *tkey, const int32_t *torder,
      const int32_t *class_off, const T *K, const T *me, const int32_t *segs, const int32_t *wgseg,
      const int32_t *items, T *part)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(T)))) T;
    using kmask_t = std::conditional_t<(KSV > 32), uint64_t, uint32_t>;
    const int lane = threadIdx.x;  // one wave per workgroup
    constexpr int UPT = 4 / NC;      // units (waves' column blocks) per tile
    // FP32 with at most four coefficient rows in the last row block (p^2 mod
    // 16 in 1..4, so that the coefficients end in k step 4 (RB - 1)): that
    // block runs as 4x4x1 instructions (16 blocks, a quarter of the cycles
    // of a 16x16x4 one).  Block 4 (lane / 16) + (lane % 16) / 4 takes the
    // lane's own B value (coefficient 4 ks + lane / 16 of column lane % 16)
    // and the A value of row lane % 4 at the same coefficient, so lane l
    // accumulates the rows at column l % 16 over the coefficients of its
    // residue l / 16 mod 4; the four residues are added across lanes at the
    // end.
    constexpr bool TAIL = sizeof(T) == 4 && KSV == 4 * (RB - 1) + 1;
    // reflection sign bits of this lane's A rows (bit rb: row 16 rb + lane %
    // 16, or lane % 4 in a 4x4 tail) and B contraction indices (bit ks:
    // coefficient 4 ks + lane / 16)
    uint32_t rsz = 0, rsy = 0, rsx = 0;
    kmask_t ksz = 0, ksy = 0, ksx = 0;
    for (int rb = 0; rb < RB; ++rb) {
        uint32_t bz, by, bx;
        coef_sign_bits(16 * rb + (TAIL && rb == RB - 1 ? (lane & 3) : (lane & 15)), bz, by, bx);
        rsz |= bz << rb;
        rsy |= by << rb;
        rsx |= bx << rb;
    }
    for (int ks = 0; ks < KSV; ++ks) {
        uint32_t bz, by, bx;
        coef_sign_bits(4 * ks + (lane >> 4), bz, by, bx);
        ksz |= (kmask_t)bz << ks;
        ksy |= (kmask_t)by << ks;
        ksx |= (kmask_t)bx << ks;
    }
    for (int sg = wgseg[blockIdx.x]; sg < wgseg[blockIdx.x + 1]; ++sg) {
        const int32_t *sd = segs + 4 * sg;  // unit, first item, end item
        const GemmTile tile = tiles[sd[0] / UPT];
        const int hq = sd[0] % UPT;       // the unit's column block in the tile
        const DevLev &lv = g.lev[tile.level];
        bool cvalid[NC];
        int bm[NC], bx[NC], by[NC], bz[NC];
        int64_t box[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int cl = (hq * NC + c) * 16 + (lane & 15);
            cvalid[c] = cl < tile.ncol;
            const int64_t col = tile.col0 + cl;
            bm[c] = (int)(col % g.B);
            box[c] = 0;
            bx[c] = by[c] = bz[c] = 0;
            if (cvalid[c]) {
                box[c] = torder[lv.tbox_off + lv.class_start[tile.cls] + col / g.B];
                const uint32_t key = tkey[lv.tbox_off + box[c]];
                bx[c] = (int)compact3(key);
                by[c] = (int)compact3(key >> 1);
                bz[c] = (int)compact3(key >> 2);
            }
        }
        vec4 acc[NC][RB];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                acc[c][rb] = vec4{0, 0, 0, 0};
        const int32_t *offs = class_off + tile.cls * kClassOffsets * 4;
        const int kr = lane >> 4;
        constexpr int PS = 16 * RB;
        constexpr int QC = (KSV + 3) / 4;  // chunks of four k steps holding coefficients
        // regathered expansions of this level: plane (q, kr) holds four
        // coefficients of every (class-split box, model), plane stride pstr
        const int64_t nB = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2] * g.B;
        const int64_t pstr = nB * 4;
        const T *mlev = me + lv.me_off * g.B * PS + kr * pstr;
        constexpr int64_t kstride = (int64_t)RB * 64 * 4 * RB;  // elements per offset matrix
        // One work item = one offset d of the unit (every item has a source
        // box for some column of the unit).  Its B pointers, operator and
        // column mask:
        struct Item {
            const T *mp[NC];
            const T *kp;
            bool have[NC];
            uint32_t rflip;   // bit rb: negate the A rows of row block rb
            kmask_t kflip;    // bit ks: negate the B entries of k step ks
        };
        auto setup = [&](int it, Item &st) {
            const int o = items[it];
            const int dx = offs[4 * o + 0], dy = offs[4 * o + 1], dz = offs[4 * o + 2];
            const int id = offs[4 * o + 3] % kReflShift;  // stored operator of |d|
            const int refl = offs[4 * o + 3] / kReflShift;
            st.rflip = ((refl & 4) ? rsz : 0u) ^ ((refl & 2) ? rsy : 0u) ^ ((refl & 1) ? rsx : 0u);
            st.kflip = ((refl & 4) ? ksz : (kmask_t)0) ^ ((refl & 2) ? ksy : (kmask_t)0) ^
                       ((refl & 1) ? ksx : (kmask_t)0);
            // the source boxes at this offset all belong to one parity class
            int first[3], cnt[3];
            const int64_t cstart =
                class_split(lv, tile.cls ^ ((dx & 1) | ((dy & 1) << 1) | ((dz & 1) << 2)), first, cnt);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int ax = bx[c] + dx, ay = by[c] + dy, az = bz[c] + dz;
                const int sx = ax - lv.s0[0], sy = ay - lv.s0[1], sz = az - lv.s0[2];
                st.have[c] = cvalid[c] && sx >= 0 && sy >= 0 && sz >= 0 && sx < lv.ns[0] && sy < lv.ns[1] &&
                             sz < lv.ns[2];
                const int64_t pos = cstart + ((int64_t)((az - first[2]) >> 1) * cnt[1] + ((ay - first[1]) >> 1)) * cnt[0] +
                                    ((ax - first[0]) >> 1);
                st.mp[c] = mlev + (st.have[c] ? (pos * g.B + bm[c]) * 4 : 0);
            }
            st.kp = K + (int64_t)id * kstride;
        };
        // two register sets (when they fit): the loads of chunk q + 1 (or of
        // the next item's first chunk) are in flight while the instructions
        // of chunk q run
        constexpr int NSET =
            NS == 2 && 4 * RB * (int)sizeof(T) <= (sizeof(T) == 4 ? 512 : GRAV_M2L_DB_BYTES64) ? 2 : 1;
        T av[NSET][4 * RB];
        T bb[NSET][NC][4];
        auto load = [&](const Item &st, int q, int set) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                load4(st.mp[c] + (int64_t)q * 4 * pstr, bb[set][c]);
            load_frags<T, 4 * RB>(st.kp + (int64_t)q * 64 * 4 * RB, lane, av[set]);
        };
        auto compute = [&](const Item &st, int q, int set) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (4 * q + u >= KSV)
                    break;  // k steps past the last coefficient are all zero
                constexpr bool kFlip = sizeof(T) == 4;  // FP64 plans store all 316 operators
                const uint32_t ks_flip = kFlip ? (uint32_t)(st.kflip >> (4 * q + u)) & 1u : 0u;
                T bv[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    bv[c] = st.have[c] ? (kFlip ? flip_sign(bb[set][c][u], ks_flip) : bb[set][c][u]) : (T)0;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const T a = kFlip ? flip_sign(av[set][u * RB + rb], (st.rflip >> rb) & 1u) : av[set][u * RB + rb];
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if constexpr (sizeof(T) == 8)
                            acc[c][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[c], acc[c][rb], 0, 0, 0);
                        else if (TAIL && rb == RB - 1)
                            acc[c][rb] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, bv[c], acc[c][rb], 0, 0, 0);
                        else
                            acc[c][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv[c], acc[c][rb], 0, 0, 0);
                    }
                }
            }
        };
        constexpr int NLD = NC + 4 * RB * (int)sizeof(T) / 16, NMF = 4 * RB * NC;
        const int ib = sd[1], ie = sd[2];
        if constexpr (NSET == 2 && sizeof(T) == 4) {
            // item k's chunk q uses register set (P0 + q) & 1, P0 = parity of
            // the chunks before it; items are handled in pairs so that P0 is
            // a compile-time constant
            auto item = [&](auto p0, int it, const Item &cur, Item &nxt) {
                constexpr int P0 = decltype(p0)::value;
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    if (q + 1 < QC) {
                        // the loads of chunk q + 1 issue one by one between
                        // this chunk's instructions
                        load(cur, q + 1, (P0 + q + 1) & 1);
                        compute(cur, q, (P0 + q) & 1);
                        interleave_loads<NLD, NMF>();
                    } else if (it + 1 < ie) {
                        // last chunk: the next item's first loads instead
                        setup(it + 1, nxt);
                        load(nxt, 0, (P0 + QC) & 1);
                        compute(cur, q, (P0 + q) & 1);
                        interleave_loads<NLD, NMF>();
                    } else {
                        compute(cur, q, (P0 + q) & 1);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            Item A, Bn;
            if (ib < ie) {
                setup(ib, A);
                load(A, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            for (int it = ib; it < ie; it += 2) {
                item(std::integral_constant<int, 0>{}, it, A, Bn);
                if (it + 1 < ie)
                    item(std::integral_constant<int, QC & 1>{}, it + 1, Bn, A);
            }
        } else if constexpr (NSET == 2) {
            // FP64: the cross-item prefetch would need the registers of a
            // second wave per SIMD; pipeline within each item only
            for (int it = ib; it < ie; ++it) {
                Item A;
                setup(it, A);
                load(A, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    if (q + 1 < QC) {
                        load(A, q + 1, (q + 1) & 1);
                        compute(A, q, q & 1);
                        interleave_loads<NLD, NMF>();
                    } else {
                        compute(A, q, q & 1);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        } else {
            for (int it = ib; it < ie; ++it) {
                Item A;
                setup(it, A);
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    load(A, q, 0);
                    __builtin_amdgcn_sched_barrier(0);
#if GRAV_M2L_PRIO
                    // a wave that has its operands keeps the matrix unit for
                    // its whole chunk (the waves of a SIMD alternate instead
                    // of interleaving and then waiting for loads together)
                    __builtin_amdgcn_s_setprio(1);
#endif
                    compute(A, q, 0);
#if GRAV_M2L_PRIO
                    __builtin_amdgcn_sched_barrier(0);
                    __builtin_amdgcn_s_setprio(0);
#endif
                }
            }
        }
        if constexpr (TAIL) {
            // the 4x4 tail: lane l holds rows 16 (RB - 1) + r of column l % 16
            // summed over its coefficient residue; add the four residues in a
            // fixed order and leave the sums in lanes 0..15, which is where
            // the 16x16x4 layout below puts those rows (the other lanes'
            // rows are padding: zero)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    T v = acc[c][RB - 1][r];
                    v += __shfl_xor(v, 16);
                    v += __shfl_xor(v, 32);
                    acc[c][RB - 1][r] = lane < 16 ? v : (T)0;
                }
        }
        // Output fragment: lane holds column lane % 16 and four rows; the FP32
        // instruction gives rows 4*(lane/16) + r, the FP64 one rows lane/16 + 4r.
        // The segment's partial LE goes to its own slot [16 NC columns][PS].
        constexpr int rstride = sizeof(T) == 8 ? 4 : 1;
        const int rbase = sizeof(T) == 8 ? kr : 4 * kr;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (!cvalid[c])
                continue;
            T *dst = part + ((int64_t)sg * (16 * NC) + c * 16 + (lane & 15)) * PS;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    dst[16 * rb + rbase + rstride * r] = acc[c][rb][r];
        }
    }
}

// --------------------------------------------------------------------------
// Reflection-orbit M2L (mixed plans whose eight sign classes hold at most 16
// coefficients each, p <= 10).  With S_r the diagonal sign matrix of
// reflection r, the offsets r(|d|) of one orbit share the canonical operator
// K = K_|d|: K_r(|d|) = S_r K S_r.  Entry (i, j) of S_r K S_r is K[i][j]
// times chi_{a^b}(r) = (-1)^popcount(r & (a ^ b)), a and b the sign classes
// of coefficients i and j.  Grouping rows and columns by class, the orbit's
// contribution to the rows of class a is
//   sum_b K[a, b] H_{a^b},   H_w = sum_r chi_w(r) ME_r[b],
// ME_r the expansion of the source box at offset r(|d|) (zero where there
// is none).  H is the Walsh-Hadamard transform of the eight ME_r (three
// butterfly stages over the reflection bits), so an orbit costs one
// operator's matrix instructions (8 x 8 blocks of 16 x 16, 256 16x16x4
// instructions per column block) instead of one per offset (up to eight).
// A work item is a (unit, canonical offset) pair; chunk q of an item is
// column class q: its A fragments are the 8 row blocks of K[:, q] and its B
// values the four k steps of class q from each of the eight source boxes.
// The regathered expansions hold class q's coefficients in planes 4 q .. 4
// q + 3 (value u of plane (q, kr): position 4 u + kr of the class).  Output
// row 4 kr + r of row block a is coefficient ccoef[a][4 kr + r] (-1: none;
// the slot's unused entries stay zero from the plan's clearing).  The
// adjoint's transposed M2L runs the same kernel on its own problem: columns
// are source boxes, K the class-blocked K_c^T, and the orbit table groups
// the reverse offset lists.
// --------------------------------------------------------------------------
#ifndef GRAV_M2L_ORB_WAVES
#define GRAV_M2L_ORB_WAVES 2
#endif
template <int NC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(GRAV_M2L_ORB_WAVES, 8)))
k_m2l_orb(DevGeom g, const GemmTile *tiles, const uint32_t *tkey, const int32_t *torder,
          const int32_t *class_off, const int32_t *orbtab, const float *K, const float *me,
          const int32_t *segs, const int32_t *wgseg, const int32_t *items, const int32_t *ccoef, float *part)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
    const int lane = threadIdx.x;  // one wave per workgroup
    constexpr int UPT = 4 / NC;
    const int kr = lane >> 4;
    const int PS = g.PS;
    for (int sg = wgseg[blockIdx.x]; sg < wgseg[blockIdx.x + 1]; ++sg) {
        const int32_t *sd = segs + 4 * sg;  // unit, first item, end item
        const GemmTile tile = tiles[sd[0] / UPT];
        const int hq = sd[0] % UPT;
        const DevLev &lv = g.lev[tile.level];
        bool cvalid[NC];
        int bm[NC], bx[NC], by[NC], bz[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int cl = (hq * NC + c) * 16 + (lane & 15);
            cvalid[c] = cl < tile.ncol;
            const int64_t col = tile.col0 + cl;
            bm[c] = (int)(col % g.B);
            bx[c] = by[c] = bz[c] = 0;
            if (cvalid[c]) {
                const int32_t box = torder[lv.tbox_off + lv.class_start[tile.cls] + col / g.B];
                const uint32_t key = tkey[lv.tbox_off + box];
                bx[c] = (int)compact3(key);
                by[c] = (int)compact3(key >> 1);
                bz[c] = (int)compact3(key >> 2);
            }
        }
        vec4 acc[NC][8];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int a = 0; a < 8; ++a)
                acc[c][a] = vec4{0, 0, 0, 0};
        const int32_t *offs = class_off + tile.cls * kClassOffsets * 4;
        const int32_t *otab = orbtab + tile.cls * kCanonOffsets * 8;
        const int64_t nB = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2] * g.B;
        const int64_t pstr = nB * 4;
        // chunk q's planes start at mlev + 4 q pstr (wave-uniform); a lane's
        // byte offsets from there hold its sub-row kr (below 2^32: the plan
        // takes this kernel only for smaller regathered buffers)
        const char *mlev = reinterpret_cast<const char *>(me + lv.me_off * g.B * 128);
        const uint32_t krb = (uint32_t)(kr * pstr * 4);
        for (int it = sd[1]; it < sd[2]; ++it) {
            const int ci = items[it];
            // per reflection r: whether the class has that offset, and per
            // column the byte offset of its source box's expansion and a
            // have bit (the offsets of an orbit share their parity, hence the
            // source class)
            uint32_t present = 0, hm = 0;
            uint32_t off[8][NC];
            int first[3] = {0, 0, 0}, cnt[3] = {0, 0, 0};
            int64_t cstart = 0;
            bool split = false;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int o = otab[ci * 8 + r];
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    off[r][c] = krb;
                if (o < 0)
                    continue;
                present |= 1u << r;
                const int dx = offs[4 * o + 0], dy = offs[4 * o + 1], dz = offs[4 * o + 2];
                if (!split) {
                    cstart = class_split(lv, tile.cls ^ ((dx & 1) | ((dy & 1) << 1) | ((dz & 1) << 2)), first, cnt);
                    split = true;
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const int ax = bx[c] + dx, ay = by[c] + dy, az = bz[c] + dz;
                    const int sx = ax - lv.s0[0], sy = ay - lv.s0[1], sz = az - lv.s0[2];
                    const bool have = cvalid[c] && sx >= 0 && sy >= 0 && sz >= 0 && sx < lv.ns[0] &&
                                      sy < lv.ns[1] && sz < lv.ns[2];
                    const int64_t pos = cstart +
                                        ((int64_t)((az - first[2]) >> 1) * cnt[1] + ((ay - first[1]) >> 1)) * cnt[0] +
                                        ((ax - first[0]) >> 1);
                    if (have) {
                        off[r][c] = krb + (uint32_t)((pos * g.B + bm[c]) * 16);
                        hm |= 1u << (r * NC + c);
                    }
                }
            }
            const float *kp = K + (int64_t)ci * (8 * 8 * 256);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float av[32];
                vec4 h[NC][8];
                load_frags<float, 32>(kp + q * (8 * 256), lane, av);
                const char *mq = mlev + (int64_t)q * 16 * pstr;
#pragma unroll
                for (int r = 0; r < 8; ++r)
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        h[c][r] = vec4{0, 0, 0, 0};
                        if (present & (1u << r)) {
                            const vec4 v = *(const vec4 *)(mq + off[r][c]);
                            if ((hm >> (r * NC + c)) & 1u)
                                h[c][r] = v;
                        }
                    }
                __builtin_amdgcn_sched_barrier(0);
#if GRAV_M2L_PRIO
                __builtin_amdgcn_s_setprio(1);
#endif
                // Walsh-Hadamard transform over the reflection bits x, y, z
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
                        for (int r = 0; r < 8; ++r)
                            if ((r & bit) == 0) {
                                const vec4 x = h[c][r], y = h[c][r | bit];
                                h[c][r] = x + y;
                                h[c][r | bit] = x - y;
                            }
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            acc[c][a] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[4 * a + u], h[c][a ^ q][u],
                                                                             acc[c][a], 0, 0, 0);
#if GRAV_M2L_PRIO
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(0);
#endif
            }
        }
        // lane: column lane % 16, rows 4 kr + r of each row block (class)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (!cvalid[c])
                continue;
            float *dst = part + ((int64_t)sg * (16 * NC) + c * 16 + (lane & 15)) * PS;
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = ccoef[16 * a + 4 * kr + r];
                    if (k >= 0)
                        dst[k] = acc[c][a][r];
                }
        }
    }
}

template <typename T>
grav_status launch_m2l(const Plan *p, const DevGeom &g, hipStream_t s, const M2LRun<T> &r)
{
    if (r.wgs == 0)
        return GRAV_OK;
    if constexpr (sizeof(T) == 4) {
        if (r.orbtab != nullptr) {
            if (r.nc != GRAV_M2L_ORB_NC)
                return GRAV_EUNSUPPORTED;
            hipLaunchKernelGGL((k_m2l_orb<GRAV_M2L_ORB_NC>), dim3(r.wgs), dim3(64), 0, s, g, r.tiles, r.keys,
                               r.order, r.class_off, r.orbtab, r.K, r.b_in, r.segs, r.wgseg, r.items, r.ccoef,
                               r.part);
            GRAV_HIP(hipGetLastError());
            return GRAV_OK;
        }
    }
    // column blocks per wave: FP64 one; FP32 the plan's (narrow or wide)
    constexpr int NCN = sizeof(T) == 8 ? GRAV_M2L_NC64 : GRAV_M2L_NC32;
    constexpr int NCW = sizeof(T) == 8 ? GRAV_M2L_NC64_WIDE : GRAV_M2L_NC32_WIDE;
    if (r.nc != NCN && r.nc != NCW)
        return GRAV_EUNSUPPORTED;
    dim3 grid(r.wgs), blk(64);
#define M2L_LAUNCH(P, NC, NS)                                                                          \
    hipLaunchKernelGGL((k_m2l<(P * P + 15) / 16, (P * P + 3) / 4, NC, T, NS>), grid, blk, 0, s, g, r.tiles, \
                       r.keys, r.order, r.class_off, r.K, r.b_in, r.segs, r.wgseg, r.items, r.part)
#define M2L_CASE(P)                                                                             \
    case P:                                                                                     \
        if (sizeof(T) == 4 && r.nset == 1 && r.nc == NCW)                                       \
            M2L_LAUNCH(P, NCW, 1);                                                              \
        else if (sizeof(T) == 4 && r.nset == 1)                                                 \
            M2L_LAUNCH(P, NCN, 1);                                                              \
        else if (r.nc == NCW)                                                                   \
            M2L_LAUNCH(P, NCW, 2);                                                              \
        else                                                                                    \
            M2L_LAUNCH(P, NCN, 2);                                                              \
        break;
    switch (p->P) {
        M2L_CASE(1)
        M2L_CASE(2)
        M2L_CASE(3)
        M2L_CASE(4)
        M2L_CASE(5)
        M2L_CASE(6)
        M2L_CASE(7)
        M2L_CASE(8)
        M2L_CASE(9)
        M2L_CASE(10)
        M2L_CASE(11)
        M2L_CASE(12)
        M2L_CASE(13)
        M2L_CASE(14)
        M2L_CASE(15)
        M2L_CASE(16)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef M2L_CASE
#undef M2L_LAUNCH
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

template grav_status launch_m2l<double>(const Plan *, const DevGeom &, hipStream_t, const M2LRun<double> &);
template grav_status launch_m2l<float>(const Plan *, const DevGeom &, hipStream_t, const M2LRun<float> &);

// One-wave workgroups of the plan's M2L kernel (with nset operand register
// sets in FP32) that the device holds at once (blocks per CU from the
// occupancy calculator, times the CUs): the size of the stream-K schedule,
// so that every worker is resident from the start.
grav_status m2l_resident_workers(const Plan *p, int nset, int nc, bool orbit, int *workers)
{
    const bool f64 = p->d.precision == GRAV_FP64;
    const bool wide = nc == (f64 ? GRAV_M2L_NC64_WIDE : GRAV_M2L_NC32_WIDE);
    const void *fn = nullptr;
    if (orbit)
        fn = reinterpret_cast<const void *>(&k_m2l_orb<GRAV_M2L_ORB_NC>);
    else
#define M2L_FN(P)                                                                                           \
    case P:                                                                                                 \
        fn = f64 ? (wide ? reinterpret_cast<const void *>(&k_m2l<(P * P + 15) / 16, (P * P + 3) / 4, GRAV_M2L_NC64_WIDE, double, 2>) \
                         : reinterpret_cast<const void *>(&k_m2l<(P * P + 15) / 16, (P * P + 3) / 4, GRAV_M2L_NC64, double, 2>)) \
             : wide ? (nset == 1 ? reinterpret_cast<const void *>(&k_m2l<(P * P + 15) / 16, (P * P + 3) / 4, GRAV_M2L_NC32_WIDE, float, 1>) \
                                 : reinterpret_cast<const void *>(&k_m2l<(P * P + 15) / 16, (P * P + 3) / 4, GRAV_M2L_NC32_WIDE, float, 2>)) \
             : nset == 1 ? reinterpret_cast<const void *>(&k_m2l<(P * P + 15) / 16, (P * P + 3) / 4, GRAV_M2L_NC32, float, 1>) \
                         : reinterpret_cast<const void *>(&k_m2l<(P * P + 15) / 16, (P * P + 3) / 4, GRAV_M2L_NC32, float, 2>); \
        break;
    switch (p->P) {
        M2L_FN(1)
        M2L_FN(2)
        M2L_FN(3)
        M2L_FN(4)
        M2L_FN(5)
        M2L_FN(6)
        M2L_FN(7)
        M2L_FN(8)
        M2L_FN(9)
        M2L_FN(10)
        M2L_FN(11)
        M2L_FN(12)
        M2L_FN(13)
        M2L_FN(14)
        M2L_FN(15)
        M2L_FN(16)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef M2L_FN
    int per_cu = 0, n_cu = 0;
    GRAV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, 0));
    GRAV_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, p->device));
    *workers = std::max(1, per_cu) * std::max(1, n_cu);
    return GRAV_OK;
}

}  // namespace grav
