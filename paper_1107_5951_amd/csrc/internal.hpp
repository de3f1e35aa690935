// Internal plan layout and shared device helpers of libgrav.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "grav.h"

namespace grav {

constexpr int kMaxP = 16;
constexpr int kMaxLevels = 10;

// M2L: 16-column blocks per wave (1, 2 or 4) for the FP32 and FP64
// kernels: each A fragment feeds this many instructions; a tile of 64
// columns holds 4 / NC units.  Small FP64 plans keep one block (two would
// leave one wave per SIMD).
#ifndef GRAV_M2L_NC32
#define GRAV_M2L_NC32 2
#endif
// FP32 plans with at least this many (box, model) columns take four blocks
// per wave (twice the operator reuse, two waves per SIMD instead of three):
// large plans gain, small ones lose their few work items per wave
#ifndef GRAV_M2L_NC32_WIDE
#define GRAV_M2L_NC32_WIDE 4
#endif
#ifndef GRAV_M2L_WIDE_COLUMNS
#define GRAV_M2L_WIDE_COLUMNS 131072
#endif
// FP64 plans with at least this many columns take two blocks per wave: the
// FP64 operators (up to 512 KB each at p = 16) are re-read half as often
// (128^3 x 32 models at p = 14: 1.46 -> 0.79 ms; 256^3 at p = 16: 267 ->
// 131 ms; the 64^3 plan at p = 12, 4,681 columns, is slower with two)
#ifndef GRAV_M2L_NC64_WIDE
#define GRAV_M2L_NC64_WIDE 2
#endif
#ifndef GRAV_M2L_WIDE_COLUMNS64
#define GRAV_M2L_WIDE_COLUMNS64 16384
#endif
#ifndef GRAV_M2L_NC64
#define GRAV_M2L_NC64 1
#endif
// 16-column blocks per wave of the reflection-orbit M2L
#ifndef GRAV_M2L_ORB_NC
#define GRAV_M2L_ORB_NC 2
#endif
// Lowest expansion order that takes the reflection-orbit M2L: it runs 8 x 8
// blocks of 16 x 16 per orbit whatever p is, so at lower orders much of each
// block is padding (256^3 volume, M2L per offset and per orbit: p = 8 4.05
// and 6.79 ms, p = 9 6.77 and 6.83 ms, p = 10 9.31 and 6.82 ms)
#ifndef GRAV_M2L_ORB_MIN_P
#define GRAV_M2L_ORB_MIN_P 10
#endif
// ... and only for plans whose (column, offset) pairs with a source number at
// least this many times their (column, orbit) pairs: an orbit item costs
// 256 instructions per column block at about two thirds of the per-offset
// kernel's MFMA occupancy, an offset item about 156 (break-even near 2.4);
// 256^3 volume workload: M2L 9.31 ms per offset, 6.82 per orbit; 128^3 x 32
// models, stations above the top face: 0.150 and 0.239 ms
#ifndef GRAV_M2L_ORB_MIN_RATIO
#define GRAV_M2L_ORB_MIN_RATIO 2.6
#endif
constexpr int kNumOffsets = 316;   // M2L offsets d with 2 <= |d|_inf <= 3
// The mixed-precision (FP32) forward M2L stores one operator per offset with
// non-negative components (56 of them): the operator of any other offset is
// that of its component-wise absolute value with the signs of a reflection
// applied to its rows and columns (see m2l.hip).  Its offset tables hold the
// operator index plus kReflShift times the reflection bits (x, y, z = bits
// 0, 1, 2).  The FP64 forward M2L stores all 316 operators (reflection bits
// zero): sign flips on 64-bit operands would cost the registers of a second
// wave per SIMD.
constexpr int kCanonOffsets = 56;
constexpr int kReflShift = 512;
constexpr int kClassOffsets = 189; // offsets valid for one child-parity class
constexpr int kTileCols = 64;      // columns (box, model) per M2L tile
constexpr int kMaxLeafCells = 8;     // leaf edge cap: a leaf's densities fit one 512-entry LDS stage
constexpr int kMaxLatticeLeaf = 4;   // largest leaf edge with lattice near-field matrices

struct LevelInfo {
    int l = 0;
    double w = 0.0;                   // box edge
    int s0[3] = {0, 0, 0};            // source block start (root-relative box coords, x,y,z)
    int ns[3] = {0, 0, 0};            // source block size
    int64_t n_src = 0;                // ns[0]*ns[1]*ns[2]
    int64_t me_off = 0;               // offset (in expansions) of this level in the ME array
    int64_t n_tgt = 0;                // boxes holding evaluation points
    int64_t tgt_off = 0;              // offset of this level in the per-target-box arrays
    int64_t class_start[9] = {0};     // class-grouped order boundaries
    int64_t tmap_off = 0;             // offset of this level's target map (source block + halo 3)
    int64_t tchild_off = 0;           // offset of this level's first-child table
    int64_t src_class[8] = {0};       // source boxes of each parity class
    int need_lo[3] = {0, 0, 0};       // box range whose expansions the M2L reads (the
    int need_hi[3] = {-1, -1, -1};    // target boxes' range widened by 3, inclusive)
    // transposed M2L (adjoint): its columns are the source boxes of the
    // column block (the source block within reach of a target box; the
    // whole block at level 2), class-grouped like the forward's target
    // boxes; its B operand is the adjoint LE regathered over the gather
    // region (the target boxes' bounding box within the source block
    // widened by 3)
    int cs0[3] = {0, 0, 0}, cns[3] = {0, 0, 0};
    int64_t col_class_start[9] = {0};
    int gs0[3] = {0, 0, 0}, gns[3] = {0, 0, 0};
    int64_t g_off = 0;                // offset (in boxes) of the level in the gathered buffer
};

// Tiled stages: the forward M2L (its tiles also give the L2L its columns).
enum TileKind { TK_M2L = 0, TK_COUNT };

struct TileRange {
    int64_t off = 0;
    int32_t n = 0;
};

struct Stage {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
};

struct Plan {
    grav_plan_desc d{};
    int device = 0;
    int P = 0, P2 = 0, PS = 0;     // order, p^2, padded stride (multiple of 16)
    int KS = 0;                    // k-steps of 4 covering P2
    int q = 1, nq3 = 1, b = 1;     // quadrature points per axis, per cell, leaf edge in cells
    int L = 0;                     // leaf level
    int B = 1, C = 3;
    double wl = 0.0;               // leaf edge
    double root0[3] = {0, 0, 0};   // root lower corner
    int shift[3] = {0, 0, 0};      // leaves between root corner and the mesh origin
    int64_t M = 0;                 // evaluation points
    int64_t n_spts = 0;            // explicit sources (0: the cells' quadrature points)
    int64_t n_leaf = 0;            // leaves holding evaluation points
    LevelInfo lev[kMaxLevels + 1];
    int64_t n_me = 0, n_le = 0;    // expansions (per model) in the ME / LE arrays
    int64_t n_tbox = 0;            // target boxes over all levels >= 2
    int64_t n_tmap = 0, n_tchild = 0;

    // device buffers
    double *d_points = nullptr;    // [n_points][3] user points (unsorted)
    // explicit sources, sorted by their leaf (dense index in the leaf
    // level's source block): lattice-frame positions, mass per unit input
    // value (volume / h^3, or 1 / h^3), sorted -> user index, and the CSR
    // of each leaf's sources
    double *d_spos = nullptr;      // [n_spts][3]
    double *d_sw = nullptr;        // [n_spts]
    uint32_t *d_sperm = nullptr;   // [n_spts]
    int64_t *d_sstart = nullptr;   // [leaves of the leaf-level source block + 1]
    uint32_t *d_perm = nullptr;    // [M] sorted position -> user index
    double *d_tpos = nullptr;      // [M][3] sorted target positions
    int32_t *d_tleaf = nullptr;    // [M] sorted target -> leaf (index in level-L list)
    int64_t *d_leaf_start = nullptr; // [n_leaf + 1]
    uint32_t *d_tkey = nullptr;    // [n_tbox_all] Morton key of every target box, per level
    int32_t *d_tparent = nullptr;  // [n_tbox_all] index (within its level) of the parent box
    int32_t *d_torder = nullptr;   // [n_tbox_all] class-grouped order -> box index (per level)
    int64_t tbox_off[kMaxLevels + 1] = {0}; // start of each level in the three arrays above
    struct GemmTile *d_tiles = nullptr;            // all M2L tiles
    // per stage: slot 0 = all levels, in launch order (each tile repeated
    // split[k] times); slot l >= 2 = level l's tiles in the unrepeated numbering
    TileRange tiles[TK_COUNT][kMaxLevels + 1];
    int split[TK_COUNT] = {1};
    // stream-K schedule of the forward M2L (see build_tiles): work items
    // (offset index per item, unit by unit), segments {unit, first item,
    // end item, 0} per workgroup (wgseg: CSR over workgroups), per unit its
    // segment slots (CSR), and LE column -> 64 * unit + column in unit
    int32_t m2l_wgs = 0, m2l_ncw = 64;  // workgroups (one wave each); columns per unit
    int32_t m2l_nset = 2;               // operand register sets of the FP32 M2L kernel (1 or 2)
    int32_t m2l_nc = 1;                 // 16-column blocks per wave of the M2L kernel
    int64_t m2l_nseg = 0, m2l_items = 0, m2l_nunit = 0;
    // reflection-orbit M2L (mixed plans with at most 16 coefficients per
    // sign class, p <= 10): work items are (unit, canonical offset) pairs
    bool m2l_orbit = false;
    int32_t m2l_npl = 0;                // (chunk, sub-row) planes of the regathered ME
    float *d_k32o = nullptr;            // [56][8 classes][8 classes][64][4] class-blocked canonical operators
    int32_t *d_orbtab = nullptr;        // [8 classes][56][8 reflections] class offset index or -1
    int32_t *d_ccoef = nullptr;         // [8][16] natural coefficient of (class, position) or -1
    int32_t *d_kmap = nullptr;          // [planes][4] natural coefficient of a regathered value or -1
    float *d_kt32o = nullptr;           // the transposed canonical operators, class-blocked like d_k32o
    int32_t *d_orbtab_t = nullptr;      // transposed M2L: [8 source classes][56][8 reflections] entry or -1
    int32_t *d_m2l_items = nullptr, *d_m2l_segs = nullptr, *d_m2l_wgseg = nullptr;
    int32_t *d_m2l_tseg_start = nullptr, *d_m2l_tsegs = nullptr, *d_m2l_colmap = nullptr;
    // the transposed M2L's schedule, in the same form (columns: source boxes
    // of the column blocks; colmap per column, colbox = its ME column
    // (me box * B + model)); keys/order index the source boxes like
    // d_tkey/d_torder the target boxes; class_off holds (-d, operator of
    // K_d^T) per source class; the operators are K_d^T in the forward's
    // panel layout (56 canonical ones in mixed plans, all 316 in FP64)
    int32_t m2lt_wgs = 0, m2lt_nset = 2, m2lt_nc = 1, m2lt_ncw = 64;
    int64_t m2lt_nseg = 0, m2lt_ncols = 0, m2lt_nunit = 0, m2lt_items = 0, n_leg = 0;
    struct GemmTile *d_m2lt_tiles = nullptr;
    int32_t *d_m2lt_items = nullptr, *d_m2lt_segs = nullptr, *d_m2lt_wgseg = nullptr;
    int32_t *d_m2lt_tseg_start = nullptr, *d_m2lt_tsegs = nullptr, *d_m2lt_colmap = nullptr;
    int64_t *d_m2lt_colbox = nullptr;
    uint32_t *d_skey = nullptr;       // [n_me] Morton key of every source box
    int32_t *d_sorder = nullptr;      // [n_me] column-block class order -> dense index, per level
    int32_t *d_tclass_off = nullptr;  // [8][189][4]
    double *d_kt64 = nullptr;
    float *d_kt32 = nullptr;
    double *d_leg = nullptr;          // regathered adjoint LE (FP32 in mixed plans)
    double *d_partt = nullptr;        // segment slots of the transposed M2L
    // near field of voxel-centre targets by lattice matrices (b <= 4)
    bool lat_near = false;
    int lat_RB = 0, lat_Q = 0;                     // row blocks (C b^3 / 16); chunks of four k steps
    double *d_tl2p = nullptr;                      // [PS/16][RB][64][4] far field (L2P) at the cell centres, FP64
    int64_t *d_lat_tab = nullptr;                  // [27 Q][2] per near chunk: density and operator offsets
    double *d_m2m_sw = nullptr;                    // [8][PS/4][RB][64] M2M as MFMA A fragments (FP64)
    double *d_l2l_sw = nullptr;                    // [8][KS][RB][64] L2L likewise
    double *d_l2l_msw = nullptr;                   // [8][PS/4][RB][64] L2L, as d_m2m_sw (forward, LDS-tiled)
    double *d_m2mt_sw = nullptr;                   // [8][PS/4][RB][64] M2M^T, as d_m2m_sw (adjoint)
    double *d_l2lt_sw = nullptr;                   // [8][PS/4][RB][64] L2L^T, as d_m2m_sw (adjoint)
    double *d_pmt_sw = nullptr;                    // [PS/4][ceil(b^3/16)][64] P2M^T fragments (adjoint)
    double *d_tn64 = nullptr;                      // [27][KS][RB][64] swizzled, FP64 plans
    float *d_tn32 = nullptr;                       // same, mixed plans
    int lat_TQ = 0;                                // adjoint: chunks of the (target, component) contraction
    double *d_tnt64 = nullptr;                     // [27][TQ][ceil(b^3/16)][64][4] transposed near field, FP64
    float *d_tnt32 = nullptr;                      // same, mixed plans
    double *d_tl2pt = nullptr;                     // [TQ][PS/16][64][4] transposed lattice L2P (FP64)
    double *d_w_blk = nullptr;                     // [TQ][4][padded leaves x B][4] adjoint weights per leaf (FP32 in mixed plans)
    int32_t *d_cell_slot = nullptr;                // [ncell] sorted slot of each voxel centre
    hipStream_t bs = nullptr;                      // plan-build stream (non-blocking), only inside grav_plan
    int direct_chunks = 1;                         // source chunks of grav_direct
    double *d_dpart = nullptr;                     // [chunks][M][B][4] its partial sums
    double *d_meg = nullptr;                       // ME regathered for the M2L's B operand (class-split,
                                                   // chunk-major; FP32 in mixed plans)
    double *d_rho_blk = nullptr;                   // [Q][4][padded leaves x B][4] densities per leaf (FP32 in mixed plans)
    int64_t *d_leaf_pend = nullptr;                // [n_leaf] end of the user points of a leaf
    int32_t *d_pt_leaves = nullptr;                // source leaves with user points in their 27 neighbours
    int64_t n_pt_leaves = 0;                       // (any order), for the adjoint's point near field
    int32_t *d_user_leaves = nullptr;              // target leaves holding user points (any order), for
    int64_t n_user_leaves = 0;                     // the point near field                  // workgroups sharing the offsets of one tile
    double *d_part = nullptr;                      // [split][expansions][PS] partial sums
    int32_t *d_class_off = nullptr;  // [8][189][4] (dx, dy, dz, offset id)
    int32_t *d_rclass_off = nullptr; // same for the transposed M2L, keyed by source class
    int32_t *d_tmap = nullptr;       // per level: target-box index over source block + halo 3
    int32_t *d_tchild = nullptr;     // per level: first child (in level l+1) of each box, + sentinel
    struct DevGeom *d_geom = nullptr;

    double *d_pm = nullptr;        // [b^3][PS] lattice P2M
    double *d_pm_sw = nullptr;     // [b^3/4][RB][64] the same as MFMA A fragments (FP64)
    double *d_m2m = nullptr;       // [8][PS][PS] M2M per child octant, row-major [out][in] (adjoint)
    double *d_l2l = nullptr;       // [8][PS][PS] L2L per child octant, row-major [out][in] (adjoint)
    double *d_k64 = nullptr;       // forward M2L operators as MFMA A fragments (FP64 plans: all 316)
    float *d_k32 = nullptr;        // same, FP32 (mixed plans: the 56 stored operators)

    double *d_me = nullptr;        // [n_me][B][PS]
    double *d_le = nullptr;        // [n_tbox][B][PS]
    double *d_near = nullptr;      // [M][B][4] near field (phi, gx, gy, gz), sorted order

    int64_t m2l_pairs = 0;         // box pairs translated by M2L (per model)
    int64_t p2p_pairs = 0;         // point pairs of the near-field sum (per model)
    size_t bytes_resident = 0, bytes_call = 0;
    hipStream_t last_stream = nullptr;
    hipEvent_t done = nullptr;
    bool has_pending = false;

    bool profiling = false;
    std::vector<Stage> stages;
    int n_stage_used = 0;
};

#define GRAV_HIP(call)                                                                 \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return GRAV_EDEVICE;                                                       \
    } while (0)

#define GRAV_CHECK(call)                                                               \
    do {                                                                               \
        grav_status s_ = (call);                                                       \
        if (s_ != GRAV_OK)                                                             \
            return s_;                                                                 \
    } while (0)

// Morton interleave of 10-bit coordinates (x in bit 0).
__host__ __device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x000003ffu;
    return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Device scans / sorts (sort.hip).
grav_status scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                               hipStream_t s);
size_t scan_tmp_words(int64_t n);
grav_status radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp,
                             uint32_t *vals_tmp, int64_t n, int bits, uint32_t *scratch,
                             hipStream_t s);
size_t radix_scratch_words(int64_t n);

// Stage helpers (eval.hip)
void stage_begin(Plan *p, const char *name, hipStream_t s);
void stage_end(Plan *p, hipStream_t s);

}  // namespace grav
