// Forward evaluation: upward sweep (P2M, M2M), downward sweep (M2L, L2L),
// evaluation (L2P and the near-field direct sum), following the stages of
// the FMM in Sec. 2.3.  All geometry is in the lattice frame (cell units,
// mesh origin at 0); see plan.hip.
#include <algorithm>
#include <cmath>

#include "harmonics.hpp"
#include "resolve.hpp"

#ifndef GRAV_M2M_LDS_MIN_WG
#define GRAV_M2M_LDS_MIN_WG 256  // 64-column M2M tiles from this many workgroups on
#endif

namespace grav {

// --------------------------------------------------------------------------
// P2M on the lattice: the scaled ME of a leaf is a fixed linear map of its
// b^3 cell densities (all leaves share the point layout), ME = Pm^T rho_leaf,
// a GEMM with rows = coefficients, contraction = the leaf's cells and
// columns = (model, leaf), leaves fastest.  FP64 MFMA: a wave owns 16
// columns and all row blocks; k step kv and sub-row kr take cell 4 kv + kr.
// With b = 4 the 64 lanes of one k step read one contiguous run of 64 cell
// densities (16 consecutive leaves along x, four cells each), and every
// density is read once.
// --------------------------------------------------------------------------
template <int RB>
__global__ void __launch_bounds__(64) k_p2m_mfma(DevGeom g, const double *rho, const double *A, int KV, double *me)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    constexpr int KB = 8;  // density loads issued together
    const DevLev &lv = g.lev[g.L];
    const int lane = threadIdx.x;
    const int b = g.b, b2 = b * b, b3 = b2 * b;
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t col = (int64_t)blockIdx.x * 16 + (lane & 15);
    const bool cvalid = col < nleaf * g.B;
    const int bm = cvalid ? (int)(col / nleaf) : 0;
    const int64_t leaf = cvalid ? col - (int64_t)bm * nleaf : 0;
    const int lx = (int)(leaf % lv.ns[0]), ly = (int)((leaf / lv.ns[0]) % lv.ns[1]),
              lz = (int)(leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
    const int cx = (lv.s0[0] + lx - g.shift[0]) * b, cy = (lv.s0[1] + ly - g.shift[1]) * b,
              cz = (lv.s0[2] + lz - g.shift[2]) * b;
    const double *rb0 = rho + (int64_t)bm * ncell;
    const int kr = lane >> 4;
    vec4 acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
        acc[r] = vec4{0, 0, 0, 0};
    for (int k0 = 0; k0 < KV; k0 += KB) {
        double rv[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int v = 4 * (k0 + u) + kr;
            rv[u] = 0.0;
            if (cvalid && k0 + u < KV && v < b3) {
                const int ix = cx + v % b, iy = cy + (v / b) % b, iz = cz + v / b2;
                if (ix >= 0 && iy >= 0 && iz >= 0 && ix < g.n[0] && iy < g.n[1] && iz < g.n[2])
                    rv[u] = rb0[((int64_t)iz * g.n[1] + iy) * g.n[0] + ix];
            }
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            if (k0 + u >= KV)
                break;
            const double *ap = A + (int64_t)(k0 + u) * RB * 64 + lane;
#pragma unroll
            for (int r = 0; r < RB; ++r)
                acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[r * 64], rv[u], acc[r], 0, 0, 0);
        }
    }
    if (!cvalid)
        return;
    // output fragment: column lane % 16, rows lane / 16 + 4 r of each block
    double *dst = me + ((lv.me_off + leaf) * g.B + bm) * PS;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            dst[16 * r + kr + 4 * i] = acc[r][i];
}

// The same GEMM with the operator staged through LDS: a workgroup of four
// waves owns 64 NCG columns (each wave NCG blocks of 16) and all row
// blocks; the operator passes through LDS in double-buffered chunks of four
// k steps (one barrier per chunk), so each chunk is read from L2 once per
// 64 NCG columns instead of once per 16.
template <int RB, int NCG>
__global__ void __launch_bounds__(256) k_p2m_lds(DevGeom g, const double *rho, const double *A, int KV, double *me)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    constexpr int CH = 4 * RB * 64;  // doubles per chunk
    __shared__ double sa[2][CH];
    const DevLev &lv = g.lev[g.L];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kr = lane >> 4;
    const int b = g.b, b2 = b * b, b3 = b2 * b;
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    bool cvalid[NCG];
    int bm[NCG], cx[NCG], cy[NCG], cz[NCG];
    int64_t leaf[NCG];
#pragma unroll
    for (int c = 0; c < NCG; ++c) {
        const int64_t col = ((int64_t)blockIdx.x * 4 + wave) * 16 * NCG + c * 16 + (lane & 15);
        cvalid[c] = col < nleaf * g.B;
        bm[c] = cvalid[c] ? (int)(col / nleaf) : 0;
        leaf[c] = cvalid[c] ? col - (int64_t)bm[c] * nleaf : 0;
        const int lx = (int)(leaf[c] % lv.ns[0]), ly = (int)((leaf[c] / lv.ns[0]) % lv.ns[1]),
                  lz = (int)(leaf[c] / ((int64_t)lv.ns[0] * lv.ns[1]));
        cx[c] = (lv.s0[0] + lx - g.shift[0]) * b;
        cy[c] = (lv.s0[1] + ly - g.shift[1]) * b;
        cz[c] = (lv.s0[2] + lz - g.shift[2]) * b;
    }
    auto density = [&](int c, int ks) -> double {
        const int v = 4 * ks + kr;
        if (!cvalid[c] || ks >= KV || v >= b3)
            return 0.0;
        const int ix = cx[c] + v % b, iy = cy[c] + (v / b) % b, iz = cz[c] + v / b2;
        if (ix < 0 || iy < 0 || iz < 0 || ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2])
            return 0.0;
        return rho[(int64_t)bm[c] * ncell + ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix];
    };
    // chunk j holds k steps 4 j .. 4 j + 3 (those past KV read zero)
    auto load_chunk = [&](int j, double (&ra)[RB]) {
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int e = i * 256 + tid;
            const int ks = 4 * j + e / (RB * 64);
            ra[i] = ks < KV ? A[(int64_t)4 * j * RB * 64 + e] : 0.0;
        }
    };
    const int NCH = (KV + 3) / 4;
    vec4 acc[NCG][RB];
#pragma unroll
    for (int c = 0; c < NCG; ++c)
#pragma unroll
        for (int r = 0; r < RB; ++r)
            acc[c][r] = vec4{0, 0, 0, 0};
    double ra[RB];
    load_chunk(0, ra);
#pragma unroll
    for (int i = 0; i < RB; ++i)
        sa[0][i * 256 + tid] = ra[i];
    double bv[NCG][4];
#pragma unroll
    for (int c = 0; c < NCG; ++c)
#pragma unroll
        for (int u = 0; u < 4; ++u)
            bv[c][u] = density(c, u);
    __syncthreads();
    for (int j = 0; j < NCH; ++j) {
        const int buf = j & 1;
        const bool more = j + 1 < NCH;
        if (more)
            load_chunk(j + 1, ra);
        double cur[NCG][4];
#pragma unroll
        for (int c = 0; c < NCG; ++c)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                cur[c][u] = bv[c][u];
                if (more)
                    bv[c][u] = density(c, 4 * (j + 1) + u);
            }
        // the densities as the A operand and the operator as B: the product
        // is the transposed tile (rows = columns, columns = coefficients),
        // so that the stores below write whole rows of 16 coefficients
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const double a = sa[buf][(u * RB + r) * 64 + lane];
#pragma unroll
                for (int c = 0; c < NCG; ++c)
                    acc[c][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[c][u], a, acc[c][r], 0, 0, 0);
            }
        if (more) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
                sa[buf ^ 1][i * 256 + tid] = ra[i];
        }
        __syncthreads();
    }
    // output fragment: rows kr + 4 i = columns of the block, column lane % 16
    // = coefficient 16 r + lane % 16: 16 lanes write 128 contiguous bytes
#pragma unroll
    for (int c = 0; c < NCG; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t col = ((int64_t)blockIdx.x * 4 + wave) * 16 * NCG + c * 16 + kr + 4 * i;
            if (col >= nleaf * g.B)
                continue;
            const int cbm = (int)(col / nleaf);
            double *dst = me + ((lv.me_off + col - (int64_t)cbm * nleaf) * g.B + cbm) * PS + (lane & 15);
#pragma unroll
            for (int r = 0; r < RB; ++r)
                dst[16 * r] = acc[c][r][i];
        }
}

// --------------------------------------------------------------------------
// M2M on MFMA (FP64): ME[parent] = sum over the 8 children c of T_c ME[child],
// a GEMM with M = p^2 rows, K = 8 p^2 and columns = (parent box, model).
// The operator is stored as 8 RB chunks of four k steps each (all row
// blocks of a k step together, 64 lanes per fragment); within a child the
// contraction order is kr * PS/4 + ks, so a lane's four k steps of a chunk
// are four consecutive coefficients of its child's expansion.  A child
// outside the source block contributes zero.
//
// Large levels: k_m2m_lds.  A workgroup owns 64 columns (16 per wave) and
// all row blocks; the chunks of the operator pass through LDS (double
// buffered, one barrier per chunk), so each is read from L2 once per 64
// columns instead of once per wave, and each wave streams its columns'
// child expansions once.
// --------------------------------------------------------------------------
template <int RB>
__global__ void __launch_bounds__(256) k_m2m_lds(DevGeom g, int l, const double *A, double *me)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    constexpr int K4 = PS / 4;
    constexpr int CH = 4 * RB * 64;  // doubles per chunk: 4 k steps x RB blocks x 64 lanes
    constexpr int NCH = 8 * RB;      // chunks: 8 children x RB chunks of 4 k steps
    __shared__ double sa[2][CH];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const DevLev &lp = g.lev[l];
    const DevLev &lc = g.lev[l + 1];
    const int64_t nbox = (int64_t)lp.ns[0] * lp.ns[1] * lp.ns[2];
    const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + (lane & 15);
    const bool cvalid = col < nbox * g.B;
    const int64_t box = cvalid ? col / g.B : 0;
    const int bm = cvalid ? (int)(col % g.B) : 0;
    const int px = lp.s0[0] + (int)(box % lp.ns[0]);
    const int py = lp.s0[1] + (int)((box / lp.ns[0]) % lp.ns[1]);
    const int pz = lp.s0[2] + (int)(box / ((int64_t)lp.ns[0] * lp.ns[1]));
    const int kr = lane >> 4;
    // the column's expansion of child c (nullptr: no such child)
    auto child = [&](int c) -> const double2 * {
        const int64_t ci = cvalid ? dense_index(lc, 2 * px + (c & 1), 2 * py + ((c >> 1) & 1),
                                                2 * pz + ((c >> 2) & 1))
                                  : -1;
        return ci >= 0 ? (const double2 *)(me + ((lc.me_off + ci) * g.B + bm) * PS + kr * K4) : nullptr;
    };
    vec4 acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
        acc[r] = vec4{0, 0, 0, 0};
    double ra[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
        ra[i] = A[i * 256 + tid];
#pragma unroll
    for (int i = 0; i < RB; ++i)
        sa[0][i * 256 + tid] = ra[i];
    const double2 *bp = child(0);
    double2 b01 = bp ? bp[0] : double2{0.0, 0.0};
    double2 b23 = bp ? bp[1] : double2{0.0, 0.0};
    __syncthreads();
    for (int j = 0; j < NCH; ++j) {
        const int buf = j & 1;
        const bool more = j + 1 < NCH;
        if (more) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
                ra[i] = A[(int64_t)(j + 1) * CH + i * 256 + tid];
        }
        const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
        if (more) {
            const int qn = (j + 1) % RB;
            if (qn == 0)
                bp = child((j + 1) / RB);
            b01 = bp ? bp[2 * qn] : double2{0.0, 0.0};
            b23 = bp ? bp[2 * qn + 1] : double2{0.0, 0.0};
        }
        // the expansions as the A operand and the operator as B: the product
        // is the transposed tile (rows = columns, columns = coefficients)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < RB; ++r)
                acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[u], sa[buf][(u * RB + r) * 64 + lane], acc[r], 0, 0,
                                                             0);
        if (more) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
                sa[buf ^ 1][i * 256 + tid] = ra[i];
        }
        __syncthreads();
    }
    // output fragment: rows kr + 4 i = columns of the wave, column lane % 16
    // = coefficient 16 r + lane % 16: 16 lanes write 128 contiguous bytes
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t oc = (int64_t)blockIdx.x * 64 + wave * 16 + kr + 4 * i;
        if (oc >= nbox * g.B)
            continue;
        double *dst = me + (lp.me_off * g.B + oc) * PS + (lane & 15);
#pragma unroll
        for (int r = 0; r < RB; ++r)
            dst[16 * r] = acc[r][i];
    }
}

// Small levels (too few columns to fill the chip with 64-column tiles):
// k_m2m_split.  A workgroup owns 16 columns and one 16-row block; its eight
// waves take one child each, so every wave runs PS/4 MFMAs behind a single
// round of loads, and the eight partial fragments are added through LDS in
// child order.
template <int RB>
__global__ void __launch_bounds__(512) k_m2m_split(DevGeom g, int l, const double *A, double *me)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    __shared__ double red[8][256];
    constexpr int PS = 16 * RB;
    constexpr int K4 = PS / 4;
    const int lane = threadIdx.x & 63;
    const int c = threadIdx.x >> 6;  // the wave's child
    const DevLev &lp = g.lev[l];
    const DevLev &lc = g.lev[l + 1];
    const int64_t cg = blockIdx.x / RB;
    const int rb = (int)(blockIdx.x % RB);
    const int64_t nbox = (int64_t)lp.ns[0] * lp.ns[1] * lp.ns[2];
    const int64_t col = cg * 16 + (lane & 15);
    const bool cvalid = col < nbox * g.B;
    const int64_t box = cvalid ? col / g.B : 0;
    const int bm = cvalid ? (int)(col % g.B) : 0;
    const int px = lp.s0[0] + (int)(box % lp.ns[0]);
    const int py = lp.s0[1] + (int)((box / lp.ns[0]) % lp.ns[1]);
    const int pz = lp.s0[2] + (int)(box / ((int64_t)lp.ns[0] * lp.ns[1]));
    const int kr = lane >> 4;
    const int64_t ci =
        cvalid ? dense_index(lc, 2 * px + (c & 1), 2 * py + ((c >> 1) & 1), 2 * pz + ((c >> 2) & 1)) : -1;
    vec4 acc = vec4{0, 0, 0, 0};
    if (__ballot(ci >= 0) != 0ull) {
        const double2 *bp = (const double2 *)(me + (ci >= 0 ? ((lc.me_off + ci) * g.B + bm) * PS : 0) + kr * K4);
        const double *ap = A + (int64_t)c * PS * PS + rb * 64 + lane;  // k step ks at ap[ks * RB * 64]
        constexpr int U = RB < 8 ? RB : 8;  // chunks of four k steps loaded together
        for (int q0 = 0; q0 < RB; q0 += U) {
            double av[U][4];
            double2 bb[U][2];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = min(q0 + u, RB - 1);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    av[u][k] = ap[(int64_t)(4 * q + k) * RB * 64];
                bb[u][0] = ci >= 0 ? bp[2 * q] : double2{0.0, 0.0};
                bb[u][1] = ci >= 0 ? bp[2 * q + 1] : double2{0.0, 0.0};
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = q0 + u < RB;
                const double bv[4] = {in ? bb[u][0].x : 0.0, in ? bb[u][0].y : 0.0, in ? bb[u][1].x : 0.0,
                                      in ? bb[u][1].y : 0.0};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][k], bv[k], acc, 0, 0, 0);
            }
        }
    }
    // the eight waves' fragments share one lane layout: add them in child order
#pragma unroll
    for (int r = 0; r < 4; ++r)
        red[c][lane * 4 + r] = acc[r];
    __syncthreads();
    if (c == 0 && cvalid) {
        double *dst = me + ((lp.me_off + box) * g.B + bm) * PS;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double v = red[0][lane * 4 + r];
#pragma unroll
            for (int w = 1; w < 8; ++w)
                v += red[w][lane * 4 + r];
            dst[16 * rb + kr + 4 * r] = v;
        }
    }
}

// --------------------------------------------------------------------------
// L2L on MFMA (FP64): LE[child] += T_c LE[parent] for the target boxes of
// level l, grouped by child octant c (the M2L tiles of the level: same
// columns, one matrix per tile).  Four waves of 16 columns per workgroup.
// --------------------------------------------------------------------------
// L2L, LDS-tiled (FP64 MFMA): a workgroup takes one M2L tile of a level (64
// target-box columns of one child octant, so one matrix) with all row
// blocks; the matrix passes through LDS in double-buffered chunks of four k
// steps, each wave streams its 16 columns' parent expansions once and adds
// the products into the children's LE.
// --------------------------------------------------------------------------
template <int RB>
__global__ void __launch_bounds__(256)
k_l2l_lds(DevGeom g, const GemmTile *tiles, int stride, const int32_t *torder, const int32_t *tparent, const double *A,
          double *le)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    constexpr int K4 = PS / 4;
    constexpr int CH = 4 * RB * 64;
    __shared__ double sa[2][CH];
    const GemmTile tile = tiles[(int64_t)blockIdx.x * stride];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kr = lane >> 4;
    const DevLev &lv = g.lev[tile.level];
    const DevLev &lp = g.lev[tile.level - 1];
    const int cl = wave * 16 + (lane & 15);
    const bool cvalid = cl < tile.ncol;
    const int64_t col = tile.col0 + cl;
    const int bm = (int)(col % g.B);
    int64_t box = 0, par = 0;
    if (cvalid) {
        box = torder[lv.tbox_off + lv.class_start[tile.cls] + col / g.B];
        par = tparent[lv.tbox_off + box];
    }
    const double2 *bp = (const double2 *)(le + ((lp.tgt_off + par) * g.B + bm) * PS + kr * K4);
    const double *Ao = A + (int64_t)tile.cls * PS * PS;
    vec4 acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
        acc[r] = vec4{0, 0, 0, 0};
    double ra[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
        ra[i] = Ao[i * 256 + tid];
#pragma unroll
    for (int i = 0; i < RB; ++i)
        sa[0][i * 256 + tid] = ra[i];
    double2 b01 = cvalid ? bp[0] : double2{0.0, 0.0};
    double2 b23 = cvalid ? bp[1] : double2{0.0, 0.0};
    __syncthreads();
    for (int j = 0; j < RB; ++j) {
        const int buf = j & 1;
        const bool more = j + 1 < RB;
        if (more) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
                ra[i] = Ao[(int64_t)(j + 1) * CH + i * 256 + tid];
        }
        const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
        if (more) {
            b01 = cvalid ? bp[2 * (j + 1)] : double2{0.0, 0.0};
            b23 = cvalid ? bp[2 * (j + 1) + 1] : double2{0.0, 0.0};
        }
        // the parents' expansions as the A operand and the matrix as B: the
        // product is the transposed tile (rows = columns, columns =
        // coefficients)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < RB; ++r)
                acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[u], sa[buf][(u * RB + r) * 64 + lane], acc[r], 0, 0,
                                                             0);
        if (more) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
                sa[buf ^ 1][i * 256 + tid] = ra[i];
        }
        __syncthreads();
    }
    // output fragment: rows kr + 4 i = columns of the wave (their boxes from
    // the lanes that own them), column lane % 16 = coefficient 16 r +
    // lane % 16: 16 lanes add into 128 contiguous bytes
    const int box32 = (int)box;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int oc = kr + 4 * i;
        const int obox = __shfl(box32, oc);
        if (wave * 16 + oc >= tile.ncol)
            continue;
        const int obm = (int)((tile.col0 + wave * 16 + oc) % g.B);
        double *dst = le + ((lv.tgt_off + obox) * g.B + obm) * PS + (lane & 15);
#pragma unroll
        for (int r = 0; r < RB; ++r)
            dst[16 * r] += acc[r][i];
    }
}

// --------------------------------------------------------------------------
// L2L on MFMA (FP64): LE[child] += T_c LE[parent] for the target boxes of
// level l, grouped by child octant c (the M2L tiles of the level: same
// columns, one matrix per tile).  A workgroup takes one tile (four waves of
// 16 columns) and one 16-row block (blockIdx.y), so a level has RB times
// as many workgroups as tiles.
// --------------------------------------------------------------------------
template <int RB>
__global__ void __launch_bounds__(256)
k_l2l_mfma(DevGeom g, const GemmTile *tiles, int stride, const uint32_t *tkey, const int32_t *torder,
           const int32_t *tparent, const double *A, double *le)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    const GemmTile tile = tiles[(int64_t)blockIdx.x * stride];
    const int rb = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const DevLev &lv = g.lev[tile.level];
    const DevLev &lp = g.lev[tile.level - 1];
    const int cl = wave * 16 + (lane & 15);
    const bool cvalid = cl < tile.ncol;
    const int64_t col = tile.col0 + cl;
    const int bm = (int)(col % g.B);
    int64_t box = 0, par = 0;
    if (cvalid) {
        box = torder[lv.tbox_off + lv.class_start[tile.cls] + col / g.B];
        par = tparent[lv.tbox_off + box];
    }
    vec4 acc = vec4{0, 0, 0, 0};
    const int kr = lane >> 4;
    // B: column (lane % 16) of the parent LE, contraction order kr * PS/4 + ks
    const double2 *bp = (const double2 *)(le + (cvalid ? ((lp.tgt_off + par) * g.B + bm) * PS : 0) + kr * (PS / 4));
    const double *ap = A + ((int64_t)tile.cls * RB * RB + rb) * 256;  // [c][q][rb] sets of 4 per lane
    // the child's LE (from the M2L) is read with the operands, not after the
    // products: no other workgroup writes these entries during the launch
    double *dst = le + ((lv.tgt_off + box) * g.B + bm) * PS;
    double old[4] = {0.0, 0.0, 0.0, 0.0};
    if (cvalid) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            old[r] = dst[16 * rb + kr + 4 * r];
    }
    constexpr int U = RB < 8 ? RB : 8;  // chunks of four k steps loaded together
    for (int q0 = 0; q0 < RB; q0 += U) {
        double av[U][4];
        double2 bb[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = min(q0 + u, RB - 1);
            load_frags<double, 4>(ap + (int64_t)q * RB * 256, lane, av[u]);
            bb[u][0] = bp[2 * q];
            bb[u][1] = bp[2 * q + 1];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = cvalid && q0 + u < RB;
            const double bv[4] = {in ? bb[u][0].x : 0.0, in ? bb[u][0].y : 0.0, in ? bb[u][1].x : 0.0,
                                  in ? bb[u][1].y : 0.0};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][k], bv[k], acc, 0, 0, 0);
        }
    }
    if (!cvalid)
        return;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        dst[16 * rb + kr + 4 * r] = old[r] + acc[r];
}

// The multipole expansions regathered for the M2L's B operand, in the
// M2L's element type.  Per level, boxes are ordered by parity class (x
// fastest within a class, see class_split) and the coefficients chunk-major
// in the M2L's interleaved contraction order:
//   out[level][q][kr][pos * B + model][u],  coefficient kmap[4 (4 q + kr) + u]
// (-1: zero), NP = 4 q + kr planes: in natural order coefficient 4 (4 q + u)
// + kr; for the reflection-orbit M2L position 4 u + kr of sign class q.
// The source boxes that one wave's 16 columns read at one interaction offset
// are boxes of a single class with consecutive x, so each B fragment load
// of the M2L covers a few contiguous runs instead of 64 scattered lines.
// Boxes farther than 3 boxes from every target box of their level (for
// surface stations, the deep part of the mesh) are skipped: the M2L reads
// only sources within its interaction offsets.  One thread per (box, model,
// chunk q, sub-row kr).
template <typename T>
__global__ void __launch_bounds__(256) k_me_gather(DevGeom g, const double *me, int64_t n_me, const int32_t *kmap,
                                                   int NP, T *out)
{
    // the coefficient map (at most PS <= 256 entries) through LDS: its
    // loads would otherwise sit in a dependent chain before the gathers
    __shared__ int32_t km[256];
    for (int e = threadIdx.x; e < 4 * NP; e += blockDim.x)
        km[e] = kmap[e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_me * g.B * NP)
        return;
    const int plane = (int)(i % NP);
    const int64_t col = i / NP;  // box * B + model
    const int bm = (int)(col % g.B);
    const int64_t box = col / g.B;
    int l = 2;
    while (l < g.L && box >= g.lev[l + 1].me_off)
        ++l;
    const DevLev &lv = g.lev[l];
    const int64_t j = box - lv.me_off;
    const int ax = lv.s0[0] + (int)(j % lv.ns[0]), ay = lv.s0[1] + (int)((j / lv.ns[0]) % lv.ns[1]),
              az = lv.s0[2] + (int)(j / ((int64_t)lv.ns[0] * lv.ns[1]));
    if (ax < lv.need_lo[0] || ax > lv.need_hi[0] || ay < lv.need_lo[1] || ay > lv.need_hi[1] ||
        az < lv.need_lo[2] || az > lv.need_hi[2])
        return;  // no target box within reach: the M2L never reads this expansion
    int first[3], cnt[3];
    const int64_t pos = class_split(lv, (ax & 1) | ((ay & 1) << 1) | ((az & 1) << 2), first, cnt) +
                        ((int64_t)((az - first[2]) >> 1) * cnt[1] + ((ay - first[1]) >> 1)) * cnt[0] +
                        ((ax - first[0]) >> 1);
    const int64_t nB = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2] * g.B;
    const double *src = me + col * g.PS;
    T *dst = out + lv.me_off * g.B * (4 * NP) + ((int64_t)plane * nB + pos * g.B + bm) * 4;
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = km[4 * plane + u];
        v[u] = k >= 0 ? (T)src[k] : (T)0;
    }
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            dst[u] = v[u];
    }
}
template __global__ void k_me_gather<double>(DevGeom, const double *, int64_t, const int32_t *, int, double *);
template __global__ void k_me_gather<float>(DevGeom, const double *, int64_t, const int32_t *, int, float *);

// out[i] = sum over s < S of part[s * n + i], in order s = 0, 1, ..., in FP64
template <typename T>
__global__ void __launch_bounds__(256) k_sum_parts(const T *part, int S, int64_t n, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double acc = (double)part[i];
    for (int s = 1; s < S; ++s)
        acc += (double)part[(int64_t)s * n + i];
    out[i] = acc;
}
template __global__ void k_sum_parts<double>(const double *, int, int64_t, double *);
template __global__ void k_sum_parts<float>(const float *, int, int64_t, double *);

// LE from the forward M2L's segment slots: element (column, k) of the LE is
// the sum, over the segments of the column's unit in their order, of the
// slot entry (column in unit, k), in FP64.  A unit without segments (no
// source box at any offset) gives zero.
template <typename T>
__global__ void __launch_bounds__(256)
k_m2l_sum(const T *part, const int32_t *colmap, const int32_t *tseg_start, const int32_t *tsegs, int64_t n, int PS,
          int ncw, double *le)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t col = i / PS;
    const int k = (int)(i - col * PS);
    const int32_t m = colmap[col];
    const int t = m >> 6, cl = m & 63;
    const int j0 = tseg_start[t], j1 = tseg_start[t + 1];
    double acc = 0.0;
    // SB slots at a time: their indices, then their values, are loaded
    // together (no chain of dependent loads); the sum stays in slot order.
    // A unit typically spans one or two workers' shares (the 256^3 plan:
    // about 400 items per worker, 189 per unit), so one round usually does.
    constexpr int SB = 4;
    for (int jb = j0; jb < j1; jb += SB) {
        int32_t sl[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u)
            sl[u] = jb + u < j1 ? tsegs[jb + u] : -1;
        T v[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u)
            v[u] = sl[u] >= 0 ? part[((int64_t)sl[u] * ncw + cl) * PS + k] : (T)0;
#pragma unroll
        for (int u = 0; u < SB; ++u)
            if (jb + u < j1)
                acc += (double)v[u];
    }
    le[i] = acc;
}
template __global__ void k_m2l_sum<double>(const double *, const int32_t *, const int32_t *, const int32_t *,
                                           int64_t, int, int, double *);
template __global__ void k_m2l_sum<float>(const float *, const int32_t *, const int32_t *, const int32_t *,
                                          int64_t, int, int, double *);

// --------------------------------------------------------------------------
// Near field (P2P): direct sum over the quadrature points of the cells of the
// 27 leaves around a target leaf (the near term of Eq. (13)); coincident
// pairs are skipped.  One workgroup per target leaf; each neighbour leaf's
// densities are staged in LDS; targets are spread over lanes and, when a leaf
// holds fewer than 256 targets, the sources over several lane groups whose
// partial sums are reduced through LDS.  Output in the lattice frame:
// near[i][model] = (sum m/r, sum m d/r^3).
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_p2p(DevGeom g, const double *rho, const double *tpos, const int64_t *leaf_start,
      const int64_t *leaf_end, const uint32_t *tkey, const int32_t *leaves, double *near)
{
    __shared__ double srho[512];
    __shared__ double red[256][4];
    const DevLev &lv = g.lev[g.L];
    const int64_t leaf = leaves[blockIdx.x];  // the target leaves holding user points
    const int64_t ts = leaf_start[leaf], te = leaf_end[leaf];
    const int64_t nt = te - ts;
    if (nt <= 0)
        return;  // no explicit points in this leaf (uniform over the workgroup)
    const uint32_t key = tkey[lv.tbox_off + leaf];
    const int lc[3] = {(int)compact3(key), (int)compact3(key >> 1), (int)compact3(key >> 2)};
    int corner[3];
    for (int a = 0; a < 3; ++a)
        corner[a] = (lc[a] - g.shift[a]) * g.b;  // cell coords of the leaf corner
    const int b = g.b, b3 = b * b * b;
    // no neighbour leaf inside the source block (e.g. stations far above the
    // mesh): the near field of these targets is zero
    bool any_nb = false;
    for (int nb = 0; nb < 27; ++nb) {
        bool inb = true;
        for (int a = 0; a < 3; ++a) {
            const int sx = lc[a] + (nb / (a == 0 ? 1 : a == 1 ? 3 : 9)) % 3 - 1 - lv.s0[a];
            inb = inb && sx >= 0 && sx < lv.ns[a];
        }
        any_nb = any_nb || inb;
    }
    if (!any_nb) {
        for (int64_t e = threadIdx.x; e < nt * g.B * 4; e += blockDim.x)
            near[ts * g.B * 4 + e] = 0.0;
        return;
    }
    int TC = 1;
    while (TC < nt && TC < 256)
        TC <<= 1;
    const int S = 256 / TC;
    const int t = threadIdx.x;
    const int ti = t % TC, si = t / TC;
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const T go = (T)(0.5 / 1.7320508075688772);  // Gauss point offset, cell units
    for (int bm = 0; bm < g.B; ++bm) {
        for (int64_t c0 = 0; c0 < nt; c0 += TC) {
            const int64_t j = ts + c0 + ti;
            const bool valid = (c0 + ti) < nt;
            T tl[3] = {0, 0, 0};
            if (valid)
                for (int a = 0; a < 3; ++a)
                    tl[a] = (T)(tpos[3 * j + a] - (double)corner[a]);
            T acc[4] = {0, 0, 0, 0};
            for (int nb = 0; nb < 27; ++nb) {
                const int d[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, nb / 9 - 1};
                bool inb = true;
                for (int a = 0; a < 3; ++a) {
                    const int s = lc[a] + d[a] - lv.s0[a];
                    if (s < 0 || s >= lv.ns[a])
                        inb = false;
                }
                if (!inb)
                    continue;  // uniform over the workgroup
                __syncthreads();
                for (int v = t; v < b3; v += 256) {
                    const int ix = corner[0] + d[0] * b + v % b;
                    const int iy = corner[1] + d[1] * b + (v / b) % b;
                    const int iz = corner[2] + d[2] * b + v / (b * b);
                    double r = 0.0;
                    if (ix >= 0 && iy >= 0 && iz >= 0 && ix < g.n[0] && iy < g.n[1] && iz < g.n[2])
                        r = rho[bm * ncell + ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix];
                    srho[v] = r;
                }
                __syncthreads();
                if (!valid)
                    continue;
                for (int v = si; v < b3; v += S) {
                    const T rv = (T)srho[v];
                    if (rv == (T)0)
                        continue;
                    const T cx = tl[0] - (T)(d[0] * b + v % b) - (T)0.5;
                    const T cy = tl[1] - (T)(d[1] * b + (v / b) % b) - (T)0.5;
                    const T cz = tl[2] - (T)(d[2] * b + v / (b * b)) - (T)0.5;
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
            }
            // reduce the S source groups
            __syncthreads();
            for (int c = 0; c < 4; ++c)
                red[t][c] = (double)acc[c];
            __syncthreads();
            if (si == 0 && valid) {
                double s4[4] = {0, 0, 0, 0};
                for (int k = 0; k < S; ++k)
                    for (int c = 0; c < 4; ++c)
                        s4[c] += red[k * TC + ti][c];
                double *o = near + (j * g.B + bm) * 4;
                for (int c = 0; c < 4; ++c)
                    o[c] = s4[c];
            }
        }
    }
}

// --------------------------------------------------------------------------
// Explicit sources (scattered points with volumes).  P2M: the expansion of
// a leaf is the sum over its sources of the mass times the multipole basis
// at the source (the lattice P2M's basis: R_n^0, Re R_n^m, -Im R_n^m at
// u = (x - centre) / b).  One workgroup per (leaf of the source block, MG
// models): sources in chunks of kSrcChunk, their harmonics and masses in
// LDS, every thread adding the products of the (model, coefficient) sums it
// owns in source order (deterministic).
// --------------------------------------------------------------------------
constexpr int kSrcChunk = 24, kSrcModels = 4;

template <int MG>
__global__ void __launch_bounds__(256)
k_p2m_src(DevGeom g, const double *spos, const double *sw, const uint32_t *sperm, const int64_t *sstart,
          int64_t nsrc, const double *rho, double *me)
{
    extern __shared__ double sh[];
    constexpr int TC = kSrcChunk;
    const int P2 = g.P2;
    double *H = sh;            // [TC][P2] harmonics of the chunk's sources
    double *W = sh + TC * P2;  // [TC][MG] their masses
    const int64_t leaf = blockIdx.x;
    const int bm0 = blockIdx.y * MG;
    const int tid = threadIdx.x;
    const DevLev &lv = g.lev[g.L];
    const int lx = (int)(leaf % lv.ns[0]), ly = (int)((leaf / lv.ns[0]) % lv.ns[1]),
              lz = (int)(leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
    const double inv_b = 1.0 / (double)g.b;
    const double centre[3] = {(lx + 0.5) * g.b, (ly + 0.5) * g.b, (lz + 0.5) * g.b};
    const int64_t ts = sstart[leaf], te = sstart[leaf + 1];
    const int NO = MG * P2;  // sums (model, h), o = mg P2 + h
    constexpr int NJ = MG;   // sums per thread (p^2 <= 256)
    double acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        acc[j] = 0.0;
    for (int64_t j0 = ts; j0 < te; j0 += TC) {
        const int nt = (int)min((int64_t)TC, te - j0);
        if (tid < nt) {
            const int64_t i = j0 + tid;
            regular_harmonics(g.P, (spos[3 * i + 0] - centre[0]) * inv_b, (spos[3 * i + 1] - centre[1]) * inv_b,
                              (spos[3 * i + 2] - centre[2]) * inv_b, H + tid * P2, 1);
        }
        for (int i = tid; i < nt * MG; i += 256) {
            const int t = i / MG, bm = bm0 + i % MG;
            W[i] = bm < g.B ? rho[(int64_t)bm * nsrc + sperm[j0 + t]] * sw[j0 + t] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int o = tid + 256 * j;
            if (o < NO) {
                const int h = o % P2, mg = o / P2;
                double v = acc[j];
                for (int t = 0; t < nt; ++t)
                    v += H[t * P2 + h] * W[t * MG + mg];
                acc[j] = v;
            }
        }
        __syncthreads();
    }
    // coefficient h: the real parts as summed, the imaginary parts negated
    // (conjugate harmonic); padding coefficients zero
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int o = tid + 256 * j;
        if (o < NO) {
            const int h = o % P2, bm = bm0 + o / P2;
            if (bm < g.B) {
                int n = 0;
                while ((n + 1) * (n + 1) <= h)
                    ++n;
                const int r = h - n * n;
                const bool im = r > 0 && (r & 1) == 0;
                me[((lv.me_off + leaf) * g.B + bm) * g.PS + h] = im ? -acc[j] : acc[j];
            }
        }
    }
    for (int i = tid; i < MG * (g.PS - P2); i += 256) {
        const int bm = bm0 + i / (g.PS - P2), k = P2 + i % (g.PS - P2);
        if (bm < g.B)
            me[((lv.me_off + leaf) * g.B + bm) * g.PS + k] = 0.0;
    }
}

// Near field with explicit sources: direct sum over the sources of the 27
// leaves around a target leaf (the near term of Eq. (13)), coincident pairs
// skipped.  One workgroup per target leaf; each neighbour leaf's sources are
// staged in LDS in chunks of 256 (positions relative to the target leaf's
// corner, and masses); targets over lanes, and when a leaf holds fewer than
// 256 targets, sources over several lane groups reduced through LDS in a
// fixed order.  Output as k_p2p: near = (sum m/r, sum m d/r^3), lattice frame.
template <typename T>
__global__ void __launch_bounds__(256)
k_p2p_src(DevGeom g, const double *rho, const double *spos, const double *sw, const uint32_t *sperm,
          const int64_t *sstart, int64_t nsrc, const double *tpos, const int64_t *leaf_start, const int64_t *leaf_end,
          const uint32_t *tkey, const int32_t *leaves, double *near)
{
    __shared__ T sp[256][4];
    __shared__ double red[256][4];
    const DevLev &lv = g.lev[g.L];
    const int64_t leaf = leaves[blockIdx.x];  // the target leaves holding user points
    const int64_t ts = leaf_start[leaf], te = leaf_end[leaf];
    const int64_t nt = te - ts;
    if (nt <= 0)
        return;
    const uint32_t key = tkey[lv.tbox_off + leaf];
    const int lc[3] = {(int)compact3(key), (int)compact3(key >> 1), (int)compact3(key >> 2)};
    double corner[3];
    for (int a = 0; a < 3; ++a)
        corner[a] = (double)((lc[a] - g.shift[a]) * g.b);
    int TC = 1;
    while (TC < nt && TC < 256)
        TC <<= 1;
    const int S = 256 / TC;
    const int t = threadIdx.x;
    const int ti = t % TC, si = t / TC;
    for (int bm = 0; bm < g.B; ++bm) {
        for (int64_t c0 = 0; c0 < nt; c0 += TC) {
            const int64_t j = ts + c0 + ti;
            const bool valid = (c0 + ti) < nt;
            T tl[3] = {0, 0, 0};
            if (valid)
                for (int a = 0; a < 3; ++a)
                    tl[a] = (T)(tpos[3 * j + a] - corner[a]);
            T acc[4] = {0, 0, 0, 0};
            for (int nb = 0; nb < 27; ++nb) {
                const int d[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, nb / 9 - 1};
                int r[3];
                bool inb = true;
                for (int a = 0; a < 3; ++a) {
                    r[a] = lc[a] + d[a] - lv.s0[a];
                    inb = inb && r[a] >= 0 && r[a] < lv.ns[a];
                }
                if (!inb)
                    continue;  // uniform over the workgroup
                const int64_t jl = ((int64_t)r[2] * lv.ns[1] + r[1]) * lv.ns[0] + r[0];
                const int64_t sa = sstart[jl], se = sstart[jl + 1];
                for (int64_t s0 = sa; s0 < se; s0 += 256) {
                    const int ns = (int)min((int64_t)256, se - s0);
                    __syncthreads();
                    if (t < ns) {
                        const int64_t i = s0 + t;
                        for (int a = 0; a < 3; ++a)
                            sp[t][a] = (T)(spos[3 * i + a] - corner[a]);
                        sp[t][3] = (T)(rho[(int64_t)bm * nsrc + sperm[i]] * sw[i]);
                    }
                    __syncthreads();
                    if (!valid)
                        continue;
                    for (int v = si; v < ns; v += S) {
                        const T cx = tl[0] - sp[v][0], cy = tl[1] - sp[v][1], cz = tl[2] - sp[v][2];
                        const T r2 = cx * cx + cy * cy + cz * cz;
                        if (r2 > coincident2<T>()) {
                            const T ri = rsqrt_t(r2);
                            const T m = sp[v][3] * ri;
                            const T m3 = m * ri * ri;
                            acc[0] += m;
                            acc[1] += m3 * cx;
                            acc[2] += m3 * cy;
                            acc[3] += m3 * cz;
                        }
                    }
                }
            }
            __syncthreads();
            for (int c = 0; c < 4; ++c)
                red[t][c] = (double)acc[c];
            __syncthreads();
            if (si == 0 && valid) {
                double s4[4] = {0, 0, 0, 0};
                for (int k = 0; k < S; ++k)
                    for (int c = 0; c < 4; ++c)
                        s4[c] += red[k * TC + ti][c];
                double *o = near + (j * g.B + bm) * 4;
                for (int c = 0; c < 4; ++c)
                    o[c] = s4[c];
            }
        }
    }
}

// --------------------------------------------------------------------------
// Densities in leaf blocks for the lattice near field, in the element type
// of the near-field contraction.  Cell v of a leaf (x fastest, v < b^3) is
// contraction index v = kr * 4Q + 4 q + u (Q chunks of four k steps per
// instruction sub-row kr); the blocks are stored chunk-major,
//   blk[q][kr][pl * B + model][u],
// pl = leaf index in the source block padded by one leaf on every side, so
// that the 16 columns of a wave (consecutive leaves) read four contiguous
// runs per chunk.  The padding and cells outside the mesh stay zero.  One
// thread per cell.
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_rho_blocks(DevGeom g, const double *rho, int Qn, int64_t nplB, T *blk)
{
    const DevLev &lv = g.lev[g.L];
    const int b = g.b, b2 = b * b, b3 = b2 * b;
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf * g.B * b3)
        return;
    const int v = (int)(i % b3);
    const int bm = (int)((i / b3) % g.B);
    const int64_t leaf = i / ((int64_t)b3 * g.B);
    const int lx = (int)(leaf % lv.ns[0]), ly = (int)((leaf / lv.ns[0]) % lv.ns[1]),
              lz = (int)(leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
    const int ix = lx * b + v % b, iy = ly * b + (v / b) % b, iz = lz * b + v / b2;
    double r = 0.0;
    if (ix < g.n[0] && iy < g.n[1] && iz < g.n[2])
        r = rho[(int64_t)bm * g.n[0] * g.n[1] * g.n[2] + ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix];
    const int64_t pl = ((int64_t)(lz + 1) * (lv.ns[1] + 2) + (ly + 1)) * (lv.ns[0] + 2) + (lx + 1);
    const int kr = v / (4 * Qn), q = (v % (4 * Qn)) / 4, u = v % 4;
    blk[((int64_t)(q * 4 + kr) * nplB + pl * g.B + bm) * 4 + u] = (T)r;
}

// Lattice near-field tile: GRAV_NEAR_RW32 (FP32) or GRAV_NEAR_RW64 (FP64)
// row blocks x GRAV_NEAR_CW column blocks of 16, a tile per wave on plans
// with at least GRAV_NEAR_WAVE_TILES tiles, else a tile per workgroup of
// four waves; chunks per software-pipeline step.
#ifndef GRAV_NEAR_WAVE_TILES
#define GRAV_NEAR_WAVE_TILES 8192
#endif
#ifndef GRAV_NEAR_RW32
#define GRAV_NEAR_RW32 4
#endif
#ifndef GRAV_NEAR_RW64
#define GRAV_NEAR_RW64 2
#endif
#ifndef GRAV_NEAR_CW
#define GRAV_NEAR_CW 2
#endif
#ifndef GRAV_NEAR_DEPTH32
#define GRAV_NEAR_DEPTH32 2
#endif
#ifndef GRAV_NEAR_DEPTH64
#define GRAV_NEAR_DEPTH64 2
#endif

// --------------------------------------------------------------------------
// The voxel-centre targets, fused: near field + far field + combine.
// Targets and Gauss points both sit on the lattice, so the near field of a
// leaf's b^3 cell centres is
//   near[leaf] = sum over the 27 neighbour offsets d of  A_d rho[leaf + d],
// with A_d a fixed (C b^3) x b^3 matrix (the direct sum over the same point
// pairs, precomputed in FP64, rows for the C requested output components
// only), and the far field is a fixed (C b^3) x PS matrix applied to the
// leaf's local expansion (L2P at fixed points, FP64).
// Over all leaves these are GEMMs with columns = (leaf, model).
//
// A tile is 16 CW columns x 16 RW rows (CW x RW MFMA blocks, so every
// fragment loaded feeds CW or RW instructions).  NW = 1 (large plans): each
// wave owns a tile, runs its 27 Q near chunks (chunk = neighbour d, four k
// steps) and the far-field chunks, and writes the tile straight to the
// output in descriptor order, G applied.  NW = 4: the four waves of a
// workgroup share one tile and split the contraction (wave w a quarter of
// the near chunks and every fourth far-field chunk); the four partial tiles
// meet in LDS and are added in wave order (fixed, so the result is
// deterministic).  Measured: 256^3 cells at leaf 4^3, 24,576 tiles: 1.82 ms
// with NW = 1 against 1.96 with NW = 4 (the 64 KB reduction buffer held the
// CU to two workgroups); 64^3 cells, 384 tiles: 0.094 ms against 0.053 (too
// few waves to fill the chip).  Operand fragments are group-major sets per (d, q, rb), the
// densities chunk-major (both read with contiguous-kilobyte vector loads).
// --------------------------------------------------------------------------
template <int RW, int CW, typename T, int NW>
__global__ void __launch_bounds__(256)
k_near_lat(DevGeom g, const T *blk, int64_t nplB, const T *A, const int64_t *ctab, int RBn, int Qn,
           const double *Lm, const int32_t *tmap, const double *le, int64_t npts, int nrg, int64_t ntile,
           double *out)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(T)))) T;
    using dvec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    const int lane = threadIdx.x & 63;
    // wave-uniform (scalar registers): everything that depends only on the
    // chunk index below is scalar arithmetic
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // NW = 4: the workgroup's four waves share one tile; NW = 1: each wave
    // owns a tile of its own
    const int64_t tile = NW == 4 ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * 4 + wave;
    if (tile >= ntile)
        return;  // NW = 1 only (no barrier there): the grid's last waves
    const int64_t cg = tile / nrg;
    const int rb0 = (int)(tile % nrg) * RW;
    const DevLev &lv = g.lev[g.L];
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int b = g.b, b2 = b * b, b3 = b2 * b;
    const int px = lv.ns[0] + 2, py = lv.ns[1] + 2;
    const int kr = lane >> 4;
    // this lane's column in each column block
    bool cvalid[CW];
    int bm[CW], lx[CW], ly[CW], lz[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        const int64_t col = (cg * CW + c) * 16 + (lane & 15);
        cvalid[c] = col < nleaf * g.B;
        const int64_t leaf = cvalid[c] ? col / g.B : 0;
        bm[c] = cvalid[c] ? (int)(col % g.B) : 0;
        lx[c] = (int)(leaf % lv.ns[0]);
        ly[c] = (int)((leaf / lv.ns[0]) % lv.ns[1]);
        lz[c] = (int)(leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
    }
    bool rvalid[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r)
        rvalid[r] = rb0 + r < RBn;
    vec4 acc[CW][RW];
    dvec4 far[CW][RW];
#pragma unroll
    for (int c = 0; c < CW; ++c)
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            acc[c][r] = vec4{0, 0, 0, 0};
            far[c][r] = dvec4{0, 0, 0, 0};
        }
    // near chunks [i0, i1) of this wave; the operands of the next chunk are
    // in flight while this chunk's instructions run
    const int NI = 27 * Qn;
    const int i0 = NW == 4 ? wave * NI / 4 : 0, i1 = NW == 4 ? (wave + 1) * NI / 4 : NI;
    // per lane: its column's density block at neighbour offset (0, 0, 0)
    // (padded coordinates) and sub-row kr; a chunk adds a uniform offset
    const T *bbase[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c)
        bbase[c] = blk + ((int64_t)kr * nplB + (((int64_t)lz[c] * py + ly[c]) * px + lx[c]) * g.B + bm[c]) * 4;
    // Chunk i's offsets come from the plan's table (scalar loads).  Rows past
    // the last row block read the last one and columns past the last column
    // read leaf 0 (both in bounds): an output element depends only on its
    // own row and column, and those are never written, so nothing needs
    // zeroing.
    auto loadc = [&](int i, T (&bb)[CW][4], T (&aa)[RW][4]) {
        const int64_t boff = ctab[2 * i], aoff = ctab[2 * i + 1];
#pragma unroll
        for (int c = 0; c < CW; ++c)
            load4(bbase[c] + boff, bb[c]);
        const T *ap = A + aoff;
#pragma unroll
        for (int r = 0; r < RW; ++r)
            load_frags<T, 4>(ap + (int64_t)min(rb0 + r, RBn - 1) * 256, lane, aa[r]);
    };
    auto compute = [&](const T (&bb)[CW][4], const T (&aa)[RW][4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    if constexpr (sizeof(T) == 8)
                        acc[c][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[r][u], bb[c][u], acc[c][r], 0, 0, 0);
                    else
                        acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(aa[r][u], bb[c][u], acc[c][r], 0, 0, 0);
                }
    };
    // Software pipeline over steps of D chunks: each step issues the loads of
    // the next step one by one between its own matrix instructions, so a
    // load has D chunks of instructions (and the other waves' work) to
    // arrive.  The chunks past the last whole step run unpipelined.
    constexpr int D = sizeof(T) == 8 ? GRAV_NEAR_DEPTH64 : GRAV_NEAR_DEPTH32;
    constexpr int NLD = D * (CW + RW * 4 * (int)sizeof(T) / 16), NMF = D * 4 * RW * CW;
    auto load_step = [&](int st, T (&bb)[D][CW][4], T (&aa)[D][RW][4]) {
#pragma unroll
        for (int j = 0; j < D; ++j)
            loadc(i0 + st * D + j, bb[j], aa[j]);
    };
    auto compute_step = [&](const T (&bb)[D][CW][4], const T (&aa)[D][RW][4]) {
#pragma unroll
        for (int j = 0; j < D; ++j)
            compute(bb[j], aa[j]);
    };
    const int nst = (i1 - i0) / D;
    if (nst > 0) {
        T bA[D][CW][4], bB[D][CW][4];
        T aA[D][RW][4], aB[D][RW][4];
        load_step(0, bA, aA);
        __builtin_amdgcn_sched_barrier(0);
        for (int st = 0; st < nst; st += 2) {
            load_step(min(st + 1, nst - 1), bB, aB);
            compute_step(bA, aA);
            interleave_loads<NLD, NMF>();
            __builtin_amdgcn_sched_barrier(0);
            if (st + 1 < nst) {
                load_step(min(st + 2, nst - 1), bA, aA);
                compute_step(bB, aB);
                interleave_loads<NLD, NMF>();
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    for (int i = i0 + nst * D; i < i1; ++i) {
        T bb[CW][4], aa[RW][4];
        loadc(i, bb, aa);
        compute(bb, aa);
    }
    // far field from the leaf's local expansion (FP64 in both precisions):
    // chunks q = wave, wave + 4, ...
    if (g.L >= 2) {
        bool hl[CW];
        const double2 *bp[CW];
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int64_t tl = cvalid[c] ? tmap_lookup(lv, tmap, 3, lv.s0[0] + lx[c], lv.s0[1] + ly[c],
                                                       lv.s0[2] + lz[c])
                                         : -1;
            hl[c] = tl >= 0;
            bp[c] = (const double2 *)(le + (hl[c] ? ((lv.tgt_off + tl) * g.B + bm[c]) * g.PS : 0) + kr * (g.PS / 4));
        }
        const int QL = g.PS / 16;
        for (int q = NW == 4 ? wave : 0; q < QL; q += NW) {
            double bv[CW][4];
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const double2 b01 = bp[c][2 * q], b23 = bp[c][2 * q + 1];
                bv[c][0] = hl[c] ? b01.x : 0.0;
                bv[c][1] = hl[c] ? b01.y : 0.0;
                bv[c][2] = hl[c] ? b23.x : 0.0;
                bv[c][3] = hl[c] ? b23.y : 0.0;
            }
            double av[RW][4];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                if (rvalid[r]) {
                    load_frags<double, 4>(Lm + ((int64_t)q * RBn + rb0 + r) * 256, lane, av[r]);
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        av[r][u] = 0.0;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int r = 0; r < RW; ++r)
#pragma unroll
                    for (int c = 0; c < CW; ++c)
                        far[c][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r][u], bv[c][u], far[c][r], 0, 0, 0);
        }
    }
    // row block R holds targets 16 (R % RBc) + row of output component
    // R / RBc (the row order of both operators, in lattice units); the
    // lane's element k is row 4 kr + k (FP32) or kr + 4 k (FP64)
    const double sg = g.G * g.h, sp = g.G * g.h * g.h;
    const int RBc = (b3 + 15) / 16;
    auto store = [&](int c, int r, auto &&value) {
        if (!cvalid[c] || !rvalid[r])
            return;
        const int comp = (rb0 + r) / RBc, tb = 16 * ((rb0 + r) % RBc);
        const double sc = g.C == 4 && comp == 0 ? sp : sg;
        double *o = out + ((int64_t)bm[c] * g.M + npts) * g.C + comp;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int t = tb + (sizeof(T) == 8 ? kr + 4 * k : 4 * kr + k);
            const int ix = lx[c] * b + t % b, iy = ly[c] * b + (t / b) % b, iz = lz[c] * b + t / b2;
            if (t >= b3 || ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2])
                continue;
            o[(((int64_t)iz * g.n[1] + iy) * g.n[0] + ix) * g.C] = sc * value(k);
        }
    };
    if constexpr (NW == 4) {
        // partial tiles to LDS (FP64), then each wave adds the four partials
        // of its blocks in wave order (fixed, so the result is deterministic)
        __shared__ double red[4][CW * RW * 4][64];
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    red[wave][(c * RW + r) * 4 + k][lane] = (double)acc[c][r][k] + far[c][r][k];
        __syncthreads();
        for (int j = wave; j < CW * RW; j += 4)
            store(j / RW, j % RW, [&](int k) {
                return ((red[0][j * 4 + k][lane] + red[1][j * 4 + k][lane]) + red[2][j * 4 + k][lane]) +
                       red[3][j * 4 + k][lane];
            });
    } else {
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int r = 0; r < RW; ++r)
                store(c, r, [&](int k) { return (double)acc[c][r][k] + far[c][r][k]; });
    }
}

// --------------------------------------------------------------------------
// L2P + combine: far field at each target from its leaf LE (phi and
// g = -grad phi), plus the near field, times G and the lattice-to-physical
// scale, scattered back to descriptor order.  One thread per (target, model),
// targets fastest.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_l2p_combine(DevGeom g, const double *tpos, const int32_t *tleaf, const uint32_t *tkey,
              const uint32_t *perm, const double *le, const double *near, int64_t first_lattice,
              double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.M * g.B)
        return;
    const int bm = (int)(t / g.M);
    const int64_t i = t - (int64_t)bm * g.M;
    const int64_t dst_t = perm[i];
    if (dst_t >= first_lattice)
        return;  // a voxel centre written by the fused lattice kernel
    const DevLev &lv = g.lev[g.L];
    const int64_t leaf = tleaf[i];
    double far[4] = {0, 0, 0, 0};
    if (g.L >= 2) {
        const uint32_t key = tkey[lv.tbox_off + leaf];
        const int lc[3] = {(int)compact3(key), (int)compact3(key >> 1), (int)compact3(key >> 2)};
        const double inv_w = 1.0 / (double)g.b;
        double u[3];
        for (int a = 0; a < 3; ++a) {
            const double centre = ((double)(lc[a] - g.shift[a]) + 0.5) * g.b;
            u[a] = (tpos[3 * i + a] - centre) * inv_w;
        }
        const double *L = le + ((lv.tgt_off + leaf) * g.B + bm) * g.PS;
        l2p_eval(g.P, L, u[0], u[1], u[2], far);
        far[0] *= inv_w;
        const double s = inv_w * inv_w;
        far[1] = -far[1] * s;  // g = -grad phi
        far[2] = -far[2] * s;
        far[3] = -far[3] * s;
    }
    const double *nr = near + (i * g.B + bm) * 4;
    double v[4];
    for (int c = 0; c < 4; ++c)
        v[c] = nr[c] + far[c];
    double *o = out + ((int64_t)bm * g.M + dst_t) * g.C;
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

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------
DevGeom make_geom(const Plan *p)
{
    DevGeom g{};
    for (int l = 0; l <= p->L && l <= kMaxLevels; ++l) {
        const LevelInfo &s = p->lev[l];
        DevLev &d = g.lev[l];
        for (int a = 0; a < 3; ++a) {
            d.s0[a] = s.s0[a];
            d.ns[a] = s.ns[a];
        }
        d.me_off = s.me_off;
        d.tgt_off = s.tgt_off;
        d.tbox_off = p->tbox_off[l];
        for (int c = 0; c < 9; ++c)
            d.class_start[c] = s.class_start[c];
        d.tmap_off = s.tmap_off;
        d.tchild_off = s.tchild_off;
        d.n_tgt = s.n_tgt;
        for (int a = 0; a < 3; ++a) {
            d.need_lo[a] = s.need_lo[a];
            d.need_hi[a] = s.need_hi[a];
        }
    }
    g.L = p->L;
    g.b = p->b;
    g.q = p->q;
    g.P = p->P;
    g.P2 = p->P2;
    g.PS = p->PS;
    g.KS = p->KS;
    g.B = p->B;
    g.C = p->C;
    g.n[0] = p->d.nx;
    g.n[1] = p->d.ny;
    g.n[2] = p->d.nz;
    for (int a = 0; a < 3; ++a)
        g.shift[a] = p->shift[a];
    g.M = p->M;
    g.G = p->d.G;
    g.h = p->d.h;
    return g;
}

void stage_begin(Plan *p, const char *name, hipStream_t s)
{
    if (!p->profiling)
        return;
    if ((int)p->stages.size() <= p->n_stage_used) {
        Stage st;
        (void)hipEventCreate(&st.a);
        (void)hipEventCreate(&st.b);
        p->stages.push_back(st);
    }
    Stage &st = p->stages[p->n_stage_used];
    st.name = name;
    (void)hipEventRecord(st.a, s);
}

void stage_end(Plan *p, hipStream_t s)
{
    if (!p->profiling)
        return;
    (void)hipEventRecord(p->stages[p->n_stage_used].b, s);
    ++p->n_stage_used;
}

template <typename T>
static M2LRun<T> forward_m2l(const Plan *p, const T *K)
{
    M2LRun<T> r;
    r.tiles = (const GemmTile *)(p->d_tiles + p->tiles[TK_M2L][0].off);
    r.keys = (const uint32_t *)p->d_tkey;
    r.order = (const int32_t *)p->d_torder;
    r.class_off = (const int32_t *)p->d_class_off;
    r.K = K;
    r.b_in = reinterpret_cast<const T *>(p->d_meg);
    r.segs = (const int32_t *)p->d_m2l_segs;
    r.wgseg = (const int32_t *)p->d_m2l_wgseg;
    r.items = (const int32_t *)p->d_m2l_items;
    r.part = reinterpret_cast<T *>(p->d_part);
    r.wgs = p->m2l_wgs;
    r.nset = p->m2l_nset;
    r.nc = p->m2l_nc;
    if (sizeof(T) == 4 && p->m2l_orbit) {
        r.K = reinterpret_cast<const T *>(p->d_k32o);
        r.orbtab = (const int32_t *)p->d_orbtab;
        r.ccoef = (const int32_t *)p->d_ccoef;
    }
    return r;
}

static grav_status launch_m2m(Plan *p, const DevGeom &g, int l, hipStream_t s)
{
    const int RB = p->PS / 16;
    const int64_t ncol = p->lev[l].n_src * p->B;
    // 64-column tiles once they give every CU a workgroup or more
    const bool lds = (ncol + 63) / 64 >= GRAV_M2M_LDS_MIN_WG;
    const dim3 grid_lds((unsigned)((ncol + 63) / 64)), grid_split((unsigned)((ncol + 15) / 16 * RB));
#define M2M_CASE(R)                                                                                          \
    case R:                                                                                                  \
        if (lds)                                                                                             \
            hipLaunchKernelGGL((k_m2m_lds<R>), grid_lds, dim3(256), 0, s, g, l, (const double *)p->d_m2m_sw, \
                               p->d_me);                                                                     \
        else                                                                                                 \
            hipLaunchKernelGGL((k_m2m_split<R>), grid_split, dim3(512), 0, s, g, l,                          \
                               (const double *)p->d_m2m_sw, p->d_me);                                        \
        break;
    switch (RB) {
        M2M_CASE(1)
        M2M_CASE(2)
        M2M_CASE(3)
        M2M_CASE(4)
        M2M_CASE(6)
        M2M_CASE(7)
        M2M_CASE(8)
        M2M_CASE(9)
        M2M_CASE(11)
        M2M_CASE(13)
        M2M_CASE(15)
        M2M_CASE(16)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef M2M_CASE
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

static grav_status launch_p2m(Plan *p, const DevGeom &g, const double *rho, hipStream_t s)
{
    const int RB = p->PS / 16;
    const int b3 = p->b * p->b * p->b;
    const int KV = (b3 + 3) / 4;
    const dim3 grid((unsigned)((p->lev[p->L].n_src * p->B + 15) / 16)), blk(64);
    // the LDS-staged GEMM once it gives every CU a few workgroups
    const int64_t ncol = p->lev[p->L].n_src * p->B;
    const bool lds = (ncol + 127) / 128 >= 1024;
    const dim3 grid2((unsigned)((ncol + 127) / 128)), grid1((unsigned)((ncol + 63) / 64));
#define P2M_CASE(R)                                                                             \
    case R:                                                                                     \
        if (lds && R <= 8)                                                                      \
            hipLaunchKernelGGL((k_p2m_lds<R, 2>), grid2, dim3(256), 0, s, g, rho, (const double *)p->d_pm_sw, KV, \
                               p->d_me);                                                        \
        else if (lds)                                                                           \
            hipLaunchKernelGGL((k_p2m_lds<R, 1>), grid1, dim3(256), 0, s, g, rho, (const double *)p->d_pm_sw, KV, \
                               p->d_me);                                                        \
        else                                                                                    \
            hipLaunchKernelGGL((k_p2m_mfma<R>), grid, blk, 0, s, g, rho, (const double *)p->d_pm_sw, KV, p->d_me); \
        break;
    switch (RB) {
        P2M_CASE(1)
        P2M_CASE(2)
        P2M_CASE(3)
        P2M_CASE(4)
        P2M_CASE(6)
        P2M_CASE(7)
        P2M_CASE(8)
        P2M_CASE(9)
        P2M_CASE(11)
        P2M_CASE(13)
        P2M_CASE(15)
        P2M_CASE(16)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef P2M_CASE
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

static grav_status launch_l2l(Plan *p, const DevGeom &g, int l, hipStream_t s)
{
    const TileRange &all = p->tiles[TK_M2L][0];
    const TileRange &r = p->tiles[TK_M2L][l];
    if (r.n == 0)
        return GRAV_OK;
    const int S = p->split[TK_M2L];
    const GemmTile *t0 = (const GemmTile *)(p->d_tiles + all.off) + r.off * S;
    dim3 grid((unsigned)r.n, (unsigned)(p->PS / 16)), blk(256);
    // one workgroup per tile with all row blocks once the level has enough
    // tiles to fill the chip; otherwise one workgroup per (tile, row block)
    const bool tiled = r.n >= GRAV_M2M_LDS_MIN_WG;
#define L2L_CASE(R)                                                                             \
    case R:                                                                                     \
        if (tiled)                                                                              \
            hipLaunchKernelGGL((k_l2l_lds<R>), dim3((unsigned)r.n), blk, 0, s, g, t0, S,        \
                               (const int32_t *)p->d_torder, (const int32_t *)p->d_tparent,     \
                               (const double *)p->d_l2l_msw, p->d_le);                          \
        else                                                                                    \
            hipLaunchKernelGGL((k_l2l_mfma<R>), grid, blk, 0, s, g, t0, S, (const uint32_t *)p->d_tkey, \
                               (const int32_t *)p->d_torder, (const int32_t *)p->d_tparent,     \
                               (const double *)p->d_l2l_sw, p->d_le);                           \
        break;
    switch (p->PS / 16) {
        L2L_CASE(1)
        L2L_CASE(2)
        L2L_CASE(3)
        L2L_CASE(4)
        L2L_CASE(6)
        L2L_CASE(7)
        L2L_CASE(8)
        L2L_CASE(9)
        L2L_CASE(11)
        L2L_CASE(13)
        L2L_CASE(15)
        L2L_CASE(16)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef L2L_CASE
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

static grav_status launch_near_lat(Plan *p, const DevGeom &g, const double *rho, double *out, hipStream_t s)
{
    const LevelInfo &lv = p->lev[p->L];
    const int b3 = p->b * p->b * p->b;
    const int64_t nfill = lv.n_src * p->B * b3;
    const int64_t nplB = (int64_t)(lv.ns[0] + 2) * (lv.ns[1] + 2) * (lv.ns[2] + 2) * p->B;
    const bool f64 = p->d.precision == GRAV_FP64;
    const dim3 fgrid((unsigned)((nfill + 255) / 256));
    if (f64)
        hipLaunchKernelGGL((k_rho_blocks<double>), fgrid, dim3(256), 0, s, g, rho, p->lat_Q, nplB,
                           p->d_rho_blk);
    else
        hipLaunchKernelGGL((k_rho_blocks<float>), fgrid, dim3(256), 0, s, g, rho, p->lat_Q, nplB,
                           reinterpret_cast<float *>(p->d_rho_blk));
    GRAV_HIP(hipGetLastError());
    const int64_t ncol = lv.n_src * p->B;
    const int RBn = p->lat_RB, Qn = p->lat_Q;
    constexpr int CW = GRAV_NEAR_CW;
    const int RW = f64 ? GRAV_NEAR_RW64 : GRAV_NEAR_RW32;
    const int nrg = (RBn + RW - 1) / RW;
    const int64_t ncg = (ncol + 16 * CW - 1) / (16 * CW);
    if (ncg * nrg > 0x7fffffffll)
        return GRAV_EUNSUPPORTED;
    const int64_t ntile = ncg * nrg;
    // a tile per wave once there are tiles for every wave slot of the chip,
    // else four waves per tile (small plans: 64^3 cells at leaf 4^3 with two
    // Gauss points have 384 tiles)
    const bool per_wave = ntile >= GRAV_NEAR_WAVE_TILES;
    dim3 grid((unsigned)(per_wave ? (ntile + 3) / 4 : ntile)), blk(256);
    const int64_t npts = p->d.n_points;
#define NEAR_LAUNCH(NW)                                                                                            \
    if (f64)                                                                                                       \
        hipLaunchKernelGGL((k_near_lat<GRAV_NEAR_RW64, CW, double, NW>), grid, blk, 0, s, g,                       \
                           (const double *)p->d_rho_blk, nplB, (const double *)p->d_tn64,                          \
                           (const int64_t *)p->d_lat_tab, RBn, Qn, (const double *)p->d_tl2p,                      \
                           (const int32_t *)p->d_tmap, (const double *)p->d_le, npts, nrg, ntile, out);            \
    else                                                                                                           \
        hipLaunchKernelGGL((k_near_lat<GRAV_NEAR_RW32, CW, float, NW>), grid, blk, 0, s, g,                        \
                           (const float *)p->d_rho_blk, nplB, (const float *)p->d_tn32,                            \
                           (const int64_t *)p->d_lat_tab, RBn, Qn, (const double *)p->d_tl2p,                      \
                           (const int32_t *)p->d_tmap, (const double *)p->d_le, npts, nrg, ntile, out);
    if (per_wave) {
        NEAR_LAUNCH(1)
    } else {
        NEAR_LAUNCH(4)
    }
#undef NEAR_LAUNCH
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

grav_status enqueue_forward(Plan *p, const double *rho, double *out, hipStream_t s)
{
    const DevGeom g = make_geom(p);
    const int L = p->L;
    if (p->M == 0)
        return GRAV_OK;
    if (L >= 2) {
        stage_begin(p, "p2m", s);
        if (p->n_spts > 0) {
            const int MG = p->B == 1 ? 1 : kSrcModels;
            const size_t lds = sizeof(double) * (size_t)std::max(kSrcChunk * (p->P2 + MG), MG * p->P2);
            const dim3 sg((unsigned)p->lev[L].n_src, (unsigned)((p->B + MG - 1) / MG));
            if (MG == 1)
                hipLaunchKernelGGL((k_p2m_src<1>), sg, dim3(256), lds, s, g, (const double *)p->d_spos,
                                   (const double *)p->d_sw, (const uint32_t *)p->d_sperm,
                                   (const int64_t *)p->d_sstart, p->n_spts, rho, p->d_me);
            else
                hipLaunchKernelGGL((k_p2m_src<kSrcModels>), sg, dim3(256), lds, s, g, (const double *)p->d_spos,
                                   (const double *)p->d_sw, (const uint32_t *)p->d_sperm,
                                   (const int64_t *)p->d_sstart, p->n_spts, rho, p->d_me);
            GRAV_HIP(hipGetLastError());
        } else {
            GRAV_CHECK(launch_p2m(p, g, rho, s));
        }
        stage_end(p, s);
        stage_begin(p, "m2m", s);
        for (int l = L - 1; l >= 2; --l)
            GRAV_CHECK(launch_m2m(p, g, l, s));
        stage_end(p, s);
        stage_begin(p, "me_gather", s);
        {
            const int64_t n = p->n_me * p->B * p->m2l_npl;
            const dim3 gg((unsigned)((n + 255) / 256));
            const int32_t *kmap = (const int32_t *)p->d_kmap;
            if (n == 0 || kmap == nullptr) {
            } else if (p->d.precision == GRAV_FP64)
                hipLaunchKernelGGL((k_me_gather<double>), gg, dim3(256), 0, s, g, (const double *)p->d_me, p->n_me,
                                   kmap, p->m2l_npl, p->d_meg);
            else
                hipLaunchKernelGGL((k_me_gather<float>), gg, dim3(256), 0, s, g, (const double *)p->d_me, p->n_me,
                                   kmap, p->m2l_npl, reinterpret_cast<float *>(p->d_meg));
            GRAV_HIP(hipGetLastError());
        }
        stage_end(p, s);
        stage_begin(p, "m2l", s);
        if (p->tiles[TK_M2L][0].n > 0) {
            // the segment slots are sized for FP64; the regathered expansions
            // are FP32 in mixed plans (see k_me_gather)
            if (p->d.precision == GRAV_FP64)
                GRAV_CHECK(launch_m2l<double>(p, g, s, forward_m2l<double>(p, p->d_k64)));
            else
                GRAV_CHECK(launch_m2l<float>(p, g, s, forward_m2l<float>(p, p->d_k32)));
        }
        stage_end(p, s);
        {
            stage_begin(p, "m2l_sum", s);
            const int64_t n = p->n_tbox * p->B * p->PS;
            const dim3 gs((unsigned)((n + 255) / 256));
            if (p->d.precision == GRAV_FP64)
                hipLaunchKernelGGL(k_m2l_sum<double>, gs, dim3(256), 0, s, (const double *)p->d_part,
                                   (const int32_t *)p->d_m2l_colmap, (const int32_t *)p->d_m2l_tseg_start,
                                   (const int32_t *)p->d_m2l_tsegs, n, p->PS, p->m2l_ncw, p->d_le);
            else
                hipLaunchKernelGGL(k_m2l_sum<float>, gs, dim3(256), 0, s, (const float *)p->d_part,
                                   (const int32_t *)p->d_m2l_colmap, (const int32_t *)p->d_m2l_tseg_start,
                                   (const int32_t *)p->d_m2l_tsegs, n, p->PS, p->m2l_ncw, p->d_le);
            GRAV_HIP(hipGetLastError());
            stage_end(p, s);
        }
        stage_begin(p, "l2l", s);
        for (int l = 3; l <= L; ++l)
            GRAV_CHECK(launch_l2l(p, g, l, s));
        stage_end(p, s);
    }
    if (p->lat_near) {
        stage_begin(p, "near_lat", s);
        GRAV_CHECK(launch_near_lat(p, g, rho, out, s));
        stage_end(p, s);
    }
    if (!p->lat_near || p->d.n_points > 0) {
        stage_begin(p, "p2p", s);
        // one workgroup per target leaf holding user points
        const dim3 pgrid((unsigned)p->n_user_leaves);
        const int32_t *ul = (const int32_t *)p->d_user_leaves;
        if (p->n_user_leaves == 0) {
        } else if (p->n_spts > 0 && p->d.precision == GRAV_FP64)
            hipLaunchKernelGGL(k_p2p_src<double>, pgrid, dim3(256), 0, s, g, rho,
                               (const double *)p->d_spos, (const double *)p->d_sw, (const uint32_t *)p->d_sperm,
                               (const int64_t *)p->d_sstart, p->n_spts, (const double *)p->d_tpos,
                               (const int64_t *)p->d_leaf_start, (const int64_t *)p->d_leaf_pend,
                               (const uint32_t *)p->d_tkey, ul, p->d_near);
        else if (p->n_spts > 0)
            hipLaunchKernelGGL(k_p2p_src<float>, pgrid, dim3(256), 0, s, g, rho,
                               (const double *)p->d_spos, (const double *)p->d_sw, (const uint32_t *)p->d_sperm,
                               (const int64_t *)p->d_sstart, p->n_spts, (const double *)p->d_tpos,
                               (const int64_t *)p->d_leaf_start, (const int64_t *)p->d_leaf_pend,
                               (const uint32_t *)p->d_tkey, ul, p->d_near);
        else if (p->d.precision == GRAV_FP64)
            hipLaunchKernelGGL(k_p2p<double>, pgrid, dim3(256), 0, s, g, rho,
                               (const double *)p->d_tpos, (const int64_t *)p->d_leaf_start,
                               (const int64_t *)p->d_leaf_pend, (const uint32_t *)p->d_tkey, ul, p->d_near);
        else
            hipLaunchKernelGGL(k_p2p<float>, pgrid, dim3(256), 0, s, g, rho,
                               (const double *)p->d_tpos, (const int64_t *)p->d_leaf_start,
                               (const int64_t *)p->d_leaf_pend, (const uint32_t *)p->d_tkey, ul, p->d_near);
        GRAV_HIP(hipGetLastError());
        stage_end(p, s);
        stage_begin(p, "l2p", s);
        hipLaunchKernelGGL(k_l2p_combine, dim3((unsigned)((p->M * p->B + 255) / 256)), dim3(256), 0, s, g,
                           (const double *)p->d_tpos, (const int32_t *)p->d_tleaf,
                           (const uint32_t *)p->d_tkey, (const uint32_t *)p->d_perm,
                           (const double *)p->d_le, (const double *)p->d_near,
                           p->lat_near ? p->d.n_points : p->M, out);
        GRAV_HIP(hipGetLastError());
        stage_end(p, s);
    }
    return GRAV_OK;
}

// Workspace lock of a plan: a call on another stream while the previous
// call's work is still in flight returns GRAV_EBUSY.  Under stream capture
// (a HIP graph being recorded) nothing is enqueued yet, so the lock is not
// consulted or updated and no event is recorded; the replays of a captured
// call are the caller's to serialise.
static bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

grav_status begin_call(Plan *p, hipStream_t s)
{
    p->n_stage_used = 0;
    if (capturing(s))
        return p->profiling ? GRAV_EUNSUPPORTED : GRAV_OK;
    if (p->has_pending && p->last_stream != s) {
        const hipError_t q = hipEventQuery(p->done);
        if (q == hipErrorNotReady)
            return GRAV_EBUSY;
        if (q != hipSuccess)
            return GRAV_EDEVICE;
    }
    return GRAV_OK;
}

grav_status end_call(Plan *p, hipStream_t s)
{
    if (capturing(s))
        return GRAV_OK;
    GRAV_HIP(hipEventRecord(p->done, s));
    p->has_pending = true;
    p->last_stream = s;
    return GRAV_OK;
}

}  // namespace grav

using namespace grav;

extern "C" grav_status grav_eval(grav_plan_t plan, const double *rho, double *g_out, void *stream)
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
    if (st == GRAV_OK)
        st = enqueue_forward(p, rho, g_out, s);
    if (st == GRAV_OK)
        st = end_call(p, s);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return st;
}

extern "C" grav_status grav_set_profiling(grav_plan_t plan, int32_t enable)
{
    if (!plan)
        return GRAV_EINVAL;
    (reinterpret_cast<Plan *>(plan))->profiling = enable != 0;
    return GRAV_OK;
}

extern "C" grav_status grav_stage_times(grav_plan_t plan, const char **names, double *ms,
                                        int32_t n, int32_t *count)
{
    if (!plan)
        return GRAV_EINVAL;
    Plan *p = reinterpret_cast<Plan *>(plan);
    int k = 0;
    for (int i = 0; i < p->n_stage_used && k < n; ++i, ++k) {
        Stage &st = p->stages[i];
        GRAV_HIP(hipEventSynchronize(st.b));
        float t = 0.f;
        GRAV_HIP(hipEventElapsedTime(&t, st.a, st.b));
        if (names)
            names[k] = st.name.c_str();
        if (ms)
            ms[k] = t;
    }
    if (count)
        *count = k;
    return GRAV_OK;
}
