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

#include "harmonics.hpp"
#include "resolve.hpp"

namespace grav {

namespace {

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// combine^T: the weights that multiply (phi, gx, gy, gz) of a target in the
// lattice frame (G and the lattice-to-physical scale of the combine folded
// in), from its residual r (C values).
__device__ __forceinline__ void combine_weights(const DevGeom &g, const double *r, double (&o)[4])
{
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

// The weights of each sorted target (one thread per (sorted target,
// model)), for the targets with descriptor index below `limit`: all of them,
// or on lattice plans the user points only (the lattice kernels form the
// cell centres' weights from the residuals themselves).
__global__ void __launch_bounds__(256)
k_t_weights(DevGeom g, const double *resid, const uint32_t *perm, int64_t limit, double *w)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.M * g.B)
        return;
    const int64_t i = t / g.B;
    const int bm = (int)(t - i * g.B);
    const int64_t u = perm[i];
    if (u >= limit)
        return;
    double *o = w + t * 4;
    if (u < 0 || u >= g.M) {
        o[0] = o[1] = o[2] = o[3] = 0.0;
        return;
    }
    double v[4];
    combine_weights(g, resid + ((int64_t)bm * g.M + u) * g.C, v);
    o[0] = v[0];
    o[1] = v[1];
    o[2] = v[2];
    o[3] = v[3];
}

// The matrix stages below give each thread up to MT density models (a
// group), so that every operator entry or pair geometry it loads serves MT
// models; groups are ceil(B / MT).

// L2P^T: the adjoint LE of a leaf is the derivative, with respect to its
// coefficients, of the sum over the leaf's targets (with `pend`, its user
// points only) of a phi - (b1 gx + b2 gy + b3 gz), with (a, b) the target's
// weights scaled as the combine scales the far field (a = w0 / w, b = w_1..3
// / w^2).  That derivative is linear in the weights: with the sums
//   S_c[h] = sum over targets of (a, b1, b2, b3)_c R_h(target)
// of the regular harmonics, coefficient (n, m) collects a R_n^m (x2 for
// m > 0) and the gradient terms of degree n-1 and orders m-1, m, m+1, as
// the evaluation pairs them (d/dz R_n^m = R_{n-1}^m, d/dx and d/dy from
// R_{n-1}^{m-1} and R_{n-1}^{m+1}).  One workgroup per (target leaf, group
// of MG models: 1 for single-model plans, else kL2PTModels); targets in
// chunks of kL2PTChunk: their harmonics
// and weights go to LDS, and every thread adds, in target order, the
// products of the (c, model, h) sums it owns (deterministic).
constexpr int kL2PTChunk = 24, kL2PTModels = 4;

template <int MG>
__device__ __forceinline__ double l2pt_gather(const double *S, int P2, int mg, int n, int m, int part)
{
    auto h = [&](int c, int nn, int mm, int pp) -> double {
        if (nn < 0 || mm > nn || (mm == 0 && pp == 1))
            return 0.0;
        return S[(c * MG + mg) * P2 + harm_index(nn, mm, pp)];
    };
    const int q = n - 1;  // degree of the gradient terms
    double v;
    if (part == 0) {
        v = (m == 0 ? 1.0 : 2.0) * h(0, n, m, 0);
        if (q >= 0) {
            if (m == 0) {
                v += -h(3, q, 0, 0) + h(1, q, 1, 0) + h(2, q, 1, 1);
            } else {
                v += -2.0 * h(3, q, m, 0);
                if (m == 1)
                    v -= h(1, q, 0, 0);
                else
                    v += h(2, q, m - 1, 1) - h(1, q, m - 1, 0);
                v += h(1, q, m + 1, 0) + h(2, q, m + 1, 1);
            }
        }
    } else {
        v = -2.0 * h(0, n, m, 1);
        if (q >= 0) {
            v += 2.0 * h(3, q, m, 1);
            if (m == 1)
                v += h(2, q, 0, 0);
            else
                v += h(1, q, m - 1, 1) + h(2, q, m - 1, 0);
            v += h(2, q, m + 1, 0) - h(1, q, m + 1, 1);
        }
    }
    return v;
}

template <int MG>
__global__ void __launch_bounds__(256)
k_t_l2p(DevGeom g, const double *tpos, const int64_t *leaf_start, const int64_t *pend, const uint32_t *tkey,
        int64_t n_leaf, const int32_t *leaves, const double *w, double *le)
{
    extern __shared__ double sh[];
    constexpr int TC = kL2PTChunk;
    const int P2 = g.P2;
    double *H = sh;             // [TC][P2] harmonics of the chunk's targets
    double *W = sh + TC * P2;   // [TC][MG][4] their scaled weights
    const int64_t leaf = leaves[blockIdx.x];  // the target leaves holding user points
    const int bm0 = blockIdx.y * MG;
    const int tid = threadIdx.x;
    const DevLev &lv = g.lev[g.L];
    const uint32_t key = tkey[lv.tbox_off + leaf];
    const int lc[3] = {(int)compact3(key), (int)compact3(key >> 1), (int)compact3(key >> 2)};
    double centre[3];
    for (int a = 0; a < 3; ++a)
        centre[a] = ((double)(lc[a] - g.shift[a]) + 0.5) * g.b;
    const double inv_w = 1.0 / (double)g.b, inv_w2 = inv_w * inv_w;
    const int64_t ts = max(leaf_start[leaf], (int64_t)0);
    const int64_t te = min(pend ? pend[leaf] : leaf_start[leaf + 1], g.M);
    const int NO = 4 * MG * P2;  // sums (c, model, h), output o = (c MG + mg) P2 + h
    constexpr int NJ = 4 * MG * 256 / 256;  // sums per thread (p^2 <= 256)
    double acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        acc[j] = 0.0;
    for (int64_t j0 = ts; j0 < te; j0 += TC) {
        const int nt = (int)min((int64_t)TC, te - j0);
        if (tid < nt) {
            const int64_t j = j0 + tid;
            regular_harmonics(g.P, (tpos[3 * j + 0] - centre[0]) * inv_w, (tpos[3 * j + 1] - centre[1]) * inv_w,
                              (tpos[3 * j + 2] - centre[2]) * inv_w, H + tid * P2, 1);
        }
        for (int i = tid; i < nt * MG * 4; i += 256) {
            const int t = i / (MG * 4), mg = (i / 4) % MG, c = i % 4;
            const int bm = bm0 + mg;
            W[i] = bm < g.B ? w[((j0 + t) * g.B + bm) * 4 + c] * (c == 0 ? inv_w : inv_w2) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int o = tid + 256 * j;
            if (o < NO) {
                const int h = o % P2, cm = o / P2;  // cm = c MG + mg
                const int c = cm / MG, mg = cm % MG;
                double v = acc[j];
                for (int t = 0; t < nt; ++t)
                    v += H[t * P2 + h] * W[(t * MG + mg) * 4 + c];
                acc[j] = v;
            }
        }
        __syncthreads();
    }
    double *S = sh;  // [4][MG][P2]
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int o = tid + 256 * j;
        if (o < NO)
            S[o] = acc[j];
    }
    __syncthreads();
    for (int i = tid; i < MG * g.PS; i += 256) {
        const int mg = i / g.PS, k = i % g.PS;
        const int bm = bm0 + mg;
        if (bm >= g.B)
            continue;
        double v = 0.0;  // padding coefficients stay zero
        if (k < P2) {
            int n = 0;
            while ((n + 1) * (n + 1) <= k)
                ++n;
            const int r = k - n * n;
            v = l2pt_gather<MG>(S, P2, mg, n, (r + 1) / 2, (r > 0 && (r & 1) == 0) ? 1 : 0);
        }
        le[((lv.tgt_off + leaf) * g.B + bm) * g.PS + k] = v;
    }
}

// The column blocks of the transposed M2L: the boxes of level l whose ME it
// writes (inclusive range); M2M^T adds to these and sets the others.
struct ColBlock {
    int lo[3], hi[3];
};

// The transposed translations M2M^T (downward over the source blocks) and
// L2L^T (upward over the target boxes) as FP64 MFMA GEMMs in the layout of
// the forward's k_m2m_lds: a workgroup owns 64 (box, model) columns, 16 per
// wave, and all row blocks; the operator chunks (four k steps, all row
// blocks) pass through LDS double-buffered, one barrier per chunk.
//
// L2L^T: LE_l[box] = sum over the box's children c of L2L_c^T LE_l+1[c];
// the children of a target box are a contiguous range of level l+1 whose
// keys give their octants.  K = 8 x p^2 (absent children read zero).
template <int RB>
__global__ void __launch_bounds__(256)
k_t_l2l(DevGeom g, int l, const uint32_t *tkey, const int32_t *tchild, const double *A, double *le)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    constexpr int K4 = PS / 4;
    constexpr int CH = 4 * RB * 64;
    constexpr int NCH = 8 * RB;
    __shared__ double sa[2][CH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kr = lane >> 4;
    const DevLev &lv = g.lev[l];
    const DevLev &lc = g.lev[l + 1];
    const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + (lane & 15);
    const bool cvalid = col < lv.n_tgt * g.B;
    const int64_t box = cvalid ? col / g.B : 0;
    const int bm = cvalid ? (int)(col % g.B) : 0;
    int32_t ca = 0, ce = 0;
    if (cvalid) {
        ca = max(tchild[lv.tchild_off + box], 0);
        ce = min(tchild[lv.tchild_off + box + 1], (int32_t)lc.n_tgt);
    }
    auto child = [&](int c) -> const double2 * {
        for (int32_t ch = ca; ch < ce; ++ch)
            if ((int)(tkey[lc.tbox_off + ch] & 7u) == c)
                return (const double2 *)(le + ((lc.tgt_off + ch) * g.B + bm) * PS + kr * K4);
        return nullptr;
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
        // the children's expansions as the A operand and the matrix as B:
        // the product is the transposed tile (rows = columns, columns =
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
    // output fragment: rows kr + 4 i = columns of the wave, column lane % 16
    // = coefficient 16 r + lane % 16: 16 lanes write 128 contiguous bytes
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t oc = (int64_t)blockIdx.x * 64 + wave * 16 + kr + 4 * i;
        if (oc >= lv.n_tgt * g.B)
            continue;
        double *dst = le + (lv.tgt_off * g.B + oc) * PS + (lane & 15);
#pragma unroll
        for (int r = 0; r < RB; ++r)
            dst[16 * r] = acc[r][i];
    }
}

// L2L^T on levels with few boxes: a workgroup owns 16 columns and one
// 16-row block; its eight waves take one child octant each (a chain of PS/4
// instructions instead of 8 PS/4) and add their fragments through LDS in
// octant order.
template <int RB>
__global__ void __launch_bounds__(512)
k_t_l2l_split(DevGeom g, int l, const uint32_t *tkey, const int32_t *tchild, const double *A, double *le)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    __shared__ double red[8][256];
    constexpr int PS = 16 * RB;
    constexpr int K4 = PS / 4;
    const int lane = threadIdx.x & 63, kr = lane >> 4;
    const int c = threadIdx.x >> 6;  // the wave's child octant
    const DevLev &lv = g.lev[l];
    const DevLev &lc = g.lev[l + 1];
    const int64_t cg = blockIdx.x / RB;
    const int rb = (int)(blockIdx.x % RB);
    const int64_t col = cg * 16 + (lane & 15);
    const bool cvalid = col < lv.n_tgt * g.B;
    const int64_t box = cvalid ? col / g.B : 0;
    const int bm = cvalid ? (int)(col % g.B) : 0;
    int64_t ci = -1;
    if (cvalid) {
        const int32_t ca = max(tchild[lv.tchild_off + box], 0);
        const int32_t ce = min(tchild[lv.tchild_off + box + 1], (int32_t)lc.n_tgt);
        for (int32_t ch = ca; ch < ce; ++ch)
            if ((int)(tkey[lc.tbox_off + ch] & 7u) == c)
                ci = ch;
    }
    vec4 acc = vec4{0, 0, 0, 0};
    if (__ballot(ci >= 0) != 0ull) {
        const double2 *bp = (const double2 *)(le + (ci >= 0 ? ((lc.tgt_off + ci) * g.B + bm) * PS : 0) + kr * K4);
        const double *ap = A + (int64_t)c * PS * PS + rb * 64 + lane;  // k step ks at ap[ks * RB * 64]
        constexpr int U = RB < 8 ? RB : 8;
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
#pragma unroll
    for (int r = 0; r < 4; ++r)
        red[c][lane * 4 + r] = acc[r];
    __syncthreads();
    if (c == 0 && cvalid) {
        double *dst = le + ((lv.tgt_off + box) * g.B + bm) * PS;
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

// M2M^T: ME_l[child] (+)= M2M_c^T ME_l-1[parent] for the children of octant c
// = blockIdx.y; the columns are the parent boxes of level l-1 (x models),
// K = p^2.  Inside the transposed M2L's column block the child's ME already
// holds the M2L^T terms and the product is added; elsewhere it is set.
template <int RB>
__global__ void __launch_bounds__(256)
k_t_m2m(DevGeom g, int l, ColBlock cb, const double *A, double *me)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    constexpr int K4 = PS / 4;
    constexpr int CH = 4 * RB * 64;
    __shared__ double sa[2][CH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kr = lane >> 4;
    const int oct = blockIdx.y;
    const DevLev &lv = g.lev[l];
    const DevLev &lp = g.lev[l - 1];
    const int64_t nbox = (int64_t)lp.ns[0] * lp.ns[1] * lp.ns[2];
    const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + (lane & 15);
    const bool cvalid = col < nbox * g.B;
    const int64_t box = cvalid ? col / g.B : 0;
    const int bm = cvalid ? (int)(col % g.B) : 0;
    const int x = 2 * (lp.s0[0] + (int)(box % lp.ns[0])) + (oct & 1);
    const int y = 2 * (lp.s0[1] + (int)((box / lp.ns[0]) % lp.ns[1])) + ((oct >> 1) & 1);
    const int z = 2 * (lp.s0[2] + (int)(box / ((int64_t)lp.ns[0] * lp.ns[1]))) + ((oct >> 2) & 1);
    const int64_t ci = cvalid ? dense_index(lv, x, y, z) : -1;
    const double2 *bp = (const double2 *)(me + ((lp.me_off + box) * g.B + bm) * PS + kr * K4);
    const double *Ao = A + (int64_t)oct * PS * PS;
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
    // output fragment: rows kr + 4 i = columns of the wave (child and add
    // flag from the lanes that own them), column lane % 16 = coefficient
    // 16 r + lane % 16: 16 lanes write 128 contiguous bytes
    const bool add = x >= cb.lo[0] && x <= cb.hi[0] && y >= cb.lo[1] && y <= cb.hi[1] && z >= cb.lo[2] &&
                     z <= cb.hi[2];
    const int ci32 = (int)ci, add32 = add ? 1 : 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int oc = kr + 4 * i;
        const int oci = __shfl(ci32, oc);
        const int oadd = __shfl(add32, oc);
        if (oci < 0)
            continue;
        const int obm = (int)(((int64_t)blockIdx.x * 64 + wave * 16 + oc) % g.B);
        double *dst = me + ((lv.me_off + oci) * g.B + obm) * PS + (lane & 15);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            double *o = dst + 16 * r;
            *o = oadd ? *o + acc[r][i] : acc[r][i];
        }
    }
}

// P2M^T: drho[cell] = sum_k Pm[v][k] ME_L[leaf][k] for the cells v of every
// leaf of the source block (each mesh cell once), as FP64 MFMA: one wave
// owns 16 (leaf, model) columns and four 16-cell row blocks (blockIdx.y
// selects the blocks), K = the coefficients in the order 16 (ks/4) +
// 4 (lane/16) + ks%4: a lane's four k steps of chunk q are the coefficients
// 16 q + 4 (lane/16) + 0..3, one 32-byte read, and the four sub-rows of a
// column read one contiguous 128 bytes.
template <int RB>
__global__ void __launch_bounds__(64)
k_t_p2m(DevGeom g, const double *A, int RBT, const double *me, double *drho)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    const int lane = threadIdx.x, kr = lane >> 4;
    const DevLev &lv = g.lev[g.L];
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    // columns leaf-fastest: a row of the output fragment is 16 neighbouring
    // leaves of one model, so the stores of x-runs of cells coalesce
    const int64_t col = (int64_t)blockIdx.x * 16 + (lane & 15);
    const bool cvalid = col < nleaf * g.B;
    const int64_t leaf = cvalid ? col % nleaf : 0;
    const int bm = cvalid ? (int)(col / nleaf) : 0;
    const int rb0 = 4 * blockIdx.y;
    const double2 *bp = (const double2 *)(me + ((lv.me_off + leaf) * g.B + bm) * PS + 4 * kr);
    vec4 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        acc[r] = vec4{0, 0, 0, 0};
    for (int q = 0; q < RB; ++q) {
        const double2 b01 = cvalid ? bp[8 * q] : double2{0.0, 0.0};
        const double2 b23 = cvalid ? bp[8 * q + 1] : double2{0.0, 0.0};
        const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double *ap = A + ((int64_t)(4 * q + u) * RBT + rb0) * 64 + lane;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (rb0 + r < RBT)
                    acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[r * 64], bv[u], acc[r], 0, 0, 0);
        }
    }
    if (!cvalid)
        return;
    const int b = g.b, b3 = b * b * b;
    const int lx = lv.s0[0] + (int)(leaf % lv.ns[0]), ly = lv.s0[1] + (int)((leaf / lv.ns[0]) % lv.ns[1]),
              lz = lv.s0[2] + (int)(leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = 16 * (rb0 + r) + kr + 4 * i;
            if (rb0 + r >= RBT || v >= b3)
                continue;
            const int ix = (lx - g.shift[0]) * b + v % b, iy = (ly - g.shift[1]) * b + (v / b) % b,
                      iz = (lz - g.shift[2]) * b + v / (b * b);
            if (ix < 0 || iy < 0 || iz < 0 || ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2])
                continue;
            drho[(int64_t)bm * ncell + ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix] = acc[r][i];
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
            int64_t n_leg, const int32_t *kmap, int NP, T *out)
{
    // the forward regather's coefficient map (value u of plane pl is
    // coefficient kmap[4 pl + u], -1: zero), through LDS
    __shared__ int32_t km[256];
    for (int e = threadIdx.x; e < 4 * NP; e += blockDim.x)
        km[e] = kmap[e];
    __syncthreads();
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
    const int64_t nB = (int64_t)lt.ns[0] * lt.ns[1] * lt.ns[2] * g.B;
    T *dst = out + lt.me_off * g.B * (4 * NP) + ((int64_t)plane * nB + pos * g.B + bm) * 4;
    const double *src = le + (tb >= 0 ? ((lv.tgt_off + tb) * g.B + bm) * g.PS : 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = km[4 * plane + u];
        dst[u] = (T)(tb >= 0 && c >= 0 ? src[c] : 0.0);
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

// The near-field transpose, per cell: drho[cell] = (with `prior`, the terms
// already in drho, else 0) plus, over the targets j (with `pend`, the user
// points only: the lattice kernel takes the cell centres) of the 27 leaves
// around the cell's leaf (the forward near field pairs every target of a
// leaf with every quadrature point of its 27 neighbours), the weights times
// the pair terms (1/r, (t - x)/r^3) of each of the cell's quadrature
// points, with the forward's coincidence rule and arithmetic type T.  One
// thread per (cell, model group): the pair geometry is computed once for the
// group's models.  With `leaves` (and `prior`), only the cells of those
// source leaves (the leaves with user points around them; the other cells
// keep their prior terms), else every cell.
template <typename T, int MT>
__global__ void __launch_bounds__(256)
k_t_cells(DevGeom g, const double *tpos, const int64_t *leaf_start, const int64_t *pend, int64_t n_leaf,
          const int32_t *tmap, int64_t n_tmap, const double *w, int prior, const int32_t *leaves, int64_t n_leaves,
          double *drho)
{
    const int NG = (g.B + MT - 1) / MT;
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = g.b;
    const DevLev &lv = g.lev[g.L];
    int grp, ix, iy, iz;
    if (leaves) {
        const int b3 = b * b * b;
        const int64_t per = n_leaves * b3;
        if (t >= per * NG)
            return;
        grp = (int)(t / per);
        const int64_t r = t - (int64_t)grp * per;
        const int64_t sl = leaves[r / b3];
        const int v = (int)(r % b3);
        ix = (lv.s0[0] + (int)(sl % lv.ns[0]) - g.shift[0]) * b + v % b;
        iy = (lv.s0[1] + (int)((sl / lv.ns[0]) % lv.ns[1]) - g.shift[1]) * b + (v / b) % b;
        iz = (lv.s0[2] + (int)(sl / ((int64_t)lv.ns[0] * lv.ns[1])) - g.shift[2]) * b + v / (b * b);
        if (ix < 0 || iy < 0 || iz < 0 || ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2])
            return;
    } else {
        if (t >= ncell * NG)
            return;
        grp = (int)(t / ncell);
        const int64_t c = t - (int64_t)grp * ncell;
        ix = (int)(c % g.n[0]);
        iy = (int)((c / g.n[0]) % g.n[1]);
        iz = (int)(c / ((int64_t)g.n[0] * g.n[1]));
    }
    const int64_t cell = ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix;
    // the cell's leaf (root-relative) and place in it
    const int lx = ix / b + g.shift[0], ly = iy / b + g.shift[1], lz = iz / b + g.shift[2];
    const int v = (ix % b) + b * ((iy % b) + b * (iz % b));
    double acc[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
        acc[u] = 0.0;
    (void)v;
    if (prior) {
        // the terms already in drho (P2M^T, the lattice near field)
#pragma unroll
        for (int u = 0; u < MT; ++u)
            if (grp * MT + u < g.B)
                acc[u] = drho[(int64_t)(grp * MT + u) * ncell + cell];
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
        const int64_t ts = max(leaf_start[tl], (int64_t)0);
        const int64_t te = min(pend ? pend[tl] : leaf_start[tl + 1], g.M);
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

// Explicit sources, the transposes of P2M and of the near field per source:
// drho[source] = mass per unit value x (the derivative of the leaf
// expansion's contribution, multipole_basis_dot against ME_L^T, plus the
// pair terms of the targets of the 27 leaves around the source's leaf with
// their weights, formed as the forward near field forms them: relative to
// the target leaf's corner, in type T, with its coincidence rule).  One
// thread per (sorted source, model group).
template <typename T, int MT>
__global__ void __launch_bounds__(256)
k_t_src(DevGeom g, const double *spos, const double *sw, const uint32_t *sperm, int64_t nsrc, const double *tpos,
        const int64_t *leaf_start, int64_t n_leaf, const int32_t *tmap, int64_t n_tmap, const double *w,
        const double *me, double *drho)
{
    const int NG = (g.B + MT - 1) / MT;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsrc * NG)
        return;
    const int grp = (int)(t / nsrc);
    const int64_t i = t - (int64_t)grp * nsrc;
    const int nm = min(MT, g.B - grp * MT);
    const int b = g.b;
    const DevLev &lv = g.lev[g.L];
    const double x[3] = {spos[3 * i + 0], spos[3 * i + 1], spos[3 * i + 2]};
    // the source's leaf (block-relative, as the sort key)
    int lc[3];
    for (int a = 0; a < 3; ++a)
        lc[a] = min(max((int)floor(x[a] / b), 0), lv.ns[a] - 1);
    double acc[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
        acc[u] = 0.0;
    if (g.L >= 2) {
        const int64_t leaf = ((int64_t)lc[2] * lv.ns[1] + lc[1]) * lv.ns[0] + lc[0];
        const double inv_b = 1.0 / (double)b;
        multipole_basis_dot<MT>(g.P, (x[0] - (lc[0] + 0.5) * b) * inv_b, (x[1] - (lc[1] + 0.5) * b) * inv_b,
                                (x[2] - (lc[2] + 0.5) * b) * inv_b,
                                me + ((lv.me_off + leaf) * g.B + grp * MT) * g.PS, g.PS, nm, acc);
    }
    const int mxl = lv.ns[0] + 6, myl = lv.ns[1] + 6, mzl = lv.ns[2] + 6;
    for (int nb = 0; nb < 27; ++nb) {
        // target leaf (root coordinates) and its place in the target map
        const int tx = lc[0] + lv.s0[0] + nb % 3 - 1, ty = lc[1] + lv.s0[1] + (nb / 3) % 3 - 1,
                  tz = lc[2] + lv.s0[2] + nb / 9 - 1;
        const int mx = tx - lv.s0[0] + 3, my = ty - lv.s0[1] + 3, mz = tz - lv.s0[2] + 3;
        if (mx < 0 || my < 0 || mz < 0 || mx >= mxl || my >= myl || mz >= mzl)
            continue;
        const int64_t mi = lv.tmap_off + ((int64_t)mz * myl + my) * mxl + mx;
        if (mi >= n_tmap)
            continue;
        const int64_t tl = tmap[mi];
        if (tl < 0 || tl >= n_leaf)
            continue;
        const double corner[3] = {(double)((tx - g.shift[0]) * b), (double)((ty - g.shift[1]) * b),
                                  (double)((tz - g.shift[2]) * b)};
        const T sx = (T)(x[0] - corner[0]), sy = (T)(x[1] - corner[1]), sz = (T)(x[2] - corner[2]);
        const int64_t ts = max(leaf_start[tl], (int64_t)0), te = min(leaf_start[tl + 1], g.M);
        T part[MT];
#pragma unroll
        for (int u = 0; u < MT; ++u)
            part[u] = 0;
        for (int64_t j = ts; j < te; ++j) {
            const T cx = (T)(tpos[3 * j + 0] - corner[0]) - sx;
            const T cy = (T)(tpos[3 * j + 1] - corner[1]) - sy;
            const T cz = (T)(tpos[3 * j + 2] - corner[2]) - sz;
            const T r2 = cx * cx + cy * cy + cz * cz;
            if (!(r2 > coincident2<T>()))
                continue;
            const T ri = rsqrt_t(r2);
            const T ri3 = ri * ri * ri;
#pragma unroll
            for (int u = 0; u < MT; ++u) {
                if (u >= nm)
                    break;
                const double *wj = w + (j * g.B + grp * MT + u) * 4;
                part[u] += (T)wj[0] * ri + ((T)wj[1] * (cx * ri3) + (T)wj[2] * (cy * ri3) + (T)wj[3] * (cz * ri3));
            }
        }
#pragma unroll
        for (int u = 0; u < MT; ++u)
            acc[u] += (double)part[u];
    }
    const uint32_t user = sperm[i];
#pragma unroll
    for (int u = 0; u < MT; ++u)
        if (u < nm)
            drho[(int64_t)(grp * MT + u) * nsrc + user] = sw[i] * acc[u];
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
    const int64_t n = p->n_leg * p->B * p->m2l_npl;
    if (n > 0 && p->d_kmap != nullptr) {
        hipLaunchKernelGGL((k_le_gather<T>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, gt, g,
                           (const int32_t *)p->d_tmap, p->n_tmap, p->n_tbox, (const double *)p->d_le, p->n_leg,
                           (const int32_t *)p->d_kmap, p->m2l_npl, leg);
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
    r.nc = p->m2lt_nc;
    if (sizeof(T) == 4 && p->m2l_orbit) {
        r.K = reinterpret_cast<const T *>(p->d_kt32o);
        r.orbtab = (const int32_t *)p->d_orbtab_t;
        r.ccoef = (const int32_t *)p->d_ccoef;
    }
    GRAV_CHECK(launch_m2l<T>(p, gt, s, r));
    const int64_t ns = p->m2lt_ncols * p->PS;
    if (ns > 0) {
        hipLaunchKernelGGL((k_m2lt_sum<T>), dim3((unsigned)ceil_div(ns, 256)), dim3(256), 0, s,
                           (const T *)p->d_partt, (const int32_t *)p->d_m2lt_colmap, (const int64_t *)p->d_m2lt_colbox,
                           (const int32_t *)p->d_m2lt_tseg_start, (const int32_t *)p->d_m2lt_tsegs, p->m2lt_ncols,
                           p->PS, p->m2lt_ncw, p->d_me);
        GRAV_HIP(hipGetLastError());
    }
    return GRAV_OK;
}

static grav_status enqueue_m2l_transposed(Plan *p, const DevGeom &g, hipStream_t s)
{
    return p->d.precision == GRAV_FP64 ? m2l_transposed_t<double>(p, g, s, p->d_kt64)
                                       : m2l_transposed_t<float>(p, g, s, p->d_kt32);
}

// Workgroups of the grouped P2M^T (each takes G groups of 64 columns so that
// about this many cover the plan: eight per CU).
constexpr int64_t kGroupedWorkgroups = 2048;

// P2M^T for leaves of at most 64 cells (four row blocks): the layout of
// k_m2m_lds, a workgroup owning groups of 64 leaf-fastest columns, G groups
// one after the other, with the chunks of the operator (four k steps, all
// row blocks) double-buffered in LDS.  The chunk sequence runs on across
// its groups (step s = chunk s % RB of group s / RB), so the loads of a
// group's first chunk are in flight during the previous group's last one:
// a short workgroup per group left the matrix units idle most of the time.
template <int RB>
__global__ void __launch_bounds__(256)
k_t_p2m_lds(DevGeom g, const double *A, int RBT, const double *me, double *drho, int G)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    __shared__ double sa[2][4 * 4 * 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kr = lane >> 4;
    const int CH = 4 * RBT * 64;  // doubles per chunk
    const DevLev &lv = g.lev[g.L];
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int64_t ncol = nleaf * g.B;
    const int64_t ngrp = (ncol + 63) / 64;
    const int64_t g0 = (int64_t)blockIdx.x * G;
    const int ng = (int)min((int64_t)G, ngrp - g0);  // >= 1: the grid covers ngrp
    const int b = g.b, b3 = b * b * b;
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    // this lane's column in group gi; chunk j reads coefficients 16 j +
    // 4 kr + 0..3 (the order of the fragments)
    struct Col {
        bool valid;
        int64_t leaf;
        int bm;
        const double2 *bp;
    };
    auto column = [&](int gi) {
        Col c;
        const int64_t col = (g0 + gi) * 64 + wave * 16 + (lane & 15);
        c.valid = col < ncol;
        c.leaf = c.valid ? col % nleaf : 0;
        c.bm = c.valid ? (int)(col / nleaf) : 0;
        c.bp = (const double2 *)(me + ((lv.me_off + c.leaf) * g.B + c.bm) * PS + 4 * kr);
        return c;
    };
    Col cur = column(0), nxt = cur;
    vec4 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        acc[r] = vec4{0, 0, 0, 0};
    double ra[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (i < RBT)
            ra[i] = A[i * 256 + tid];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (i < RBT)
            sa[0][i * 256 + tid] = ra[i];
    double2 b01 = cur.valid ? cur.bp[0] : double2{0.0, 0.0};
    double2 b23 = cur.valid ? cur.bp[1] : double2{0.0, 0.0};
    __syncthreads();
    const int S = ng * RB;
    for (int s = 0; s < S; ++s) {
        const int buf = s & 1, j = s % RB;
        const bool more = s + 1 < S;
        const int jn = j + 1 < RB ? j + 1 : 0;  // chunk of step s + 1
        if (more) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (i < RBT)
                    ra[i] = A[(int64_t)jn * CH + i * 256 + tid];
        }
        const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
        if (more) {
            if (jn == 0)
                nxt = column(s / RB + 1);
            b01 = nxt.valid ? nxt.bp[8 * jn] : double2{0.0, 0.0};
            b23 = nxt.valid ? nxt.bp[8 * jn + 1] : double2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < RBT)
                    acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[buf][(u * RBT + r) * 64 + lane], bv[u], acc[r], 0,
                                                                 0, 0);
        if (more) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (i < RBT)
                    sa[buf ^ 1][i * 256 + tid] = ra[i];
        }
        if (j == RB - 1) {
            // the group is done: its cells, then the next group's sums
            if (cur.valid) {
                const int lx = lv.s0[0] + (int)(cur.leaf % lv.ns[0]),
                          ly = lv.s0[1] + (int)((cur.leaf / lv.ns[0]) % lv.ns[1]),
                          lz = lv.s0[2] + (int)(cur.leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int v = 16 * r + kr + 4 * i;
                        if (r >= RBT || v >= b3)
                            continue;
                        const int ix = (lx - g.shift[0]) * b + v % b, iy = (ly - g.shift[1]) * b + (v / b) % b,
                                  iz = (lz - g.shift[2]) * b + v / (b * b);
                        if (ix < 0 || iy < 0 || iz < 0 || ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2])
                            continue;
                        drho[(int64_t)cur.bm * ncell + ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix] = acc[r][i];
                    }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[r] = vec4{0, 0, 0, 0};
            cur = nxt;
        }
        __syncthreads();
    }
}

// The lattice transposes for voxel-centre targets (see k_near_lat): with w_T
// the combine^T weights of target leaf T's b^3 cell centres (4 per centre),
//   drho[S] (+)= sum over the 27 neighbours d of A_d^T w_{S - d}   (near^T)
//   LE[T]   (+)= Lm^T w_T                                          (L2P^T)
// GEMMs with columns = (leaf, model) and contraction over (centre t,
// component) of the target leaf.  L2P^T: chunk q and k step u take t =
// (lane/16) TQ + q and component u, so a lane's four k steps are the four
// weights of one centre.  near^T: only the C output components, value e =
// C t + c in chunk q, sub-row kr and k step u with e = 4 KQ kr + 4 q + u,
// read from the weight blocks.  A centre's weights come straight from its
// residual (the centres follow the npts user points in descriptor order, x
// fastest); centres outside the mesh or past b^3 read zero.
__device__ __forceinline__ void lattice_weights(const DevGeom &g, const double *resid, int64_t npts, int tx, int ty,
                                                int tz, int t, int bm, bool in, double (&v)[4])
{
    const int b = g.b;
    v[0] = v[1] = v[2] = v[3] = 0.0;
    if (!in || t >= b * b * b)
        return;
    const int ix = tx * b + t % b, iy = ty * b + (t / b) % b, iz = tz * b + t / (b * b);
    if (ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2])
        return;
    const int64_t cell = ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix;
    combine_weights(g, resid + ((int64_t)bm * g.M + npts + cell) * g.C, v);
}

// The weights of the cell centres in leaf blocks for near^T, as k_rho_blocks
// lays out the densities, for the C output components only: value e =
// C t + c (centre t, component c of the C) of a leaf sits at
// blk[q][kr][pl * B + model][u] with e = 4 KQ kr + 4 q + u, pl = the leaf's
// index in the source block padded by one leaf per side (padding and
// e >= C b^3 zero).  One thread per (leaf, model, centre).
template <typename T>
__global__ void __launch_bounds__(256)
k_t_wblocks(DevGeom g, const double *resid, int64_t npts, int KQ, int64_t nplB, T *blk)
{
    const DevLev &lv = g.lev[g.L];
    const int b = g.b, b3 = b * b * b;
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf * g.B * b3)
        return;
    const int t = (int)(i % b3);
    const int bm = (int)((i / b3) % g.B);
    const int64_t leaf = i / ((int64_t)b3 * g.B);
    const int lx = (int)(leaf % lv.ns[0]), ly = (int)((leaf / lv.ns[0]) % lv.ns[1]),
              lz = (int)(leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
    double v[4];
    lattice_weights(g, resid, npts, lx, ly, lz, t, bm, true, v);
    const int64_t pl = ((int64_t)(lz + 1) * (lv.ns[1] + 2) + (ly + 1)) * (lv.ns[0] + 2) + (lx + 1);
    for (int c = 0; c < g.C; ++c) {
        const int e = g.C * t + c, kr = e / (4 * KQ), q = (e / 4) % KQ;
        blk[((int64_t)(q * 4 + kr) * nplB + pl * g.B + bm) * 4 + e % 4] = (T)v[c + 4 - g.C];
    }
}

// near^T: a workgroup owns CW blocks of 16 (source leaf, model) columns and
// four 16-cell row blocks (blockIdx.y); its four waves split the 27 KQ
// chunks (neighbour d, chunk q of the target leaf's C b^3 weights) and add
// their partial tiles through LDS in wave order (deterministic), as
// k_near_lat does.  Target leaf T = S - d reads the padded weight blocks (no
// bounds test).
template <int CW, typename T>
__global__ void __launch_bounds__(256)
k_t_near_lat(DevGeom g, const T *blk, int64_t nplB, const T *A, int RBt, int KQ, int add, double *drho)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(T)))) T;
    __shared__ double red[4][CW * 4 * 4][64];
    const int lane = threadIdx.x & 63, kr = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const DevLev &lv = g.lev[g.L];
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int b = g.b, b3 = b * b * b;
    const int px = lv.ns[0] + 2, py = lv.ns[1] + 2;
    const int rb0 = 4 * blockIdx.y;
    bool cvalid[CW];
    int bm[CW], sx[CW], sy[CW], sz[CW];
    const T *bbase[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        const int64_t col = ((int64_t)blockIdx.x * CW + c) * 16 + (lane & 15);
        cvalid[c] = col < nleaf * g.B;
        const int64_t leaf = cvalid[c] ? col / g.B : 0;
        bm[c] = cvalid[c] ? (int)(col % g.B) : 0;
        sx[c] = (int)(leaf % lv.ns[0]);
        sy[c] = (int)((leaf / lv.ns[0]) % lv.ns[1]);
        sz[c] = (int)(leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
        bbase[c] = blk + ((int64_t)kr * nplB + (((int64_t)(sz[c] + 1) * py + (sy[c] + 1)) * px + (sx[c] + 1)) * g.B +
                          bm[c]) * 4;
    }
    vec4 acc[CW][4];
#pragma unroll
    for (int c = 0; c < CW; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[c][r] = vec4{0, 0, 0, 0};
    const int NI = 27 * KQ;
    const int i0 = wave * NI / 4, i1 = (wave + 1) * NI / 4;
    for (int i = i0; i < i1; ++i) {
        const int nb = i / KQ, q = i - nb * KQ;
        // the forward pairs target leaf T with source leaf T + d: T = S - d
        const int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = nb / 9 - 1;
        const int64_t boff = ((int64_t)q * 4 * nplB + (((int64_t)(-dz) * py - dy) * px - dx) * g.B) * 4;
        T bb[CW][4];
#pragma unroll
        for (int c = 0; c < CW; ++c)
            load4(bbase[c] + boff, bb[c]);
        T av[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            load_frags<T, 4>(A + (((int64_t)nb * KQ + q) * RBt + min(rb0 + r, RBt - 1)) * 256, lane, av[r]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    if constexpr (sizeof(T) == 8)
                        acc[c][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r][u], bb[c][u], acc[c][r], 0, 0, 0);
                    else
                        acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][u], bb[c][u], acc[c][r], 0, 0, 0);
                }
    }
#pragma unroll
    for (int c = 0; c < CW; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                red[wave][(c * 4 + r) * 4 + k][lane] = (double)acc[c][r][k];
    __syncthreads();
    // output rows: FP32 instruction rows 4 (lane/16) + i, FP64 rows lane/16 + 4 i
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    for (int j = wave; j < CW * 4; j += 4) {
        const int c = j / 4, r = j % 4;
        if (!cvalid[c] || rb0 + r >= RBt)
            continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = 16 * (rb0 + r) + (sizeof(T) == 8 ? kr + 4 * i : 4 * kr + i);
            if (v >= b3)
                continue;
            const int ix = sx[c] * b + v % b, iy = sy[c] * b + (v / b) % b, iz = sz[c] * b + v / (b * b);
            if (ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2])
                continue;
            const double sum = ((red[0][j * 4 + i][lane] + red[1][j * 4 + i][lane]) + red[2][j * 4 + i][lane]) +
                               red[3][j * 4 + i][lane];
            double *o = drho + (int64_t)bm[c] * ncell + ((int64_t)iz * g.n[1] + iy) * g.n[0] + ix;
            *o = add ? *o + sum : sum;
        }
    }
}

// L2P^T at the cell centres (FP64): one wave owns 16 (leaf, model) columns
// and all RB coefficient blocks; the column's target leaf is found in the
// leaf level's target map.  With `add`, the LE of a leaf that also holds
// user points (written by k_t_l2p) is added to, every other one set.
template <int RB>
__global__ void __launch_bounds__(64)
k_t_l2p_lat(DevGeom g, const double *A, int TQ, const int32_t *tmap, const double *resid, int64_t npts,
            int add, const int64_t *leaf_start, const int64_t *pend, double *le)
{
    using vec4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    constexpr int PS = 16 * RB;
    const int lane = threadIdx.x, kr = lane >> 4;
    const DevLev &lv = g.lev[g.L];
    const int64_t nleaf = (int64_t)lv.ns[0] * lv.ns[1] * lv.ns[2];
    const int64_t col = (int64_t)blockIdx.x * 16 + (lane & 15);
    const bool cvalid = col < nleaf * g.B;
    const int64_t leaf = cvalid ? col / g.B : 0;
    const int bm = cvalid ? (int)(col % g.B) : 0;
    const int sx = (int)(leaf % lv.ns[0]), sy = (int)((leaf / lv.ns[0]) % lv.ns[1]),
              sz = (int)(leaf / ((int64_t)lv.ns[0] * lv.ns[1]));
    const int64_t tl =
        cvalid ? tmap_lookup(lv, tmap, 3, lv.s0[0] + sx, lv.s0[1] + sy, lv.s0[2] + sz) : -1;
    vec4 acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
        acc[r] = vec4{0, 0, 0, 0};
    for (int q = 0; q < TQ; ++q) {
        double bv[4];
        lattice_weights(g, resid, npts, sx, sy, sz, kr * TQ + q, bm, tl >= 0, bv);
        double av[RB][4];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            load_frags<double, 4>(A + ((int64_t)q * RB + r) * 256, lane, av[r]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < RB; ++r)
                acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r][u], bv[u], acc[r], 0, 0, 0);
    }
    if (tl < 0 || tl >= lv.n_tgt)
        return;
    const bool addc = add && pend[tl] > max(leaf_start[tl], (int64_t)0);
    double *dst = le + ((lv.tgt_off + tl) * g.B + bm) * PS;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double *o = dst + 16 * r + kr + 4 * i;
            *o = addc ? *o + acc[r][i] : acc[r][i];
        }
}

#define GRAV_T_RB_CASES(X) X(1) X(2) X(3) X(4) X(6) X(7) X(8) X(9) X(11) X(13) X(15) X(16)

// levels with fewer 64-column workgroups than this take the split kernel
constexpr int64_t kTileWgsMin = 256;

static grav_status launch_t_l2l(Plan *p, const DevGeom &g, int l, hipStream_t s)
{
    const int64_t ncol = p->lev[l].n_tgt * p->B;
    const int RB = p->PS / 16;
    const bool tiled = ceil_div(ncol, 64) >= kTileWgsMin;
    const dim3 grid((unsigned)ceil_div(ncol, 64)), grid_split((unsigned)(ceil_div(ncol, 16) * RB));
#define CASE(R)                                                                                            \
    case R:                                                                                                \
        if (tiled)                                                                                         \
            hipLaunchKernelGGL((k_t_l2l<R>), grid, dim3(256), 0, s, g, l, (const uint32_t *)p->d_tkey,     \
                               (const int32_t *)p->d_tchild, (const double *)p->d_l2lt_sw, p->d_le);       \
        else                                                                                               \
            hipLaunchKernelGGL((k_t_l2l_split<R>), grid_split, dim3(512), 0, s, g, l,                      \
                               (const uint32_t *)p->d_tkey, (const int32_t *)p->d_tchild,                  \
                               (const double *)p->d_l2lt_sw, p->d_le);                                     \
        break;
    switch (RB) {
        GRAV_T_RB_CASES(CASE)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef CASE
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

static grav_status launch_t_m2m(Plan *p, const DevGeom &g, int l, hipStream_t s)
{
    const LevelInfo &lv = p->lev[l];
    ColBlock cb;
    for (int a = 0; a < 3; ++a) {
        cb.lo[a] = lv.cs0[a];
        cb.hi[a] = lv.cs0[a] + lv.cns[a] - 1;
    }
    const dim3 grid((unsigned)ceil_div(p->lev[l - 1].n_src * p->B, 64), 8);
#define CASE(R)                                                                                             \
    case R:                                                                                                 \
        hipLaunchKernelGGL((k_t_m2m<R>), grid, dim3(256), 0, s, g, l, cb, (const double *)p->d_m2mt_sw, p->d_me); \
        break;
    switch (p->PS / 16) {
        GRAV_T_RB_CASES(CASE)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef CASE
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

static grav_status launch_t_p2m(Plan *p, const DevGeom &g, double *drho, hipStream_t s)
{
    const int b3 = p->b * p->b * p->b, RBT = (b3 + 15) / 16;
    const int64_t ncol = p->lev[p->L].n_src * p->B;
    // LDS kernel: groups of 64 columns, about kGroupedWorkgroups workgroups
    const int64_t ngrp = ceil_div(ncol, 64);
    const int G = (int)std::max<int64_t>(1, ceil_div(ngrp, kGroupedWorkgroups));
    const dim3 grid((unsigned)ceil_div(ncol, 16), (unsigned)ceil_div(RBT, 4)), grid_lds((unsigned)ceil_div(ngrp, G));
#define CASE(R)                                                                                             \
    case R:                                                                                                 \
        if (RBT <= 4)                                                                                       \
            hipLaunchKernelGGL((k_t_p2m_lds<R>), grid_lds, dim3(256), 0, s, g, (const double *)p->d_pmt_sw, RBT, \
                               (const double *)p->d_me, drho, G);                                           \
        else                                                                                                \
            hipLaunchKernelGGL((k_t_p2m<R>), grid, dim3(64), 0, s, g, (const double *)p->d_pmt_sw, RBT,     \
                               (const double *)p->d_me, drho);                                              \
        break;
    switch (p->PS / 16) {
        GRAV_T_RB_CASES(CASE)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef CASE
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

static grav_status launch_t_l2p_lat(Plan *p, const DevGeom &g, const double *resid, int add, hipStream_t s)
{
    const dim3 grid((unsigned)ceil_div(p->lev[p->L].n_src * p->B, 16));
#define CASE(R)                                                                                             \
    case R:                                                                                                 \
        hipLaunchKernelGGL((k_t_l2p_lat<R>), grid, dim3(64), 0, s, g, (const double *)p->d_tl2pt, p->lat_TQ, \
                           (const int32_t *)p->d_tmap, resid, p->d.n_points,                              \
                           add, (const int64_t *)p->d_leaf_start, (const int64_t *)p->d_leaf_pend, p->d_le); \
        break;
    switch (p->PS / 16) {
        GRAV_T_RB_CASES(CASE)
    default:
        return GRAV_EUNSUPPORTED;
    }
#undef CASE
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
}

static grav_status launch_t_near_lat(Plan *p, const DevGeom &g, const double *resid, int add, double *drho,
                                     hipStream_t s)
{
    constexpr int CW = 2;
    const LevelInfo &lv = p->lev[p->L];
    const int b3 = p->b * p->b * p->b, RBt = (int)ceil_div(b3, 16);
    // chunks of 16 weights over the C b^3 (centre, component) pairs of a leaf
    const int KQ = (int)ceil_div((int64_t)p->d.components * b3, 16);
    const int64_t nplB = (int64_t)(lv.ns[0] + 2) * (lv.ns[1] + 2) * (lv.ns[2] + 2) * p->B;
    const bool f64 = p->d.precision == GRAV_FP64;
    const dim3 fgrid((unsigned)ceil_div(lv.n_src * p->B * b3, 256));
    const dim3 grid((unsigned)ceil_div(lv.n_src * p->B, 16 * CW), (unsigned)ceil_div(RBt, 4));
    if (f64) {
        hipLaunchKernelGGL((k_t_wblocks<double>), fgrid, dim3(256), 0, s, g, resid, p->d.n_points, KQ, nplB,
                           p->d_w_blk);
        hipLaunchKernelGGL((k_t_near_lat<CW, double>), grid, dim3(256), 0, s, g, (const double *)p->d_w_blk, nplB,
                           (const double *)p->d_tnt64, RBt, KQ, add, drho);
    } else {
        float *wb = reinterpret_cast<float *>(p->d_w_blk);
        hipLaunchKernelGGL((k_t_wblocks<float>), fgrid, dim3(256), 0, s, g, resid, p->d.n_points, KQ, nplB,
                           wb);
        hipLaunchKernelGGL((k_t_near_lat<CW, float>), grid, dim3(256), 0, s, g, (const float *)wb, nplB,
                           (const float *)p->d_tnt32, RBt, KQ, add, drho);
    }
    GRAV_HIP(hipGetLastError());
    return GRAV_OK;
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
    if (ncell * NG > 0x7fffffffll * 256 || p->n_me > 0x7fffffffll || p->P2 > 256)
        return GRAV_EUNSUPPORTED;
    stage_begin(p, "weights", s);
    hipLaunchKernelGGL(k_t_weights, grid(p->M * p->B), blk, 0, s, g, resid, (const uint32_t *)p->d_perm,
                       p->lat_near ? p->d.n_points : p->M, p->d_near);
    GRAV_HIP(hipGetLastError());
    stage_end(p, s);
    if (L >= 2) {
        stage_begin(p, "l2pT", s);
        // user points by the transposed recurrence; cell centres of lattice
        // plans by the transposed lattice L2P
        const bool pts = !p->lat_near || p->d.n_points > 0;
        if (p->n_leaf > 0 && pts) {
            const int MG = p->B == 1 ? 1 : kL2PTModels;
            const size_t lds = sizeof(double) * std::max(kL2PTChunk * (p->P2 + 4 * MG), 4 * MG * p->P2);
            // one workgroup per target leaf holding user points (the LE of
            // the other leaves, cell centres only, is set by the lattice
            // L2P^T below)
            const dim3 lgrid((unsigned)p->n_user_leaves, (unsigned)ceil_div(p->B, MG));
            const int64_t *pend = p->lat_near ? (const int64_t *)p->d_leaf_pend : nullptr;
            const int32_t *ul = (const int32_t *)p->d_user_leaves;
            if (p->n_user_leaves == 0) {
            } else if (MG == 1)
                hipLaunchKernelGGL((k_t_l2p<1>), lgrid, dim3(256), lds, s, g, (const double *)p->d_tpos,
                                   (const int64_t *)p->d_leaf_start, pend, (const uint32_t *)p->d_tkey, p->n_leaf,
                                   ul, (const double *)p->d_near, p->d_le);
            else
                hipLaunchKernelGGL((k_t_l2p<kL2PTModels>), lgrid, dim3(256), lds, s, g, (const double *)p->d_tpos,
                                   (const int64_t *)p->d_leaf_start, pend, (const uint32_t *)p->d_tkey, p->n_leaf,
                                   ul, (const double *)p->d_near, p->d_le);
            GRAV_HIP(hipGetLastError());
        }
        if (p->lat_near)
            GRAV_CHECK(launch_t_l2p_lat(p, g, resid, pts ? 1 : 0, s));
        stage_end(p, s);
        stage_begin(p, "l2lT", s);
        for (int l = L - 1; l >= 2; --l)
            if (p->lev[l].n_tgt > 0)
                GRAV_CHECK(launch_t_l2l(p, g, l, s));
        stage_end(p, s);
        stage_begin(p, "m2lT", s);
        GRAV_CHECK(enqueue_m2l_transposed(p, g, s));
        stage_end(p, s);
        stage_begin(p, "m2mT", s);
        for (int l = 3; l <= L; ++l)
            GRAV_CHECK(launch_t_m2m(p, g, l, s));
        stage_end(p, s);
        if (p->n_spts == 0) {
            stage_begin(p, "p2mT", s);
            GRAV_CHECK(launch_t_p2m(p, g, drho, s));
            stage_end(p, s);
        }
    }
    if (p->n_spts > 0) {
        // explicit sources: P2M^T and near^T per source
        stage_begin(p, "srcT", s);
        const int64_t n = p->n_spts * NG;
        if (p->d.precision == GRAV_FP64)
            hipLaunchKernelGGL((k_t_src<double, MT>), grid(n), blk, 0, s, g, (const double *)p->d_spos,
                               (const double *)p->d_sw, (const uint32_t *)p->d_sperm, p->n_spts,
                               (const double *)p->d_tpos, (const int64_t *)p->d_leaf_start, p->n_leaf,
                               (const int32_t *)p->d_tmap, p->n_tmap, (const double *)p->d_near,
                               (const double *)p->d_me, drho);
        else
            hipLaunchKernelGGL((k_t_src<float, MT>), grid(n), blk, 0, s, g, (const double *)p->d_spos,
                               (const double *)p->d_sw, (const uint32_t *)p->d_sperm, p->n_spts,
                               (const double *)p->d_tpos, (const int64_t *)p->d_leaf_start, p->n_leaf,
                               (const int32_t *)p->d_tmap, p->n_tmap, (const double *)p->d_near,
                               (const double *)p->d_me, drho);
        GRAV_HIP(hipGetLastError());
        stage_end(p, s);
        return GRAV_OK;
    }
    // the near field's transpose (with no far field it also sets drho):
    // cell centres of lattice plans on MFMA, user points (or all targets of
    // other plans) pair by pair
    if (p->lat_near) {
        stage_begin(p, "nearT", s);
        GRAV_CHECK(launch_t_near_lat(p, g, resid, L >= 2 ? 1 : 0, drho, s));
        stage_end(p, s);
    }
    const bool pts = p->lat_near ? p->d.n_points > 0 : (p->p2p_pairs > 0 || L < 2);
    if (pts) {
        const int prior = (L >= 2 || p->lat_near) ? 1 : 0;
        const int64_t *pend = p->lat_near ? (const int64_t *)p->d_leaf_pend : nullptr;
        stage_begin(p, "nearT_pts", s);
        // with prior terms only the cells of the leaves near user points
        // change (none when the points lie away from the mesh)
        const int32_t *leaves = prior ? p->d_pt_leaves : nullptr;
        const int64_t nthr = leaves ? p->n_pt_leaves * p->b * p->b * p->b * NG : ncell * NG;
        if (nthr > 0) {
            if (p->d.precision == GRAV_FP64)
                hipLaunchKernelGGL((k_t_cells<double, MT>), grid(nthr), blk, 0, s, g, (const double *)p->d_tpos,
                                   (const int64_t *)p->d_leaf_start, pend, p->n_leaf, (const int32_t *)p->d_tmap,
                                   p->n_tmap, (const double *)p->d_near, prior, leaves, p->n_pt_leaves, drho);
            else
                hipLaunchKernelGGL((k_t_cells<float, MT>), grid(nthr), blk, 0, s, g, (const double *)p->d_tpos,
                                   (const int64_t *)p->d_leaf_start, pend, p->n_leaf, (const int32_t *)p->d_tmap,
                                   p->n_tmap, (const double *)p->d_near, prior, leaves, p->n_pt_leaves, drho);
            GRAV_HIP(hipGetLastError());
        }
        stage_end(p, s);
    }
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
            const int64_t n = (p->n_spts > 0 ? p->n_spts : (int64_t)p->d.nx * p->d.ny * p->d.nz) * p->B;
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
