// Kernel-side geometry and helpers shared by the forward and adjoint passes.
#pragma once

#include "internal.hpp"

namespace grav {

struct DevLev {
    int s0[3];
    int ns[3];
    int64_t me_off;
    int64_t tgt_off;
    int64_t tbox_off;
    int64_t class_start[9];
    int64_t tmap_off;
    int64_t tchild_off;
    int64_t n_tgt;       // target boxes of the level
    int need_lo[3];      // box range (inclusive) whose expansions the M2L reads
    int need_hi[3];
};

struct DevGeom {
    DevLev lev[kMaxLevels + 1];
    int L, b, q, P, P2, PS, KS, B, C;
    int n[3];
    int shift[3];
    int64_t M;
    double G, h;
};

// Boxes of one parity class (bit a of cls = parity of coordinate a) of a
// level's source block, in x-fastest order; classes follow each other in
// order 0..7.  Returns the class's first box position and, per axis, its
// first absolute coordinate and box count.
__host__ __device__ inline int64_t class_split(const DevLev &lv, int cls, int first[3], int cnt[3])
{
    int64_t start = 0;
    for (int c = 0; c <= cls; ++c) {
        int64_t n = 1;
        for (int a = 0; a < 3; ++a) {
            const int f = lv.s0[a] + ((((c >> a) & 1) - lv.s0[a]) & 1);
            const int k = (lv.ns[a] - (f - lv.s0[a]) + 1) / 2;
            const int kk = k > 0 ? k : 0;
            if (c == cls) {
                first[a] = f;
                cnt[a] = kk;
            }
            n *= kk;
        }
        if (c < cls)
            start += n;
    }
    return start;
}

DevGeom make_geom(const Plan *p);
template <typename T>
__global__ void k_sum_parts(const T *part, int S, int64_t n, double *out);
// One M2L problem on the stream-K kernel: the forward M2L (columns are
// target boxes, B the regathered multipole expansions) or the adjoint's
// transposed M2L (columns are source boxes, B the regathered adjoint local
// expansions, operators K_d^T).
template <typename T>
struct M2LRun {
    const GemmTile *tiles;
    const uint32_t *keys;      // Morton key of each column box (per level, from lev.tbox_off)
    const int32_t *order;      // class-grouped column order -> box (per level, from lev.tbox_off)
    const int32_t *class_off;  // [8][189][4] (dx, dy, dz, operator) per column class
    const T *K;                // operators in the panel layout
    const T *b_in;             // regathered B operand
    const int32_t *segs, *wgseg, *items;
    T *part;                   // segment slots
    int32_t wgs;               // workgroups (0: nothing to do)
    int nset;                  // operand register sets of the FP32 kernel
    int nc;                    // 16-column blocks per wave (FP32: 2 or 4; FP64: 1)
    // the reflection-orbit M2L (forward, mixed plans): items are canonical
    // offsets, K the class-blocked canonical operators, orbtab the class
    // offset of each reflection, ccoef the coefficient of each class row
    const int32_t *orbtab = nullptr, *ccoef = nullptr;
};
template <typename T>
grav_status launch_m2l(const Plan *p, const DevGeom &g, hipStream_t s, const M2LRun<T> &r);
grav_status m2l_resident_workers(const Plan *p, int nset, int nc, bool orbit, int *workers);
grav_status begin_call(Plan *p, hipStream_t s);
grav_status end_call(Plan *p, hipStream_t s);

// Pairs closer than this (squared, in cell units) count as coincident and
// contribute nothing: 1e-10 cells in FP64, 1e-5 cells in FP32 (the offset
// of a point from a cell corner is only known to ~1e-6 cells in FP32).
template <typename T> __device__ constexpr T coincident2();
template <> __device__ constexpr double coincident2<double>() { return 1e-20; }
template <> __device__ constexpr float coincident2<float>() { return 1e-10f; }

// Four consecutive values from a 16-byte (float) or 32-byte (double)
// aligned address, as vector loads.
__device__ inline void load4(const float *p, float v[4])
{
    const float4 x = *(const float4 *)p;
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
}
__device__ inline void load4(const double *p, double v[4])
{
    const double2 a = ((const double2 *)p)[0], b = ((const double2 *)p)[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}

// Scheduling pattern for one software-pipelined step that issues NLD vector
// loads (of the next step's operands) and NMF matrix instructions (of this
// step): load, NMF / NLD instructions, load, ..., then the rest.  Without it
// the compiler either issues every load in one block ahead of the matrix
// instructions (the matrix pipe idles while the loads issue) or moves each
// load next to its single use (no overlap at all).  Place it at the end of
// the scheduling region that holds those loads and instructions.
template <int NLD, int NMF>
__device__ __forceinline__ void interleave_loads()
{
    constexpr int K = NMF / NLD > 0 ? NMF / NLD : 1;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // one VMEM read
        __builtin_amdgcn_sched_group_barrier(0x008, K, 0);  // K MFMA
    }
    if constexpr (NMF > K * NLD)
        __builtin_amdgcn_sched_group_barrier(0x008, NMF - K * NLD, 0);
}

// Per-lane MFMA operand fragments in HBM, group-major: a set of E values per
// lane is stored as [E / G][64 lanes][G] with G = 16 bytes / sizeof(T), so
// every 16-byte vector load of a wave reads one contiguous kilobyte (eight
// cache lines).  The set must start on a 16-byte boundary.
template <typename T, int E>
__device__ __forceinline__ void load_frags(const T *set, int lane, T (&v)[E])
{
    constexpr int G = 16 / (int)sizeof(T);
    static_assert(E % G == 0, "fragment set not a whole number of 16-byte groups");
    using g16 = __attribute__((__vector_size__(16))) T;
    const g16 *p = reinterpret_cast<const g16 *>(set) + lane;
#pragma unroll
    for (int j = 0; j < E / G; ++j) {
        const g16 x = p[j * 64];
#pragma unroll
        for (int t = 0; t < G; ++t)
            v[j * G + t] = x[t];
    }
}

__device__ inline double rsqrt_t(double x) { return rsqrt(x); }
__device__ inline float rsqrt_t(float x) { return rsqrtf(x); }

// Coefficient accessors of the local-expansion evaluation: the real and
// imaginary parts of coefficient (n, m) in the library's real order (degree
// n block of 2n+1 values: real part of order 0, then real and imaginary
// parts of orders 1..n).
struct CoefArray {
    const double *L;
    __host__ __device__ double re(int n, int m) const { return m == 0 ? L[n * n] : L[n * n + 2 * m - 1]; }
    __host__ __device__ double im(int n, int m) const { return m == 0 ? 0.0 : L[n * n + 2 * m]; }
};
// The unit vector of coefficient k: evaluating with it gives the derivatives
// of the evaluation with respect to coefficient k (the transposed L2P).
struct CoefUnit {
    int k;
    __host__ __device__ double re(int n, int m) const { return (m == 0 ? n * n : n * n + 2 * m - 1) == k ? 1.0 : 0.0; }
    __host__ __device__ double im(int n, int m) const { return (m != 0 && n * n + 2 * m == k) ? 1.0 : 0.0; }
};

// Local expansion evaluation at u (box-width units from the box centre):
// out[0] = sum L_j^k R_j^k(u), out[1..3] = its gradient with respect to u.
// The regular harmonics are generated by the order-m recurrences one column
// at a time, so only two previous values are live; with
// d/dz R_n^m = R_{n-1}^m, d/dx R_n^m = (R_{n-1}^{m-1} - R_{n-1}^{m+1})/2 and
// d/dy R_n^m = i (R_{n-1}^{m-1} + R_{n-1}^{m+1})/2, each R_n^m pairs with
// degree-(n+1) coefficients for the gradient.
template <class Coef>
__host__ __device__ inline void l2p_eval_t(int P, const Coef &L, double x, double y, double z, double out[4])
{
    double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    const double r2 = x * x + y * y + z * z;
    double mmr = 1.0, mmi = 0.0;
    for (int m = 0; m < P; ++m) {
        if (m > 0) {
            const double s = 1.0 / (2.0 * m);
            const double nr = (x * mmr - y * mmi) * s;
            const double ni = (x * mmi + y * mmr) * s;
            mmr = nr;
            mmi = ni;
        }
        double p1r = 0.0, p1i = 0.0, p2r = 0.0, p2i = 0.0;
        for (int n = m; n < P; ++n) {
            double Rr, Ri;
            if (n == m) {
                Rr = mmr;
                Ri = mmi;
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
            if (m == 0)
                phi += L.re(n, 0) * Rr;
            else
                phi += 2.0 * (L.re(n, m) * Rr - L.im(n, m) * Ri);
            if (n + 1 < P) {
                const int n1 = n + 1;
                if (m == 0) {
                    gz += Rr * L.re(n1, 0);
                    gx += Rr * L.re(n1, 1);
                    gy -= Rr * L.im(n1, 1);
                } else {
                    gz += 2.0 * (Rr * L.re(n1, m) - Ri * L.im(n1, m));
                    const double ar = L.re(n1, m + 1) - L.re(n1, m - 1);
                    const double ai = L.im(n1, m + 1) - L.im(n1, m - 1);
                    gx += Rr * ar - Ri * ai;
                    const double br = L.re(n1, m + 1) + L.re(n1, m - 1);
                    const double bi = L.im(n1, m + 1) + L.im(n1, m - 1);
                    gy -= Rr * bi + Ri * br;
                }
            }
        }
    }
    out[0] = phi;
    out[1] = gx;
    out[2] = gy;
    out[3] = gz;
}

__host__ __device__ inline void l2p_eval(int P, const double *L, double x, double y, double z, double out[4])
{
    l2p_eval_t(P, CoefArray{L}, x, y, z, out);
}

// Derivatives of l2p_eval's four outputs with respect to coefficient k.
__host__ __device__ inline void l2p_coef(int P, int k, double x, double y, double z, double out[4])
{
    l2p_eval_t(P, CoefUnit{k}, x, y, z, out);
}

}  // namespace grav
