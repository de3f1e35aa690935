// Device exclusive scan and stable LSD radix sort of (key, value) pairs.
//
// Used at plan time to order the evaluation points by the Morton key of
// their leaf (the hierarchical decomposition of Sec. 2.3) and to group the
// boxes of each level by child-parity class.
#include "internal.hpp"

namespace grav {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t *total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        uint32_t a = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    uint32_t incl = sh[t];
    if (total)
        *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_tile(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *sums)
{
    __shared__ uint32_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0u;
        run += v[i];
    }
    uint32_t total = 0;
    uint32_t pre = block_exclusive_scan(run, sh, &total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (idx < n)
            out[idx] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0 && sums)
        sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_add(uint32_t *out, int64_t n, const uint32_t *sums)
{
    const uint32_t add = sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
        const int64_t idx = base + i;
        if (idx < n)
            out[idx] += add;
    }
}

constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 8;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;  // 2048

__global__ void __launch_bounds__(kRadixThreads)
k_radix_hist(const uint32_t *keys, int64_t n, int shift, uint32_t *hist, int nblk)
{
    __shared__ uint32_t cnt[256];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t i = base + r * kRadixThreads + t;
        if (i < n)
            atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * nblk + blockIdx.x] = cnt[t];
}

// Stable scatter: elements of a tile are taken in rounds of 256 (round r
// holds tile positions r*256 .. r*256+255 in thread order); within a wave
// the rank among equal digits comes from ballots over the digit bits, and
// waves of a round are ordered by index.
__global__ void __launch_bounds__(kRadixThreads)
k_radix_scatter(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                int64_t n, int shift, const uint32_t *offs, int nblk)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][257];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    base[t] = offs[(int64_t)t * nblk + blockIdx.x];
    for (int w = 0; w < 4; ++w)
        wcnt[w][t] = 0;
    if (t < 4)
        wcnt[t][256] = 0;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * kRadixTile;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t i = tile + r * kRadixThreads + t;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = valid ? ((key >> shift) & 255u) : 256u;
        uint64_t same = ~0ull;
#pragma unroll
        for (int bit = 0; bit < 9; ++bit) {
            const int mine = (d >> bit) & 1u;
            const uint64_t bs = __ballot(mine);
            same &= mine ? bs : ~bs;
        }
        const uint32_t rank = __popcll(same & lt);
        if (rank == 0)
            wcnt[wave][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w)
                pre += wcnt[w][d];
            const uint32_t pos = base[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        base[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        for (int w = 0; w < 4; ++w)
            wcnt[w][t] = 0;
        if (t < 4)
            wcnt[t][256] = 0;
        __syncthreads();
    }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t scan_tmp_words(int64_t n)
{
    size_t words = 0;
    int64_t m = ceil_div(n, kScanTile);
    while (m > 1) {
        words += (size_t)m;
        m = ceil_div(m, kScanTile);
    }
    return words + 1;
}

grav_status scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                               hipStream_t s)
{
    if (n <= 0)
        return GRAV_OK;
    const int64_t nblk = ceil_div(n, kScanTile);
    if (nblk > 0x7fffffff)
        return GRAV_EUNSUPPORTED;
    uint32_t *sums = nblk > 1 ? tmp : nullptr;
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, in, out, n,
                       sums);
    GRAV_HIP(hipGetLastError());
    if (nblk > 1) {
        GRAV_CHECK(scan_exclusive_u32(sums, sums, nblk, tmp + nblk, s));
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, out, n,
                           (const uint32_t *)sums);
        GRAV_HIP(hipGetLastError());
    }
    return GRAV_OK;
}

size_t radix_scratch_words(int64_t n)
{
    const int64_t nblk = ceil_div(n > 0 ? n : 1, kRadixTile);
    return (size_t)(2 * 256 * nblk) + scan_tmp_words(256 * nblk);
}

grav_status radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp,
                             uint32_t *vals_tmp, int64_t n, int bits, uint32_t *scratch,
                             hipStream_t s)
{
    if (n <= 1 || bits <= 0)
        return GRAV_OK;
    const int64_t nblk64 = ceil_div(n, kRadixTile);
    if (nblk64 > 0x7fffffff || n > 0xffffffffll)
        return GRAV_EUNSUPPORTED;
    const int nblk = (int)nblk64;
    uint32_t *hist = scratch;
    uint32_t *offs = scratch + 256 * nblk64;
    uint32_t *tmp = scratch + 2 * 256 * nblk64;
    uint32_t *kin = keys, *vin = vals, *kout = keys_tmp, *vout = vals_tmp;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8, ++passes) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kRadixThreads), 0, s,
                           (const uint32_t *)kin, n, shift, hist, nblk);
        GRAV_HIP(hipGetLastError());
        GRAV_CHECK(scan_exclusive_u32(hist, offs, 256 * nblk64, tmp, s));
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kRadixThreads), 0, s,
                           (const uint32_t *)kin, (const uint32_t *)vin, kout, vout, n, shift,
                           (const uint32_t *)offs, nblk);
        GRAV_HIP(hipGetLastError());
        uint32_t *tk = kin, *tv = vin;
        kin = kout;
        vin = vout;
        kout = tk;
        vout = tv;
    }
    if (passes & 1) {
        GRAV_HIP(hipMemcpyAsync(keys, kin, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
        GRAV_HIP(hipMemcpyAsync(vals, vin, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    return GRAV_OK;
}

}  // namespace grav
