// Device-wide scans and the stable LSD radix sort used by the depth presort
// and the tile sort (the sort's design is described at its kernels below).
// Counts live in device memory (read by every kernel and clamped to the
// capacity the grid was sized for), so no stage needs a host round trip.
#include "gsr_internal.hpp"
#include "radix_rank.hpp"

namespace gsr {

// ------------------------------------------------------------------- scans
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T *in, int64_t m, uint64_t *parts,
                                                              DevExtent ext, int64_t *total) {
    __shared__ T wt[kScanThreads / kWave];
    m = ext.resolve(m);
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    // the total of an empty input; k_scan_down's last live block overwrites it
    if (total && blockIdx.x == 0 && threadIdx.x == 0) *total = 0;
    if (base >= m) {  // past the live elements: contributes nothing
        if (threadIdx.x == 0) parts[blockIdx.x] = 0;
        return;
    }
    T v[kScanItems], acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) v[i] = load_or_zero(in, base + (int64_t)i * kScanThreads + threadIdx.x, m);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) acc += v[i];
    T tot;
    block_exclusive_scan<kScanThreads, T>(acc, wt, &tot);
    if (threadIdx.x == 0) parts[blockIdx.x] = (uint64_t)tot;
}

// Each block rescans its chunk: thread t owns kScanItems consecutive elements.
// The block's offset, the sum of the partials of the blocks before it, is
// reduced here (the partial count is small), so no separate pass scans them;
// the last live block stores the grand total.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const T *in, T *out, int64_t m,
                                                            const uint64_t *parts, DevExtent ext,
                                                            int64_t *total) {
    __shared__ T wt[kScanThreads / kWave];
    __shared__ uint64_t wt64[kScanThreads / kWave];
    m = ext.resolve(m);
    if ((int64_t)blockIdx.x * kScanChunk >= m) return;
    // the chunk and the partials before it are requested together
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < m ? in[idx] : 0;
    }
    uint64_t before = 0;
    for (int64_t i0 = threadIdx.x; i0 < (int64_t)blockIdx.x; i0 += 4 * kScanThreads) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            before += i0 + k * kScanThreads < (int64_t)blockIdx.x ? parts[i0 + k * kScanThreads] : 0ull;
    }
    uint64_t btot;
    block_exclusive_scan<kScanThreads, uint64_t>(before, wt64, &btot);
    T acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) acc += v[i];
    T tot;
    T run = block_exclusive_scan<kScanThreads, T>(acc, wt, &tot) + (T)btot;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (idx < m) out[idx] = run;
        run += v[i];
    }
    if (total && threadIdx.x == 0 && ((int64_t)blockIdx.x + 1) * kScanChunk >= m)
        *total = (int64_t)(btot + (uint64_t)tot);
}

__global__ void k_set_total(int64_t *total) { *total = 0; }

template <typename T>
static hipError_t scan_exclusive(const T *in, T *out, int64_t m, uint64_t *parts, int64_t *total,
                                 DevExtent ext, hipStream_t s) {
    const int64_t nparts = (m + kScanChunk - 1) / kScanChunk;
    if (nparts == 0) {
        if (total) k_set_total<<<1, 1, 0, s>>>(total);
        return hipGetLastError();
    }
    k_scan_reduce<T><<<(unsigned)nparts, kScanThreads, 0, s>>>(in, m, parts, ext, total);
    k_scan_down<T><<<(unsigned)nparts, kScanThreads, 0, s>>>(in, out, m, parts, ext, total);
    return hipGetLastError();
}

hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t m, uint64_t *parts,
                              int64_t *total, hipStream_t s, DevExtent ext) {
    return scan_exclusive<uint32_t>(in, out, m, parts, total, ext, s);
}

__global__ void k_fill_u32(uint32_t *p, int64_t m, uint32_t v);

// ------------------------------------------------------------------ LSD sort
// Stable LSD radix sort of (key, value) pairs, 8-bit digits, two kernels per
// pass and no device-wide scan kernels or atomics that many blocks aim at one
// address (global atomics on one address serialise, about 50 ns each):
//   k_lsd_hist     per-block digit histogram in LDS, stored block-major, and
//                  added to sums over groups of blocks, group-major
//                  (Regime::group blocks per sum, so an address takes that
//                  many atomics);
//   k_lsd_scatter  forms its offsets itself -- the sum over all groups is a
//                  digit's total, the sum over the earlier groups plus the
//                  earlier blocks of its own group its start within the digit
//                  -- re-reads its keys and ranks them stably (radix_rank.hpp):
//                  each wave walks its part of the chunk 64 items at a time,
//                  finds the lanes holding the same digit with 8 ballots and
//                  keeps a running per-digit count in LDS; wave prefixes then
//                  order the waves.
// Up to kLsdSmallMax live items the blocks hold 1024 (about one block per
// compute unit at a few hundred thousand items, so the per-block ranking,
// bound by LDS latency, runs on the whole chip); above, 4096.  The regime is
// chosen on the device from the count, uniformly for all blocks; the grid is
// sized for the small blocks.  The group sums of consecutive passes alternate
// between two buffers: a pass's histogram kernel clears the next pass's
// (whose last reader, the previous pass's scatter, has finished).
constexpr int64_t kLsdSmallMax = 512 * 1024;
template <int ITEMS>
struct LsdRegime {
    static constexpr int items = ITEMS;
    static constexpr int64_t chunk = (int64_t)ITEMS * kSortThreads;
    static constexpr int group = ITEMS == 4 ? 16 : 32;  // blocks per group sum
};
using LsdSmall = LsdRegime<4>;
using LsdLarge = LsdRegime<16>;
static_assert(LsdLarge::chunk == kSortChunk, "LDS staging is sized for the large blocks");
static_assert(kLsdSmallMax / LsdSmall::chunk <= 32 * LsdSmall::group,
              "small regime: at most 32 group sums");

int64_t lsd_pass_blocks(int64_t cap) { return cap > 0 ? (cap + LsdSmall::chunk - 1) / LsdSmall::chunk : 1; }
int64_t lsd_pass_groups(int64_t cap) {
    return (lsd_pass_blocks(cap) + LsdSmall::group - 1) / LsdSmall::group;
}

template <class Rg>
__device__ __forceinline__ void lsd_hist_body(const uint32_t *keys, int64_t n, int shift, uint32_t *hist,
                                              int64_t nb, uint32_t *gsum, int64_t ngroups,
                                              uint32_t (*h)[256]) {
    const int64_t b = blockIdx.x, base = b * Rg::chunk;
    if (base >= n) return;  // uniform
    const int wid = threadIdx.x / kWave;
    uint32_t k[Rg::items];
#pragma unroll
    for (int i = 0; i < Rg::items; ++i) {
        const int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        k[i] = idx < n ? keys[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < Rg::items; ++i) {
        const int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[wid][(k[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) c += h[w][d];
    hist[b * 256 + d] = c;
    if (c) atomicAdd(gsum + (b / Rg::group) * 256 + d, c);
}

__global__ __launch_bounds__(kSortThreads) void k_lsd_hist(const uint32_t *keys, const int64_t *count,
                                                           int64_t cap, int empty_if_over, int shift,
                                                           uint32_t *hist, int64_t nb, uint32_t *gsum,
                                                           uint32_t *gsum_next, int64_t ngroups) {
    __shared__ uint32_t h[kSortThreads / kWave][256];
    for (int i = threadIdx.x; i < (kSortThreads / kWave) * 256; i += kSortThreads) (&h[0][0])[i] = 0;
    if (gsum_next)
        for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < 256 * ngroups;
             i += (int64_t)gridDim.x * kSortThreads)
            gsum_next[i] = 0u;
    __syncthreads();
    const int64_t n = live_count(count, cap, empty_if_over);
    if (n <= kLsdSmallMax)
        lsd_hist_body<LsdSmall>(keys, n, shift, hist, nb, gsum, ngroups, h);
    else
        lsd_hist_body<LsdLarge>(keys, n, shift, hist, nb, gsum, ngroups, h);
}

template <class Rg>
__device__ __forceinline__ void lsd_scatter_body(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                                 uint32_t *vout, int64_t n, int shift,
                                                 const uint32_t *hist, int64_t nb, const uint32_t *gsum,
                                                 int64_t ngroups, RankSmem &sm, uint32_t *skey,
                                                 uint32_t *sval, uint32_t *s_wt) {
    const int64_t b = blockIdx.x, base = b * Rg::chunk;
    if (base >= n) return;  // uniform
    // the chunk's keys and this digit's counts are all requested before any
    // of them is used (one round trip, mostly to other XCDs' writes)
    const int cnt = (int)(n - base < Rg::chunk ? n - base : Rg::chunk);
    uint32_t key[Rg::items], val[Rg::items];
#pragma unroll
    for (int i = 0; i < Rg::items; ++i) {
        const int p = rank_pos<Rg::items>(i);
        key[i] = p < cnt ? kin[base + p] : 0u;
        val[i] = p < cnt ? vin[base + p] : 0u;
    }
    const int d = threadIdx.x;
    const int64_t live = (n + Rg::chunk - 1) / Rg::chunk;
    const int64_t lg = (live + Rg::group - 1) / Rg::group, g = b / Rg::group;
    const int in_group = (int)(b - g * Rg::group);
    // block-major counts and group-major sums: a wave's 64 digits are
    // consecutive words of each row
    const uint32_t *hrow = hist + g * Rg::group * 256 + d;
    const uint32_t *grow = gsum + d;
    uint32_t pre = 0, t = 0;
    constexpr int kBatch = Rg::items == LsdSmall::items ? 32 : 16;
    for (int64_t i0 = 0; i0 < lg; i0 += kBatch) {  // one batch in the small regime
        uint32_t c[kBatch], e[Rg::group - 1];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) c[i] = i0 + i < lg ? grow[(i0 + i) * 256] : 0u;
        if (i0 == 0) {
#pragma unroll
            for (int i = 0; i < Rg::group - 1; ++i) e[i] = i < in_group ? hrow[i * 256] : 0u;
#pragma unroll
            for (int i = 0; i < Rg::group - 1; ++i) pre += e[i];
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            t += c[i];
            pre += i0 + i < g ? c[i] : 0u;
        }
    }
    uint32_t all;
    sm.gbase[d] = block_exclusive_scan<kSortThreads, uint32_t>(t, s_wt, &all) + pre;
    __syncthreads();
    rank_stage_write<Rg::items>(
        key, val, cnt, shift, sm, skey, sval, [](uint32_t, uint32_t v) { return v; },
        [&](int64_t dst, uint32_t k, uint32_t v) {
            kout[dst] = k;
            vout[dst] = v;
        });
}

__global__ __launch_bounds__(kSortThreads) void k_lsd_scatter(const uint32_t *kin, const uint32_t *vin,
                                                              uint32_t *kout, uint32_t *vout,
                                                              const int64_t *count, int64_t cap,
                                                              int empty_if_over, int shift,
                                                              const uint32_t *hist, int64_t nb,
                                                              const uint32_t *gsum, int64_t ngroups) {
    __shared__ RankSmem sm;
    __shared__ uint32_t skey[kSortChunk];
    __shared__ uint32_t sval[kSortChunk];
    __shared__ uint32_t s_wt[kSortThreads / kWave];
    rank_init(sm);
    const int64_t n = live_count(count, cap, empty_if_over);
    if (n <= kLsdSmallMax)
        lsd_scatter_body<LsdSmall>(kin, vin, kout, vout, n, shift, hist, nb, gsum, ngroups, sm, skey, sval,
                                   s_wt);
    else
        lsd_scatter_body<LsdLarge>(kin, vin, kout, vout, n, shift, hist, nb, gsum, ngroups, sm, skey, sval,
                                   s_wt);
}

hipError_t radix_sort_u32(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                          uint32_t *ktmp, uint32_t *vtmp, const int64_t *count, int64_t cap,
                          int bits, uint32_t *hist, uint32_t *gsum, hipStream_t s, int first_bit,
                          int empty_if_over, bool gsum_zeroed) {
    const int passes = bits <= first_bit ? 1 : (bits - first_bit + 7) / 8;
    const int64_t nb = lsd_pass_blocks(cap), ng = lsd_pass_groups(cap);
    if (!gsum_zeroed) k_fill_u32<<<(unsigned)((256 * ng + 255) / 256), 256, 0, s>>>(gsum, 256 * ng, 0u);
    // choose buffers so the last pass lands in (kout, vout)
    const uint32_t *srck = kin, *srcv = vin;
    for (int p = 0; p < passes; ++p) {
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        uint32_t *dk = to_out ? kout : ktmp, *dv = to_out ? vout : vtmp;
        const int shift = first_bit + 8 * p;
        uint32_t *cur = gsum + (p % 2) * 256 * ng, *next = gsum + ((p + 1) % 2) * 256 * ng;
        k_lsd_hist<<<(unsigned)nb, kSortThreads, 0, s>>>(srck, count, cap, empty_if_over, shift, hist, nb, cur,
                                                        p + 1 < passes ? next : nullptr, ng);
        k_lsd_scatter<<<(unsigned)nb, kSortThreads, 0, s>>>(srck, srcv, dk, dv, count, cap, empty_if_over,
                                                           shift, hist, nb, cur, ng);
        srck = dk;
        srcv = dv;
    }
    return hipGetLastError();
}

hipError_t depth_sort(const Workspace &ws, const int64_t *count, hipStream_t s) {
    // dkey/dval[0] -> [1], [2] as the pass scratch; the group sums were cleared
    // by the visibility count
    return radix_sort_u32(ws.dkey[0], ws.dval[0], ws.dkey[1], ws.dval[1], ws.dkey[2], ws.dval[2], count,
                          ws.nb_dpass * LsdSmall::chunk, 32, ws.dhist, ws.dgsum, s, 0, 0, true);
}

// ------------------------------------------------------------- tile ranges
__global__ void k_fill_u32(uint32_t *p, int64_t m, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = v;
}

// Thread i tests the boundary between items i-1 and i, for four consecutive i
// per thread (one 16-byte load plus the item before).
// Tile ids at or beyond the tile count (none from the emitters) write nothing.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t *tiles, const int64_t *count,
                                                     int64_t cap, uint32_t *ranges, uint32_t ntiles,
                                                     int empty_if_over) {
    const int64_t n = live_count(count, cap, empty_if_over);
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    uint32_t t[5];
    t[0] = i0 > 0 ? tiles[i0 - 1] : 0xffffffffu;
    if (i0 + 4 <= n) {
        const uint4 q = *reinterpret_cast<const uint4 *>(tiles + i0);
        t[1] = q.x; t[2] = q.y; t[3] = q.z; t[4] = q.w;
    } else {
        for (int k = 0; k < 4; ++k) t[1 + k] = i0 + k < n ? tiles[i0 + k] : 0xffffffffu;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = i0 + k;
        if (i >= n) break;
        if (t[k + 1] != t[k]) {
            if (t[k + 1] < ntiles) ranges[2 * (int64_t)t[k + 1]] = (uint32_t)i;
            if (i > 0 && t[k] < ntiles) ranges[2 * (int64_t)t[k] + 1] = (uint32_t)i;
        }
    }
    if (i0 + 4 >= n && i0 < n) {
        const uint32_t last = tiles[n - 1];
        if (last < ntiles) ranges[2 * (int64_t)last + 1] = (uint32_t)n;
    }
}

hipError_t launch_tile_ranges(const uint32_t *sorted_tiles, const int64_t *num_pairs, int64_t cap,
                              uint32_t *ranges, int num_tiles, hipStream_t s, int empty_if_over,
                              bool ranges_zeroed) {
    const int64_t m = 2 * (int64_t)num_tiles;
    if (!ranges_zeroed) k_fill_u32<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(ranges, m, 0u);
    if (cap > 0)
        k_tile_ranges<<<(unsigned)((cap + 1023) / 1024), 256, 0, s>>>(sorted_tiles, num_pairs, cap, ranges,
                                                                      (uint32_t)num_tiles, empty_if_over);
    return hipGetLastError();
}

}  // namespace gsr
