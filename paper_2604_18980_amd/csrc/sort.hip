// Device-wide scans and the stable LSD radix sort used by stages 2 and 3.
//
// The radix sort is a reduce-then-scan LSD sort with 8-bit digits:
//   k_radix_hist     per-block digit histogram in LDS (one 256-bin histogram per
//                    wave, merged), written digit-major so that
//   scan             one flat exclusive scan turns it into per-(digit, block)
//                    output offsets, and
//   k_radix_scatter  re-reads the block's keys and ranks them stably: each wave
//                    walks its quarter of the chunk 64 items at a time, finds
//                    the lanes holding the same digit with 8 ballots, and keeps
//                    a running per-digit count in LDS; wave prefixes then order
//                    the four waves.
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
    T acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;
        if (idx < m) acc += in[idx];
    }
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
hipError_t scan_exclusive_u64(const uint64_t *in, uint64_t *out, int64_t m, uint64_t *parts,
                              int64_t *total, hipStream_t s, DevExtent ext) {
    return scan_exclusive<uint64_t>(in, out, m, parts, total, ext, s);
}

// ------------------------------------------------------------------ radix sort


__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *keys, const int64_t *count,
                                                             int64_t cap, int shift, uint32_t *hist,
                                                             int64_t nblocks, int empty_if_over) {
    __shared__ uint32_t h[kSortThreads / kWave][256];
    const int wid = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < (kSortThreads / kWave) * 256; i += kSortThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t n = live_count(count, cap, empty_if_over);
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    if (base >= n) return;  // idle block (uniform): holds no items, owns no histogram column
    const int64_t nb_live = (n + kSortChunk - 1) / kSortChunk;
    if (base + kSortChunk <= n) {
        // full chunk: 16-byte loads, four keys each
        const uint4 *k4 = reinterpret_cast<const uint4 *>(keys + base);
#pragma unroll
        for (int i = 0; i < kSortItems / 4; ++i) {
            const uint4 q = k4[i * kSortThreads + threadIdx.x];
            atomicAdd(&h[wid][(q.x >> shift) & 255u], 1u);
            atomicAdd(&h[wid][(q.y >> shift) & 255u], 1u);
            atomicAdd(&h[wid][(q.z >> shift) & 255u], 1u);
            atomicAdd(&h[wid][(q.w >> shift) & 255u], 1u);
        }
    } else {
        for (int i = 0; i < kSortItems; ++i) {
            const int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
            if (idx < n) atomicAdd(&h[wid][(keys[idx] >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    const int d = threadIdx.x;  // kSortThreads == 256 digits
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) tot += h[w][d];
    hist[(int64_t)d * nb_live + blockIdx.x] = tot;
}

// Scatter: re-reads the block's keys, ranks them stably by the digit and
// writes each digit's run contiguously (radix_rank.hpp).
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, const int64_t *count,
    int64_t cap, int shift, const uint32_t *offs, int64_t nblocks, int empty_if_over) {
    __shared__ RankSmem sm;
    __shared__ uint32_t skey[kSortChunk];
    __shared__ uint32_t sval[kSortChunk];
    rank_init(sm);
    const int64_t n = live_count(count, cap, empty_if_over);
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    if (base >= n) return;  // whole block idle (uniform across the block)
    const int64_t nb_live = (n + kSortChunk - 1) / kSortChunk;
    sm.gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * nb_live + blockIdx.x];
    __syncthreads();
    const int cnt = (int)(n - base < kSortChunk ? n - base : kSortChunk);
    uint32_t key[kSortItems], val[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int p = rank_pos(i);
        key[i] = p < cnt ? kin[base + p] : 0u;
        val[i] = p < cnt ? vin[base + p] : 0u;
    }
    rank_stage_write(
        key, val, cnt, shift, sm, skey, sval, [](uint32_t, uint32_t v) { return v; },
        [&](int64_t dst, uint32_t k, uint32_t v) {
            if (kout) kout[dst] = k;
            vout[dst] = v;
        });
}

hipError_t radix_sort_u32(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                          uint32_t *ktmp, uint32_t *vtmp, const int64_t *count, int64_t cap,
                          int bits, uint32_t *hist, int64_t nblocks, uint64_t *parts,
                          hipStream_t s, int first_bit, int empty_if_over) {
    const int passes = bits <= first_bit ? 1 : (bits - first_bit + 7) / 8;
    // choose buffers so the last pass lands in (kout, vout)
    const uint32_t *srck = kin, *srcv = vin;
    for (int p = 0; p < passes; ++p) {
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        uint32_t *dk = to_out ? kout : ktmp, *dv = to_out ? vout : vtmp;
        const int shift = first_bit + 8 * p;
        radix_pass(srck, srcv, dk, dv, count, cap, shift, hist, nblocks, parts, s, empty_if_over);
        srck = dk;
        srcv = dv;
    }
    return hipGetLastError();
}

void radix_hist(const uint32_t *keys, const int64_t *count, int64_t cap, int shift, uint32_t *hist,
                int64_t nblocks, uint64_t *parts, hipStream_t s, int empty_if_over) {
    k_radix_hist<<<(unsigned)nblocks, kSortThreads, 0, s>>>(keys, count, cap, shift, hist, nblocks,
                                                            empty_if_over);
    // histogram columns exist for live blocks only: 256 x ceil(count / chunk)
    scan_exclusive_u32(hist, hist, 256 * nblocks, parts, nullptr, s,
                       DevExtent{count, cap, kSortChunk, 256, empty_if_over != 0});
}

void radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                const int64_t *count, int64_t cap, int shift, uint32_t *hist, int64_t nblocks,
                uint64_t *parts, hipStream_t s, int empty_if_over) {
    radix_hist(kin, count, cap, shift, hist, nblocks, parts, s, empty_if_over);
    k_radix_scatter<<<(unsigned)nblocks, kSortThreads, 0, s>>>(kin, vin, kout, vout, count, cap,
                                                                shift, hist, nblocks, empty_if_over);
}

// ---------------------------------------------------------- depth presort
// The same LSD passes without device-wide scan kernels and without atomics
// that many blocks aim at one address (global atomics on one address
// serialise, about 50 ns each).  The histogram kernel stores each block's
// digit counts (digit-major) and adds them to sums over groups of blocks
// (DepthRegime::group blocks per sum, so an address takes that many atomics);
// each scatter block forms its offsets from its group's earlier counts and
// every group sum: the sum over all groups is the digit's total, the sum over
// the earlier groups plus the earlier blocks of its own group its start
// within the digit.  Up to kDepthSmallMax visible keys the blocks hold 1024
// keys (about one block per compute unit at a few hundred thousand keys, so
// the per-block ranking, which is bound by LDS latency, runs on the whole
// chip); above, 4096.  The regime is chosen on the device from the count,
// uniformly for all blocks; the grid is sized for the small blocks.
constexpr int64_t kDepthSmallMax = 512 * 1024;
template <int ITEMS>
struct DepthRegime {
    static constexpr int items = ITEMS;
    static constexpr int64_t chunk = (int64_t)ITEMS * kSortThreads;
    static constexpr int group = ITEMS == 4 ? 16 : 32;  // blocks per group sum
};
using DepthSmall = DepthRegime<4>;
using DepthLarge = DepthRegime<16>;
static_assert(DepthLarge::chunk == kSortChunk, "LDS staging is sized for the large blocks");
static_assert(kDepthSmallMax / DepthSmall::chunk <= 32 * DepthSmall::group,
              "small regime: at most 32 group sums");

template <class Rg>
__device__ __forceinline__ void dhist_body(const uint32_t *keys, int64_t n, int shift,
                                           uint32_t *hist, int64_t nb, uint32_t *gsum,
                                           int64_t ngroups, uint32_t (*h)[256]) {
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
    hist[(int64_t)d * nb + b] = c;
    if (c) atomicAdd(gsum + (int64_t)d * ngroups + b / Rg::group, c);
}

__global__ __launch_bounds__(kSortThreads) void k_dhist(const uint32_t *keys, const int64_t *count,
                                                        int shift, uint32_t *hist, int64_t nb,
                                                        uint32_t *gsum, int64_t ngroups) {
    __shared__ uint32_t h[kSortThreads / kWave][256];
    for (int i = threadIdx.x; i < (kSortThreads / kWave) * 256; i += kSortThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t n = *count;
    if (n <= kDepthSmallMax)
        dhist_body<DepthSmall>(keys, n, shift, hist, nb, gsum, ngroups, h);
    else
        dhist_body<DepthLarge>(keys, n, shift, hist, nb, gsum, ngroups, h);
}

template <class Rg>
__device__ __forceinline__ void dscatter_body(const uint32_t *kin, const uint32_t *vin,
                                              uint32_t *kout, uint32_t *vout, int64_t n, int shift,
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
    const uint32_t *hrow = hist + (int64_t)d * nb + g * Rg::group;
    const uint32_t *grow = gsum + (int64_t)d * ngroups;
    uint32_t pre = 0, t = 0;
    constexpr int kBatch = Rg::items == DepthSmall::items ? 32 : 16;
    for (int64_t i0 = 0; i0 < lg; i0 += kBatch) {  // one batch in the small regime
        uint32_t c[kBatch], e[Rg::group - 1];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) c[i] = i0 + i < lg ? grow[i0 + i] : 0u;
        if (i0 == 0) {
#pragma unroll
            for (int i = 0; i < Rg::group - 1; ++i) e[i] = i < in_group ? hrow[i] : 0u;
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

__global__ __launch_bounds__(kSortThreads) void k_dscatter(const uint32_t *kin, const uint32_t *vin,
                                                           uint32_t *kout, uint32_t *vout,
                                                           const int64_t *count, int shift,
                                                           const uint32_t *hist, int64_t nb,
                                                           const uint32_t *gsum, int64_t ngroups) {
    __shared__ RankSmem sm;
    __shared__ uint32_t skey[kSortChunk];
    __shared__ uint32_t sval[kSortChunk];
    __shared__ uint32_t s_wt[kSortThreads / kWave];
    rank_init(sm);
    const int64_t n = *count;
    if (n <= kDepthSmallMax)
        dscatter_body<DepthSmall>(kin, vin, kout, vout, n, shift, hist, nb, gsum, ngroups, sm, skey,
                                  sval, s_wt);
    else
        dscatter_body<DepthLarge>(kin, vin, kout, vout, n, shift, hist, nb, gsum, ngroups, sm, skey,
                                  sval, s_wt);
}

int64_t depth_pass_blocks(int64_t n) { return n > 0 ? (n + DepthSmall::chunk - 1) / DepthSmall::chunk : 1; }
int64_t depth_pass_groups(int64_t n) {
    return (depth_pass_blocks(n) + DepthSmall::group - 1) / DepthSmall::group;
}

hipError_t depth_sort(const Workspace &ws, const int64_t *count, hipStream_t s) {
    // 0 -> 2 -> 1 -> 2 -> 1: the fourth pass lands in buffer 1
    const int src[4] = {0, 2, 1, 2}, dst[4] = {2, 1, 2, 1};
    const unsigned nb = (unsigned)ws.nb_dpass;
    for (int p = 0; p < 4; ++p) {
        uint32_t *gsum = ws.dgsum + (int64_t)p * 256 * ws.nb_dgroups;
        k_dhist<<<nb, kSortThreads, 0, s>>>(ws.dkey[src[p]], count, 8 * p, ws.dhist, ws.nb_dpass, gsum,
                                           ws.nb_dgroups);
        k_dscatter<<<nb, kSortThreads, 0, s>>>(ws.dkey[src[p]], ws.dval[src[p]], ws.dkey[dst[p]],
                                              ws.dval[dst[p]], count, 8 * p, ws.dhist, ws.nb_dpass,
                                              gsum, ws.nb_dgroups);
    }
    return hipGetLastError();
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
                              uint32_t *ranges, int num_tiles, hipStream_t s, int empty_if_over) {
    const int64_t m = 2 * (int64_t)num_tiles;
    k_fill_u32<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(ranges, m, 0u);
    if (cap > 0)
        k_tile_ranges<<<(unsigned)((cap + 1023) / 1024), 256, 0, s>>>(sorted_tiles, num_pairs, cap, ranges,
                                                                      (uint32_t)num_tiles, empty_if_over);
    return hipGetLastError();
}

}  // namespace gsr
