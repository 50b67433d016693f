// Stages 2+3 fused (paper Sec. 2.1: pair generation, sorting, tile ranges):
// the per-tile depth-ordered lists without the emission-order pair arrays.
//
// After the depth presort of the visible Gaussians (launch_emit_prepare), the
// pairs are defined implicitly: pair k belongs to the depth-sorted Gaussian j
// with off[j] <= k < off[j+1] and lies on tile number k - off[j] of j's
// rectangle (rows outer).  A stable sort by tile id of that sequence is the
// result.  With at most 2^16 tiles and fewer than 2^24 Gaussians it runs as two
// 8-bit LSD passes whose first pass generates its items instead of reading
// them and writes one 32-bit word per pair:
//
//   k_bin_hist       per 4096-pair slice: low-byte histogram of the pairs' tiles
//   scan
//   k_bin_scatter1   regenerate the slice, rank by the low byte (radix_rank.hpp),
//                    write (tile >> 8) << 24 | depth rank j
//   k_bin_hist2      high-byte histogram of the packed words, scan
//   k_bin_scatter2   rank by the high byte, write sorted_gids = id of rank j
//                    (and, optionally, the tile id: high byte from the word, low
//                    byte from the pass-1 bucket that held it)
//
// Pass 2 runs bucket-aligned: each of its blocks holds items of a single
// pass-1 bucket (one low byte l), so the digit-major exclusive offsets of its
// histogram give the lists for free -- tile (h, l) occupies
// [offs(h, first block of l), offs(h, first block of l + 1)).  With at most 256
// tiles, pass 1 writes the final lists directly and its bucket starts are the
// ranges.  Beyond the packed limits, and under the ellipse and oriented-box
// extent rules (whose per-Gaussian pairs are row spans, not a rectangle), the
// path emits pairs and sorts them.
//
// If the pair count exceeds the capacity, nothing is binned: every range is
// empty and num_pairs holds the required count.
#include "gsr_internal.hpp"
#include "radix_rank.hpp"

namespace gsr {

static_assert(kEmitChunk == kSortChunk, "one emission slice per ranking block");

constexpr int kRankBits = 24;  // depth-rank bits of a packed pass-1 word
constexpr uint32_t kRankMask = (1u << kRankBits) - 1u;

bool bin_packed(int64_t n, int tiles_x, int tiles_y) {
    return n < ((int64_t)1 << kRankBits) && (int64_t)tiles_x * tiles_y <= 65536;
}

namespace {

// The depth-sorted Gaussians owning the pairs of one slice [p0, p1), in LDS:
// for owner o (Gaussian ja + o), where its pairs start relative to p0 (0 for
// the first owner, whose pairs may start before p0: m0 = p0 - off[ja]), its
// rectangle's first tile column and row and its width.  A bitmap marks the
// slice positions where an owner's pairs start, so the owner of position k is
// the number of marks at or before k, less one.
struct Owners {
    uint16_t rel[kEmitChunk], x0[kEmitChunk], y0[kEmitChunk], w[kEmitChunk];
    uint32_t marks[kEmitChunk / 32];
    uint32_t mark_prefix[kEmitChunk / 32];
    uint32_t wt[kSortThreads / kWave];
    uint32_t ja, m0;
};

struct SliceArgs {
    const uint32_t *sorted_ids;  // depth-sorted visible Gaussians
    const int64_t *num_vis;
    const uint64_t *rects;
    const uint64_t *pair_off;    // exclusive prefix of the pair counts, by depth rank
    const uint32_t *slice_start; // owner of each slice's first pair
    const int64_t *num_pairs;
    int64_t cap;
    int tiles_x;
};

// Loads the owners of slice b (pairs [p0, p1), P = total pairs <= cap).
// Contains barriers.
__device__ void load_owners(const SliceArgs &a, int64_t b, int64_t p0, int64_t p1, int64_t P,
                            Owners &ow) {
    const uint32_t ja = a.slice_start[b];
    uint32_t jb;
    if (p1 < P) {  // the next slice's owner, unless its pairs start exactly at p1
        const uint32_t jn = a.slice_start[b + 1];
        jb = a.pair_off[jn] == (uint64_t)p1 ? jn - 1u : jn;
    } else {
        jb = (uint32_t)(*a.num_vis - 1);
    }
    // every owner after the first starts strictly inside the slice, so
    // no <= p1 - p0 <= kEmitChunk (clamped all the same: the LDS table holds
    // kEmitChunk owners)
    int no = (int)(jb - ja) + 1;
    no = no < 1 ? 1 : (no > kEmitChunk ? kEmitChunk : no);
    for (int i = threadIdx.x; i < kEmitChunk / 32; i += kSortThreads) ow.marks[i] = 0u;
    __syncthreads();
    const int64_t V = *a.num_vis;
    for (int o = threadIdx.x; o < no; o += kSortThreads) {
        const uint32_t j = ja + (uint32_t)o;
        if ((int64_t)j >= V) break;  // cannot happen with consistent offsets; keeps reads in bounds
        const uint64_t r = a.rects[a.sorted_ids[j]];
        const uint32_t x0 = r & 0xffff, y0 = (r >> 16) & 0xffff, x1 = (r >> 32) & 0xffff;
        const uint64_t off = a.pair_off[j];
        const uint64_t rel64 = o == 0 ? 0ull : off - (uint64_t)p0;
        if (rel64 >= (uint64_t)kEmitChunk) continue;  // likewise impossible; keeps LDS in bounds
        const uint32_t rel = (uint32_t)rel64;
        ow.rel[o] = (uint16_t)rel;
        ow.x0[o] = (uint16_t)x0;
        ow.y0[o] = (uint16_t)y0;
        ow.w[o] = (uint16_t)(x1 - x0);
        atomicOr(&ow.marks[rel >> 5], 1u << (rel & 31));
        if (o == 0) {
            ow.ja = ja;
            ow.m0 = (uint32_t)((uint64_t)p0 - off);
        }
    }
    __syncthreads();
    const uint32_t c = threadIdx.x < kEmitChunk / 32 ? (uint32_t)__popc(ow.marks[threadIdx.x]) : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kSortThreads, uint32_t>(c, ow.wt, &tot);
    if (threadIdx.x < kEmitChunk / 32) ow.mark_prefix[threadIdx.x] = ex;
    __syncthreads();
}

// Tile and depth rank of pair p0 + k (k < p1 - p0).
__device__ __forceinline__ void slice_pair(const Owners &ow, int k, int tiles_x, uint32_t &tile,
                                           uint32_t &j) {
    const int wi = k >> 5;
    const uint32_t upto = ow.marks[wi] & (0xffffffffu >> (31 - (k & 31)));
    const int o = (int)ow.mark_prefix[wi] + __popc(upto) - 1;
    const uint32_t m = o == 0 ? ow.m0 + (uint32_t)k : (uint32_t)k - ow.rel[o];
    const uint32_t w = ow.w[o];
    // m / w by the hardware reciprocal (within an ulp), corrected by one step:
    // m < 2^22 here, so the truncated estimate is off by at most one
    int q = (int)((float)m * __builtin_amdgcn_rcpf((float)w));
    int r = (int)m - q * (int)w;
    if (r < 0) { --q; r += (int)w; } else if (r >= (int)w) { ++q; r -= (int)w; }
    tile = ((uint32_t)ow.y0[o] + (uint32_t)q) * (uint32_t)tiles_x + ow.x0[o] + (uint32_t)r;
    j = ow.ja + (uint32_t)o;
}

__device__ __forceinline__ bool slice_bounds(const SliceArgs &a, int64_t &P, int64_t &p0,
                                             int64_t &p1, int64_t &nb_live) {
    P = live_count(a.num_pairs, a.cap, 1);
    p0 = (int64_t)blockIdx.x * kEmitChunk;
    if (p0 >= P) return false;
    p1 = p0 + kEmitChunk < P ? p0 + kEmitChunk : P;
    nb_live = (P + kEmitChunk - 1) / kEmitChunk;
    return true;
}
}  // namespace

// Low-byte histogram of the tiles of one slice, digit-major [256][live slices].
__global__ __launch_bounds__(kSortThreads) void k_bin_hist(const SliceArgs a, uint32_t *hist) {
    __shared__ Owners ow;
    __shared__ uint32_t h[kSortThreads / kWave][256];
    int64_t P, p0, p1, nb_live;
    if (!slice_bounds(a, P, p0, p1, nb_live)) return;
    for (int i = threadIdx.x; i < (kSortThreads / kWave) * 256; i += kSortThreads) (&h[0][0])[i] = 0;
    load_owners(a, blockIdx.x, p0, p1, P, ow);
    const int wid = threadIdx.x / kWave;
    const int cnt = (int)(p1 - p0);
    for (int k = threadIdx.x; k < cnt; k += kSortThreads) {
        uint32_t tile, j;
        slice_pair(ow, k, a.tiles_x, tile, j);
        atomicAdd(&h[wid][tile & 255u], 1u);
    }
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) tot += h[w][d];
    hist[(int64_t)d * nb_live + blockIdx.x] = tot;
}

// Pass 1: regenerate the slice, rank by the tile's low byte, write.  FINAL
// (all tiles < 256): the output is the final list (ids, optional tiles);
// otherwise one packed word per pair.
template <bool FINAL>
__global__ __launch_bounds__(kSortThreads) void k_bin_scatter1(const SliceArgs a, const uint32_t *offs,
                                                               uint32_t *packed, uint32_t *sorted_gids,
                                                               uint32_t *sorted_tiles) {
    __shared__ RankSmem sm;
    __shared__ union {
        Owners ow;
        uint32_t stage[2][kSortChunk];
    } u;
    int64_t P, p0, p1, nb_live;
    if (!slice_bounds(a, P, p0, p1, nb_live)) return;
    rank_init(sm);
    sm.gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * nb_live + blockIdx.x];
    load_owners(a, blockIdx.x, p0, p1, P, u.ow);
    const int cnt = (int)(p1 - p0);
    uint32_t key[kSortItems], val[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int k = rank_pos(i);
        uint32_t tile = 0, j = 0;
        if (k < cnt) slice_pair(u.ow, k, a.tiles_x, tile, j);
        key[i] = FINAL ? tile : ((tile >> 8) << kRankBits) | j;
        val[i] = FINAL ? j : (tile & 255u);
    }
    // the ranking digit is the low tile byte: key bits 0..7 when FINAL, else
    // carried in val -- rank on a key whose low byte is that digit.  The owner
    // table is dead from here on; rank_stage_write stages into the same LDS
    // only after its own barriers.
    uint32_t rkey[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) rkey[i] = FINAL ? key[i] : val[i];
    if (FINAL) {
        rank_stage_write(
            rkey, val, cnt, 0, sm, u.stage[0], u.stage[1],
            [&](uint32_t, uint32_t j) { return a.sorted_ids[j]; },
            [&](int64_t dst, uint32_t tile, uint32_t gid) {
                sorted_gids[dst] = gid;
                if (sorted_tiles) sorted_tiles[dst] = tile;
            });
    } else {
        rank_stage_write(
            rkey, key, cnt, 0, sm, u.stage[0], u.stage[1], [](uint32_t, uint32_t word) { return word; },
            [&](int64_t dst, uint32_t, uint32_t word) { packed[dst] = word; });
    }
}

// Pass-2 plan (one block): bucket starts B[l] (the pass-1 offsets of slice
// 0; B[256] = P) and the first pass-2 block of each bucket, bfirst[l]
// (bfirst[256] = number of pass-2 blocks, also stored in *nb2).
__global__ __launch_bounds__(256) void k_bin_plan2(const uint32_t *hist1, const int64_t *num_pairs,
                                                   int64_t cap, uint32_t *plan, int64_t *nb2) {
    __shared__ uint32_t wt[256 / kWave];
    const int64_t P = live_count(num_pairs, cap, 1);
    const int64_t nb1 = (P + kSortChunk - 1) / kSortChunk;
    const int l = threadIdx.x;
    const uint32_t b0 = P > 0 ? hist1[(int64_t)l * nb1] : 0u;
    const uint32_t b1 = P > 0 ? (l < 255 ? hist1[(int64_t)(l + 1) * nb1] : (uint32_t)P) : 0u;
    const uint32_t blocks = (b1 - b0 + kSortChunk - 1) / kSortChunk;
    uint32_t tot;
    const uint32_t first = block_exclusive_scan<256, uint32_t>(blocks, wt, &tot);
    plan[l] = b0;
    plan[257 + l] = first;
    if (l == 0) {
        plan[256] = (uint32_t)P;
        plan[257 + 256] = tot;
        *nb2 = tot;
    }
}

struct Pass2Block {
    int l;             // the bucket (tile low byte)
    int64_t base;      // first item
    int cnt;           // items
    int64_t nb2;
};

// Which bucket and items pass-2 block b holds (false for an idle block, the
// same for the whole block).  s_bfirst: LDS copy of bfirst[0..256].
// Contains a barrier.
__device__ __forceinline__ bool pass2_block(const uint32_t *plan, const int64_t *nb2_p,
                                            uint32_t *s_bfirst, Pass2Block &pb) {
    const int64_t nb2 = *nb2_p;
    const uint32_t b = blockIdx.x;
    if ((int64_t)b >= nb2) return false;
    s_bfirst[threadIdx.x] = plan[257 + threadIdx.x];
    if (threadIdx.x == 0) s_bfirst[256] = plan[257 + 256];
    __syncthreads();
    int lo = 0, hi = 255;  // last bucket whose first block is <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_bfirst[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const int64_t start = (int64_t)plan[lo] + (int64_t)(b - s_bfirst[lo]) * kSortChunk;
    const int64_t end = plan[lo + 1];
    pb.l = lo;
    pb.base = start;
    pb.cnt = (int)(end - start < kSortChunk ? end - start : kSortChunk);
    pb.nb2 = nb2;
    return true;
}

// Pass-2 histogram of the high byte, digit-major [256][nb2].
__global__ __launch_bounds__(kSortThreads) void k_bin_hist2(const uint32_t *packed, const uint32_t *plan,
                                                            const int64_t *nb2_p, uint32_t *hist) {
    __shared__ uint32_t h[kSortThreads / kWave][256];
    __shared__ uint32_t s_bfirst[257];
    Pass2Block pb;
    if (!pass2_block(plan, nb2_p, s_bfirst, pb)) return;
    for (int i = threadIdx.x; i < (kSortThreads / kWave) * 256; i += kSortThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int wid = threadIdx.x / kWave;
    uint32_t w[kSortItems];  // all loads in flight before the first count
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int k = threadIdx.x + i * kSortThreads;
        // (an index past the block's items reads the block's first item: pb.cnt >= 1)
        w[i] = load_or_zero(packed + pb.base, (int64_t)k, (int64_t)pb.cnt);
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i)
        if (threadIdx.x + i * kSortThreads < pb.cnt) atomicAdd(&h[wid][w[i] >> kRankBits], 1u);
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) tot += h[w][d];
    hist[(int64_t)d * pb.nb2 + blockIdx.x] = tot;
}

// Pass 2: rank the packed words by their high byte and write the Gaussian id
// of each word's depth rank (and optionally the tile id, high byte << 8 | the
// block's bucket).
template <bool TILES>
__global__ __launch_bounds__(kSortThreads) void k_bin_scatter2(const uint32_t *packed, const uint32_t *plan,
                                                               const int64_t *nb2_p, const uint32_t *offs,
                                                               const uint32_t *sorted_ids,
                                                               uint32_t *sorted_gids,
                                                               uint32_t *sorted_tiles) {
    __shared__ RankSmem sm;
    __shared__ uint32_t skey[kSortChunk];
    __shared__ uint32_t s_bfirst[257];
    Pass2Block pb;
    if (!pass2_block(plan, nb2_p, s_bfirst, pb)) return;
    rank_init(sm);
    sm.gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * pb.nb2 + blockIdx.x];
    __syncthreads();
    uint32_t key[kSortItems], val[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int p = rank_pos(i);
        key[i] = p < pb.cnt ? packed[pb.base + p] : 0u;
        val[i] = 0u;
    }
    const uint32_t l = (uint32_t)pb.l;
    rank_stage_write(
        key, val, pb.cnt, kRankBits, sm, skey, nullptr,
        [&](uint32_t word, uint32_t) { return sorted_ids[word & kRankMask]; },
        [&](int64_t dst, uint32_t word, uint32_t gid) {
            sorted_gids[dst] = gid;
            if (TILES) sorted_tiles[dst] = ((word >> kRankBits) << 8) | l;
        });
}

// ranges[t] for t = (h, l): [offs(h, bfirst[l]), offs(h, bfirst[l + 1])), the
// flat digit-major index h * nb2 + bfirst[256] being the next digit's start
// (or P past the last).  (0, 0) for an empty tile, and for every tile when the
// pairs overflowed.
__global__ __launch_bounds__(256) void k_bin_ranges2(const uint32_t *offs, const uint32_t *plan,
                                                     const int64_t *nb2_p, const int64_t *num_pairs,
                                                     int64_t cap, int64_t ntiles, uint32_t *ranges) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= ntiles) return;
    const int64_t P = live_count(num_pairs, cap, 1);
    const int64_t nb2 = *nb2_p;
    uint32_t s = 0, e = 0;
    if (P > 0 && nb2 > 0) {
        const int64_t h = t >> 8, l = t & 255;
        const uint32_t *bfirst = plan + 257;
        if (bfirst[l] < bfirst[l + 1]) {
            const int64_t i0 = h * nb2 + bfirst[l], i1 = h * nb2 + bfirst[l + 1];
            s = offs[i0];
            e = i1 < 256 * nb2 ? offs[i1] : (uint32_t)P;
        }
        if (s == e) s = e = 0;
    }
    reinterpret_cast<uint2 *>(ranges)[t] = make_uint2(s, e);
}

// One-pass route (at most 256 tiles): tile t is bucket t, [B[t], B[t + 1]).
__global__ __launch_bounds__(256) void k_bin_ranges1(const uint32_t *plan, int64_t ntiles,
                                                     uint32_t *ranges) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= ntiles) return;
    uint32_t s = plan[t], e = plan[t + 1];
    if (s == e) s = e = 0;
    reinterpret_cast<uint2 *>(ranges)[t] = make_uint2(s, e);
}

__global__ __launch_bounds__(256) void k_zero_ranges(uint32_t *ranges, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) ranges[i] = 0u;
}

hipError_t launch_bin(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                      int n, int tiles_x, int tiles_y, int extent_rule, uint32_t *sorted_gids,
                      uint32_t *sorted_tiles, uint32_t *ranges, int64_t cap, int64_t *num_pairs,
                      const Workspace &ws, hipStream_t s) {
    const int64_t ntiles = (int64_t)tiles_x * tiles_y;
    const bool packed = bin_packed(n, tiles_x, tiles_y);
    const bool generic = !packed || extent_rule != 0;
    // the generic route's tile-sort group sums and ranges are cleared by the
    // emission preparation's first kernel (no fill launches)
    hipError_t e = launch_emit_prepare(splats, rects, tiles_touched, n, extent_rule, cap, num_pairs,
                                       ws, s, generic ? ws.psum : nullptr, 256 * lsd_pass_groups(cap),
                                       generic ? ranges : nullptr, 2 * ntiles);
    if (e != hipSuccess) return e;
    if (n == 0 || cap == 0) {  // no pairs can be binned: every range empty
        k_zero_ranges<<<(unsigned)((2 * ntiles + 255) / 256), 256, 0, s>>>(ranges, 2 * ntiles);
        return hipGetLastError();
    }
    const int64_t nb = ws.nb_psort;  // slices = sort blocks = ceil(cap / 4096)
    if (generic) {
        // generic route (and the ellipse and oriented-box rules, whose pairs are
        // not a rectangle enumeration): emit the pairs, sort them by tile
        // (nothing if over), ranges
        uint32_t *kout = sorted_tiles ? sorted_tiles : ws.bpacked;
        int bits = 0;
        while (bits < 63 && ((int64_t)1 << bits) < ntiles) ++bits;
        const int passes = bits <= 0 ? 1 : (bits + 7) / 8;
        // Emit into the buffers the sort's first pass reads.  Beyond the packed
        // limits the workspace has its own pair arrays; within them (at most
        // two passes) an odd count reads the sort scratch, and an even count the
        // outputs, which the first pass leaves for the scratch before the
        // second pass writes them.
        uint32_t *ek = ws.bkey, *ev = ws.bval;
        if (packed) {
            ek = passes % 2 ? ws.ptile_tmp : kout;
            ev = passes % 2 ? ws.pgid_tmp : sorted_gids;
        }
        e = launch_emit_pairs(splats, rects, tiles_x, extent_rule, ek, ev, cap, num_pairs, ws, s);
        if (e != hipSuccess) return e;
        e = radix_sort_u32(ek, ev, kout, sorted_gids, ws.ptile_tmp, ws.pgid_tmp, num_pairs, cap,
                           bits, ws.phist, ws.psum, s, 0, 1, true);
        if (e != hipSuccess) return e;
        return launch_tile_ranges(kout, num_pairs, cap, ranges, (int)ntiles, s, 1, true);
    }
    SliceArgs a;
    a.sorted_ids = ws.dval[1];
    a.num_vis = ws.counters;
    a.rects = rects;
    a.pair_off = ws.pair_off;
    a.slice_start = ws.slice_start;
    a.num_pairs = num_pairs;
    a.cap = cap;
    a.tiles_x = tiles_x;
    k_bin_hist<<<(unsigned)nb, kSortThreads, 0, s>>>(a, ws.bhist);
    e = scan_exclusive_u32(ws.bhist, ws.bhist, 256 * nb, ws.scan_part, nullptr, s,
                           DevExtent{num_pairs, cap, kSortChunk, 256, true});
    if (e != hipSuccess) return e;
    int64_t *nb2 = ws.counters + 2;
    k_bin_plan2<<<1, 256, 0, s>>>(ws.bhist, num_pairs, cap, ws.bplan, nb2);
    const unsigned ranges_grid = (unsigned)((ntiles + 255) / 256);
    if (ntiles <= 256) {
        k_bin_scatter1<true><<<(unsigned)nb, kSortThreads, 0, s>>>(a, ws.bhist, nullptr, sorted_gids,
                                                                  sorted_tiles);
        k_bin_ranges1<<<ranges_grid, 256, 0, s>>>(ws.bplan, ntiles, ranges);
        return hipGetLastError();
    }
    k_bin_scatter1<false><<<(unsigned)nb, kSortThreads, 0, s>>>(a, ws.bhist, ws.bpacked, nullptr,
                                                               nullptr);
    const int64_t nb2max = nb + 256;  // bucket alignment adds at most one partial block per bucket
    k_bin_hist2<<<(unsigned)nb2max, kSortThreads, 0, s>>>(ws.bpacked, ws.bplan, nb2, ws.bhist2);
    e = scan_exclusive_u32(ws.bhist2, ws.bhist2, 256 * nb2max, ws.scan_part, nullptr, s,
                           DevExtent{nb2, nb2max, 1, 256});
    if (e != hipSuccess) return e;
    if (sorted_tiles)
        k_bin_scatter2<true><<<(unsigned)nb2max, kSortThreads, 0, s>>>(
            ws.bpacked, ws.bplan, nb2, ws.bhist2, ws.dval[1], sorted_gids, sorted_tiles);
    else
        k_bin_scatter2<false><<<(unsigned)nb2max, kSortThreads, 0, s>>>(
            ws.bpacked, ws.bplan, nb2, ws.bhist2, ws.dval[1], sorted_gids, nullptr);
    k_bin_ranges2<<<ranges_grid, 256, 0, s>>>(ws.bhist2, ws.bplan, nb2, num_pairs, cap, ntiles, ranges);
    return hipGetLastError();
}

}  // namespace gsr
