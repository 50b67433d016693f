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
//   radix_hist       high-byte histogram of the packed words, scan
//   k_bin_scatter2   rank by the high byte, write sorted_gids = id of rank j
//                    (and, optionally, the tile id: high byte from the word, low
//                    byte from the pass-1 bucket that held it)
//
// The ranges come from per-tile counts: each rectangle adds its four corners
// to a (tiles_y+1) x (tiles_x+1) difference array, whose 2D prefix sum is the
// list length of every tile; the exclusive scan of those is the list starts.
// With at most 256 tiles, pass 1 writes the final lists directly.  Beyond the
// packed limits the path falls back to emitting the pairs and sorting them.
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
    // m / w by a float reciprocal, corrected by one step (m < 2^22 here)
    int q = (int)((float)m * (1.0f / (float)w));
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
        rank_stage_write(rkey, val, cnt, 0, sm, u.stage[0], u.stage[1],
                         [&](int64_t dst, uint32_t tile, uint32_t j) {
                             sorted_gids[dst] = a.sorted_ids[j];
                             if (sorted_tiles) sorted_tiles[dst] = tile;
                         });
    } else {
        rank_stage_write(rkey, key, cnt, 0, sm, u.stage[0], u.stage[1],
                         [&](int64_t dst, uint32_t, uint32_t word) { packed[dst] = word; });
    }
}

// Pass 2: rank the packed words by their high byte (the tile's high byte),
// write the Gaussian id of the word's depth rank, and optionally the tile id,
// whose low byte is the pass-1 bucket the word was read from (bucket starts:
// the pass-1 offsets of slice 0, lo_offs[d * nb1]).
template <bool TILES>
__global__ __launch_bounds__(kSortThreads) void k_bin_scatter2(
    const uint32_t *packed, const int64_t *num_pairs, int64_t cap, const uint32_t *offs,
    const uint32_t *sorted_ids, uint32_t *sorted_gids, uint32_t *sorted_tiles,
    const uint32_t *lo_offs) {
    __shared__ RankSmem sm;
    __shared__ uint32_t skey[kSortChunk];
    __shared__ uint32_t sval[kSortChunk];
    __shared__ uint32_t lo_start[256];
    rank_init(sm);
    const int64_t n = live_count(num_pairs, cap, 1);
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    if (base >= n) return;
    const int64_t nb_live = (n + kSortChunk - 1) / kSortChunk;
    sm.gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * nb_live + blockIdx.x];
    if (TILES) lo_start[threadIdx.x] = lo_offs[(int64_t)threadIdx.x * nb_live];
    __syncthreads();
    const int cnt = (int)(n - base < kSortChunk ? n - base : kSortChunk);
    uint32_t key[kSortItems], val[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int p = rank_pos(i);
        key[i] = p < cnt ? packed[base + p] : 0u;
        val[i] = (uint32_t)p;
    }
    rank_stage_write(key, val, cnt, kRankBits, sm, skey, sval,
                     [&](int64_t dst, uint32_t word, uint32_t p) {
                         sorted_gids[dst] = sorted_ids[word & kRankMask];
                         if (TILES) {
                             // last bucket whose start is <= the word's input position
                             const uint32_t pos = (uint32_t)(base + p);
                             int lo = 0, hi = 255;
                             while (lo < hi) {
                                 const int mid = (lo + hi + 1) >> 1;
                                 if (lo_start[mid] <= pos) lo = mid; else hi = mid - 1;
                             }
                             sorted_tiles[dst] = ((word >> kRankBits) << 8) | (uint32_t)lo;
                         }
                     });
}

// ---------------------------------------------------------------- tile counts
__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) p[i] = 0;
}

// Each visible rectangle [x0, x1) x [y0, y1) adds +1 at (y0, x0) and (y1, x1)
// and -1 at (y0, x1) and (y1, x0) of the difference array.
__global__ __launch_bounds__(256) void k_rect_corners(const uint32_t *sorted_ids, const int64_t *num_vis,
                                                      const uint64_t *rects, int tiles_x, int32_t *diff,
                                                      int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n || j >= *num_vis) return;
    const uint64_t r = rects[sorted_ids[j]];
    const uint32_t x0 = r & 0xffff, y0 = (r >> 16) & 0xffff, x1 = (r >> 32) & 0xffff, y1 = r >> 48;
    const int64_t W = tiles_x + 1;
    atomicAdd(&diff[y0 * W + x0], 1);
    atomicAdd(&diff[y0 * W + x1], -1);
    atomicAdd(&diff[y1 * W + x0], -1);
    atomicAdd(&diff[y1 * W + x1], 1);
}

// Inclusive prefix along x of rows 0 .. tiles_y - 1 (one block per row).
__global__ __launch_bounds__(256) void k_prefix_rows(int32_t *diff, int tiles_x) {
    __shared__ int32_t wt[256 / kWave];
    int32_t *row = diff + (int64_t)blockIdx.x * (tiles_x + 1);
    int32_t carry = 0;
    for (int c0 = 0; c0 < tiles_x; c0 += 256 * 8) {
        int32_t v[8], s = 0;
        const int c = c0 + threadIdx.x * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            v[i] = c + i < tiles_x ? row[c + i] : 0;
            s += v[i];
        }
        int32_t tot;
        int32_t run = carry + block_exclusive_scan<256, int32_t>(s, wt, &tot);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            run += v[i];
            if (c + i < tiles_x) row[c + i] = run;
        }
        carry += tot;
    }
}

// Inclusive prefix along y (one thread per column): the list length of every
// tile, written densely; zero for all tiles when the pairs overflowed.
__global__ __launch_bounds__(256) void k_prefix_cols(const int32_t *diff, int tiles_x, int tiles_y,
                                                     const int64_t *num_pairs, int64_t cap,
                                                     uint32_t *count) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= tiles_x) return;
    const bool over = *num_pairs > cap;
    int32_t acc = 0;
    for (int y = 0; y < tiles_y; ++y) {
        acc += diff[(int64_t)y * (tiles_x + 1) + x];
        count[(int64_t)y * tiles_x + x] = over ? 0u : (uint32_t)acc;
    }
}

__global__ __launch_bounds__(256) void k_ranges_from_counts(const uint32_t *count, const uint32_t *off,
                                                            int64_t ntiles, uint32_t *ranges) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= ntiles) return;
    const uint32_t c = count[t], s = c ? off[t] : 0u;  // an empty tile's range is (0, 0)
    reinterpret_cast<uint2 *>(ranges)[t] = make_uint2(s, s + c);
}

// Counts -> starts -> ranges.  Needs launch_emit_prepare's outputs.
static hipError_t bin_ranges(const uint64_t *rects, int n, int tiles_x, int tiles_y, int64_t cap,
                             const int64_t *num_pairs, uint32_t *ranges, const Workspace &ws,
                             hipStream_t s) {
    const int64_t ntiles = (int64_t)tiles_x * tiles_y;
    const int64_t md = (int64_t)(tiles_x + 1) * (tiles_y + 1);
    k_fill_i32<<<(unsigned)((md + 255) / 256), 256, 0, s>>>(ws.tdiff, md);
    if (n > 0)
        k_rect_corners<<<(unsigned)ws.nb_gauss, 256, 0, s>>>(ws.dval[1], ws.counters, rects, tiles_x,
                                                             ws.tdiff, n);
    k_prefix_rows<<<(unsigned)tiles_y, 256, 0, s>>>(ws.tdiff, tiles_x);
    k_prefix_cols<<<(unsigned)((tiles_x + 255) / 256), 256, 0, s>>>(ws.tdiff, tiles_x, tiles_y,
                                                                    num_pairs, cap, ws.tcount);
    hipError_t e = scan_exclusive_u32(ws.tcount, ws.toff, ntiles, ws.scan_part, nullptr, s);
    if (e != hipSuccess) return e;
    k_ranges_from_counts<<<(unsigned)((ntiles + 255) / 256), 256, 0, s>>>(ws.tcount, ws.toff, ntiles,
                                                                         ranges);
    return hipGetLastError();
}

hipError_t launch_bin(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                      int n, int tiles_x, int tiles_y, uint32_t *sorted_gids, uint32_t *sorted_tiles,
                      uint32_t *ranges, int64_t cap, int64_t *num_pairs, const Workspace &ws,
                      hipStream_t s) {
    hipError_t e = launch_emit_prepare(splats, rects, tiles_touched, n, cap, num_pairs, ws, s);
    if (e != hipSuccess) return e;
    e = bin_ranges(rects, n, tiles_x, tiles_y, cap, num_pairs, ranges, ws, s);
    if (e != hipSuccess || n == 0 || cap == 0) return e;
    const int64_t nb = ws.nb_psort;  // slices = sort blocks = ceil(cap / 4096)
    const int64_t ntiles = (int64_t)tiles_x * tiles_y;
    if (!bin_packed(n, tiles_x, tiles_y)) {
        // generic route: emit the pairs, then sort them by tile (empty if over)
        e = launch_emit_pairs(rects, tiles_x, ws.bkey, ws.bval, cap, num_pairs, ws, s);
        if (e != hipSuccess) return e;
        uint32_t *kout = sorted_tiles ? sorted_tiles : ws.bpacked;
        int bits = 0;
        while (bits < 63 && ((int64_t)1 << bits) < ntiles) ++bits;
        return radix_sort_u32(ws.bkey, ws.bval, kout, sorted_gids, ws.ptile_tmp, ws.pgid_tmp,
                              num_pairs, cap, bits, ws.phist, nb, ws.scan_part, s, 0, 1);
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
    if (ntiles <= 256) {
        k_bin_scatter1<true><<<(unsigned)nb, kSortThreads, 0, s>>>(a, ws.bhist, nullptr, sorted_gids,
                                                                  sorted_tiles);
        return hipGetLastError();
    }
    k_bin_scatter1<false><<<(unsigned)nb, kSortThreads, 0, s>>>(a, ws.bhist, ws.bpacked, nullptr,
                                                               nullptr);
    radix_hist(ws.bpacked, num_pairs, cap, kRankBits, ws.phist, nb, ws.scan_part, s, 1);
    if (sorted_tiles)
        k_bin_scatter2<true><<<(unsigned)nb, kSortThreads, 0, s>>>(
            ws.bpacked, num_pairs, cap, ws.phist, ws.dval[1], sorted_gids, sorted_tiles, ws.bhist);
    else
        k_bin_scatter2<false><<<(unsigned)nb, kSortThreads, 0, s>>>(
            ws.bpacked, num_pairs, cap, ws.phist, ws.dval[1], sorted_gids, nullptr, ws.bhist);
    return hipGetLastError();
}

}  // namespace gsr
