// Stage 2: Gaussian-tile pair generation (paper Sec. 2.1, Fig. 1).
//
// The paper's pipeline emits pairs Gaussian by Gaussian and then sorts
// (tile | depth) keys.  Here the Gaussians are first put in depth order (a
// radix sort of one 32-bit key per visible Gaussian, a few MB), and pairs are
// emitted in that order.  The per-tile depth order then only needs a stable
// sort by tile id (16 bits at 4608x3456) instead of a 48-bit (tile | depth)
// sort of every pair; the sorted result is the same sequence.
//
//   k_vis_count / k_vis_compact         visible Gaussians -> (depth bits, id)
//   depth_sort                          by depth bits (stable: ties keep id order)
//   k_pair_counts / k_pair_offsets      pairs per sorted Gaussian, their prefix,
//                                       the owner of each emission slice
//   k_emit                              each block writes its pairs contiguously,
//                                       one pair per thread per step, after an LDS
//                                       scan of its Gaussians' tile counts
//   k_emit_spans                        extent rules 1 and 2: per wave 32
//                                       Gaussians' row spans (tile_shapes.hpp),
//                                       64 (Gaussian, row) items per step,
//                                       written by the whole wave
#include <type_traits>

#include "tile_shapes.hpp"
#include "gsr_internal.hpp"

namespace gsr {

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

// Sum over the blocks before this one of a per-block total (a short array:
// the offset of this block's chunk).  Contains barriers.
template <typename T>
__device__ __forceinline__ T sum_before(const T *tot, int64_t b, T *wt) {
    T acc = 0;
    for (int64_t i0 = threadIdx.x; i0 < b; i0 += 4 * 256) {  // four loads in flight
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += i0 + 256 * k < b ? tot[i0 + 256 * k] : (T)0;
    }
    T all;
    block_exclusive_scan<256, T>(acc, wt, &all);
    return all;
}

// Visible Gaussians per chunk of 4096 ids; also clears the depth passes'
// group sums (accumulated by k_lsd_hist), the pair totals per chunk
// (accumulated by k_pair_counts) and up to two further word ranges.
__global__ __launch_bounds__(256) void k_vis_count(const uint32_t *tiles_touched, int n,
                                                   uint32_t *vis_count, uint32_t *clear,
                                                   int64_t nclear, uint64_t *clear64,
                                                   int64_t nclear64, uint32_t *xclear, int64_t nxclear,
                                                   uint32_t *xclear2, int64_t nxclear2) {
    __shared__ uint32_t wt[4];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nclear; i += (int64_t)gridDim.x * 256)
        clear[i] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nxclear; i += (int64_t)gridDim.x * 256)
        xclear[i] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nxclear2; i += (int64_t)gridDim.x * 256)
        xclear2[i] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nclear64; i += (int64_t)gridDim.x * 256)
        clear64[i] = 0ull;
    const int64_t base = (int64_t)blockIdx.x * kSortChunk + threadIdx.x;
    uint32_t t[kSortItems], c = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) t[i] = load_or_zero(tiles_touched, base + (int64_t)i * 256, n);
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) c += t[i] > 0u ? 1u : 0u;
    uint32_t tot;
    block_exclusive_scan<256, uint32_t>(c, wt, &tot);
    if (threadIdx.x == 0) vis_count[blockIdx.x] = tot;
}

// Visible Gaussians in id order as (depth bits, id).  Block b owns ids
// [4096 b, 4096 b + 4096): wave w the 1024 from 4096 b + 1024 w, lane l item
// i at ... + 64 i + l, so ballots order each wave's items; the block's output
// offset is the sum of the earlier blocks' counts.  The last block stores the
// visible count.
__global__ __launch_bounds__(256) void k_vis_compact(const uint32_t *tiles_touched, const float *splats,
                                                     int n, const uint32_t *vis_count, uint32_t *dkey,
                                                     uint32_t *dval, int64_t *num_vis) {
    __shared__ uint32_t wt[4], s_wcnt[4];
    const int64_t b = blockIdx.x;
    const uint32_t before = sum_before<uint32_t>(vis_count, b, wt);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int64_t wbase = b * kSortChunk + (int64_t)wid * (kSortItems * kWave) + lane;
    const uint64_t lt = lanemask_lt();
    uint64_t m[kSortItems];
    uint32_t t[kSortItems], pos[kSortItems], wc = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) t[i] = load_or_zero(tiles_touched, wbase + 64 * i, n);
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        m[i] = __ballot(t[i] > 0u);
        pos[i] = wc + (uint32_t)__popcll(m[i] & lt);
        wc += (uint32_t)__popcll(m[i]);
    }
    if (lane == 0) s_wcnt[wid] = wc;
    __syncthreads();
    uint32_t woff = before, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        woff += w < wid ? s_wcnt[w] : 0u;
        tot += s_wcnt[w];
    }
    // every depth requested before the first store (lanes without a visible
    // Gaussian read Gaussian 0's: one line, shared)
    uint32_t dk[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t g = ((m[i] >> lane) & 1ull) ? wbase + 64 * i : 0;
        dk[i] = __float_as_uint(splats[(size_t)g * 12 + 6]);  // depth > 0.2: bits order = value order
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if ((m[i] >> lane) & 1ull) {
            dkey[woff + pos[i]] = dk[i];
            dval[woff + pos[i]] = (uint32_t)(wbase + 64 * i);
        }
    }
    if (threadIdx.x == 0 && b == (int64_t)gridDim.x - 1) *num_vis = (int64_t)(before + tot);
}

// Inclusive prefix sum over the wave in DPP lane moves, no LDS round trip:
// shifts by 1, 2, 4 and 8 lanes inside each row of 16 lanes (lanes shifted in
// from outside the row read 0), then lane 15's sum added to row 1 and lane
// 47's to row 3 (row_bcast:15 on rows 1 and 3), then lane 31's to rows 2 and
// 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Inclusive running maximum over the wave, the same DPP lane moves.
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
    return x;
}

// Exclusive prefix over the wave of one value per lane, and the wave's total.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t v, uint32_t &total) {
    const uint32_t x = wave_inclusive_sum(v);
    total = lane_u32(x, kWave - 1);
    return x - v;
}

// One wave's Gaussians for the flattened row walk of the span kernels.  The
// rows of the wave's 64 Gaussians (lane-major: lane 0's band, then lane 1's,
// ...) are numbered 0 .. total-1 and taken 64 per step, one per lane, so every
// lane computes a span whatever the lengths of the bands.  Item q belongs to
// the last lane whose band prefix p is <= q and is row ra + q - p of its band:
// per step each Gaussian whose band starts in the step marks that item's slot
// (tagged with the step), and a running maximum over the lanes hands every
// item the last mark at or before it; items before the step's first mark
// continue the previous step's last Gaussian.
template <class Shape>
struct RowTable {
    Shape sh[kWave];
    int x0[kWave], x1[kWave], ra[kWave], rb[kWave];
    uint32_t p[kWave];     // exclusive prefix of the band lengths
    uint32_t acc[kWave];   // the count's pair totals
    uint32_t mark[kWave];  // step << 8 | (lane + 1) of the Gaussian whose band starts here
    uint64_t k[kWave];     // output index of the Gaussian's first pair
    uint32_t g[kWave];
};

// Loads this lane's Gaussian into the wave's table: shape, columns [x0, x1),
// row band [ra, rb) (empty when the shape has no tiles).  Returns the number
// of items (rows) of the whole wave; p = this lane's band prefix.  Contains
// wave barriers.
template <class Shape>
__device__ __forceinline__ uint32_t row_table_fill(RowTable<Shape> &tb, const Shape &e, int x0, int x1,
                                                   int ra, int rb, uint64_t k, uint32_t g, uint32_t &p) {
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t total;
    p = wave_exclusive_scan((uint32_t)(rb - ra), total);
    tb.sh[lane] = e;
    tb.x0[lane] = x0;
    tb.x1[lane] = x1;
    tb.ra[lane] = ra;
    tb.rb[lane] = rb;
    tb.p[lane] = p;
    tb.acc[lane] = 0u;
    tb.mark[lane] = 0xffffffffu;  // a step tag no step has
    tb.k[lane] = k;
    tb.g[lane] = g;
    wave_sync_lds();
    return total;
}

// Owner (lane) of item q0 + lane of the step starting at item q0; `carry` is
// the owner of the previous step's last item and is advanced to this step's;
// `first` tells whether the item is its Gaussian's first row.  This lane's
// Gaussian has band prefix p and nb rows.  Called by the whole wave; contains
// wave barriers.
template <class Shape>
__device__ __forceinline__ int step_owner(RowTable<Shape> &tb, uint32_t q0, uint32_t p, uint32_t nb,
                                          int &carry, bool &first) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t tag = q0 / kWave;
    if (nb > 0u && p >= q0 && p - q0 < (uint32_t)kWave) tb.mark[p - q0] = (tag << 8) | (uint32_t)(lane + 1);
    wave_sync_lds();
    const uint32_t m = tb.mark[lane];
    first = (m >> 8) == tag;
    const uint32_t last = wave_inclusive_max(first ? (m & 0xffu) : 0u);
    const int o = last ? (int)last - 1 : carry;
    carry = lane_i32(o, kWave - 1);
    return o;
}

// Span of item q of Gaussian (lane) o: the tile row and its inclusive column
// span [a, b]; false when the row misses the shape or q is not in o's band.
template <class Shape>
__device__ __forceinline__ bool row_item_span(const RowTable<Shape> &tb, uint32_t q, int o, int &ty,
                                              int &a, int &b) {
    const uint32_t r = q - tb.p[o];
    if (r >= (uint32_t)(tb.rb[o] - tb.ra[o])) return false;
    ty = tb.ra[o] + (int)r;
    return tb.sh[o].row_span(ty, tb.x0[o], tb.x1[o] - 1, a, b);
}

// Pair count of one visible Gaussian under a shape rule: its tiles meeting the
// shape, the spans of the wave's rows summed per Gaussian in LDS.
template <class Shape>
__device__ __forceinline__ uint64_t shape_pair_count(const float *splats, const uint64_t *rects,
                                                     uint32_t g, bool valid, RowTable<Shape> &tb) {
    const int lane = threadIdx.x & (kWave - 1);
    Shape e{};
    int x0 = 0, x1 = 0, ra = 0, rb = 0;
    if (valid) {
        const uint64_t r = rects[g];
        SplatRec rec = SplatRec::load(splats + (size_t)g * 12, Shape::kThird);
        rec.pin(Shape::kThird);
        if (e.setup(rec)) {
            x0 = (int)(r & 0xffff);
            x1 = (int)((r >> 32) & 0xffff);
            e.row_band((int)((r >> 16) & 0xffff), (int)(r >> 48), ra, rb);
        }
    }
    uint32_t p;
    const uint32_t total = row_table_fill(tb, e, x0, x1, ra, rb, 0ull, g, p);
    int carry = 0;
    for (uint32_t q0 = 0; q0 < total; q0 += kWave) {  // wave-uniform
        const uint32_t q = q0 + (uint32_t)lane;
        bool first;
        const int o = step_owner(tb, q0, p, (uint32_t)(rb - ra), carry, first);
        int ty, a, b;
        if (q < total && row_item_span(tb, q, o, ty, a, b)) atomicAdd(&tb.acc[o], (uint32_t)(b - a + 1));
    }
    wave_sync_lds();
    return tb.acc[lane];
}

// Pairs of each depth-sorted visible Gaussian (one per thread), added to the
// total of its chunk of 4096 (cleared by k_vis_count): the rectangle's area
// (tiles_touched) under extent rule 0, the count of its tiles that meet the
// ellipse (rule 1) or the oriented box (rule 2).  The visible Gaussians are
// dense here, and the flattened row walk keeps every lane on a span.
// Gaussians per wave in the span emitter: the flattened walk takes 64 items
// per step whatever the count, so fewer Gaussians per wave mean more, shorter
// waves over the visible Gaussians (their steps are latency-bound FP64 chains,
// and a few hundred thousand Gaussians at 64 per wave leave about four waves
// per SIMD).  Measured on a 6M city frame (259K visible Gaussians): emission
// 55 us at 64, 50 at 32, 56 at 16; the pair count is fastest at 64 (its
// steps are shorter), so it keeps one Gaussian per lane.
#ifndef GSR_SPAN_LANES
#define GSR_SPAN_LANES 32
#endif
constexpr int kSpanLanes = GSR_SPAN_LANES;
static_assert(kSpanLanes >= 1 && kSpanLanes <= kWave && kSortChunk % (4 * kSpanLanes) == 0,
              "a block's Gaussians lie in one 4096-chunk");

template <int RULE>
__global__ __launch_bounds__(256) void k_pair_counts(const uint32_t *sorted_ids, const int64_t *num_vis,
                                                     const uint32_t *tiles_touched, const float *splats,
                                                     const uint64_t *rects, uint64_t *cnt,
                                                     uint64_t *chunk_tot) {
    __shared__ uint64_t wt[4];
    using Shape = typename std::conditional<RULE == 2, OrientedBox, Ellipse>::type;
    __shared__ RowTable<Shape> s_rows[RULE == 0 ? 1 : 4];
    const int64_t V = *num_vis;
    const int wid = threadIdx.x / kWave;
    const int64_t j0 = (int64_t)blockIdx.x * 256;
    if (j0 >= V) return;  // uniform
    const int64_t j = j0 + threadIdx.x;
    const bool mine = j < V;
    uint64_t c = 0;
    const uint32_t g = mine ? sorted_ids[j] : 0u;
    if constexpr (RULE == 0) {
        if (mine) c = tiles_touched[g];
    } else {
        c = shape_pair_count<Shape>(splats, rects, g, mine, s_rows[wid]);
    }
    if (mine) cnt[j] = c;
    uint64_t tot;
    block_exclusive_scan<256, uint64_t>(c, wt, &tot);
    if (threadIdx.x == 0 && tot)
        atomicAdd((unsigned long long *)&chunk_tot[j0 / kSortChunk], (unsigned long long)tot);
}

// Exclusive prefix of the pair counts (the chunk's offset is the sum of the
// earlier chunks' totals), the first Gaussian of each emission slice that
// starts below the capacity, and the total (stored by the last live chunk).
__global__ __launch_bounds__(256) void k_pair_offsets(const uint64_t *cnt, const uint64_t *chunk_tot,
                                                      const int64_t *num_vis, uint64_t *off,
                                                      uint32_t *bstart, int64_t *num_pairs, int64_t cap) {
    __shared__ uint64_t wt[4];
    const int64_t V = *num_vis;
    const int64_t b = blockIdx.x;
    if (V == 0) {
        if (b == 0 && threadIdx.x == 0) *num_pairs = 0;
        return;
    }
    if (b * kSortChunk >= V) return;  // uniform
    const uint64_t before = sum_before<uint64_t>(chunk_tot, b, wt);
    const int64_t j0 = b * kSortChunk + (int64_t)threadIdx.x * kSortItems;  // 16 consecutive
    uint64_t c[kSortItems], acc = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        c[i] = j0 + i < V ? cnt[j0 + i] : 0ull;
        acc += c[i];
    }
    uint64_t tot;
    uint64_t run = before + block_exclusive_scan<256, uint64_t>(acc, wt, &tot);
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (j0 + i < V) {
            off[j0 + i] = run;
            const uint64_t p1 = run + c[i];
            for (uint64_t s = (run + kEmitChunk - 1) / kEmitChunk;
                 s * kEmitChunk < p1 && (int64_t)(s * kEmitChunk) < cap; ++s)
                bstart[s] = (uint32_t)(j0 + i);
        }
        run += c[i];
    }
    if (threadIdx.x == 0 && (b + 1) * kSortChunk >= V) *num_pairs = (int64_t)(before + tot);
}

// Emission is split into fixed slices of kEmitChunk pairs, one per workgroup,
// so a few huge Gaussians cannot serialise one block.  bstart[b] = the sorted
// Gaussian that owns pair b * kEmitChunk (k_pair_offsets marks the slices
// that begin inside each Gaussian's pair range).

__global__ __launch_bounds__(256) void k_emit(const uint32_t *sorted_ids, const int64_t *num_vis,
                                              const uint64_t *rects, const uint64_t *off,
                                              const uint32_t *bstart, const int64_t *num_pairs,
                                              int tiles_x, uint32_t *pair_tiles, uint32_t *pair_gids,
                                              int64_t cap) {
    __shared__ uint64_t s_off[257];
    __shared__ uint32_t gid_s[256], x0_s[256], y0_s[256], w_s[256];
    __shared__ float rw_s[256];
    const int64_t P = *num_pairs < cap ? *num_pairs : cap;
    const int64_t p0 = (int64_t)blockIdx.x * kEmitChunk;
    if (p0 >= P) return;
    const int64_t p1 = p0 + kEmitChunk < P ? p0 + kEmitChunk : P;
    const int64_t V = *num_vis;
    int64_t j0 = bstart[blockIdx.x];
    for (;;) {  // Gaussians j0 .. j0+255 in LDS; their pairs intersected with [p0, p1)
        const int64_t j = j0 + threadIdx.x;
        if (j < V) {
            const uint32_t g = sorted_ids[j];
            const uint64_t r = rects[g];
            const uint32_t x0 = r & 0xffff, y0 = (r >> 16) & 0xffff, x1 = (r >> 32) & 0xffff;
            s_off[threadIdx.x] = off[j];
            gid_s[threadIdx.x] = g;
            x0_s[threadIdx.x] = x0;
            y0_s[threadIdx.x] = y0;
            w_s[threadIdx.x] = x1 - x0;
            rw_s[threadIdx.x] = 1.0f / (float)(x1 - x0);
        } else {
            s_off[threadIdx.x] = ~0ull;  // past the last Gaussian
        }
        if (threadIdx.x == 0) s_off[256] = j0 + 256 < V ? off[j0 + 256] : ~0ull;
        __syncthreads();
        const uint64_t lo = s_off[0] > (uint64_t)p0 ? s_off[0] : (uint64_t)p0;
        const uint64_t hi = s_off[256] < (uint64_t)p1 ? s_off[256] : (uint64_t)p1;
        for (uint64_t k = lo + threadIdx.x; k < hi; k += 256) {
            // owner: the last Gaussian of the batch whose first pair is <= k
            int a = 0, b = 255;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (s_off[mid] <= k) a = mid; else b = mid - 1;
            }
            const uint32_t m = (uint32_t)(k - s_off[a]);
            const uint32_t w = w_s[a];
            int q = (int)((float)m * rw_s[a]);  // m / w, corrected below
            int rr = (int)m - q * (int)w;
            if (rr < 0) { --q; rr += (int)w; } else if (rr >= (int)w) { ++q; rr -= (int)w; }
            pair_tiles[k] = (y0_s[a] + (uint32_t)q) * (uint32_t)tiles_x + x0_s[a] + (uint32_t)rr;
            pair_gids[k] = gid_s[a];
        }
        const bool more = s_off[256] < (uint64_t)p1;
        __syncthreads();
        if (!more) break;
        j0 += 256;
    }
}

hipError_t launch_emit_prepare(const float *splats, const uint64_t *rects,
                               const uint32_t *tiles_touched, int n, int extent_rule, int64_t cap,
                               int64_t *num_pairs, const Workspace &ws, hipStream_t s,
                               uint32_t *xclear, int64_t nxclear, uint32_t *xclear2, int64_t nxclear2) {
    int64_t *num_vis = ws.counters;
    if (n == 0) {
        k_set_i64<<<1, 1, 0, s>>>(num_pairs, 0);
        k_set_i64<<<1, 1, 0, s>>>(num_vis, 0);
        return hipGetLastError();
    }
    const unsigned nb = (unsigned)ws.nb_dsort;  // chunks of 4096 (ids, then visible Gaussians)
    // also clears the depth passes' digit group sums
    k_vis_count<<<nb, 256, 0, s>>>(tiles_touched, n, ws.vis_count, ws.dgsum,
                                   256 * ws.nb_dgroups, ws.pair_tot, ws.nb_dsort,
                                   xclear, xclear ? nxclear : 0, xclear2, xclear2 ? nxclear2 : 0);
    k_vis_compact<<<nb, 256, 0, s>>>(tiles_touched, splats, n, ws.vis_count, ws.dkey[0], ws.dval[0],
                                     num_vis);
    hipError_t e = depth_sort(ws, num_vis, s);  // dkey/dval[0] -> [1]
    if (e != hipSuccess) return e;
    const unsigned span_blocks = (unsigned)ws.nb_gauss;
    if (extent_rule == 1)
        k_pair_counts<1><<<span_blocks, 256, 0, s>>>(ws.dval[1], num_vis, tiles_touched,
                                                              splats, rects, ws.pair_cnt, ws.pair_tot);
    else if (extent_rule == 2)
        k_pair_counts<2><<<span_blocks, 256, 0, s>>>(ws.dval[1], num_vis, tiles_touched,
                                                              splats, rects, ws.pair_cnt, ws.pair_tot);
    else
        k_pair_counts<0><<<(unsigned)ws.nb_gauss, 256, 0, s>>>(ws.dval[1], num_vis, tiles_touched,
                                                              splats, rects, ws.pair_cnt, ws.pair_tot);
    k_pair_offsets<<<nb, 256, 0, s>>>(ws.pair_cnt, ws.pair_tot, num_vis, ws.pair_off, ws.slice_start,
                                      num_pairs, cap);
    return hipGetLastError();
}

// Extent rules 1 and 2: each wave takes kSpanLanes consecutive depth-sorted
// visible Gaussians, one per lane (the other lanes hold none), and walks their
// rows flattened, 64 (Gaussian, row) items per step (RowTable): every lane
// recomputes the span of its item exactly as k_pair_counts counted it, the
// item's first pair follows the Gaussian's earlier rows (a wave prefix sum
// carried over the steps, less its value at the Gaussian's first row), and the
// whole wave writes the step's spans.
// Pairs at or beyond the capacity are not written.

// spans of up to this many pairs are written by their own lanes
#ifndef GSR_SHORT_SPAN
#define GSR_SHORT_SPAN 16
#endif

// Writes one step's spans (lane l's span: len pairs from output index k, tiles
// t0, t0 + 1, ..., Gaussian gid).  Short spans by their own lanes, pair i of
// every short span in iteration i (the step's spans lie end to end, so each
// store covers a short stretch of the output); longer ones one after another
// by the whole wave, consecutive lanes on consecutive pairs.
__device__ __forceinline__ void wave_write_spans(uint32_t len, uint64_t k, uint32_t t0, uint32_t gid,
                                                 uint32_t *pair_tiles, uint32_t *pair_gids, int64_t cap) {
    const int lane = threadIdx.x & (kWave - 1);
    const bool short_span = len <= (uint32_t)GSR_SHORT_SPAN;
    // the span's pairs below the capacity
    const uint64_t room = k < (uint64_t)cap ? (uint64_t)cap - k : 0ull;
    const uint32_t n = room < (uint64_t)len ? (uint32_t)room : len;
    const uint32_t ns = short_span ? n : 0u;
    uint32_t *pt = pair_tiles + (ns ? k : 0ull), *pg = pair_gids + (ns ? k : 0ull);
    for (uint32_t i = 0; __ballot(i < ns); ++i) {  // wave-uniform
        if (i < ns) {
            pt[i] = t0 + i;
            pg[i] = gid;
        }
    }
    for (uint64_t m = __ballot(!short_span && n > 0u); m; m &= m - 1) {  // wave-uniform
        const int src = __ffsll((long long)m) - 1;
        const uint32_t nn = lane_u32(n, src), tb = lane_u32(t0, src), gb = lane_u32(gid, src);
        const uint64_t kb = lane_u64(k, src);
        uint32_t *ptb = pair_tiles + kb, *pgb = pair_gids + kb;
        for (uint32_t i = (uint32_t)lane; i < nn; i += kWave) {
            ptb[i] = tb + i;
            pgb[i] = gb;
        }
    }
}

template <class Shape>
__global__ __launch_bounds__(256) void k_emit_spans(const uint32_t *sorted_ids, const int64_t *num_vis,
                                                    const float *splats, const uint64_t *rects,
                                                    const uint64_t *off, int tiles_x,
                                                    uint32_t *pair_tiles, uint32_t *pair_gids,
                                                    int64_t cap) {
    __shared__ RowTable<Shape> s_rows[4];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int64_t V = *num_vis;
    const int64_t jw = ((int64_t)blockIdx.x * 4 + wid) * kSpanLanes;  // this wave's first Gaussian
    if (jw >= V) return;  // wave-uniform
    const int64_t j = jw + lane;
    RowTable<Shape> &tb = s_rows[wid];
    uint64_t k = 0;
    uint32_t g = 0;
    int ra = 0, rb = 0, x0 = 0, x1 = 0;
    Shape e{};
    if (lane < kSpanLanes && j < V) {
        k = off[j];
        g = sorted_ids[j];
        const uint64_t r = rects[g];
        SplatRec rec = SplatRec::load(splats + (size_t)g * 12, Shape::kThird);
        rec.pin(Shape::kThird);
        x0 = (int)(r & 0xffff);
        x1 = (int)((r >> 32) & 0xffff);
        if (k < (uint64_t)cap && e.setup(rec))
            e.row_band((int)((r >> 16) & 0xffff), (int)(r >> 48), ra, rb);
    }
    uint32_t p;
    const uint32_t total = row_table_fill(tb, e, x0, x1, ra, rb, k, g, p);
    uint32_t carry = 0;  // pairs of the earlier steps
    int carry_owner = 0;
    uint32_t carry_g0 = 0;  // prefix at the first row of the previous step's last Gaussian
    for (uint32_t q0 = 0; q0 < total; q0 += kWave) {  // wave-uniform
        const uint32_t q = q0 + (uint32_t)lane;
        const bool item = q < total;
        bool first;
        const int o = step_owner(tb, q0, p, (uint32_t)(rb - ra), carry_owner, first);
        uint32_t len = 0, t0 = 0;
        int ty, a, b;
        if (item && row_item_span(tb, q, o, ty, a, b)) {
            len = (uint32_t)(b - a + 1);
            t0 = (uint32_t)ty * (uint32_t)tiles_x + (uint32_t)a;
        }
        uint32_t step;
        const uint32_t G = carry + wave_exclusive_scan(len, step);
        // the prefix at the Gaussian's first row: the prefix never decreases
        // along the items, so it is the running maximum over the first rows
        const uint32_t f = wave_inclusive_max(first ? G + 1u : 0u);
        const uint32_t G0 = f ? f - 1u : carry_g0;
        carry_g0 = lane_u32(G0, kWave - 1);
        uint64_t kk = 0;
        uint32_t gid = 0;
        if (item) {
            kk = tb.k[o] + (uint64_t)(G - G0);
            gid = tb.g[o];
        }
        wave_write_spans(len, kk, t0, gid, pair_tiles, pair_gids, cap);
        wave_sync_lds();  // the table's reads before the next step's writes
        carry += step;
    }
}

hipError_t launch_emit_pairs(const float *splats, const uint64_t *rects, int tiles_x,
                             int extent_rule, uint32_t *pair_tiles, uint32_t *pair_gids,
                             int64_t cap, const int64_t *num_pairs, const Workspace &ws,
                             hipStream_t s) {
    if (cap <= 0) return hipGetLastError();
    const unsigned span_blocks =
        (unsigned)(((int64_t)ws.nb_gauss * 256 + 4 * kSpanLanes - 1) / (4 * kSpanLanes));
    if (extent_rule == 1)
        k_emit_spans<Ellipse><<<span_blocks, 256, 0, s>>>(
            ws.dval[1], ws.counters, splats, rects, ws.pair_off, tiles_x, pair_tiles, pair_gids, cap);
    else if (extent_rule == 2)
        k_emit_spans<OrientedBox><<<span_blocks, 256, 0, s>>>(
            ws.dval[1], ws.counters, splats, rects, ws.pair_off, tiles_x, pair_tiles, pair_gids, cap);
    else
        k_emit<<<(unsigned)((cap + kEmitChunk - 1) / kEmitChunk), 256, 0, s>>>(
            ws.dval[1], ws.counters, rects, ws.pair_off, ws.slice_start, num_pairs, tiles_x,
            pair_tiles, pair_gids, cap);
    return hipGetLastError();
}

hipError_t launch_emit(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                       int n, int tiles_x, int extent_rule, uint32_t *pair_tiles,
                       uint32_t *pair_gids, int64_t cap, int64_t *num_pairs, const Workspace &ws,
                       hipStream_t s) {
    hipError_t e = launch_emit_prepare(splats, rects, tiles_touched, n, extent_rule, cap, num_pairs,
                                       ws, s);
    if (e != hipSuccess || n == 0) return e;
    return launch_emit_pairs(splats, rects, tiles_x, extent_rule, pair_tiles, pair_gids, cap,
                             num_pairs, ws, s);
}

int emit_chunk() { return kEmitChunk; }

}  // namespace gsr
