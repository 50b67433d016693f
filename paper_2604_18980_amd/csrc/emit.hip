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
//   k_emit_spans                        extent rules 1 and 2: per wave 64
//                                       Gaussians' row spans (tile_shapes.hpp),
//                                       written by the whole wave
//                                       (Gaussians with long row bands: one at a
//                                       time by the whole wave, a row per lane)
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
// digit totals and group sums (accumulated by k_dhist) and the pair totals
// per chunk (accumulated by k_pair_counts).
__global__ __launch_bounds__(256) void k_vis_count(const uint32_t *tiles_touched, int n,
                                                   uint32_t *vis_count, uint32_t *clear,
                                                   int64_t nclear, uint64_t *clear64,
                                                   int64_t nclear64) {
    __shared__ uint32_t wt[4];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nclear; i += (int64_t)gridDim.x * 256)
        clear[i] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nclear64; i += (int64_t)gridDim.x * 256)
        clear64[i] = 0ull;
    const int64_t base = (int64_t)blockIdx.x * kSortChunk + threadIdx.x;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t g = base + (int64_t)i * 256;
        c += (g < n && tiles_touched[g] > 0u) ? 1u : 0u;
    }
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
    uint32_t pos[kSortItems], wc = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t g = wbase + 64 * i;
        m[i] = __ballot(g < n && tiles_touched[g] > 0u);
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
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if ((m[i] >> lane) & 1ull) {
            const int64_t g = wbase + 64 * i;
            dkey[woff + pos[i]] = __float_as_uint(splats[(size_t)g * 12 + 6]);  // depth > 0.2: bits order = value order
            dval[woff + pos[i]] = (uint32_t)g;
        }
    }
    if (threadIdx.x == 0 && b == (int64_t)gridDim.x - 1) *num_vis = (int64_t)(before + tot);
}

// Broadcast of one lane's shape and row range to the whole wave.
template <class Shape>
struct WaveShape {
    Shape e;
    int x0, x1, ra, rb;
};
template <class Shape>
__device__ __forceinline__ WaveShape<Shape> wave_broadcast(const Shape &e, int x0, int x1, int ra, int rb,
                                                           int src) {
    WaveShape<Shape> w;
    w.e = e;
    w.e.broadcast(src);
    w.x0 = lane_i32(x0, src);
    w.x1 = lane_i32(x1, src);
    w.ra = lane_i32(ra, src);
    w.rb = lane_i32(rb, src);
    return w;
}

// Pairs of each depth-sorted visible Gaussian (one per thread), added to the
// total of its chunk of 4096 (cleared by k_vis_count): the rectangle's area
// (tiles_touched) under extent rule 0, the count of its tiles that meet the
// ellipse under rule 1.  The visible Gaussians are dense here, so the FP64
// span arithmetic of rule 1 keeps the lanes busy.  A Gaussian whose row band
// is longer than kSmallRows is counted afterwards by its whole wave, one row
// per lane, so no lane walks a giant's rows alone.
// Pair count of one visible Gaussian under a shape rule: its tiles meeting the
// shape, or the whole wave's long-band Gaussians afterwards (see below).
template <class Shape>
__device__ __forceinline__ uint64_t shape_pair_count(const float *splats, const uint64_t *rects,
                                                     uint32_t g, bool valid) {
    const int lane = threadIdx.x & (kWave - 1);
    Shape e;
    int x0 = 0, x1 = 0, ra = 0, rb = 0;
    bool big = false;
    uint64_t c = 0;
    if (valid) {
        const uint64_t r = rects[g];
        if (e.setup(splats + (size_t)g * 12)) {
            x0 = (int)(r & 0xffff);
            x1 = (int)((r >> 32) & 0xffff);
            e.row_band((int)((r >> 16) & 0xffff), (int)(r >> 48), ra, rb);
            big = rb - ra > kSmallRows;
            if (!big) {
                for (int ty = ra; ty < rb; ++ty) {
                    int a, b;
                    if (e.row_span(ty, x0, x1 - 1, a, b)) c += (uint64_t)(b - a + 1);
                }
            }
        }
    }
    // the wave's long-band Gaussians, one at a time, a row per lane
    for (uint64_t m = __ballot(big); m; m &= m - 1) {  // wave-uniform
        const int src = __ffsll((long long)m) - 1;
        const WaveShape<Shape> w = wave_broadcast(e, x0, x1, ra, rb, src);
        uint32_t part = 0;
        for (int ty = w.ra + lane; ty < w.rb; ty += kWave) {
            int a, b;
            if (w.e.row_span(ty, w.x0, w.x1 - 1, a, b)) part += (uint32_t)(b - a + 1);
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
        if (lane == src) c = part;
    }
    return c;
}

// Pairs of each depth-sorted visible Gaussian (one per thread), added to the
// total of its chunk of 4096 (cleared by k_vis_count): the rectangle's area
// (tiles_touched) under extent rule 0, the count of its tiles that meet the
// ellipse (rule 1) or the oriented box (rule 2).  The visible Gaussians are
// dense here, so the FP64 span arithmetic keeps the lanes busy.  A Gaussian
// whose row band is longer than kSmallRows is counted afterwards by its whole
// wave, one row per lane, so no lane walks a giant's rows alone.
template <int RULE>
__global__ __launch_bounds__(256) void k_pair_counts(const uint32_t *sorted_ids, const int64_t *num_vis,
                                                     const uint32_t *tiles_touched, const float *splats,
                                                     const uint64_t *rects, uint64_t *cnt,
                                                     uint64_t *chunk_tot) {
    __shared__ uint64_t wt[4];
    const int64_t V = *num_vis;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((int64_t)blockIdx.x * 256 >= V) return;  // uniform
    uint64_t c = 0;
    const uint32_t g = j < V ? sorted_ids[j] : 0u;
    if constexpr (RULE == 0) {
        if (j < V) c = tiles_touched[g];
    } else if constexpr (RULE == 1) {
        c = shape_pair_count<Ellipse>(splats, rects, g, j < V);
    } else {
        c = shape_pair_count<OrientedBox>(splats, rects, g, j < V);
    }
    if (j < V) cnt[j] = c;
    uint64_t tot;
    block_exclusive_scan<256, uint64_t>(c, wt, &tot);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)&chunk_tot[(int64_t)blockIdx.x * 256 / kSortChunk],
                                           (unsigned long long)tot);
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
                               int64_t *num_pairs, const Workspace &ws, hipStream_t s) {
    int64_t *num_vis = ws.counters;
    if (n == 0) {
        k_set_i64<<<1, 1, 0, s>>>(num_pairs, 0);
        k_set_i64<<<1, 1, 0, s>>>(num_vis, 0);
        return hipGetLastError();
    }
    const unsigned nb = (unsigned)ws.nb_dsort;  // chunks of 4096 (ids, then visible Gaussians)
    // the depth passes' digit group sums and totals are contiguous: clear both
    k_vis_count<<<nb, 256, 0, s>>>(tiles_touched, n, ws.vis_count, ws.dgsum,
                                   4 * 256 * (ws.nb_dgroups + 1), ws.pair_tot, ws.nb_dsort);
    k_vis_compact<<<nb, 256, 0, s>>>(tiles_touched, splats, n, ws.vis_count, ws.dkey[0], ws.dval[0],
                                     num_vis);
    hipError_t e = depth_sort(ws, num_vis, s);  // dkey/dval[0] -> [1]
    if (e != hipSuccess) return e;
    if (extent_rule == 1)
        k_pair_counts<1><<<(unsigned)ws.nb_gauss, 256, 0, s>>>(ws.dval[1], num_vis, tiles_touched,
                                                              splats, rects, ws.pair_cnt, ws.pair_tot);
    else if (extent_rule == 2)
        k_pair_counts<2><<<(unsigned)ws.nb_gauss, 256, 0, s>>>(ws.dval[1], num_vis, tiles_touched,
                                                              splats, rects, ws.pair_cnt, ws.pair_tot);
    else
        k_pair_counts<0><<<(unsigned)ws.nb_gauss, 256, 0, s>>>(ws.dval[1], num_vis, tiles_touched,
                                                              splats, rects, ws.pair_cnt, ws.pair_tot);
    k_pair_offsets<<<nb, 256, 0, s>>>(ws.pair_cnt, ws.pair_tot, num_vis, ws.pair_off, ws.slice_start,
                                      num_pairs, cap);
    return hipGetLastError();
}

// Extent rule 1: each wave takes 64 consecutive depth-sorted visible
// Gaussians, one per lane.  Those with short row bands are walked in lockstep:
// per step every lane recomputes the ellipse span of its next row (exactly as
// k_pair_counts counted it), a wave prefix sum lays the spans end to end, and
// the whole wave writes them -- lane l takes pairs l, l + 64, ..., finding the
// span that holds each by binary search over the 64 span starts in LDS.  Then
// the long-band Gaussians follow one at a time, 64 of their rows per step, one
// row per lane, written the same way.  Pairs at or beyond the capacity are not
// written.
struct SpanTable {
    uint32_t start[kWave];  // exclusive prefix of the step's span lengths
    uint64_t k[kWave];      // output index of each span's first pair
    uint32_t t0[kWave];     // tile id of each span's first tile
    uint32_t gid[kWave];
};

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// mean span length from which a step's spans are written one at a time
#ifndef GSR_LONG_SPAN
#define GSR_LONG_SPAN 16
#endif

// Writes one step's spans (lane l's span: len pairs from output index k, tiles
// t0, t0 + 1, ..., Gaussian gid).  Long spans are written one after another by
// the whole wave (the span's values read from its lane, consecutive lanes on
// consecutive pairs); many short ones together, each lane finding the span of
// its pair by binary search over the span starts in LDS.  Contains wave
// barriers.
__device__ __forceinline__ void wave_write_spans(SpanTable &st, uint32_t len, uint64_t k, uint32_t t0,
                                                 uint32_t gid, uint32_t *pair_tiles,
                                                 uint32_t *pair_gids, int64_t cap) {
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t x = len;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    const uint32_t total = lane_u32(x, kWave - 1);
    const uint64_t spans = __ballot(len > 0u);
    if (total >= (uint32_t)GSR_LONG_SPAN * (uint32_t)__popcll(spans)) {  // long spans: one at a time
        for (uint64_t m = spans; m; m &= m - 1) {  // wave-uniform
            const int src = __ffsll((long long)m) - 1;
            const uint32_t n = lane_u32(len, src), tb = lane_u32(t0, src), gb = lane_u32(gid, src);
            const uint64_t kb = lane_u64(k, src);
            for (uint32_t i = (uint32_t)lane; i < n; i += kWave) {
                if (kb + i < (uint64_t)cap) {
                    pair_tiles[kb + i] = tb + i;
                    pair_gids[kb + i] = gb;
                }
            }
        }
        return;
    }
    st.start[lane] = x - len;
    st.k[lane] = k;
    st.t0[lane] = t0;
    st.gid[lane] = gid;
    wave_sync_lds();
    for (uint32_t i = (uint32_t)lane; i < total; i += kWave) {
        // the span holding pair i: the last lane whose start is <= i (a lane
        // with an empty span shares its start with the next lane)
        int lo = 0, hi = kWave - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (st.start[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const uint32_t m = i - st.start[lo];
        const uint64_t kk = st.k[lo] + m;
        if (kk < (uint64_t)cap) {
            pair_tiles[kk] = st.t0[lo] + m;
            pair_gids[kk] = st.gid[lo];
        }
    }
    wave_sync_lds();  // every lane has read the table before it is rewritten
}

template <class Shape>
__global__ __launch_bounds__(256) void k_emit_spans(const uint32_t *sorted_ids, const int64_t *num_vis,
                                                    const float *splats, const uint64_t *rects,
                                                    const uint64_t *off, int tiles_x,
                                                    uint32_t *pair_tiles, uint32_t *pair_gids,
                                                    int64_t cap) {
    __shared__ SpanTable s_tab[4];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int64_t V = *num_vis;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((int64_t)blockIdx.x * 256 + wid * kWave >= V) return;  // wave-uniform
    SpanTable &st = s_tab[wid];
    bool live = false, big = false;
    uint64_t k = 0;
    uint32_t g = 0;
    int ra = 0, rb = 0, x0 = 0, x1 = 0;
    Shape e;
    if (j < V) {
        k = off[j];
        g = sorted_ids[j];
        const uint64_t r = rects[g];
        x0 = (int)(r & 0xffff);
        x1 = (int)((r >> 32) & 0xffff);
        const float *rec = splats + (size_t)g * 12;
        if (k < (uint64_t)cap && e.setup(rec)) {
            e.row_band((int)((r >> 16) & 0xffff), (int)(r >> 48), ra, rb);
            big = rb - ra > kSmallRows;
            live = !big;
        }
    }
    // short bands: every lane its own rows, in lockstep
    uint64_t ks = k;
    for (int ty = ra;;) {
        const bool act = live && ty < rb;
        if (!__ballot(act)) break;  // wave-uniform
        uint32_t len = 0, t0 = 0;
        if (act) {
            int a, b;
            if (e.row_span(ty, x0, x1 - 1, a, b)) {
                len = (uint32_t)(b - a + 1);
                t0 = (uint32_t)ty * (uint32_t)tiles_x + (uint32_t)a;
            }
            ++ty;
        }
        wave_write_spans(st, len, ks, t0, g, pair_tiles, pair_gids, cap);
        ks += len;
    }
    // long bands: one Gaussian at a time, a row per lane
    for (uint64_t m = __ballot(big); m; m &= m - 1) {  // wave-uniform
        const int src = __ffsll((long long)m) - 1;
        const WaveShape<Shape> w = wave_broadcast(e, x0, x1, ra, rb, src);
        uint64_t kb = lane_u64(k, src);
        const uint32_t gb = lane_u32(g, src);
        for (int t = w.ra; t < w.rb; t += kWave) {  // wave-uniform
            const int ty = t + lane;
            uint32_t len = 0, t0 = 0;
            int a, b;
            if (ty < w.rb && w.e.row_span(ty, w.x0, w.x1 - 1, a, b)) {
                len = (uint32_t)(b - a + 1);
                t0 = (uint32_t)ty * (uint32_t)tiles_x + (uint32_t)a;
            }
            // this lane's row starts after the rows of the lanes below it
            uint32_t x = len;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, kWave);
                if (lane >= o) x += y;
            }
            const uint32_t total = lane_u32(x, kWave - 1);
            wave_write_spans(st, len, kb + (x - len), t0, gb, pair_tiles, pair_gids, cap);
            kb += total;
        }
    }
}

hipError_t launch_emit_pairs(const float *splats, const uint64_t *rects, int tiles_x,
                             int extent_rule, uint32_t *pair_tiles, uint32_t *pair_gids,
                             int64_t cap, const int64_t *num_pairs, const Workspace &ws,
                             hipStream_t s) {
    if (cap <= 0) return hipGetLastError();
    if (extent_rule == 1)
        k_emit_spans<Ellipse><<<(unsigned)ws.nb_gauss, 256, 0, s>>>(
            ws.dval[1], ws.counters, splats, rects, ws.pair_off, tiles_x, pair_tiles, pair_gids, cap);
    else if (extent_rule == 2)
        k_emit_spans<OrientedBox><<<(unsigned)ws.nb_gauss, 256, 0, s>>>(
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
