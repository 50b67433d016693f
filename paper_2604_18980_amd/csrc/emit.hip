// Stage 2: Gaussian-tile pair generation (paper Sec. 2.1, Fig. 1).
//
// The paper's pipeline emits pairs Gaussian by Gaussian and then sorts
// (tile | depth) keys.  Here the Gaussians are first put in depth order (a
// radix sort of one 32-bit key per visible Gaussian, a few MB), and pairs are
// emitted in that order.  The per-tile depth order then only needs a stable
// sort by tile id (16 bits at 4608x3456) instead of a 48-bit (tile | depth)
// sort of every pair; the sorted result is the same sequence.
//
//   k_vis_count / scan / k_vis_compact   visible Gaussians -> (depth bits, id)
//   radix_sort_u32                      by depth bits (stable: ties keep id order)
//   k_pair_block_counts / scan          pairs per block of 256 sorted Gaussians
//   k_emit                              each block writes its pairs contiguously,
//                                       one pair per thread per step, after an LDS
//                                       scan of its Gaussians' tile counts
#include "gsr_internal.hpp"

namespace gsr {

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

__global__ __launch_bounds__(256) void k_vis_count(const uint32_t *tiles_touched, int n,
                                                   uint32_t *vis_count) {
    __shared__ uint32_t wt[4];
    const int g = blockIdx.x * 256 + threadIdx.x;
    const uint32_t v = (g < n && tiles_touched[g] > 0) ? 1u : 0u;
    uint32_t tot;
    block_exclusive_scan<256, uint32_t>(v, wt, &tot);
    if (threadIdx.x == 0) vis_count[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_vis_compact(const uint32_t *tiles_touched, const float *splats,
                                                     int n, const uint32_t *vis_off, uint32_t *dkey,
                                                     uint32_t *dval) {
    __shared__ uint32_t wt[4];
    const int g = blockIdx.x * 256 + threadIdx.x;
    const bool vis = g < n && tiles_touched[g] > 0;
    uint32_t tot;
    const uint32_t pos = vis_off[blockIdx.x] +
                         block_exclusive_scan<256, uint32_t>(vis ? 1u : 0u, wt, &tot);
    if (vis) {
        dkey[pos] = __float_as_uint(splats[(size_t)g * 12 + 6]);  // depth > 0.2: bits order = value order
        dval[pos] = (uint32_t)g;
    }
}

__device__ __forceinline__ uint32_t rect_tiles(uint64_t r) {
    const uint32_t x0 = r & 0xffff, y0 = (r >> 16) & 0xffff, x1 = (r >> 32) & 0xffff, y1 = r >> 48;
    return (x1 - x0) * (y1 - y0);
}

// Pairs of each depth-sorted visible Gaussian.
__global__ __launch_bounds__(256) void k_pair_counts(const uint32_t *sorted_ids, const int64_t *num_vis,
                                                     const uint64_t *rects, uint64_t *cnt, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n || j >= *num_vis) return;
    cnt[j] = (uint64_t)rect_tiles(rects[sorted_ids[j]]);
}

// Emission is split into fixed slices of kEmitChunk pairs, one per workgroup,
// so a few huge Gaussians cannot serialise one block.  bstart[b] = the sorted
// Gaussian that owns pair b * kEmitChunk (each Gaussian marks the slices that
// begin inside its pair range).

__global__ __launch_bounds__(256) void k_slice_starts(const uint64_t *off, const uint64_t *cnt,
                                                      const int64_t *num_vis, uint32_t *bstart,
                                                      int64_t n, int64_t cap) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n || j >= *num_vis) return;
    const uint64_t p0 = off[j], p1 = p0 + cnt[j];
    // only slices that start below the capacity are ever emitted
    for (uint64_t b = (p0 + kEmitChunk - 1) / kEmitChunk; b * kEmitChunk < p1 && (int64_t)(b * kEmitChunk) < cap; ++b)
        bstart[b] = (uint32_t)j;
}

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
                               const uint32_t *tiles_touched, int n, int64_t cap, int64_t *num_pairs,
                               const Workspace &ws, hipStream_t s) {
    const int64_t nb = ws.nb_gauss;
    int64_t *num_vis = ws.counters;
    if (n == 0) {
        k_set_i64<<<1, 1, 0, s>>>(num_pairs, 0);
        k_set_i64<<<1, 1, 0, s>>>(num_vis, 0);
        return hipGetLastError();
    }
    k_vis_count<<<(unsigned)nb, 256, 0, s>>>(tiles_touched, n, ws.vis_count);
    hipError_t e = scan_exclusive_u32(ws.vis_count, ws.vis_off, nb, ws.scan_part, num_vis, s);
    if (e != hipSuccess) return e;
    k_vis_compact<<<(unsigned)nb, 256, 0, s>>>(tiles_touched, splats, n, ws.vis_off, ws.dkey[0],
                                              ws.dval[0]);
    e = radix_sort_u32(ws.dkey[0], ws.dval[0], ws.dkey[1], ws.dval[1], ws.dkey[2], ws.dval[2],
                       num_vis, n, 32, ws.dhist, ws.nb_dsort, ws.scan_part, s);
    if (e != hipSuccess) return e;
    k_pair_counts<<<(unsigned)nb, 256, 0, s>>>(ws.dval[1], num_vis, rects, ws.pair_cnt, n);
    // only the num_vis leading entries are live
    e = scan_exclusive_u64(ws.pair_cnt, ws.pair_off, n, ws.scan_part, num_pairs, s,
                           DevExtent{num_vis, n, 1, 1});
    if (e != hipSuccess) return e;
    if (cap > 0)
        k_slice_starts<<<(unsigned)nb, 256, 0, s>>>(ws.pair_off, ws.pair_cnt, num_vis, ws.slice_start,
                                                   n, cap);
    return hipGetLastError();
}

hipError_t launch_emit_pairs(const uint64_t *rects, int tiles_x, uint32_t *pair_tiles,
                             uint32_t *pair_gids, int64_t cap, const int64_t *num_pairs,
                             const Workspace &ws, hipStream_t s) {
    if (cap > 0)
        k_emit<<<(unsigned)((cap + kEmitChunk - 1) / kEmitChunk), 256, 0, s>>>(
            ws.dval[1], ws.counters, rects, ws.pair_off, ws.slice_start, num_pairs, tiles_x,
            pair_tiles, pair_gids, cap);
    return hipGetLastError();
}

hipError_t launch_emit(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                       int n, int tiles_x, uint32_t *pair_tiles, uint32_t *pair_gids, int64_t cap,
                       int64_t *num_pairs, const Workspace &ws, hipStream_t s) {
    hipError_t e = launch_emit_prepare(splats, rects, tiles_touched, n, cap, num_pairs, ws, s);
    if (e != hipSuccess || n == 0) return e;
    return launch_emit_pairs(rects, tiles_x, pair_tiles, pair_gids, cap, num_pairs, ws, s);
}

int emit_chunk() { return kEmitChunk; }

}  // namespace gsr
