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

__global__ __launch_bounds__(256) void k_pair_block_counts(const uint32_t *sorted_ids,
                                                           const int64_t *num_vis,
                                                           const uint64_t *rects, uint64_t *cnt) {
    __shared__ uint64_t wt[4];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t c = j < *num_vis ? (uint64_t)rect_tiles(rects[sorted_ids[j]]) : 0ull;
    uint64_t tot;
    block_exclusive_scan<256, uint64_t>(c, wt, &tot);
    if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_emit(const uint32_t *sorted_ids, const int64_t *num_vis,
                                              const uint64_t *rects, const uint64_t *block_off,
                                              int tiles_x, uint32_t *pair_tiles, uint32_t *pair_gids,
                                              int64_t cap) {
    __shared__ uint32_t start[257];
    __shared__ uint32_t gid_s[256], x0_s[256], y0_s[256], w_s[256];
    __shared__ float rw_s[256];
    __shared__ uint32_t wt[4];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t c = 0;
    if (j < *num_vis) {
        const uint32_t g = sorted_ids[j];
        const uint64_t r = rects[g];
        const uint32_t x0 = r & 0xffff, y0 = (r >> 16) & 0xffff, x1 = (r >> 32) & 0xffff, y1 = r >> 48;
        c = (x1 - x0) * (y1 - y0);
        gid_s[threadIdx.x] = g;
        x0_s[threadIdx.x] = x0;
        y0_s[threadIdx.x] = y0;
        w_s[threadIdx.x] = x1 - x0;
        rw_s[threadIdx.x] = 1.0f / (float)(x1 - x0);
    }
    uint32_t total;
    start[threadIdx.x] = block_exclusive_scan<256, uint32_t>(c, wt, &total);
    if (threadIdx.x == 0) start[256] = total;
    __syncthreads();
    const int64_t base = (int64_t)block_off[blockIdx.x];
    for (uint32_t k = threadIdx.x; k < total; k += 256) {
        // owner: the last Gaussian whose start is <= k (binary search in LDS)
        int lo = 0, hi = 255;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const uint32_t m = k - start[lo];
        const uint32_t w = w_s[lo];
        int q = (int)((float)m * rw_s[lo]);  // m / w, corrected below
        int rr = (int)m - q * (int)w;
        if (rr < 0) { --q; rr += (int)w; } else if (rr >= (int)w) { ++q; rr -= (int)w; }
        const int64_t dst = base + k;
        if (dst < cap) {
            pair_tiles[dst] = (y0_s[lo] + (uint32_t)q) * (uint32_t)tiles_x + x0_s[lo] + (uint32_t)rr;
            pair_gids[dst] = gid_s[lo];
        }
    }
}

hipError_t launch_emit(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                       int n, int tiles_x, uint32_t *pair_tiles, uint32_t *pair_gids, int64_t cap,
                       int64_t *num_pairs, const Workspace &ws, hipStream_t s) {
    const int64_t nb = ws.nb_gauss;
    int64_t *num_vis = ws.counters;
    if (n == 0) {
        k_set_i64<<<1, 1, 0, s>>>(num_pairs, 0);
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
    k_pair_block_counts<<<(unsigned)nb, 256, 0, s>>>(ws.dval[1], num_vis, rects, ws.pair_cnt);
    e = scan_exclusive_u64(ws.pair_cnt, ws.pair_off, nb, ws.scan_part, num_pairs, s);
    if (e != hipSuccess) return e;
    k_emit<<<(unsigned)nb, 256, 0, s>>>(ws.dval[1], num_vis, rects, ws.pair_off, tiles_x, pair_tiles,
                                       pair_gids, cap);
    return hipGetLastError();
}

}  // namespace gsr
