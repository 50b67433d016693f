// Internal declarations shared by the HIP translation units of libgsr.
// Device helpers are written for 64-wide wavefronts (CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsr.h"

namespace gsr {

constexpr int kTile = GS_TILE;
constexpr int kWave = 64;
constexpr int kLutBins = GS_LUT_BINS;

// ---------------------------------------------------------------- launch args
struct PreprocessArgs {
    const float *means, *log_scales, *quats, *opacity_logits, *sh;
    int n, sh_degree;
    double R[9], t[3], campos[3];
    double fx, fy, cx, cy, limx, limy;
    int width, height, tiles_x, tiles_y;
    int adagscale, force_unit_scale;
    int extent_rule;  // 0, 2: scaled extent's rectangle (rule 2: oriented box at emission);
                      // 1: plain rectangle (ellipse test at emission)
    double K, lut_depth_max;
    float lut[kLutBins];
    // float32 copies for the preprocess' float32 prefilter (proves culls)
    float Rf[9], tf[3], fxf, fyf, cxf, cyf, limxf, limyf, Kf, lut_scalef;  // lut_scalef = 20 / D_max
    double shc[16];  // real-SH normalisation constants, see preprocess.hip
    float shcf[16];  // the same, rounded to float32 (colour is evaluated in float32)
    float *splats;
    uint64_t *rects;
    uint32_t *tiles_touched;
};

// Workspace layout, computed identically by the size query and every stage.
struct Workspace {
    // emit
    uint32_t *vis_count;   // [nb_dsort] visible Gaussians per chunk of 4096 ids
    uint64_t *pair_tot;    // [nb_dsort] pairs per chunk of 4096 depth-sorted visible Gaussians
    uint32_t *dgsum;       // [2][nb_dgroups][256] depth-pass digit sums per block group
    int64_t nb_dpass;      // blocks of the depth passes' grid (lsd_pass_blocks(n))
    int64_t nb_dgroups;    // group sums per digit row (lsd_pass_groups(n))
    uint64_t *pair_cnt;    // [n] pairs of each depth-sorted visible Gaussian
    uint64_t *pair_off;    // [n] their exclusive prefix
    uint32_t *slice_start; // [cap / emit chunk + 1] first Gaussian of each emission slice
    uint32_t *dkey[3];     // [n] depth keys: input, sorted output, pass scratch
    uint32_t *dval[3];     // [n] Gaussian ids, same roles
    uint32_t *dhist;       // [nb_dpass][256]
    // sort
    uint32_t *ptile_tmp;   // [cap]
    uint32_t *pgid_tmp;    // [cap]
    uint32_t *phist;       // [lsd_pass_blocks(cap)][256]
    uint32_t *psum;        // [2][lsd_pass_groups(cap)][256]
    // fused binning (bin.hip)
    uint32_t *bpacked;     // [cap] pass-1 output: tile >> 8 in bits 24..31, depth rank below
    uint32_t *bhist;       // [256][nb_psort] pass-1 histogram / offsets
    uint32_t *bhist2;      // [256][nb_psort + 256] pass-2 histogram / offsets
    uint32_t *bplan;       // [2][257] pass-1 bucket starts, first pass-2 block per bucket
    uint32_t *bkey, *bval; // [cap] each, only when the packed path does not apply
    // device-wide scan partials (large enough for any scan above)
    uint64_t *scan_part;   // [max_parts]
    int64_t *counters;     // [0] visible Gaussians, [1] scratch, [2] pass-2 blocks
    int64_t nb_gauss, nb_dsort, nb_psort, max_parts;
    int tiles_x, tiles_y;
    size_t bytes;
};
// tiles_x = tiles_y = 0 leaves out the binning buffers (emit and sort alone).
bool workspace_layout(int64_t n, int64_t cap, void *base, Workspace *ws, int tiles_x = 0,
                      int tiles_y = 0);
// whether launch_bin takes the packed two-pass route for this problem
bool bin_packed(int64_t n, int tiles_x, int tiles_y);
int emit_chunk();

// ------------------------------------------------------------ sort constants
constexpr int kSortThreads = 256;
#ifndef GSR_SORT_ITEMS
#define GSR_SORT_ITEMS 16
#endif
constexpr int kSortItems = GSR_SORT_ITEMS;                // per thread
constexpr int kSortChunk = kSortThreads * kSortItems;     // 4096 items per block
// pairs per emission slice (one workgroup each); slice_start[b] is the
// depth-sorted Gaussian that owns pair b * kEmitChunk
constexpr int kEmitChunk = kSortChunk;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;     // 4096 elements per block

// ------------------------------------------------------------------ launchers
hipError_t launch_preprocess(const PreprocessArgs &a, hipStream_t s);

// Number of live elements of a device-wide pass whose launch was sized on the
// host for the capacity m: with `count` set, mul * ceil(min(*count, cap) / chunk)
// (at most m), read on the device so no host round trip is needed.
// A count read on the device, clamped to the capacity cap that launches were
// sized for; with empty_if_over, a count above cap counts as zero (a pass that
// must not run on a partial set).
__device__ __forceinline__ int64_t live_count(const int64_t *count, int64_t cap, int empty_if_over) {
    const int64_t c = *count;
    if (c > cap) return empty_if_over ? 0 : cap;
    return c < 0 ? 0 : c;
}

struct DevExtent {
    const int64_t *count = nullptr;
    int64_t cap = 0, chunk = 1, mul = 1;
    bool empty_if_over = false;
    __device__ __forceinline__ int64_t resolve(int64_t m) const {
        if (!count) return m;
        const int64_t c = live_count(count, cap, empty_if_over);
        const int64_t e = ((c + chunk - 1) / chunk) * mul;
        return e < m ? e : m;
    }
};

// device-wide exclusive scan of m elements (m known on the host, or fewer as
// given by ext); if total is non-null the grand total is stored there (as int64).
hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t m, uint64_t *parts,
                              int64_t *total, hipStream_t s, DevExtent ext = DevExtent{});

// Stable LSD radix sort of (key, val) pairs by key bits [first_bit, bits),
// count in device memory (clamped to cap, or taken as zero when above cap with
// empty_if_over).  Reads (kin, vin), leaves them unchanged, and puts the result
// in (kout, vout); (ktmp, vtmp) is pass scratch distinct from both.  hist:
// [lsd_pass_blocks(cap)][256]; gsum: [2][lsd_pass_groups(cap)][256], whose
// first half the caller may have cleared already (gsum_zeroed).
hipError_t radix_sort_u32(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                          uint32_t *ktmp, uint32_t *vtmp, const int64_t *count, int64_t cap,
                          int bits, uint32_t *hist, uint32_t *gsum, hipStream_t s, int first_bit = 0,
                          int empty_if_over = 0, bool gsum_zeroed = false);
int64_t lsd_pass_blocks(int64_t cap);
int64_t lsd_pass_groups(int64_t cap);

hipError_t launch_emit(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                       int n, int tiles_x, int extent_rule, uint32_t *pair_tiles,
                       uint32_t *pair_gids, int64_t cap, int64_t *num_pairs, const Workspace &ws,
                       hipStream_t s);
// Everything of launch_emit before the pairs are written: visible Gaussians in
// depth order (ws.dval[1], count in ws.counters[0]), their pair counts and
// offsets (ws.pair_cnt, ws.pair_off), the pair total, and the emission slice
// owners (ws.slice_start, when cap > 0).
// Stable sort of the visible Gaussians' depth keys dkey/dval[0] (count in
// device memory) into dkey/dval[1]: four 8-bit LSD passes of two kernels
// each (digit offsets from block-group sums, no device-wide scan kernels).
hipError_t depth_sort(const Workspace &ws, const int64_t *count, hipStream_t s);
// xclear / xclear2 (nullable): further words its first kernel zeroes (for
// later kernels of the same call, in place of fill launches).
hipError_t launch_emit_prepare(const float *splats, const uint64_t *rects,
                               const uint32_t *tiles_touched, int n, int extent_rule, int64_t cap,
                               int64_t *num_pairs, const Workspace &ws, hipStream_t s,
                               uint32_t *xclear = nullptr, int64_t nxclear = 0,
                               uint32_t *xclear2 = nullptr, int64_t nxclear2 = 0);
// The pair-writing part of launch_emit, after launch_emit_prepare: whole
// rectangles (extent rule 0) or each rectangle row's ellipse (rule 1) or
// oriented-box (rule 2) span, recomputed from the splat records.
hipError_t launch_emit_pairs(const float *splats, const uint64_t *rects, int tiles_x,
                             int extent_rule, uint32_t *pair_tiles, uint32_t *pair_gids,
                             int64_t cap, const int64_t *num_pairs, const Workspace &ws,
                             hipStream_t s);
// Emission and tile sort fused (bin.hip): the sorted ids, optionally the sorted
// tile ids, and the ranges, without the emission-order pair arrays.
hipError_t launch_bin(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                      int n, int tiles_x, int tiles_y, int extent_rule, uint32_t *sorted_gids,
                      uint32_t *sorted_tiles, uint32_t *ranges, int64_t cap, int64_t *num_pairs,
                      const Workspace &ws, hipStream_t s);

// ranges_zeroed: the caller has cleared the ranges (no fill launch).
hipError_t launch_tile_ranges(const uint32_t *sorted_tiles, const int64_t *num_pairs, int64_t cap,
                              uint32_t *ranges, int num_tiles, hipStream_t s, int empty_if_over = 0,
                              bool ranges_zeroed = false);

struct RasterArgs {
    const float *splats;
    const uint32_t *gids;
    const uint32_t *ranges;
    int width, height, tiles_x, tiles_y;
    float bg[3];
    float *image, *final_T;
    uint32_t *n_contrib;
    uint32_t *n_evaluated;  // nullable
    unsigned long long *work;  // nullable; set: count work instead of writing pixels
    // T_upper calibration (set lut_bits: no pixels written): per depth bin
    // (kLutBins over [0, lut_depth_max)) and optionally per Gaussian, the
    // largest transmittance in front of a Gaussian where it blends, as float
    // bits raised with atomicMax
    uint32_t *lut_bits;
    uint32_t *max_t_bits;
    double lut_depth_max;
    // contribution-skip rendering (skip_kind >= 0; pixels written): a blend
    // whose contribution alpha x (T, skip_weight[i] or skip_lut[depth bin of i],
    // for kinds 0, 1, 2) is below skip_theta is skipped; work, if set, then
    // receives [0] the skipped and [1] the kept blends (added)
    int skip_kind;  // -1: off
    float skip_theta;
    const float *skip_weight;
    float skip_lut[kLutBins];
    // contribution profile (prof_sum set; no pixels written): per bin of the
    // Mahalanobis distance m between pixel and mean, bin = min(floor(m /
    // width), prof_bins - 1), the sum and count of the blends' alpha T (added)
    float *prof_sum;
    unsigned long long *prof_cnt;
    int prof_bins;  // 1 .. kProfBins
    float prof_inv_width;
};
constexpr int kProfBins = 64;
hipError_t launch_raster(const RasterArgs &a, const gs_raster_cfg &cfg, hipStream_t s);

struct ViewsArgs {
    const gs_view_target *views;  // device
    float bg[3];
    const uint32_t *items;        // (view << 26 | tile), longest list first
    int64_t n_items;
    uint32_t *next;               // work ticket
    uint32_t *view_left;          // [n_views] tiles not yet finished
    uint64_t *clock;              // nullable, [1 + n_views]
};
hipError_t launch_raster_views(const ViewsArgs &q, const gs_raster_cfg &cfg, int grid, hipStream_t s);
int raster_views_grid(const gs_raster_cfg &cfg);

struct ViewsPlan {
    int n_views;
    int parts;                            // raster work items per tile (1, or 2 half tiles)
    uint32_t tile_off[GS_MAX_VIEWS + 1];  // prefix of tiles per view
    uint32_t tiles_x[GS_MAX_VIEWS];
};
hipError_t launch_views_plan(const ViewsPlan &p, const gs_view_target *d_views, uint32_t *keys,
                             uint32_t *vals, uint32_t *next, uint32_t *view_left, uint64_t *clock,
                             hipStream_t s);

struct RasterBwdArgs {
    const float *splats;
    const uint32_t *gids;
    const uint32_t *ranges;
    int width, height, tiles_x, tiles_y;
    float bg[3];
    const float *final_T;
    const uint32_t *n_contrib;
    const float *dL_dimage;
    float *grad_splats;
};
hipError_t launch_raster_backward(const RasterBwdArgs &a, int64_t n, hipStream_t s);

struct PreprocessBwdArgs {
    const float *means, *log_scales, *quats, *opacity_logits, *sh;
    int n, sh_degree;
    double R[9], t[3], campos[3];
    double fx, fy, limx, limy;
    double shc[16];
    float shcf[16];
    const uint32_t *tiles_touched;
    const float *grad_splats;
    float *d_means, *d_log_scales, *d_quats, *d_opacity_logits, *d_sh;
};
hipError_t launch_preprocess_backward(const PreprocessBwdArgs &a, hipStream_t s);

// Offset of element g of plane k of a [C][n] structure-of-arrays parameter,
// computed in 64 bits: k n + g passes 2^31 for n above about 7.2e8 (k = 3).
__host__ __device__ __forceinline__ size_t plane_at(int k, int n, int g) {
    return (size_t)k * (size_t)n + (size_t)g;
}

// ------------------------------------------------------------ device helpers
// p[i] for i < n, else zero, with the load made unconditionally (from p[0]
// past the end, so p must hold at least one element): a load under a
// per-lane condition compiles to a branch that waits for it, so a loop of
// guarded loads would make one memory round trip per element.
template <typename T>
__device__ __forceinline__ T load_or_zero(const T *p, int64_t i, int64_t n) {
    const T v = p[i < n ? i : 0];
    return i < n ? v : (T)0;
}

// An empty asm that claims to modify x: the value must exist in a register at
// this point, so the compiler neither sinks its computation nor recomputes it.
__device__ __forceinline__ void pin_vgpr(float &x) { __asm__ volatile("" : "+v"(x)); }

// The wave's LDS writes before this point are visible to its reads after it.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Exclusive scan across one block (BLOCK threads, multiple of 64) of a
// per-thread value; `wave_tot` is LDS scratch of BLOCK/64 entries.  Returns the
// exclusive prefix and writes the block total to *total.  Contains barriers.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wave_tot, T *total) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    T x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wave_tot[wid] = x;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / kWave; ++w) {
        T t = wave_tot[w];
        if (w < wid) pre += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

}  // namespace gsr
