// C-ABI of libgsr: argument validation, workspace layout and launches.
// Every entry point validates on the host, then enqueues on the caller's
// stream; nothing here synchronises or allocates.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "gsr_internal.hpp"

namespace {
thread_local std::string g_last_error;

gs_status fail(gs_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

gs_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return GS_OK;
    return fail(GS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_f(float x) { return isfinite(x) != 0; }

gs_status check_camera(const gs_camera *cam) {
    if (!cam) return fail(GS_ERR_INVALID_ARGUMENT, "camera is NULL");
    if (cam->width < 1 || cam->height < 1 || cam->width > GS_MAX_IMAGE_SIDE ||
        cam->height > GS_MAX_IMAGE_SIDE)
        return fail(GS_ERR_INVALID_ARGUMENT, "image size %dx%d outside 1..%d", cam->width,
                    cam->height, GS_MAX_IMAGE_SIDE);
    for (int i = 0; i < 12; ++i)
        if (!finite_f(cam->viewmat[i])) return fail(GS_ERR_INVALID_ARGUMENT, "viewmat[%d] not finite", i);
    if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f) || !finite_f(cam->fx) || !finite_f(cam->fy))
        return fail(GS_ERR_INVALID_ARGUMENT, "focal lengths must be finite and positive");
    if (!finite_f(cam->cx) || !finite_f(cam->cy))
        return fail(GS_ERR_INVALID_ARGUMENT, "principal point not finite");
    return GS_OK;
}

int tiles_x(const gs_camera *c) { return (c->width + GS_TILE - 1) / GS_TILE; }
int tiles_y(const gs_camera *c) { return (c->height + GS_TILE - 1) / GS_TILE; }

int bits_for(int64_t count) {
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) < count) ++b;
    return b;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Raster geometries with a compiled kernel: one wave per tile with 4 pixels
// per lane, two waves per tile with 2 pixels per lane (each wave walks the
// list in batches of 64 for its 16x8 half), or one 256-thread workgroup per
// tile staging 64/128/256 records.
bool geometry_built(const gs_raster_cfg &c) {
    const bool block = c.threads_per_tile == 256 && c.pixels_per_thread == 1 &&
                       (c.lds_batch == 64 || c.lds_batch == 128 || c.lds_batch == 256);
    const bool wave = c.threads_per_tile == 64 && c.pixels_per_thread == 4 && c.lds_batch == 64;
    const bool half = c.threads_per_tile == 128 && c.pixels_per_thread == 2 && c.lds_batch == 64;
    return block || wave || half;
}

// Real-SH normalisation constants (Condon-Shortley phase) for the polynomial
// forms used by the device code:
//   c0 = sqrt(1/4pi), c1 = sqrt(3/4pi), c2 = sqrt(15/4pi), c3 = sqrt(5/16pi),
//   c4 = sqrt(15/16pi), c5 = sqrt(35/32pi), c6 = sqrt(105/4pi), c7 = sqrt(21/32pi),
//   c8 = sqrt(7/16pi), c9 = sqrt(105/16pi).
void sh_constants(double *c) {
    const double pi = 3.14159265358979323846;
    c[0] = sqrt(1.0 / (4.0 * pi));
    c[1] = sqrt(3.0 / (4.0 * pi));
    c[2] = sqrt(15.0 / (4.0 * pi));
    c[3] = sqrt(5.0 / (16.0 * pi));
    c[4] = sqrt(15.0 / (16.0 * pi));
    c[5] = sqrt(35.0 / (32.0 * pi));
    c[6] = sqrt(105.0 / (4.0 * pi));
    c[7] = sqrt(21.0 / (32.0 * pi));
    c[8] = sqrt(7.0 / (16.0 * pi));
    c[9] = sqrt(105.0 / (16.0 * pi));
    for (int i = 10; i < 16; ++i) c[i] = 0.0;
}

void camera_to_double(const gs_camera *cam, double R[9], double t[3], double campos[3]) {
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) R[3 * i + j] = cam->viewmat[4 * i + j];
        t[i] = cam->viewmat[4 * i + 3];
    }
    for (int j = 0; j < 3; ++j) campos[j] = -(R[j] * t[0] + R[3 + j] * t[1] + R[6 + j] * t[2]);
}

gs_status check_scene(const gs_scene *sc) {
    if (!sc) return fail(GS_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (sc->n < 0 || sc->n >= ((int64_t)1 << 31))
        return fail(GS_ERR_INVALID_ARGUMENT, "n = %lld outside [0, 2^31)", (long long)sc->n);
    if (sc->sh_degree < 0 || sc->sh_degree > GS_MAX_SH_DEGREE)
        return fail(GS_ERR_INVALID_ARGUMENT, "sh_degree %d outside 0..%d", sc->sh_degree, GS_MAX_SH_DEGREE);
    if (sc->n > 0 && (!sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits || !sc->sh))
        return fail(GS_ERR_INVALID_ARGUMENT, "scene has a NULL parameter array");
    if (((uintptr_t)sc->sh & 15) != 0)
        return fail(GS_ERR_INVALID_ARGUMENT, "sh is not 16-byte aligned");
    return GS_OK;
}

gs_status check_mode(const gs_mode *mode) {
    if (!mode) return fail(GS_ERR_INVALID_ARGUMENT, "mode is NULL");
    if (mode->adagscale != 0 && mode->adagscale != 1)
        return fail(GS_ERR_INVALID_ARGUMENT, "mode.adagscale must be 0 or 1");
    if (mode->adagscale) {
        if (!(mode->K >= 0.0f) || !finite_f(mode->K))
            return fail(GS_ERR_INVALID_ARGUMENT, "mode.K must be finite and >= 0");
        if (!(mode->lut_depth_max > 0.0f) || !finite_f(mode->lut_depth_max))
            return fail(GS_ERR_INVALID_ARGUMENT, "mode.lut_depth_max must be finite and > 0");
        for (int i = 0; i < GS_LUT_BINS; ++i)
            if (!(mode->t_upper[i] >= 0.0f && mode->t_upper[i] <= 1.0f))
                return fail(GS_ERR_INVALID_ARGUMENT, "mode.t_upper[%d] outside [0, 1]", i);
    }
    if (mode->extent_rule < 0 || mode->extent_rule > 2)
        return fail(GS_ERR_INVALID_ARGUMENT, "mode.extent_rule must be 0, 1 or 2");
    return GS_OK;
}

// The scene and method parts of the preprocess arguments (validated).
void fill_preprocess_args(const gs_scene *scene, const gs_mode *mode, gsr::PreprocessArgs *a) {
    memset(a, 0, sizeof *a);
    a->means = scene->means;
    a->log_scales = scene->log_scales;
    a->quats = scene->quats;
    a->opacity_logits = scene->opacity_logits;
    a->sh = scene->sh;
    a->n = (int)scene->n;
    a->sh_degree = scene->sh_degree;
    a->adagscale = mode->adagscale;
    a->force_unit_scale = mode->force_unit_scale ? 1 : 0;
    a->extent_rule = mode->extent_rule;
    a->K = mode->K;
    a->lut_depth_max = mode->lut_depth_max;
    a->Kf = mode->K;
    a->lut_scalef = (float)((double)GS_LUT_BINS / (double)mode->lut_depth_max);
    for (int i = 0; i < GS_LUT_BINS; ++i) a->lut[i] = mode->t_upper[i];
    sh_constants(a->shc);
    for (int i = 0; i < 16; ++i) a->shcf[i] = (float)a->shc[i];
}

// The camera part (validated camera).
void set_preprocess_camera(const gs_camera *cam, gsr::PreprocessArgs *a) {
    camera_to_double(cam, a->R, a->t, a->campos);
    a->fx = cam->fx;
    a->fy = cam->fy;
    a->cx = cam->cx;
    a->cy = cam->cy;
    a->limx = 1.3 * ((0.5 * cam->width) / a->fx);
    a->limy = 1.3 * ((0.5 * cam->height) / a->fy);
    a->width = cam->width;
    a->height = cam->height;
    a->tiles_x = tiles_x(cam);
    a->tiles_y = tiles_y(cam);
    for (int i = 0; i < 9; ++i) a->Rf[i] = (float)a->R[i];
    for (int i = 0; i < 3; ++i) a->tf[i] = (float)a->t[i];
    a->fxf = (float)a->fx;
    a->fyf = (float)a->fy;
    a->cxf = (float)a->cx;
    a->cyf = (float)a->cy;
    a->limxf = (float)a->limx;
    a->limyf = (float)a->limy;
}
}  // namespace

__global__ void k_set_count(int64_t *p, int64_t v) { *p = v; }

namespace gsr {
// Sort region (depends on the pair capacity only) first, then the emit region.
bool workspace_layout(int64_t n, int64_t cap, void *base, Workspace *ws, int tx, int ty) {
    if (n < 0 || cap < 0 || tx < 0 || ty < 0) return false;
    memset(ws, 0, sizeof *ws);
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) -> char * {
        off = align256(off);
        char *p = b ? b + off : nullptr;
        off += bytes;
        return p;
    };
    const bool bin = tx > 0 && ty > 0;
    const int64_t ntiles = (int64_t)tx * ty;
    ws->tiles_x = tx;
    ws->tiles_y = ty;
    ws->nb_psort = cap > 0 ? (cap + kSortChunk - 1) / kSortChunk : 1;
    ws->nb_gauss = n > 0 ? (n + 255) / 256 : 1;
    ws->nb_dsort = n > 0 ? (n + kSortChunk - 1) / kSortChunk : 1;
    const int64_t parts_sort = (256 * ws->nb_psort + kScanChunk - 1) / kScanChunk + 1;
    const int64_t parts_emit = (256 * ws->nb_dsort + kScanChunk - 1) / kScanChunk +
                               (n + kScanChunk - 1) / kScanChunk + 1;
    const int64_t parts_bin = (256 * (ws->nb_psort + 256) + kScanChunk - 1) / kScanChunk + 1;
    ws->max_parts = parts_sort > parts_emit ? parts_sort : parts_emit;
    if (parts_bin > ws->max_parts) ws->max_parts = parts_bin;
    // sort region
    ws->ptile_tmp = (uint32_t *)take(sizeof(uint32_t) * (size_t)cap);
    ws->pgid_tmp = (uint32_t *)take(sizeof(uint32_t) * (size_t)cap);
    ws->phist = (uint32_t *)take(sizeof(uint32_t) * 256 * (size_t)lsd_pass_blocks(cap));
    ws->psum = (uint32_t *)take(sizeof(uint32_t) * 2 * 256 * (size_t)lsd_pass_groups(cap));
    ws->scan_part = (uint64_t *)take(sizeof(uint64_t) * (size_t)ws->max_parts);
    ws->counters = (int64_t *)take(sizeof(int64_t) * 4);
    const size_t sort_bytes = align256(off);
    // emit region
    ws->nb_dpass = lsd_pass_blocks(n);
    ws->nb_dgroups = lsd_pass_groups(n);
    ws->vis_count = (uint32_t *)take(sizeof(uint32_t) * (size_t)ws->nb_dsort);
    ws->pair_tot = (uint64_t *)take(sizeof(uint64_t) * (size_t)ws->nb_dsort);
    ws->dgsum = (uint32_t *)take(sizeof(uint32_t) * 2 * 256 * (size_t)ws->nb_dgroups);
    ws->pair_cnt = (uint64_t *)take(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    ws->pair_off = (uint64_t *)take(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    ws->slice_start = (uint32_t *)take(sizeof(uint32_t) * (size_t)(cap / kEmitChunk + 2));
    for (int i = 0; i < 3; ++i) {
        ws->dkey[i] = (uint32_t *)take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
        ws->dval[i] = (uint32_t *)take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    }
    ws->dhist = (uint32_t *)take(sizeof(uint32_t) * 256 * (size_t)ws->nb_dpass);
    const size_t emit_bytes = align256(off);
    if (!bin) {
        ws->bytes = n > 0 ? emit_bytes : sort_bytes;
        return true;
    }
    // binning region
    ws->bpacked = (uint32_t *)take(sizeof(uint32_t) * (size_t)cap);
    ws->bhist = (uint32_t *)take(sizeof(uint32_t) * 256 * (size_t)ws->nb_psort);
    ws->bhist2 = (uint32_t *)take(sizeof(uint32_t) * 256 * (size_t)(ws->nb_psort + 256));
    ws->bplan = (uint32_t *)take(sizeof(uint32_t) * 2 * 257);
    if (!bin_packed(n, tx, ty)) {
        ws->bkey = (uint32_t *)take(sizeof(uint32_t) * (size_t)cap);
        ws->bval = (uint32_t *)take(sizeof(uint32_t) * (size_t)cap);
    }
    ws->bytes = align256(off);
    return true;
}
}  // namespace gsr


using namespace gsr;

namespace {
struct ViewsWs {
    uint32_t *key[3], *val[3], *hist, *gsum, *next, *view_left;
    size_t bytes;
};
void views_layout(int n_views, int64_t total, void *base, ViewsWs *w) {
    size_t off = 0;
    char *b = static_cast<char *>(base);
    auto take = [&](size_t bytes) -> char * {
        off = align256(off);
        char *p = b ? b + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t m = (size_t)(total > 0 ? total : 1);
    for (int i = 0; i < 3; ++i) {
        w->key[i] = (uint32_t *)take(4 * m);
        w->val[i] = (uint32_t *)take(4 * m);
    }
    w->hist = (uint32_t *)take(4 * 256 * (size_t)lsd_pass_blocks((int64_t)m));
    w->gsum = (uint32_t *)take(4 * 2 * 256 * (size_t)lsd_pass_groups((int64_t)m));
    w->next = (uint32_t *)take(4);
    w->view_left = (uint32_t *)take(4 * (size_t)(n_views > 0 ? n_views : 1));
    w->bytes = align256(off) + 256;  // + room for the item count
}

// The views' raster targets, written into the workspace by one kernel whose
// argument carries them (a captured graph replays the kernel with the values
// baked in; no host-to-device copy).
struct ViewTable {
    gs_view_target v[GS_MAX_VIEWS];
    int n_views;
};
constexpr size_t kViewTableBytes = (sizeof(gs_view_target) * GS_MAX_VIEWS + 255) & ~(size_t)255;
static_assert(sizeof(ViewTable) <= 4000, "kernel argument limit");

__global__ void k_view_table(const ViewTable t, gs_view_target *dst) {
    const int v = threadIdx.x;
    if (v < t.n_views) dst[v] = t.v[v];
}

hipError_t launch_view_table(const ViewTable &t, gs_view_target *dst, hipStream_t s) {
    k_view_table<<<1, GS_MAX_VIEWS, 0, s>>>(t, dst);
    return hipGetLastError();
}

// Streams and events of gs_render_views' per-view chains, one set per device,
// created on first use and kept for the life of the process.
constexpr int kMaxLanes = 8;
constexpr int kMaxDevices = 64;
struct LaneSet {
    hipStream_t s[kMaxLanes];
    hipEvent_t fork, join[kMaxLanes];
};
std::mutex g_lane_mutex;
LaneSet *g_lanes[kMaxDevices];

gs_status lane_set(LaneSet **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_UNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lock(g_lane_mutex);
    if (!g_lanes[dev]) {
        LaneSet *ls = new LaneSet();
        for (int l = 0; l < kMaxLanes && e == hipSuccess; ++l) {
            e = hipStreamCreateWithFlags(&ls->s[l], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ls->join[l], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ls->fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_check(e, "gs_render_views lane streams");
        g_lanes[dev] = ls;
    }
    *out = g_lanes[dev];
    return GS_OK;
}

// bits of the view index in the views queue's sort key (GS_MAX_VIEWS views)
constexpr int kViewBits = 6;
static_assert((1 << kViewBits) >= GS_MAX_VIEWS, "view index fits the key");

gs_status rasterize_views(const gs_view_target *views, const gs_view_target *d_views, int n_views,
                          const float *bg, const gs_raster_cfg *cfg, uint64_t *clock, void *ws,
                          size_t ws_bytes, hipStream_t s, const char *who) {
    if (!views || !d_views || !bg) return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (n_views < 1 || n_views > GS_MAX_VIEWS)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_views %d outside 1..%d", n_views, GS_MAX_VIEWS);
    ViewsPlan p;
    memset(&p, 0, sizeof p);
    p.n_views = n_views;
    int64_t total = 0;
    for (int v = 0; v < n_views; ++v) {
        const gs_view_target &t = views[v];
        if (t.width < 1 || t.height < 1 || t.width > GS_MAX_IMAGE_SIDE || t.height > GS_MAX_IMAGE_SIDE)
            return fail(GS_ERR_INVALID_ARGUMENT, "view %d: image size %dx%d", v, t.width, t.height);
        if (!t.ranges || !t.image || !t.final_T || !t.n_contrib)
            return fail(GS_ERR_INVALID_ARGUMENT, "view %d: NULL array", v);
        p.tile_off[v] = (uint32_t)total;
        p.tiles_x[v] = (uint32_t)((t.width + GS_TILE - 1) / GS_TILE);
        total += (int64_t)p.tiles_x[v] * ((t.height + GS_TILE - 1) / GS_TILE);
    }
    if (total >= ((int64_t)1 << 26)) return fail(GS_ERR_INVALID_ARGUMENT, "more than 2^26 tiles");
    p.tile_off[n_views] = (uint32_t)total;
    gs_raster_cfg c = {64, 4, 64};
    if (cfg && (cfg->threads_per_tile || cfg->pixels_per_thread || cfg->lds_batch)) {
        c = *cfg;
        if (!geometry_built(c))
            return fail(GS_ERR_UNSUPPORTED, "raster geometry %d/%d/%d not built", c.threads_per_tile,
                        c.pixels_per_thread, c.lds_batch);
    }
    p.parts = c.threads_per_tile == 128 ? 2 : 1;  // half tiles are separate work items
    ViewsWs w;
    views_layout(n_views, total, ws, &w);
    if (!ws || ws_bytes < w.bytes)
        return fail(GS_ERR_CAPACITY, "workspace of %zu bytes, %zu needed", ws_bytes, w.bytes);
    int64_t *count = (int64_t *)((char *)ws + w.bytes - 256);
    hipError_t e = launch_views_plan(p, d_views, w.key[0], w.val[0], w.next, w.view_left, clock, s);
    if (e == hipSuccess) {
        // the item count is a host-known constant; the sort reads it from device memory
        k_set_count<<<1, 1, 0, s>>>(count, total);
        e = radix_sort_u32(w.key[0], w.val[0], w.key[1], w.val[1], w.key[2], w.val[2], count, total,
                           24 + kViewBits, w.hist, w.gsum, s);
    }
    if (e != hipSuccess) return hip_check(e, who);
    ViewsArgs q;
    q.views = d_views;
    for (int i = 0; i < 3; ++i) q.bg[i] = bg[i];
    q.items = w.val[1];
    q.n_items = total;
    q.next = w.next;
    q.view_left = w.view_left;
    q.clock = clock;
    // persistent grid per (device, geometry), from the occupancy query
    static thread_local int grid_cache[kMaxDevices][5];
    const int gi = c.threads_per_tile == 256   ? (c.lds_batch == 64 ? 1 : c.lds_batch == 128 ? 2 : 3)
                   : c.threads_per_tile == 128 ? 4
                                               : 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    int &grid = grid_cache[dev][gi];
    if (!grid) grid = raster_views_grid(c);
    return hip_check(launch_raster_views(q, c, grid, s), who);
}

// Argument checks of gs_sort and gs_sort_noalloc (host only).
gs_status check_sort(const uint32_t *pair_tiles, const uint32_t *pair_gids,
                     const int64_t *num_pairs, int64_t pair_capacity, const gs_camera *cam,
                     const uint32_t *sorted_tiles, const uint32_t *sorted_gids,
                     const uint32_t *ranges) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (pair_capacity < 0 || pair_capacity > (int64_t)0xffffffffLL)
        return fail(GS_ERR_INVALID_ARGUMENT, "pair_capacity outside [0, 2^32)");
    if (!num_pairs || !ranges) return fail(GS_ERR_INVALID_ARGUMENT, "num_pairs or ranges is NULL");
    if (pair_capacity > 0 && (!pair_tiles || !pair_gids || !sorted_tiles || !sorted_gids))
        return fail(GS_ERR_INVALID_ARGUMENT, "pair arrays are NULL");
    if (pair_capacity > 0 && (sorted_tiles == pair_tiles || sorted_gids == pair_gids))
        return fail(GS_ERR_INVALID_ARGUMENT, "sorted arrays must not alias the inputs");
    return GS_OK;
}

// The sort's launches on a workspace of ws_bytes at ws.
gs_status enqueue_sort(const uint32_t *pair_tiles, const uint32_t *pair_gids,
                       const int64_t *num_pairs, int64_t pair_capacity, const gs_camera *cam,
                       uint32_t *sorted_tiles, uint32_t *sorted_gids, uint32_t *ranges, void *ws,
                       size_t ws_bytes, hipStream_t s, const char *who) {
    Workspace w;
    workspace_layout(0, pair_capacity, ws, &w);
    if (!ws || ws_bytes < w.bytes)
        return fail(GS_ERR_CAPACITY, "%s: workspace of %zu bytes, %zu needed", who, ws_bytes, w.bytes);
    const int ntiles = tiles_x(cam) * tiles_y(cam);
    gs_status st;
    if (pair_capacity > 0) {
        hipError_t e = radix_sort_u32(pair_tiles, pair_gids, sorted_tiles, sorted_gids, w.ptile_tmp,
                                      w.pgid_tmp, num_pairs, pair_capacity, bits_for(ntiles), w.phist,
                                      w.psum, s);
        if ((st = hip_check(e, who)) != GS_OK) return st;
    }
    return hip_check(launch_tile_ranges(sorted_tiles, num_pairs, pair_capacity, ranges, ntiles, s),
                     who);
}

// gs_sort_noalloc's workspace: a fixed device array of this library, held on
// every device the library runs on for the life of the process.  In host code
// `scratch` names a host-side stand-in, never the device memory: its device
// address is looked up once per device (with that device current) and kept.
// Every call of gs_sort_noalloc on a device shares that device's array.
constexpr size_t kScratchBytes = GS_SORT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mutex;
void *g_scratch[kMaxDevices];

gs_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_UNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(GS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return GS_OK;
}
}  // namespace

extern "C" {

const char *gs_status_string(gs_status s) {
    switch (s) {
        case GS_OK: return "ok";
        case GS_ERR_INVALID_ARGUMENT: return "invalid argument";
        case GS_ERR_CAPACITY: return "capacity exceeded";
        case GS_ERR_HIP: return "HIP error";
        case GS_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *gs_last_error(void) { return g_last_error.c_str(); }

const char *gs_version(void) { return "gsr 0.1 gfx950"; }

size_t gs_workspace_size(int64_t n, int64_t pair_capacity, int width, int height) {
    Workspace ws;
    const bool img = width >= 1 && height >= 1 && width <= GS_MAX_IMAGE_SIDE &&
                     height <= GS_MAX_IMAGE_SIDE;
    const int tx = img ? (width + GS_TILE - 1) / GS_TILE : 0;
    const int ty = img ? (height + GS_TILE - 1) / GS_TILE : 0;
    if (!workspace_layout(n, pair_capacity, nullptr, &ws, tx, ty)) return 0;
    return ws.bytes;
}

gs_status gs_preprocess(const gs_scene *scene, const gs_camera *cam, const gs_mode *mode,
                        float *splats, uint64_t *rects, uint32_t *tiles_touched, void *stream) {
    gs_status st;
    if ((st = check_scene(scene)) != GS_OK) return st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if ((st = check_mode(mode)) != GS_OK) return st;
    if (scene->n > 0 && (!splats || !rects || !tiles_touched))
        return fail(GS_ERR_INVALID_ARGUMENT, "output array is NULL");
    PreprocessArgs a;
    fill_preprocess_args(scene, mode, &a);
    set_preprocess_camera(cam, &a);
    a.splats = splats;
    a.rects = rects;
    a.tiles_touched = tiles_touched;
    return hip_check(launch_preprocess(a, (hipStream_t)stream), "gs_preprocess");
}

gs_status gs_emit_pairs(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                        int64_t n, const gs_camera *cam, int extent_rule, uint32_t *pair_tiles,
                        uint32_t *pair_gids, int64_t pair_capacity, int64_t *num_pairs, void *ws,
                        size_t ws_bytes, void *stream) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (extent_rule < 0 || extent_rule > 2)
        return fail(GS_ERR_INVALID_ARGUMENT, "extent_rule must be 0, 1 or 2");
    if (n < 0 || n >= ((int64_t)1 << 31))
        return fail(GS_ERR_INVALID_ARGUMENT, "n = %lld outside [0, 2^31)", (long long)n);
    if (pair_capacity < 0 || pair_capacity > (int64_t)0xffffffffLL)
        return fail(GS_ERR_INVALID_ARGUMENT, "pair_capacity outside [0, 2^32)");
    if (!num_pairs) return fail(GS_ERR_INVALID_ARGUMENT, "num_pairs is NULL");
    if (n > 0 && (!splats || !rects || !tiles_touched))
        return fail(GS_ERR_INVALID_ARGUMENT, "input array is NULL");
    if (pair_capacity > 0 && (!pair_tiles || !pair_gids))
        return fail(GS_ERR_INVALID_ARGUMENT, "pair arrays are NULL");
    Workspace w;
    workspace_layout(n, pair_capacity, ws, &w);
    if (!ws || ws_bytes < w.bytes)
        return fail(GS_ERR_CAPACITY, "workspace of %zu bytes, %zu needed", ws_bytes, w.bytes);
    return hip_check(launch_emit(splats, rects, tiles_touched, (int)n, tiles_x(cam), extent_rule,
                                 pair_tiles, pair_gids, pair_capacity, num_pairs, w,
                                 (hipStream_t)stream),
                     "gs_emit_pairs");
}

gs_status gs_bin_pairs(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                       int64_t n, const gs_camera *cam, int extent_rule, uint32_t *sorted_gids,
                       uint32_t *sorted_tiles, uint32_t *ranges, int64_t pair_capacity,
                       int64_t *num_pairs, void *ws, size_t ws_bytes, void *stream) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (extent_rule < 0 || extent_rule > 2)
        return fail(GS_ERR_INVALID_ARGUMENT, "extent_rule must be 0, 1 or 2");
    if (n < 0 || n >= ((int64_t)1 << 31))
        return fail(GS_ERR_INVALID_ARGUMENT, "n = %lld outside [0, 2^31)", (long long)n);
    if (pair_capacity < 0 || pair_capacity > (int64_t)0xffffffffLL)
        return fail(GS_ERR_INVALID_ARGUMENT, "pair_capacity outside [0, 2^32)");
    if (!num_pairs || !ranges) return fail(GS_ERR_INVALID_ARGUMENT, "num_pairs or ranges is NULL");
    if (n > 0 && (!splats || !rects || !tiles_touched))
        return fail(GS_ERR_INVALID_ARGUMENT, "input array is NULL");
    if (pair_capacity > 0 && !sorted_gids)
        return fail(GS_ERR_INVALID_ARGUMENT, "sorted_gids is NULL");
    Workspace w;
    workspace_layout(n, pair_capacity, ws, &w, tiles_x(cam), tiles_y(cam));
    if (!ws || ws_bytes < w.bytes)
        return fail(GS_ERR_CAPACITY, "workspace of %zu bytes, %zu needed", ws_bytes, w.bytes);
    return hip_check(launch_bin(splats, rects, tiles_touched, (int)n, tiles_x(cam), tiles_y(cam),
                                extent_rule, sorted_gids, sorted_tiles, ranges, pair_capacity,
                                num_pairs, w, (hipStream_t)stream),
                     "gs_bin_pairs");
}

gs_status gs_sort(const uint32_t *pair_tiles, const uint32_t *pair_gids, const int64_t *num_pairs,
                  int64_t pair_capacity, const gs_camera *cam, uint32_t *sorted_tiles,
                  uint32_t *sorted_gids, uint32_t *ranges, void *ws, size_t ws_bytes,
                  void *stream) {
    gs_status st = check_sort(pair_tiles, pair_gids, num_pairs, pair_capacity, cam, sorted_tiles,
                              sorted_gids, ranges);
    if (st != GS_OK) return st;
    return enqueue_sort(pair_tiles, pair_gids, num_pairs, pair_capacity, cam, sorted_tiles,
                        sorted_gids, ranges, ws, ws_bytes, (hipStream_t)stream, "gs_sort");
}

gs_status gs_sort_noalloc(const uint32_t *pair_tiles, const uint32_t *pair_gids,
                          const int64_t *num_pairs, int64_t pair_capacity, const gs_camera *cam,
                          uint32_t *sorted_tiles, uint32_t *sorted_gids, uint32_t *ranges,
                          void *stream) {
    gs_status st = check_sort(pair_tiles, pair_gids, num_pairs, pair_capacity, cam, sorted_tiles,
                              sorted_gids, ranges);
    if (st != GS_OK) return st;
    if (pair_capacity > GS_SORT_NOALLOC_MAX_PAIRS)
        return fail(GS_ERR_INVALID_ARGUMENT,
                    "gs_sort_noalloc: pair_capacity %lld above its fixed scratch's limit of %lld pairs",
                    (long long)pair_capacity, (long long)GS_SORT_NOALLOC_MAX_PAIRS);
    void *ptr = nullptr;
    if ((st = scratch_address(&ptr)) != GS_OK) return st;
    return enqueue_sort(pair_tiles, pair_gids, num_pairs, pair_capacity, cam, sorted_tiles,
                        sorted_gids, ranges, ptr, kScratchBytes, (hipStream_t)stream,
                        "gs_sort_noalloc");
}

gs_status gs_rasterize(const float *splats, int64_t n, const uint32_t *sorted_gids,
                       const uint32_t *ranges, const gs_camera *cam, const float *bg,
                       const gs_raster_cfg *cfg, float *image, float *final_T,
                       uint32_t *n_contrib, uint32_t *n_evaluated, void *stream) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (!ranges || !image || !final_T || !n_contrib || !bg)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n > 0 && (!splats || !sorted_gids)) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    gs_raster_cfg c = {64, 4, 64};
    if (cfg && (cfg->threads_per_tile || cfg->pixels_per_thread || cfg->lds_batch)) {
        c = *cfg;
        if (!geometry_built(c))
            return fail(GS_ERR_UNSUPPORTED, "raster geometry %d/%d/%d not built", c.threads_per_tile,
                        c.pixels_per_thread, c.lds_batch);
    }
    RasterArgs a;
    a.splats = splats;
    a.gids = sorted_gids;
    a.ranges = ranges;
    a.width = cam->width;
    a.height = cam->height;
    a.tiles_x = tiles_x(cam);
    a.tiles_y = tiles_y(cam);
    for (int i = 0; i < 3; ++i) a.bg[i] = bg[i];
    a.image = image;
    a.final_T = final_T;
    a.n_contrib = n_contrib;
    a.n_evaluated = n_evaluated;
    a.work = nullptr;
    a.lut_bits = a.max_t_bits = nullptr;
    a.skip_kind = -1;
    a.prof_sum = nullptr;
    a.lut_depth_max = 0.0;
    return hip_check(launch_raster(a, c, (hipStream_t)stream), "gs_rasterize");
}

gs_status gs_raster_work(const float *splats, int64_t n, const uint32_t *sorted_gids,
                         const uint32_t *ranges, const gs_camera *cam, uint64_t *work,
                         void *stream) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (!ranges || !work) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n > 0 && (!splats || !sorted_gids)) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    RasterArgs a;
    a.splats = splats;
    a.gids = sorted_gids;
    a.ranges = ranges;
    a.width = cam->width;
    a.height = cam->height;
    a.tiles_x = tiles_x(cam);
    a.tiles_y = tiles_y(cam);
    for (int i = 0; i < 3; ++i) a.bg[i] = 0.0f;
    a.image = a.final_T = nullptr;
    a.n_contrib = nullptr;
    a.n_evaluated = nullptr;
    a.work = reinterpret_cast<unsigned long long *>(work);
    a.lut_bits = a.max_t_bits = nullptr;
    a.skip_kind = -1;
    a.prof_sum = nullptr;
    a.lut_depth_max = 0.0;
    const gs_raster_cfg c = {64, 4, 64};
    return hip_check(launch_raster(a, c, (hipStream_t)stream), "gs_raster_work");
}

gs_status gs_calibrate_t_upper(const float *splats, int64_t n, const uint32_t *sorted_gids,
                               const uint32_t *ranges, const gs_camera *cam, float lut_depth_max,
                               uint32_t *t_upper_bits, uint32_t *max_t_bits, void *stream) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (!ranges || !t_upper_bits) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n > 0 && (!splats || !sorted_gids)) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (!(lut_depth_max > 0.0f) || !finite_f(lut_depth_max))
        return fail(GS_ERR_INVALID_ARGUMENT, "lut_depth_max must be finite and > 0");
    RasterArgs a;
    a.splats = splats;
    a.gids = sorted_gids;
    a.ranges = ranges;
    a.width = cam->width;
    a.height = cam->height;
    a.tiles_x = tiles_x(cam);
    a.tiles_y = tiles_y(cam);
    for (int i = 0; i < 3; ++i) a.bg[i] = 0.0f;
    a.image = a.final_T = nullptr;
    a.n_contrib = nullptr;
    a.n_evaluated = nullptr;
    a.work = nullptr;
    a.lut_bits = t_upper_bits;
    a.max_t_bits = max_t_bits;
    a.lut_depth_max = (double)lut_depth_max;
    a.skip_kind = -1;
    a.prof_sum = nullptr;
    const gs_raster_cfg c = {64, 4, 64};
    return hip_check(launch_raster(a, c, (hipStream_t)stream), "gs_calibrate_t_upper");
}

gs_status gs_rasterize_skip(const float *splats, int64_t n, const uint32_t *sorted_gids,
                            const uint32_t *ranges, const gs_camera *cam, const float *bg,
                            int kind, float theta, const float *weight, const float *t_upper,
                            float lut_depth_max, float *image, float *final_T, uint32_t *n_contrib,
                            unsigned long long *counts, void *stream) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (!ranges || !image || !final_T || !n_contrib || !bg)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n > 0 && (!splats || !sorted_gids)) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (kind < 0 || kind > 2) return fail(GS_ERR_INVALID_ARGUMENT, "kind must be 0, 1 or 2");
    if (!(theta >= 0.0f) || !finite_f(theta))
        return fail(GS_ERR_INVALID_ARGUMENT, "theta must be finite and >= 0");
    if (kind == 1 && n > 0 && !weight) return fail(GS_ERR_INVALID_ARGUMENT, "kind 1 needs weight");
    if (kind == 2) {
        if (!t_upper) return fail(GS_ERR_INVALID_ARGUMENT, "kind 2 needs t_upper");
        if (!(lut_depth_max > 0.0f) || !finite_f(lut_depth_max))
            return fail(GS_ERR_INVALID_ARGUMENT, "lut_depth_max must be finite and > 0");
    }
    RasterArgs a;
    a.splats = splats;
    a.gids = sorted_gids;
    a.ranges = ranges;
    a.width = cam->width;
    a.height = cam->height;
    a.tiles_x = tiles_x(cam);
    a.tiles_y = tiles_y(cam);
    for (int i = 0; i < 3; ++i) a.bg[i] = bg[i];
    a.image = image;
    a.final_T = final_T;
    a.n_contrib = n_contrib;
    a.n_evaluated = nullptr;
    a.work = counts;
    a.lut_bits = a.max_t_bits = nullptr;
    a.lut_depth_max = kind == 2 ? (double)lut_depth_max : 1.0;
    a.skip_kind = kind;
    a.prof_sum = nullptr;
    a.skip_theta = theta;
    a.skip_weight = weight;
    for (int i = 0; i < GS_LUT_BINS; ++i) a.skip_lut[i] = kind == 2 ? t_upper[i] : 1.0f;
    const gs_raster_cfg c = {64, 4, 64};
    return hip_check(launch_raster(a, c, (hipStream_t)stream), "gs_rasterize_skip");
}

gs_status gs_contribution_profile(const float *splats, int64_t n, const uint32_t *sorted_gids,
                                  const uint32_t *ranges, const gs_camera *cam, int nbins,
                                  float bin_width, float *sums, unsigned long long *counts,
                                  void *stream) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (!ranges || !sums || !counts) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n > 0 && (!splats || !sorted_gids)) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (nbins < 1 || nbins > kProfBins)
        return fail(GS_ERR_INVALID_ARGUMENT, "nbins must be in [1, %d]", kProfBins);
    if (!(bin_width > 0.0f) || !finite_f(bin_width))
        return fail(GS_ERR_INVALID_ARGUMENT, "bin_width must be finite and > 0");
    RasterArgs a;
    a.splats = splats;
    a.gids = sorted_gids;
    a.ranges = ranges;
    a.width = cam->width;
    a.height = cam->height;
    a.tiles_x = tiles_x(cam);
    a.tiles_y = tiles_y(cam);
    for (int i = 0; i < 3; ++i) a.bg[i] = 0.0f;
    a.image = a.final_T = nullptr;
    a.n_contrib = nullptr;
    a.n_evaluated = nullptr;
    a.work = nullptr;
    a.lut_bits = a.max_t_bits = nullptr;
    a.lut_depth_max = 1.0;
    a.skip_kind = -1;
    a.prof_sum = sums;
    a.prof_cnt = counts;
    a.prof_bins = nbins;
    a.prof_inv_width = 1.0f / bin_width;
    const gs_raster_cfg c = {64, 4, 64};
    return hip_check(launch_raster(a, c, (hipStream_t)stream), "gs_contribution_profile");
}

gs_status gs_rasterize_backward(const float *splats, int64_t n, const uint32_t *sorted_gids,
                                const uint32_t *ranges, const gs_camera *cam, const float *bg,
                                const float *final_T, const uint32_t *n_contrib,
                                const float *dL_dimage, float *grad_splats, void *stream) {
    gs_status st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GS_ERR_INVALID_ARGUMENT, "n outside [0, 2^31)");
    if (!ranges || !final_T || !n_contrib || !dL_dimage || !bg)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (n > 0 && (!splats || !sorted_gids || !grad_splats))
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    RasterBwdArgs a;
    a.splats = splats;
    a.gids = sorted_gids;
    a.ranges = ranges;
    a.width = cam->width;
    a.height = cam->height;
    a.tiles_x = tiles_x(cam);
    a.tiles_y = tiles_y(cam);
    for (int i = 0; i < 3; ++i) a.bg[i] = bg[i];
    a.final_T = final_T;
    a.n_contrib = n_contrib;
    a.dL_dimage = dL_dimage;
    a.grad_splats = grad_splats;
    return hip_check(launch_raster_backward(a, n, (hipStream_t)stream), "gs_rasterize_backward");
}

gs_status gs_preprocess_backward(const gs_scene *scene, const gs_camera *cam,
                                 const uint32_t *tiles_touched, const float *grad_splats,
                                 const gs_scene_grads *out, void *stream) {
    gs_status st;
    if ((st = check_scene(scene)) != GS_OK) return st;
    if ((st = check_camera(cam)) != GS_OK) return st;
    if (!out) return fail(GS_ERR_INVALID_ARGUMENT, "gradient struct is NULL");
    if (scene->n > 0 && (!tiles_touched || !grad_splats || !out->d_means || !out->d_log_scales ||
                         !out->d_quats || !out->d_opacity_logits || !out->d_sh))
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array argument");
    if (((uintptr_t)out->d_sh & 15) != 0)
        return fail(GS_ERR_INVALID_ARGUMENT, "d_sh is not 16-byte aligned");
    PreprocessBwdArgs a;
    memset(&a, 0, sizeof a);
    a.means = scene->means;
    a.log_scales = scene->log_scales;
    a.quats = scene->quats;
    a.opacity_logits = scene->opacity_logits;
    a.sh = scene->sh;
    a.n = (int)scene->n;
    a.sh_degree = scene->sh_degree;
    camera_to_double(cam, a.R, a.t, a.campos);
    a.fx = cam->fx;
    a.fy = cam->fy;
    a.limx = 1.3 * ((0.5 * cam->width) / a.fx);
    a.limy = 1.3 * ((0.5 * cam->height) / a.fy);
    sh_constants(a.shc);
    for (int i = 0; i < 16; ++i) a.shcf[i] = (float)a.shc[i];
    a.tiles_touched = tiles_touched;
    a.grad_splats = grad_splats;
    a.d_means = out->d_means;
    a.d_log_scales = out->d_log_scales;
    a.d_quats = out->d_quats;
    a.d_opacity_logits = out->d_opacity_logits;
    a.d_sh = out->d_sh;
    return hip_check(launch_preprocess_backward(a, (hipStream_t)stream), "gs_preprocess_backward");
}


int gs_wall_clock_khz(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, device) != hipSuccess) return 0;
    return v;
}

size_t gs_views_workspace_size(int n_views, int64_t total_tiles) {
    if (n_views < 0 || total_tiles < 0) return 0;
    ViewsWs w;
    views_layout(n_views, total_tiles, nullptr, &w);
    return w.bytes;
}

gs_status gs_rasterize_views(const gs_view_target *views, const gs_view_target *d_views,
                             int n_views, const float *bg, const gs_raster_cfg *cfg,
                             uint64_t *clock, void *ws, size_t ws_bytes, void *stream) {
    return rasterize_views(views, d_views, n_views, bg, cfg, clock, ws, ws_bytes,
                           (hipStream_t)stream, "gs_rasterize_views");
}

size_t gs_render_views_workspace_size(int n_views, int64_t total_tiles) {
    if (n_views < 0 || total_tiles < 0) return 0;
    ViewsWs w;
    views_layout(n_views, total_tiles, nullptr, &w);
    return kViewTableBytes + w.bytes;
}

gs_status gs_render_views(const gs_scene *scene, const gs_mode *mode, const gs_view_frame *views,
                          int n_views, const float *bg, const gs_raster_cfg *cfg, int lanes,
                          uint64_t *clock, void *ws, size_t ws_bytes, void *stream) {
    gs_status st;
    if ((st = check_scene(scene)) != GS_OK) return st;
    if ((st = check_mode(mode)) != GS_OK) return st;
    if (!views || !bg) return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (n_views < 1 || n_views > GS_MAX_VIEWS)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_views %d outside 1..%d", n_views, GS_MAX_VIEWS);
    if (lanes < 1 || lanes > kMaxLanes)
        return fail(GS_ERR_INVALID_ARGUMENT, "lanes %d outside 1..%d", lanes, kMaxLanes);
    const int64_t n = scene->n;
    ViewTable table;
    memset(&table, 0, sizeof table);
    table.n_views = n_views;
    int64_t total = 0;
    for (int v = 0; v < n_views; ++v) {
        const gs_view_frame &f = views[v];
        if ((st = check_camera(&f.cam)) != GS_OK)
            return fail(st, "view %d: %s", v, g_last_error.c_str());
        if (f.pair_capacity < 0 || f.pair_capacity > (int64_t)0xffffffffLL)
            return fail(GS_ERR_INVALID_ARGUMENT, "view %d: pair_capacity outside [0, 2^32)", v);
        if (!f.num_pairs || !f.ranges || !f.image || !f.final_T || !f.n_contrib)
            return fail(GS_ERR_INVALID_ARGUMENT, "view %d: NULL output array", v);
        if (n > 0 && (!f.splats || !f.rects || !f.tiles_touched))
            return fail(GS_ERR_INVALID_ARGUMENT, "view %d: NULL per-Gaussian array", v);
        if (f.pair_capacity > 0 && !f.sorted_gids)
            return fail(GS_ERR_INVALID_ARGUMENT, "view %d: sorted_gids is NULL", v);
        Workspace w;
        workspace_layout(n, f.pair_capacity, f.ws, &w, tiles_x(&f.cam), tiles_y(&f.cam));
        if (!f.ws || f.ws_bytes < w.bytes)
            return fail(GS_ERR_CAPACITY, "view %d: workspace of %zu bytes, %zu needed", v,
                        f.ws_bytes, w.bytes);
        gs_view_target &t = table.v[v];
        t.splats = f.splats;
        t.sorted_gids = f.sorted_gids;
        t.ranges = f.ranges;
        t.image = f.image;
        t.final_T = f.final_T;
        t.n_contrib = f.n_contrib;
        t.width = f.cam.width;
        t.height = f.cam.height;
        total += (int64_t)tiles_x(&f.cam) * tiles_y(&f.cam);
    }
    const size_t need = gs_render_views_workspace_size(n_views, total);
    if (!ws || ws_bytes < need)
        return fail(GS_ERR_CAPACITY, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    hipStream_t main = (hipStream_t)stream;
    LaneSet *ls = nullptr;
    if (lanes > 1 && (st = lane_set(&ls)) != GS_OK) return st;
    gs_view_target *d_table = static_cast<gs_view_target *>(ws);
    hipError_t e = launch_view_table(table, d_table, main);
    if (e != hipSuccess) return hip_check(e, "gs_render_views table");
    // fork: every lane starts after the work already on `stream`
    if (lanes > 1) {
        if ((e = hipEventRecord(ls->fork, main)) != hipSuccess) return hip_check(e, "gs_render_views fork");
        for (int l = 0; l < lanes; ++l)
            if ((e = hipStreamWaitEvent(ls->s[l], ls->fork, 0)) != hipSuccess)
                return hip_check(e, "gs_render_views fork");
    }
    PreprocessArgs pa;
    fill_preprocess_args(scene, mode, &pa);
    hipError_t err = hipSuccess;
    for (int v = 0; v < n_views && err == hipSuccess; ++v) {
        const gs_view_frame &f = views[v];
        hipStream_t s = lanes > 1 ? ls->s[v % lanes] : main;
        set_preprocess_camera(&f.cam, &pa);
        pa.splats = f.splats;
        pa.rects = f.rects;
        pa.tiles_touched = f.tiles_touched;
        err = launch_preprocess(pa, s);
        if (err != hipSuccess) break;
        Workspace w;
        workspace_layout(n, f.pair_capacity, f.ws, &w, tiles_x(&f.cam), tiles_y(&f.cam));
        err = launch_bin(f.splats, f.rects, f.tiles_touched, (int)n, tiles_x(&f.cam),
                         tiles_y(&f.cam), mode->extent_rule, f.sorted_gids, nullptr, f.ranges,
                         f.pair_capacity, f.num_pairs, w, s);
    }
    // join, whatever happened above, so a capture stays well formed
    if (lanes > 1) {
        for (int l = 0; l < lanes; ++l) {
            hipError_t j = hipEventRecord(ls->join[l], ls->s[l]);
            if (j == hipSuccess) j = hipStreamWaitEvent(main, ls->join[l], 0);
            if (j != hipSuccess && err == hipSuccess) err = j;
        }
    }
    if (err != hipSuccess) return hip_check(err, "gs_render_views");
    return rasterize_views(table.v, d_table, n_views, bg, cfg, clock,
                           static_cast<char *>(ws) + kViewTableBytes, ws_bytes - kViewTableBytes,
                           main, "gs_render_views");
}

}  // extern "C"
