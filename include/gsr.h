/*
 * gsr.h -- C-ABI of the MI355X (gfx950) 3D Gaussian Splatting tile renderer
 * with AdaGScale viewpoint-adaptive scaling.
 *
 * The paper (Jo et al., AdaGScale, arXiv 2604.18980) splits a frame into four
 * stages (Sec. 2.1, Fig. 1): preprocessing, Gaussian-tile pair generation,
 * sorting and rasterization.  AdaGScale changes only the first two: the
 * preprocess computes a per-Gaussian alpha threshold Th (eq. 10), drops
 * Gaussians whose Th exceeds their opacity (Sec. 3.3), and the pair test uses
 * the smaller extent that Th implies; the rasterizer keeps the original
 * covariance and tau = 1/255 ("dual size", Sec. 3.3).
 *
 * General rules for every entry point
 * -----------------------------------
 * - Every pointer argument is DEVICE memory unless marked "host".  Buffers are
 *   owned by the caller; the library never allocates, frees or retains them.
 * - All work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *   default stream).  No entry point synchronises the host.
 * - Arguments are validated on the host before anything is enqueued.  On
 *   failure the call returns a non-zero gs_status, enqueues nothing, and
 *   gs_last_error() returns a message (thread-local).
 * - Pair counts live in device memory so that a frame can be enqueued (and
 *   captured in a HIP graph) without a host round trip; see gs_emit_pairs.
 *
 * Layouts
 * -------
 * scene  : float32.  Geometry as structure of arrays, [C][n] contiguous:
 *          means [3][n], log_scales [3][n], quats [4][n] (w, x, y, z; need not
 *          be normalised), opacity_logits [n].  Colour Gaussian-major:
 *          sh [n][(d+1)^2][3] (SH coefficient k of colour channel c of
 *          Gaussian i at (i*(d+1)^2 + k)*3 + c), 16-byte aligned, so a
 *          Gaussian's coefficients are read only if it survives the cull.
 * splat  : array of structures, float32 [n][12], one 48-byte record per
 *          Gaussian, written by gs_preprocess:
 *            [0] mean x (pixels)   [1] mean y     [2] A         [3] beta
 *            [4] gamma             [5] opacity    [6] depth     [7] Th
 *            [8] red   [9] green   [10] blue      [11] extent scale s
 *          A, beta, gamma hold the inverse 2D covariance of eq. (1) as a sum
 *          of squares: with dx = mean x - px, dy = mean y - py,
 *            d^T Sigma2^-1 d = A (dx + beta dy)^2 + gamma dy^2,
 *          A = c/det, beta = -b/c, gamma = 1/c for Sigma2 = [[a, b], [b, c]]
 *          (no cancellation for thin Gaussians far from their centre); the
 *          alpha exponent is minus half of it.  Fields of Gaussians with
 *          tiles_touched == 0 are unspecified.
 * rect   : uint64 per Gaussian: x0 | y0 << 16 | x1 << 32 | y1 << 48, the
 *          half-open rectangle of 16x16 tiles the Gaussian is paired with.
 * pairs  : two parallel uint32 arrays, tile id (ty * TX + tx) and Gaussian id.
 * ranges : uint32 [num_tiles][2] = [first, one-past-last) into the sorted pairs.
 * image  : float32 [3][H][W]; final_T float32 [H][W]; n_contrib uint32 [H][W].
 * Tiles are 16x16 pixels; TX = ceil(W/16), TY = ceil(H/16).
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

/* Only the entry points declared here are exported from libgsr.so (it is
 * built with hidden visibility by default). */
#define GS_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARGUMENT = 1, /* a pointer, size or option is out of range */
    GS_ERR_CAPACITY = 2,         /* a caller buffer is too small */
    GS_ERR_HIP = 3,              /* a HIP runtime call failed (message has the HIP text) */
    GS_ERR_UNSUPPORTED = 4       /* valid request the library does not implement */
} gs_status;

#define GS_TILE 16
#define GS_LUT_BINS 20
#define GS_MAX_SH_DEGREE 3
#define GS_MAX_IMAGE_SIDE 32768 /* tile coordinates are stored in 16 bits */

/* Scene parameters (device float32, see layouts above). */
typedef struct {
    const float *means;
    const float *log_scales;
    const float *quats;
    const float *opacity_logits;
    const float *sh;
    int64_t n;     /* number of Gaussians, 0 <= n < 2^31 */
    int sh_degree; /* 0..3 */
} gs_scene;

/* Pinhole camera (host struct).  viewmat is the row-major 3x4 [R | t] mapping
 * world to camera coordinates (x right, y down, z forward).  Pixel (px, py)
 * is sampled at its integer coordinates. */
typedef struct {
    float viewmat[12];
    float fx, fy, cx, cy;
    int width, height; /* 1 .. GS_MAX_IMAGE_SIDE */
} gs_camera;

/* Per-call method switch (host struct).
 * adagscale = 0: plain 3D-GS extent (3 standard deviations, tau = 1/255).
 * adagscale = 1: AdaGScale (Sec. 3.2-3.3).  Th = K / (T_up(depth) 2 pi
 *   sqrt(det Sigma2)) + tau (eq. 10) with T_up looked up in t_upper over 20
 *   uniform bins of [0, lut_depth_max] (Sec. 3.4; depths beyond use the last
 *   bin).  A Gaussian with Th >= opacity, or whose bin holds T_up <= 0, gets no
 *   pairs; otherwise its extent is scaled by s = sqrt(ln(opacity/Th) /
 *   ln(opacity/tau)), the factor that maps the alpha = tau contour onto the
 *   alpha = Th contour.  force_unit_scale = 1 keeps s = 1 (testing aid).
 * extent_rule = 0: the pairs are the tile rectangle of that (scaled) extent.
 * extent_rule = 1: the ellipse test of the prior work the paper builds on
 *   (Sec. 2.3 Fig. 3(c), Sec. 4.1), applied at pair generation as Sec. 3.3
 *   applies Th there: gs_preprocess writes the plain (unscaled) rectangle and
 *   its area as the candidates, and gs_emit_pairs / gs_bin_pairs keep only the
 *   candidate tiles whose pixel box [16 tx, 16 tx + 15] x [16 ty, 16 ty + 15]
 *   meets the ellipse alpha >= t, t = Th under AdaGScale and tau otherwise,
 *   evaluated in double from the float32 splat record.
 * extent_rule = 2: the oriented-box test of the prior work (GSCore, Sec. 2.3
 *   Fig. 3(b)): gs_preprocess writes rule 0's rectangle and area as the
 *   candidates, and pair generation keeps the candidate tiles whose pixel box
 *   meets the box of half-lengths 3 s sqrt(lambda_i) along the eigenvectors of
 *   the 2D covariance (recovered from the record), s the AdaGScale scale (1
 *   plain).
 * The same rule must be passed to gs_emit_pairs / gs_bin_pairs. */
typedef struct {
    int adagscale;
    float K;                       /* peripheral-loss budget, >= 0 (eq. 5) */
    float t_upper[GS_LUT_BINS];    /* T_up per depth bin, in [0, 1]; all 1 = uncalibrated */
    float lut_depth_max;           /* > 0; the paper's range is 100 */
    int force_unit_scale;
    int extent_rule;               /* 0 rectangle, 1 ellipse, 2 oriented box; others rejected */
} gs_mode;

/* Raster launch geometry.  Tiles stay 16x16 so pair sets are comparable.
 * Built: (64, 4, 64) one wave per tile, 4 pixels per lane (the default; the
 * grid's last twentieth of the tiles, dispatched last, get two waves each);
 * (128, 2, 64) two waves per tile, 2 pixels per lane, each wave walking the
 * list for its 16x8 half; (256, 1, B) one 256-thread workgroup per tile
 * staging B in {64, 128, 256} records.  A zeroed struct (or NULL) selects the
 * default; any other triple is GS_ERR_UNSUPPORTED. */
typedef struct {
    int threads_per_tile;
    int pixels_per_thread;
    int lds_batch;
} gs_raster_cfg;

/* Gradients of the scene parameters (device float32, same layouts as
 * gs_scene, d_sh 16-byte aligned; every value is overwritten). */
typedef struct {
    float *d_means;
    float *d_log_scales;
    float *d_quats;
    float *d_opacity_logits;
    float *d_sh;
} gs_scene_grads;

/* Bytes of scratch ("workspace") that gs_emit_pairs, gs_sort and gs_bin_pairs
 * need for n Gaussians, pair_capacity pairs and a width x height image.  The
 * same workspace may be reused by consecutive calls on one stream. */
GS_API size_t gs_workspace_size(int64_t n, int64_t pair_capacity, int width, int height);

/* Stage 1 (Sec. 2.1 preprocessing; Sec. 3.3 AdaGScale preprocessing).
 * One thread per Gaussian: near-plane cull (z <= 0.2), EWA projection of the
 * 3D covariance R S S^T R^T to Sigma2 = J W Sigma3 W^T J^T + 0.3 I, conic =
 * Sigma2^-1, pixel mean, depth = camera z, opacity = sigmoid(logit), colour =
 * max(0, SH(view direction) + 0.5), plain extent 3 sqrt(lambda_max) or the
 * AdaGScale-scaled extent (extent_rule 0; rule 1 keeps the plain extent), and
 * the tile rectangle.  Geometry that decides discrete outputs is evaluated in
 * double precision (a float32 prefilter with error bounds only skips that
 * work for Gaussians it proves get no tiles).
 * Out: splats [n][12], rects [n], tiles_touched [n] = the rectangle's area
 * (0 = no pairs; under rule 1 an upper bound of the pairs).  The record and
 * the rectangle of a Gaussian with tiles_touched == 0 are unspecified. */
GS_API gs_status gs_preprocess(const gs_scene *scene, const gs_camera *cam, const gs_mode *mode,
                        float *splats, uint64_t *rects, uint32_t *tiles_touched, void *stream);

/* Stage 2 (Sec. 2.1 Gaussian-tile pair generation; Sec. 3.3: the rectangle
 * already reflects AdaGScale's extent under rule 0, and the ellipse of Th is
 * applied here under rule 1).  Emits one (tile, Gaussian) pair per tile of
 * each rectangle (extent_rule 0), or per rectangle tile that meets the
 * Gaussian's ellipse (extent_rule 1) or oriented box (extent_rule 2), from the
 * splat records; pass the rule gs_preprocess ran with.  Pairs
 * are emitted Gaussian by Gaussian in ascending (float32 depth, Gaussian id)
 * order, tile rows outer, columns inner; a stable sort by tile of this list is
 * therefore the paper's per-tile depth order.  extent_rule outside 0..2 is
 * rejected (GS_ERR_INVALID_ARGUMENT).
 * num_pairs (device int64) receives the number of pairs REQUIRED; at most
 * pair_capacity pairs are written.  When *num_pairs > pair_capacity the
 * caller must grow the buffers and run the frame again (stages 3-4 then see a
 * truncated list and their output is meaningless).
 * ws: workspace of at least gs_workspace_size(n, pair_capacity, W, H) bytes. */
GS_API gs_status gs_emit_pairs(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                        int64_t n, const gs_camera *cam, int extent_rule, uint32_t *pair_tiles,
                        uint32_t *pair_gids, int64_t pair_capacity, int64_t *num_pairs, void *ws,
                        size_t ws_bytes, void *stream);

/* Stage 3 (Sec. 2.1 sorting).  Stable LSD radix sort (8-bit digits, LDS
 * histograms) of the pairs by tile id, so each tile's run keeps the depth
 * order of emission.  Reads min(*num_pairs, pair_capacity) pairs from
 * (pair_tiles, pair_gids), which are left unchanged; writes the sorted tile
 * ids to sorted_tiles and the Gaussian ids to sorted_gids (both distinct from
 * the inputs, pair_capacity entries each), and ranges [num_tiles][2] as
 * (start, end), (0, 0) for a tile with no pairs. */
GS_API gs_status gs_sort(const uint32_t *pair_tiles, const uint32_t *pair_gids, const int64_t *num_pairs,
                  int64_t pair_capacity, const gs_camera *cam, uint32_t *sorted_tiles,
                  uint32_t *sorted_gids, uint32_t *ranges, void *ws, size_t ws_bytes,
                  void *stream);

/* gs_sort without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, allocation-free serving loops,
 * harnesses that forbid hipMalloc).  It allocates nothing: its workspace is a
 * fixed array of GS_SORT_NOALLOC_SCRATCH_BYTES (64 MiB) inside libgsr, which
 * every device the library runs on holds for the life of the process.
 * Arguments, outputs and errors as gs_sort; in addition pair_capacity above
 * GS_SORT_NOALLOC_MAX_PAIRS returns GS_ERR_INVALID_ARGUMENT.  All calls on one
 * device share that device's array: calls that overlap in time on one device
 * (on different streams, or from different threads) race and give undefined
 * results; calls in stream order are safe (each call rewrites every scratch
 * entry it reads).  The first call on a device looks up the array's address
 * there (the device must be current). */
#define GS_SORT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
#define GS_SORT_NOALLOC_MAX_PAIRS 7000000LL
GS_API gs_status gs_sort_noalloc(const uint32_t *pair_tiles, const uint32_t *pair_gids,
                                 const int64_t *num_pairs, int64_t pair_capacity,
                                 const gs_camera *cam, uint32_t *sorted_tiles,
                                 uint32_t *sorted_gids, uint32_t *ranges, void *stream);

/* Stages 2 and 3 fused (Sec. 2.1 pair generation, sorting and tile ranges;
 * Sec. 3.3: the rectangles already carry AdaGScale's extent).  Produces the
 * same per-tile lists as gs_emit_pairs followed by gs_sort with the same
 * extent_rule -- every tile's Gaussians in ascending (float32 depth, Gaussian
 * id) order -- without writing the emission-order pair arrays.  Under rule 0
 * the pairs are generated on the fly from the depth-ordered rectangles and
 * sorted by tile with two 8-bit passes of one 32-bit word per pair (one pass
 * when the image has at most 256 tiles; with more than 65536 tiles or
 * n >= 2^24 it emits and sorts pairs internally); under rules 1 and 2 the
 * pairs are emitted into the workspace and sorted by tile.
 * The ranges come from per-tile counts of the rectangles.
 * Out: sorted_gids [pair_capacity]; sorted_tiles [pair_capacity] or NULL when
 * not wanted; ranges [num_tiles][2] as (start, end), (0, 0) for a tile with no
 * pairs, as gs_sort writes them; num_pairs (device int64)
 * receives the number of pairs REQUIRED.  When *num_pairs > pair_capacity
 * nothing is binned: every range is empty and the caller must grow the
 * buffers and run the frame again.
 * ws: workspace of at least gs_workspace_size(n, pair_capacity, W, H) bytes for
 * this camera's W x H. */
GS_API gs_status gs_bin_pairs(const float *splats, const uint64_t *rects, const uint32_t *tiles_touched,
                       int64_t n, const gs_camera *cam, int extent_rule, uint32_t *sorted_gids,
                       uint32_t *sorted_tiles, uint32_t *ranges, int64_t pair_capacity,
                       int64_t *num_pairs, void *ws, size_t ws_bytes, void *stream);

/* Stage 4 (Sec. 2.1 rasterization, eq. 1-2; dual size, Sec. 3.3).  Per 16x16
 * tile, front to back over its sorted list: alpha = min(0.99, opacity *
 * exp(power)), skipped when power > 0 or alpha < 1/255; a pixel stops before
 * a Gaussian that would bring T below 1e-4; colour += alpha T rgb.  Writes
 * image = colour + T * bg (bg: host float[3]), final_T and n_contrib (1 + list
 * position of the last blended Gaussian, 0 if none).  n_evaluated (nullable,
 * uint32 [H][W]) receives the number of list entries the pixel evaluated: up
 * to and including the one that stopped it, else the whole list. */
GS_API gs_status gs_rasterize(const float *splats, int64_t n, const uint32_t *sorted_gids,
                       const uint32_t *ranges, const gs_camera *cam, const float *bg,
                       const gs_raster_cfg *cfg, float *image, float *final_T,
                       uint32_t *n_contrib, uint32_t *n_evaluated, void *stream);

/* Work of the default (one wave per tile) rasterizer on these lists, for
 * measurement: runs its walk without writing pixels and ADDS to work[0..3]
 * (device uint64[4]; the caller zeroes it, the counts accumulate over calls):
 *   [0] list entries evaluated, summed over pixels -- the n_evaluated total of
 *       gs_rasterize: per pixel, eq. (1)-(2) entries up to and including the
 *       one that stopped it, else the whole list;
 *   [1] strip evaluations executed: (16x4 pixel strip, list entry) pairs the
 *       rasterizer's conservative per-strip bound did not rule out, each one
 *       evaluation of eq. (1)-(2) at the strip's 64 pixels;
 *   [2] pixel evaluations that blended a Gaussian (alpha >= tau on a live
 *       pixel, not the stopping one);
 *   [3] list entries loaded (read and bounded before the tile finished).
 * Same argument rules as gs_rasterize. */
GS_API gs_status gs_raster_work(const float *splats, int64_t n, const uint32_t *sorted_gids,
                         const uint32_t *ranges, const gs_camera *cam, uint64_t *work,
                         void *stream);

/* T_upper calibration (Sec. 3.2, transmittance approximation; Sec. 3.4):
 * runs the default rasterizer's walk over these lists (plain-mode lists of a
 * calibration view) without writing pixels, and for every Gaussian it blends
 * takes the largest transmittance in front of it over the pixels where it is
 * blended, max(T^i).  That value, as float bits, raises
 *   t_upper_bits[bin]   (device uint32[GS_LUT_BINS]; required) with bin =
 *                       min(floor(GS_LUT_BINS * depth / lut_depth_max),
 *                       GS_LUT_BINS - 1) of the record's float32 depth,
 *                       evaluated in double;
 *   max_t_bits[i]       (device uint32[n]; nullable) per Gaussian.
 * Both are raised with atomic max and never cleared: the caller zeroes them
 * once and calls once per calibration view.  A bin left at 0 saw no blended
 * Gaussian (take 1.0, the trivial bound, for it).  lut_depth_max > 0. */
GS_API gs_status gs_calibrate_t_upper(const float *splats, int64_t n, const uint32_t *sorted_gids,
                               const uint32_t *ranges, const gs_camera *cam, float lut_depth_max,
                               uint32_t *t_upper_bits, uint32_t *max_t_bits, void *stream);

/* Stage 4 with low-contribution blends skipped: the analysis of Sec. 2.4
 * (Fig. 4(a)) and its approximations in Sec. 3.2 (Fig. 5).  As
 * gs_rasterize with the default geometry, except that a blend of Gaussian i
 * at a pixel (alpha >= 1/255) is skipped -- no colour, no transmittance
 * update, not counted in n_contrib -- when its contribution is below theta:
 *   kind 0: alpha T, T the pixel's running transmittance (eq. 3);
 *   kind 1: alpha weight[i] (device float[n]; e.g. max(T^i) of this view, as
 *           gs_calibrate_t_upper's max_t_bits give it);
 *   kind 2: alpha t_upper[bin] (host float[GS_LUT_BINS]) of the record's
 *           float32 depth, bin = min(floor(GS_LUT_BINS * depth /
 *           lut_depth_max), GS_LUT_BINS - 1) evaluated in double.
 * theta = 0 renders exactly as gs_rasterize.  counts (nullable, device
 * uint64[2]) is added to: [0] skipped blends, [1] kept blends (the caller
 * zeroes it).  theta must be finite and >= 0, kind 0..2 (else
 * GS_ERR_INVALID_ARGUMENT). */
GS_API gs_status gs_rasterize_skip(const float *splats, int64_t n, const uint32_t *sorted_gids,
                            const uint32_t *ranges, const gs_camera *cam, const float *bg,
                            int kind, float theta, const float *weight, const float *t_upper,
                            float lut_depth_max, float *image, float *final_T, uint32_t *n_contrib,
                            unsigned long long *counts, void *stream);

/* Contribution profile (Sec. 2.4, Fig. 4(b)): the default rasterizer's walk
 * over these lists without writing pixels; every blend (alpha >= 1/255, not a
 * stopping entry) adds its contribution alpha T to sums[bin] and 1 to
 * counts[bin], bin = min(floor(m / bin_width), nbins - 1) of the Mahalanobis
 * distance m = sqrt(d^T Sigma2^-1 d) between the pixel and the Gaussian's
 * mean (float32).  sums (device float[nbins]) and counts (device
 * uint64[nbins]) are added to (the caller zeroes them).  1 <= nbins <= 64,
 * bin_width > 0 (else GS_ERR_INVALID_ARGUMENT). */
GS_API gs_status gs_contribution_profile(const float *splats, int64_t n, const uint32_t *sorted_gids,
                                  const uint32_t *ranges, const gs_camera *cam, int nbins,
                                  float bin_width, float *sums, unsigned long long *counts,
                                  void *stream);

/* Adjoint of stage 4 with the pair set and every blend decision of the
 * forward pass frozen.  Walks each pixel's list back to front from n_contrib,
 * recovering T_i = T_{i+1} / (1 - alpha_i) from final_T instead of storing
 * per-pixel lists.  dL_dimage [3][H][W]; grad_splats [n][12] receives, at the
 * splat record's offsets, d mean x, d mean y, d A, d beta, d gamma,
 * d opacity, d red, d green, d blue (other slots 0).  grad_splats is
 * overwritten. */
GS_API gs_status gs_rasterize_backward(const float *splats, int64_t n, const uint32_t *sorted_gids,
                                const uint32_t *ranges, const gs_camera *cam, const float *bg,
                                const float *final_T, const uint32_t *n_contrib,
                                const float *dL_dimage, float *grad_splats, void *stream);

/* Adjoint of stage 1 for Gaussians with tiles_touched > 0 (others get zero
 * gradients): chains grad_splats through the projection, the covariance, the
 * quaternion normalisation, the scale exponential, the opacity sigmoid and
 * the SH colour (clamped channels pass no gradient).  The tile extent (and
 * with it Th and s) passes no gradient. */
GS_API gs_status gs_preprocess_backward(const gs_scene *scene, const gs_camera *cam,
                                 const uint32_t *tiles_touched, const float *grad_splats,
                                 const gs_scene_grads *out, void *stream);

/* ---------------------------------------------------------------------------
 * Many views in one launch.  The per-view stages (gs_preprocess, gs_emit_pairs,
 * gs_sort) run per view; the rasterization of all views then runs as ONE
 * persistent launch over a queue of (view, tile) work items ordered longest
 * tile list first, so the tail of the frame is short whatever the mix of
 * resolutions.  Every call is graph-capturable (no host synchronisation, no
 * allocation, no memset nodes).
 * ------------------------------------------------------------------------- */
#define GS_MAX_VIEWS 64

/* One view's inputs (outputs of its own gs_preprocess / gs_sort) and outputs;
 * all pointers are device memory, layouts as for gs_rasterize. */
typedef struct {
    const float *splats;
    const uint32_t *sorted_gids;
    const uint32_t *ranges;
    float *image;
    float *final_T;
    uint32_t *n_contrib;
    int width, height;
} gs_view_target;

/* Workspace bytes for gs_rasterize_views over total_tiles (view, tile) items. */
GS_API size_t gs_views_workspace_size(int n_views, int64_t total_tiles);

/* Rasterize n_views views (1..GS_MAX_VIEWS) in one persistent launch.
 * views: HOST array (validated, and used to size the work queue); d_views: the
 * same array in DEVICE memory (read by the kernels; caller-owned, must stay
 * unchanged until the work completes).  bg: host float[3] shared by all views.
 * cfg: raster geometry as for gs_rasterize.  clock (nullable, device uint64
 * [1 + n_views]): [0] receives the device wall clock at the start of the
 * launch, [1 + v] the clock when view v's last tile finished (the clock runs
 * at hipDeviceAttributeWallClockRate kHz).  The work queue takes the views in
 * order, each view's longest tile lists first, so views complete one after
 * another.  Results are identical to calling gs_rasterize once per view. */
GS_API gs_status gs_rasterize_views(const gs_view_target *views, const gs_view_target *d_views,
                             int n_views, const float *bg, const gs_raster_cfg *cfg,
                             uint64_t *clock, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * A whole batched frame in one call: for every view, the preprocess (Sec. 2.1
 * preprocessing; AdaGScale Sec. 3.2-3.3) and the fused pair generation, sort
 * and tile ranges of gs_bin_pairs, then the rasterization (eq. 1-2, dual size
 * Sec. 3.3) of every view's tiles in ONE persistent launch over a longest-first
 * (view, tile) queue, as gs_rasterize_views.  The views' preprocess and
 * binning chains are independent, so they are spread over `lanes` streams
 * the library owns (created on the first call on a device, default priority),
 * forked from and joined back to `stream` with events; the whole call is
 * graph-capturable (no allocation, no host synchronisation, no memset nodes).
 * Make the first call on a device outside graph capture (it creates the
 * streams and events).  Calls that overlap on one device share those streams
 * and must be serialised by the caller.
 * ------------------------------------------------------------------------- */

/* One view of a batched frame (host struct; every pointer is device memory,
 * caller-owned, laid out as for gs_preprocess / gs_bin_pairs /
 * gs_rasterize).  num_pairs (device int64) receives the view's REQUIRED pair
 * count; when it exceeds pair_capacity the view's ranges are empty (its image
 * is the background) and the caller grows that view's buffers and renders
 * again.  ws: gs_workspace_size(scene n, pair_capacity, W, H) bytes. */
typedef struct {
    gs_camera cam;
    float *splats;           /* [n][12] */
    uint64_t *rects;         /* [n] */
    uint32_t *tiles_touched; /* [n] */
    uint32_t *sorted_gids;   /* [pair_capacity] */
    uint32_t *ranges;        /* [tiles][2] */
    int64_t pair_capacity;   /* 0 .. 2^32 - 1 */
    int64_t *num_pairs;
    void *ws;
    size_t ws_bytes;
    float *image;            /* [3][H][W] */
    float *final_T;          /* [H][W] */
    uint32_t *n_contrib;     /* [H][W] */
} gs_view_frame;

/* Workspace bytes of gs_render_views for n_views views of total_tiles
 * (view, tile) items in all (the per-view binning workspaces are separate). */
GS_API size_t gs_render_views_workspace_size(int n_views, int64_t total_tiles);

/* Render n_views (1..GS_MAX_VIEWS) views of one scene with one method switch
 * (mode, as for gs_preprocess; its extent_rule also applies to the binning).
 * views: HOST array of n_views gs_view_frame.  bg: host float[3].  cfg: raster
 * geometry as for gs_rasterize.  lanes: 1..8 streams for the per-view chains
 * (1 runs everything on `stream`).  clock: as for gs_rasterize_views
 * (nullable).  ws: gs_render_views_workspace_size bytes.  Results equal
 * gs_preprocess + gs_bin_pairs + gs_rasterize per view. */
GS_API gs_status gs_render_views(const gs_scene *scene, const gs_mode *mode,
                                 const gs_view_frame *views, int n_views, const float *bg,
                                 const gs_raster_cfg *cfg, int lanes, uint64_t *clock, void *ws,
                                 size_t ws_bytes, void *stream);

/* Frequency of the device wall clock stamped by gs_rasterize_views, in kHz
 * (0 if the query fails). */
GS_API int gs_wall_clock_khz(int device);

GS_API const char *gs_status_string(gs_status s);
GS_API const char *gs_last_error(void);
/* Library version string, e.g. "gsr 0.1 gfx950". */
GS_API const char *gs_version(void);

#ifdef __cplusplus
}
#endif
#endif
