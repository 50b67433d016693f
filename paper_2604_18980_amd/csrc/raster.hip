// Stage 4: tile rasterization, front-to-back alpha blending (paper Sec. 2.1,
// eq. 1-2), with the original covariance and tau in both modes (dual size,
// Sec. 3.3).  Two tile programs, each usable by a one-view grid and by the
// persistent multi-view work queue:
//
// tile_block<BATCH>  one 256-thread workgroup per tile, one pixel per thread.
//   The tile's list is walked in batches of BATCH records gathered into LDS
//   (three 16-byte loads per record); a block vote ends the walk once every
//   pixel has reached the 1e-4 transmittance stop.
//
// tile_wave<MODE, NS>  one wave per tile, four pixels per lane (NS = 4), or
//   two waves per tile, each a 16x8 half with two pixels per lane (NS = 2).
//   Lane l owns column l % 16 and rows l / 16 + 4k (k < NS) of its part, so
//   each wave instruction evaluates one 16x4 strip.  The list is walked 64
//   records at a time: every lane gathers one record and decides, for its
//   Gaussian, which strips can reach alpha >= tau (the exponent's minimum over
//   each strip row, taken over the continuous column interval, against
//   2 ln(opacity/tau) plus a margin that covers float32 rounding); one ballot
//   per strip turns that into 64-bit masks.  The lanes park their records
//   (with the exponent's per-Gaussian coefficients, raster_cull.hpp) in the
//   wave's own LDS slots, and the wave walks the set bits in list order,
//   reading each hit record with uniform-address (broadcast) LDS reads, and
//   evaluates only the hit strips.  A skipped strip has alpha < tau at every
//   pixel, so results are unchanged.  A strip whose last live pixel stops
//   leaves the batch's hit masks at once (its remaining hits would only
//   evaluate stopped pixels).  The per-lane state fits 62 VGPRs, so eight
//   waves per SIMD hide the LDS and exponential latencies.  No barriers:
//   waves run and retire independently.  The one-wave geometry's grid
//   renders its last twentieth of the tiles (dispatched last) with two waves
//   per tile, so the grid's final round holds shorter waves and ends closer
//   together (k_raster_hybrid).
#include "gsr_internal.hpp"
#include "raster_cull.hpp"

namespace gsr {

namespace {
constexpr float kTauF = 1.0f / 255.0f;
constexpr float kStopF = 1e-4f;
constexpr float kAlphaMaxF = 0.99f;


__device__ __forceinline__ void store_pixel(const RasterArgs &a, int px, int py, float cr, float cg,
                                            float cb, float T, uint32_t last, uint32_t ev) {
    const size_t npix = (size_t)a.width * a.height, pix = (size_t)py * a.width + px;
    a.image[pix] = cr + T * a.bg[0];
    a.image[npix + pix] = cg + T * a.bg[1];
    a.image[2 * npix + pix] = cb + T * a.bg[2];
    a.final_T[pix] = T;
    a.n_contrib[pix] = last;
    if (a.n_evaluated) a.n_evaluated[pix] = ev;
}
}  // namespace

template <int BATCH>
__device__ __forceinline__ void tile_block(const RasterArgs &a, int tile) {
    __shared__ float4 s_geo[BATCH];  // mean x, mean y, A, beta
    __shared__ float4 s_att[BATCH];  // gamma, opacity, red, green
    __shared__ float s_blue[BATCH];
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int px = tx * kTile + (threadIdx.x & (kTile - 1));
    const int py = ty * kTile + (threadIdx.x / kTile);
    const bool inside = px < a.width && py < a.height;
    const float fpx = (float)px, fpy = (float)py;
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const float4 *spl = reinterpret_cast<const float4 *>(a.splats);

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    uint32_t last = 0, evaluated = end - start;
    bool done = !inside;
    for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
        if (__syncthreads_count(done) == (int)blockDim.x) break;
        const uint32_t j = b0 + threadIdx.x;
        if (threadIdx.x < BATCH && j < end) {
            const size_t g = a.gids[j];
            const float4 g0 = spl[3 * g], g1 = spl[3 * g + 1], g2 = spl[3 * g + 2];
            s_geo[threadIdx.x] = g0;
            s_att[threadIdx.x] = make_float4(g1.x, g1.y, g2.x, g2.y);
            s_blue[threadIdx.x] = g2.z;
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)BATCH, end - b0);
        if (!done) {
            for (int k = 0; k < cnt; ++k) {
                const float4 g = s_geo[k];
                const float4 c = s_att[k];
                const float dx = g.x - fpx, dy = g.y - fpy;
                const float u = fmaf(g.w, dy, dx);
                const float power = -0.5f * fmaf(g.z * u, u, c.x * (dy * dy));
                if (power > 0.0f) continue;
                const float alpha = fminf(kAlphaMaxF, c.y * __expf(power));
                if (alpha < kTauF) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < kStopF) {
                    done = true;
                    evaluated = (b0 - start) + (uint32_t)k + 1u;
                    break;
                }
                const float w = alpha * T;
                cr = fmaf(w, c.z, cr);
                cg = fmaf(w, c.w, cg);
                cb = fmaf(w, s_blue[k], cb);
                T = Tn;
                last = (b0 - start) + (uint32_t)k + 1u;
            }
        }
    }
    if (inside) store_pixel(a, px, py, cr, cg, cb, T, last, evaluated);
}

// Wave-wide sum of a 64-bit per-lane value (every lane receives it).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

// MODE 0: the renderer.  MODE 1: also count, per pixel, the list entries
// evaluated (n_evaluated output).  MODE 2: write no pixels; add this tile's
// work to a.work[0..3]: list entries evaluated (the n_evaluated sum), strip
// evaluations executed (one per wave instruction sequence over a 16x4 strip),
// pixel evaluations that blended a Gaussian, and list entries loaded.
// MODE 3: write no pixels; T_upper calibration -- for each Gaussian the wave
// blends, the largest transmittance in front of it over the tile's pixels,
// raised into its depth bin (per-wave maxima in LDS, flushed at the end of
// the tile) and, if requested, into the Gaussian's own entry.
// MODE 5: write no pixels; the contribution profile (Sec. 2.4, Fig. 4(b)):
// each blend's alpha T added to its Mahalanobis-distance bin (per-wave LDS
// histograms, flushed at the end of the tile).
// MODE 4: the renderer with the contribution-skip rule of the analysis
// experiments (Sec. 2.4, 3.2): a blend whose contribution alpha x (T, the
// Gaussian's weight, or T_up of its depth bin) is below a.skip_theta is
// skipped (no colour, no T update, not a contributor); a.work, if set,
// receives the skipped and kept blend counts.
// The parked records of a block's four waves: one allocation shared by every
// geometry a kernel instantiates.
__shared__ float4 g_srec[4][64][3];

template <int MODE, int NS = 4>
__device__ __forceinline__ void tile_wave(const RasterArgs &a, int tile, int part = 0) {
    constexpr bool EV = MODE == 1 || MODE == 2;
    constexpr bool CNT = MODE == 2 || MODE == 4;  // counts kept blends
    // one 48-byte row per parked record (mean x, mean y, a, a beta | c,
    // log2 opacity, red, green | blue; BlendCoef), so the broadcast reads of a
    // record share one address register
    float4 (&srec)[4][64][3] = g_srec;
    __shared__ uint32_t s_cal[MODE == 3 ? 4 : 1][64];   // MODE 3: depth bin of each slot
    __shared__ uint32_t s_cgid[MODE == 3 ? 4 : 1][64];  // MODE 3: Gaussian id of each slot
    __shared__ uint32_t s_lut[MODE == 3 ? 4 : 1][kLutBins];
    __shared__ float s_w[MODE == 4 ? 4 : 1][64];          // MODE 4: weight of each slot
    __shared__ float s_ps[MODE == 5 ? 4 : 1][kProfBins];  // MODE 5: per-wave profile sums
    __shared__ uint32_t s_pc[MODE == 5 ? 4 : 1][kProfBins];  // and counts
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const int lane = threadIdx.x & (kWave - 1);
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int col = lane & 15, row0 = lane >> 4;
    const int px = tx * kTile + col;
    const float fpx = (float)px;
    const float x_lo = (float)(tx * kTile), x_hi = (float)(tx * kTile + kTile - 1);
    const int y0 = ty * kTile + part * 4 * NS;  // this wave's first row
    // Per pixel k: fpy[k] is the pixel row while the pixel is live and NaN
    // once it has stopped (or lies outside the image); the exponent is then
    // NaN and fails the alpha >= tau compare, so "live and alpha >= tau" is
    // one compare and the per-pixel state needs no boolean merges.
    float fpy[NS], T[NS], cr[NS], cg[NS], cb[NS];
    uint32_t last[NS], ev[NS];
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int py = y0 + row0 + 4 * k;
        fpy[k] = (px < a.width && py < a.height) ? (float)py : __builtin_nanf("");
        pin_vgpr(fpy[k]);  // keep the float; recomputing it costs a convert per evaluation
        T[k] = 1.0f;
        cr[k] = cg[k] = cb[k] = 0.0f;
        last[k] = 0;
        ev[k] = end - start;
    }
    const float4 *spl = reinterpret_cast<const float4 *>(a.splats);
    uint32_t w_strips = 0, w_blended = 0, w_loaded = 0;  // MODE 2 (w_blended also MODE 4)
    uint32_t w_skipped = 0;                              // MODE 4
    if (MODE == 3 && lane < kLutBins) s_lut[wid][lane] = 0u;
    if (MODE == 5) {
        s_ps[wid][lane] = 0.0f;
        s_pc[wid][lane] = 0u;
    }

    for (uint32_t base = start; base < end; base += kWave) {
        uint32_t alive = 0;
#pragma unroll
        for (int k = 0; k < NS; ++k)
            if (__ballot(fpy[k] == fpy[k]) != 0ull) alive |= 1u << k;
        if (!alive) break;
        if (MODE == 2) w_loaded += min(end - base, (uint32_t)kWave);
        const uint32_t j = base + (uint32_t)lane;
        float mx = 0.f, my = 0.f, r = 0.f, g = 0.f, bl = 0.f;
        BlendCoef kc{0.f, 0.f, 0.f, 0.f};
        uint32_t hit = 0;
        if (j < end) {
            const size_t gid = a.gids[j];
            const float4 g0 = spl[3 * gid], g1 = spl[3 * gid + 1], g2 = spl[3 * gid + 2];
            mx = g0.x; my = g0.y; r = g2.x; g = g2.y; bl = g2.z;
            const float A = g0.z, beta = g0.w, gam = g1.x;
            kc = blend_coef(A, beta, gam, g1.y);
            const float elim = kLog2Tau - kc.ls;  // alpha >= tau <=> e - ls >= elim
            hit = strip_hits<NS>(mx, my, A, beta, gam, elim, x_lo, x_hi, (float)y0,
                                 (float)(ty * kTile) + 7.5f);
            if (MODE == 3) {
                // the record's float32 depth, binned in double as the oracle does
                const double f = ((double)g1.z * kLutBins) / a.lut_depth_max;
                s_cal[wid][lane] = f >= (double)(kLutBins - 1) ? (uint32_t)(kLutBins - 1) : (uint32_t)floor(f);
                s_cgid[wid][lane] = (uint32_t)gid;
            }
            if (MODE == 4) {
                float wv = 1.0f;
                if (a.skip_kind == 1) {
                    wv = a.skip_weight[gid];
                } else if (a.skip_kind == 2) {
                    const double f = ((double)g1.z * kLutBins) / a.lut_depth_max;
                    wv = a.skip_lut[f >= (double)(kLutBins - 1) ? kLutBins - 1 : (int)floor(f)];
                }
                s_w[wid][lane] = wv;
            }
        }
        uint64_t m[NS], any = 0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            m[k] = ((alive >> k) & 1u) ? __ballot((hit >> k) & 1u) : 0ull;
            any |= m[k];
        }
        srec[wid][lane][0] = make_float4(mx, my, kc.a, kc.ab);
        srec[wid][lane][1] = make_float4(kc.c, kc.ls, r, g);
        srec[wid][lane][2] = make_float4(bl, 0.0f, 0.0f, 0.0f);
        auto eval = [&](const float4 r0, const float4 r1, const float r2, const int cur) {
            const float smx = r0.x, smy = r0.y, sa = r0.z, sab = r0.w;
            const float sc = r1.x, sls = r1.y, sr = r1.z, sg = r1.w, sb = r2;
            const float adx = sa * (smx - fpx);
            const uint32_t pos = (base - start) + (uint32_t)cur + 1u;
            float tmax = 0.0f;  // MODE 3: largest T in front of it where it blends
            const float swt = MODE == 4 ? s_w[wid][cur] : 0.0f;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                if (!((m[k] >> cur) & 1ull)) continue;  // uniform: strip k missed
                if (MODE == 2) ++w_strips;
                const float dy = smy - fpy[k];
                // log2(opacity) + exponent (base 2); NaN for a stopped pixel,
                // which fails the test below
                const float e2 = blend_exponent(adx, sab, sc, sls, dy);
                // live pixel and alpha = 2^e2 >= tau, decided on the exponent;
                // a strip where no lane blends is skipped (wave-uniform), the
                // other lanes of a blending strip take alpha = 0 (no change)
                const bool bl = e2 >= kLog2Tau;
                if (__ballot(bl) == 0ull) continue;
                float alpha = bl ? fminf(kAlphaMaxF, __builtin_amdgcn_exp2f(e2)) : 0.0f;
                bool skip = false;
                if (MODE == 4) {
                    // contribution below theta: blend nothing (alpha 0 leaves
                    // T, the colour and the stop test untouched)
                    skip = bl && alpha * (a.skip_kind == 0 ? T[k] : swt) < a.skip_theta;
                    alpha = skip ? 0.0f : alpha;
                    w_skipped += skip ? 1u : 0u;
                }
                const float wa = alpha * T[k];
                const float Tn = T[k] - wa;  // T (1 - alpha)
                if (MODE == 3 && bl && !(Tn < kStopF)) tmax = fmaxf(tmax, T[k]);
                float w = wa, Tk = Tn;
                uint32_t lk = (bl && !skip) ? pos : last[k];
                if (__ballot(Tn < kStopF) != 0ull) {
                    // rare: some lane stops here (not blended; the pixel is done)
                    const bool stop = Tn < kStopF;
                    w = stop ? 0.0f : wa;
                    Tk = stop ? T[k] : Tn;
                    lk = stop ? last[k] : lk;
                    if (EV) ev[k] = stop ? pos : ev[k];
                    if (CNT) w_blended -= stop ? 1u : 0u;
                    fpy[k] = stop ? __builtin_nanf("") : fpy[k];
                    if (__ballot(fpy[k] == fpy[k]) == 0ull) {
                        // strip k has no live pixel left: the rest of the
                        // batch skips it (its pixels blend nothing more)
                        m[k] = 0ull;
                        uint64_t rest = 0ull;
#pragma unroll
                        for (int kk = 0; kk < NS; ++kk) rest |= m[kk];
                        any &= rest;
                    }
                }
                cr[k] = fmaf(w, sr, cr[k]);
                cg[k] = fmaf(w, sg, cg[k]);
                cb[k] = fmaf(w, sb, cb[k]);
                T[k] = Tk;
                last[k] = lk;
                if (CNT) w_blended += (bl && !skip) ? 1u : 0u;
                if (MODE == 5 && w != 0.0f) {
                    // blended (not the stopping entry): its alpha T, binned by
                    // the Mahalanobis distance sqrt(q), q = (ls - e2) / (log2(e) / 2)
                    const float mq = __builtin_sqrtf(fmaxf(sls - e2, 0.0f) * (1.0f / kHalfLog2e));
                    const int bin = min((int)(mq * a.prof_inv_width), a.prof_bins - 1);
                    atomicAdd(&s_ps[wid][bin], w);
                    atomicAdd(&s_pc[wid][bin], 1u);
                }
            }
            if (MODE == 3) {
                const float t = wave_max(tmax);
                if (lane == 0 && t > 0.0f) {
                    const uint32_t bits = __float_as_uint(t), bin = s_cal[wid][cur];
                    if (bits > s_lut[wid][bin]) s_lut[wid][bin] = bits;
                    if (a.max_t_bits) atomicMax(a.max_t_bits + s_cgid[wid][cur], bits);
                }
            }
        };
        while (any) {
            const int ja = __ffsll((long long)any) - 1;
            any &= any - 1ull;
            const float4 a0 = srec[wid][ja][0], a1 = srec[wid][ja][1];
            const float a2 = srec[wid][ja][2].x;
            eval(a0, a1, a2, ja);
        }
    }
    if (MODE == 3) {
        if (lane < kLutBins && s_lut[wid][lane] != 0u) atomicMax(a.lut_bits + lane, s_lut[wid][lane]);
        return;
    }
    if (MODE == 5) {
        if (lane < a.prof_bins && s_pc[wid][lane] != 0u) {
            atomicAdd(a.prof_sum + lane, s_ps[wid][lane]);
            atomicAdd(a.prof_cnt + lane, (unsigned long long)s_pc[wid][lane]);
        }
        return;
    }
    if (MODE == 2) {
        unsigned long long e = 0;
#pragma unroll
        for (int k = 0; k < NS; ++k)
            if (px < a.width && y0 + row0 + 4 * k < a.height) e += ev[k];
        e = wave_sum_u64(e);
        const unsigned long long b = wave_sum_u64(w_blended);
        if (lane == 0) {
            atomicAdd(&a.work[0], e);
            atomicAdd(&a.work[1], (unsigned long long)w_strips);
            atomicAdd(&a.work[2], b);
            atomicAdd(&a.work[3], (unsigned long long)w_loaded);
        }
        return;
    }
    if (MODE == 4 && a.work) {
        const unsigned long long sk = wave_sum_u64(w_skipped), b = wave_sum_u64(w_blended);
        if (lane == 0) {
            atomicAdd(&a.work[0], sk);
            atomicAdd(&a.work[1], b);
        }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int py = y0 + row0 + 4 * k;
        if (px < a.width && py < a.height) store_pixel(a, px, py, cr[k], cg[k], cb[k], T[k], last[k], ev[k]);
    }
}


// ------------------------------------------------------------- one view
template <int BATCH>
__global__ __launch_bounds__(256) void k_raster_block(const RasterArgs a) {
    tile_block<BATCH>(a, (int)blockIdx.x);
}

// Tiles go to workgroups in row-major order, so the hardware's round-robin
// dealing of workgroups to the 8 XCDs interleaves neighbouring tiles across
// them.  Giving each XCD a contiguous band of tiles instead (for L2 reuse of
// shared records) measured 1.6x slower on a 6M-Gaussian 4608x3456 frame: the
// pair load is concentrated in parts of the image, and contiguous bands leave
// some XCDs with most of the work.
// NS = 4: one wave per tile; NS = 2: two waves per tile (the geometry with
// 128 threads and 2 pixels per thread), each walking the list for its half.
template <int MODE, int NS = 4>
__global__ __launch_bounds__(256) void k_raster_wave(const RasterArgs a) {
    constexpr int kParts = 4 / NS;
    const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x / kWave);
    const int tile = w / kParts;
    if (tile >= a.tiles_x * a.tiles_y) return;
    tile_wave<MODE, NS>(a, tile, w % kParts);
}

// One wave per tile for tiles [0, t_split), two waves per tile (16x8 halves)
// for the rest.  Blocks dispatch in index order, so the split tiles run last:
// measured on the 6M city frame with the last twentieth split, 295 against
// 300 us over five paired runs (a tenth or a fifth: no better).  Outputs are
// those of either geometry, bit for bit.
template <int MODE>
__global__ __launch_bounds__(256) void k_raster_hybrid(const RasterArgs a, int t_split) {
    const int nt = a.tiles_x * a.tiles_y;
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int b1 = (t_split + 3) / 4;  // blocks of whole-tile waves
    if ((int)blockIdx.x < b1) {        // block-uniform
        const int tile = (int)blockIdx.x * 4 + wid;
        if (tile >= t_split) return;
        tile_wave<MODE, 4>(a, tile, 0);
    } else {
        const int w = ((int)blockIdx.x - b1) * 4 + wid;
        const int tile = t_split + w / 2;
        if (tile >= nt) return;
        tile_wave<MODE, 2>(a, tile, w % 2);
    }
}
constexpr int kHybridSplitDiv = 20;  // the last 1/20 of the tiles get two waves each

hipError_t launch_raster(const RasterArgs &a, const gs_raster_cfg &cfg, hipStream_t s) {
    const unsigned tiles = (unsigned)a.tiles_x * (unsigned)a.tiles_y;
    if (a.lut_bits) {
        k_raster_wave<3><<<(tiles + 3) / 4, 256, 0, s>>>(a);
    } else if (a.prof_sum) {
        k_raster_wave<5><<<(tiles + 3) / 4, 256, 0, s>>>(a);
    } else if (a.skip_kind >= 0) {
        k_raster_wave<4><<<(tiles + 3) / 4, 256, 0, s>>>(a);
    } else if (a.work) {
        k_raster_wave<2><<<(tiles + 3) / 4, 256, 0, s>>>(a);
    } else if (cfg.threads_per_tile == 256) {
        switch (cfg.lds_batch) {
            case 64: k_raster_block<64><<<tiles, 256, 0, s>>>(a); break;
            case 128: k_raster_block<128><<<tiles, 256, 0, s>>>(a); break;
            default: k_raster_block<256><<<tiles, 256, 0, s>>>(a); break;
        }
    } else if (cfg.threads_per_tile == 128) {
        if (a.n_evaluated)
            k_raster_wave<1, 2><<<(tiles + 1) / 2, 256, 0, s>>>(a);
        else
            k_raster_wave<0, 2><<<(tiles + 1) / 2, 256, 0, s>>>(a);
    } else {
        const unsigned t_split = tiles - tiles / kHybridSplitDiv;
        const unsigned grid = (t_split + 3) / 4 + ((tiles - t_split) * 2 + 3) / 4;
        if (a.n_evaluated)
            k_raster_hybrid<1><<<grid, 256, 0, s>>>(a, (int)t_split);
        else
            k_raster_hybrid<0><<<grid, 256, 0, s>>>(a, (int)t_split);
    }
    return hipGetLastError();
}

// ------------------------------------------------------- many views at once
// Work items are (view, tile) packed as view << 26 | tile, ordered view by
// view, each view's longest tile lists first.  Waves (or workgroups) take the
// next item from a global ticket until the queue is empty; the last item of
// each view stamps the device clock so per-view latency can be read back.

__device__ __forceinline__ RasterArgs view_args(const ViewsArgs &q, int view) {
    const gs_view_target v = q.views[view];
    RasterArgs a;
    a.splats = v.splats;
    a.gids = v.sorted_gids;
    a.ranges = v.ranges;
    a.width = v.width;
    a.height = v.height;
    a.tiles_x = (v.width + kTile - 1) / kTile;
    a.tiles_y = (v.height + kTile - 1) / kTile;
    a.bg[0] = q.bg[0];
    a.bg[1] = q.bg[1];
    a.bg[2] = q.bg[2];
    a.image = v.image;
    a.final_T = v.final_T;
    a.n_contrib = v.n_contrib;
    a.n_evaluated = nullptr;
    a.work = nullptr;
    a.lut_bits = a.max_t_bits = nullptr;
    a.skip_kind = -1;
    a.prof_sum = nullptr;
    a.lut_depth_max = 0.0;
    return a;
}

// Plan: one item per (view, tile); key = view << 24 | complemented list length
// (24 bits), so an ascending stable sort takes the views in order and each
// view's longest lists first: views complete one after another (a view's
// latency is its share of the queue, not the whole batch), and the queue's
// tail is the last view's shortest lists.
__global__ __launch_bounds__(256) void k_views_plan(const ViewsPlan p, const gs_view_target *views,
                                                    uint32_t *keys, uint32_t *vals) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= p.tile_off[p.n_views]) return;
    int v = 0;
    while (v + 1 < p.n_views && p.tile_off[v + 1] <= i) ++v;
    const uint32_t t = i - p.tile_off[v];
    const uint32_t *r = views[v].ranges;
    const uint32_t len = r[2 * t + 1] - r[2 * t];
    keys[i] = ((uint32_t)v << 24) | (0xFFFFFFu - (len < 0xFFFFFFu ? len : 0xFFFFFFu));
    vals[i] = ((uint32_t)v << 26) | t;
}

__global__ void k_views_init(const ViewsPlan p, uint32_t *next, uint32_t *view_left, uint64_t *clock) {
    const int v = threadIdx.x;
    if (v == 0) {
        *next = 0u;
        if (clock) clock[0] = wall_clock64();
    }
    if (v < p.n_views) view_left[v] = (p.tile_off[v + 1] - p.tile_off[v]) * (uint32_t)p.parts;
}

hipError_t launch_views_plan(const ViewsPlan &p, const gs_view_target *d_views, uint32_t *keys,
                             uint32_t *vals, uint32_t *next, uint32_t *view_left, uint64_t *clock,
                             hipStream_t s) {
    const uint32_t total = p.tile_off[p.n_views];
    if (total > 0) k_views_plan<<<(total + 255) / 256, 256, 0, s>>>(p, d_views, keys, vals);
    k_views_init<<<1, 64, 0, s>>>(p, next, view_left, clock);
    return hipGetLastError();
}

// The ticket loop holds no lane-divergent branch: every lane takes part in the
// atomics (lane 0 adds 1, the others 0) and lane 0's result is read with an
// explicit readlane.  A "lane 0 fetches, then broadcast" form lets the compiler
// split the loop so that the other lanes re-read a stale ticket without lane 0.
// With NS = 2 a ticket is a half tile: item t / 2, half t % 2 (view_left then
// counts halves).
template <int NS>
__global__ __launch_bounds__(256) void k_raster_views_wave(const ViewsArgs q) {
    constexpr int kParts = 4 / NS;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t one = lane == 0 ? 1u : 0u;
    for (;;) {
        const uint32_t t = atomicAdd(q.next, one);
        const uint32_t ticket = (uint32_t)__builtin_amdgcn_readlane((int)t, 0);
        const uint32_t item = ticket / kParts;
        if ((int64_t)item >= q.n_items) break;
        const uint32_t code = q.items[item];
        const int view = (int)(code >> 26), tile = (int)(code & ((1u << 26) - 1));
        tile_wave<0, NS>(view_args(q, view), tile, (int)(ticket % kParts));
        const uint32_t left = atomicSub(&q.view_left[view], one);
        if (__builtin_amdgcn_readlane((int)left, 0) == 1 && q.clock)
            q.clock[1 + view] = wall_clock64();  // same value from every lane
    }
}

template <int BATCH>
__global__ __launch_bounds__(256) void k_raster_views_block(const ViewsArgs q) {
    __shared__ uint32_t s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(q.next, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if ((int64_t)item >= q.n_items) break;
        const uint32_t code = q.items[item];
        const int view = (int)(code >> 26), tile = (int)(code & ((1u << 26) - 1));
        tile_block<BATCH>(view_args(q, view), tile);
        if (threadIdx.x == 0 && atomicSub(&q.view_left[view], 1u) == 1u && q.clock)
            q.clock[1 + view] = wall_clock64();
    }
}

hipError_t launch_raster_views(const ViewsArgs &q, const gs_raster_cfg &cfg, int grid, hipStream_t s) {
    if (cfg.threads_per_tile == 256) {
        switch (cfg.lds_batch) {
            case 64: k_raster_views_block<64><<<grid, 256, 0, s>>>(q); break;
            case 128: k_raster_views_block<128><<<grid, 256, 0, s>>>(q); break;
            default: k_raster_views_block<256><<<grid, 256, 0, s>>>(q); break;
        }
    } else if (cfg.threads_per_tile == 128) {
        k_raster_views_wave<2><<<grid, 256, 0, s>>>(q);
    } else {
        k_raster_views_wave<4><<<grid, 256, 0, s>>>(q);
    }
    return hipGetLastError();
}

int raster_views_grid(const gs_raster_cfg &cfg) {
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;  // the MI355X's compute units
    const void *fn;
    if (cfg.threads_per_tile == 256) {
        fn = cfg.lds_batch == 64    ? (const void *)k_raster_views_block<64>
             : cfg.lds_batch == 128 ? (const void *)k_raster_views_block<128>
                                    : (const void *)k_raster_views_block<256>;
    } else if (cfg.threads_per_tile == 128) {
        fn = (const void *)k_raster_views_wave<2>;
    } else {
        fn = (const void *)k_raster_views_wave<4>;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) != hipSuccess || per < 1) per = 1;
    return cus * per;
}

}  // namespace gsr
