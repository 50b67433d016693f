// Stage 4: tile rasterization, front-to-back alpha blending (paper Sec. 2.1,
// eq. 1-2), with the original covariance and tau in both modes (dual size,
// Sec. 3.3).
//
// One workgroup per 16x16 tile, one pixel per thread.  The tile's sorted list
// is walked in batches: each thread gathers one 48-byte splat record (three
// 16-byte loads) into LDS, then every pixel scans the batch with wave-uniform
// LDS broadcasts.  A block-wide vote ends the walk once every pixel has hit
// the 1e-4 transmittance stop.
#include "gsr_internal.hpp"

namespace gsr {

namespace {
constexpr float kTauF = 1.0f / 255.0f;
constexpr float kStopF = 1e-4f;
constexpr float kAlphaMaxF = 0.99f;
constexpr int kBatch = 256;
}  // namespace

__global__ __launch_bounds__(256) void k_raster(const RasterArgs a) {
    __shared__ float4 s_geo[kBatch];  // mean x, mean y, A, beta
    __shared__ float4 s_att[kBatch];  // gamma, opacity, red, green
    __shared__ float s_blue[kBatch];
    const int tile = blockIdx.x;
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
    for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
        if (__syncthreads_count(done) == (int)blockDim.x) break;
        const uint32_t j = b0 + threadIdx.x;
        if (j < end) {
            const size_t g = a.gids[j];
            const float4 g0 = spl[3 * g], g1 = spl[3 * g + 1], g2 = spl[3 * g + 2];
            s_geo[threadIdx.x] = g0;
            s_att[threadIdx.x] = make_float4(g1.x, g1.y, g2.x, g2.y);
            s_blue[threadIdx.x] = g2.z;
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)kBatch, end - b0);
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
                cr += w * c.z;
                cg += w * c.w;
                cb += w * s_blue[k];
                T = Tn;
                last = (b0 - start) + (uint32_t)k + 1u;
            }
        }
    }
    if (inside) {
        const size_t npix = (size_t)a.width * a.height, pix = (size_t)py * a.width + px;
        a.image[pix] = cr + T * a.bg[0];
        a.image[npix + pix] = cg + T * a.bg[1];
        a.image[2 * npix + pix] = cb + T * a.bg[2];
        a.final_T[pix] = T;
        a.n_contrib[pix] = last;
        if (a.n_evaluated) a.n_evaluated[pix] = evaluated;
    }
}

hipError_t launch_raster(const RasterArgs &a, const gs_raster_cfg &cfg, hipStream_t s) {
    (void)cfg;
    const unsigned tiles = (unsigned)a.tiles_x * (unsigned)a.tiles_y;
    k_raster<<<tiles, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace gsr
