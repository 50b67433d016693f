// Stage 1: per-Gaussian preprocess (paper Sec. 2.1; AdaGScale Sec. 3.2-3.3).
//
// One thread per Gaussian, structure-of-arrays float32 loads (each wave reads
// 64 consecutive floats per parameter plane).  Everything that decides a
// discrete output -- the cull, the tile rectangle, the AdaGScale threshold and
// scale -- is computed in double precision with a fixed operation order, so
// the rectangles are reproducible on any IEEE machine; gfx950 runs FP64 add,
// multiply and FMA at half the FP32 rate (divisions and square roots are
// multi-instruction sequences), affordable once per Gaussian.  SH colour is
// only fetched for Gaussians that get tiles.
//
// The inverse covariance is stored as the sum of squares
//     d^T Sigma2^-1 d = A (dx + beta dy)^2 + gamma dy^2,
//     A = c / det, beta = -b / c, gamma = 1 / c  (Sigma2 = [[a, b], [b, c]]),
// which is exact algebra (block LDL^T of Sigma2^-1) and has no cancellation:
// the expanded A dx^2 + 2B dx dy + C dy^2 of a thin Gaussian evaluated far
// from its centre loses most of its float32 digits.
//
// Most Gaussians of a view get no tiles: under AdaGScale their threshold Th
// reaches their opacity (Sec. 3.3), or they project outside the image.  A
// float32 prefilter with error bounds proves that for most of them, and only
// the rest (kept in an LDS queue, so the double-precision lanes stay busy)
// take the double-precision path, which alone decides every output.  A
// Gaussian the prefilter drops is one the double-precision path would give no
// tiles; its rectangle is not written (unspecified when tiles_touched is 0).
#include <math.h>

#include "gsr_internal.hpp"
#include "prefilter.hpp"

namespace gsr {

namespace {
constexpr double kTau = 1.0 / 255.0;            // alpha threshold
constexpr double kTwoPi = 6.283185307179586;    // 2 pi (eq. 9-10)
constexpr double kNearZ = 0.2;
constexpr double kDilation = 0.3;
constexpr double kLambdaFloor = 0.1;
constexpr double kMaxRadius = 1073741824.0;     // 2^30 px

__device__ __forceinline__ void store_splat(float *dst, float4 a, float4 b, float4 c) {
    float4 *p = reinterpret_cast<float4 *>(dst);
    p[0] = a;
    p[1] = b;
    p[2] = c;
}


// Real spherical harmonics (Condon-Shortley phase, coefficient k = l^2+l+m)
// at the unit direction (x, y, z), as polynomials; c[] holds the
// normalisation constants computed on the host (see sh_constants()).
template <typename R>
__device__ __forceinline__ void sh_eval(int degree, R x, R y, R z, const R *c, R *Y) {
    Y[0] = c[0];
    if (degree < 1) return;
    Y[1] = -c[1] * y;
    Y[2] = c[1] * z;
    Y[3] = -c[1] * x;
    if (degree < 2) return;
    const R xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c[2] * (x * y);
    Y[5] = -c[2] * (y * z);
    Y[6] = c[3] * (R(3) * zz - R(1));
    Y[7] = -c[2] * (x * z);
    Y[8] = c[4] * (xx - yy);
    if (degree < 3) return;
    Y[9] = -c[5] * (y * (R(3) * xx - yy));
    Y[10] = c[6] * (x * y * z);
    Y[11] = -c[7] * (y * (R(5) * zz - R(1)));
    Y[12] = c[8] * (z * (R(5) * zz - R(3)));
    Y[13] = -c[7] * (x * (R(5) * zz - R(1)));
    Y[14] = c[9] * (z * (xx - yy));
    Y[15] = -c[5] * (x * (xx - R(3) * yy));
}
}  // namespace

// The double-precision path for Gaussian g (parameters as loaded): every
// output of the stage.
template <int DEG>
__device__ __forceinline__ void preprocess_exact(const PreprocessArgs &a, const int g, const float fmx,
                                                 const float fmy, const float fmz, const float fl0,
                                                 const float fl1, const float fl2, const float fqw,
                                                 const float fqx, const float fqy, const float fqz,
                                                 const float fop) {
    uint32_t tiles = 0;
    uint64_t rect = 0;

    // view transform: p = R mu + t
    const double mx = fmx, my = fmy, mz = fmz;
    const double px = a.R[0] * mx + a.R[1] * my + a.R[2] * mz + a.t[0];
    const double py = a.R[3] * mx + a.R[4] * my + a.R[5] * mz + a.t[1];
    const double pz = a.R[6] * mx + a.R[7] * my + a.R[8] * mz + a.t[2];

    if (pz > kNearZ) {
        // scales and normalised rotation
        const double sx = exp((double)fl0);
        const double sy = exp((double)fl1);
        const double sz = exp((double)fl2);
        double qw = fqw, qx = fqx, qy = fqy, qz = fqz;
        const double qn = qw * qw + qx * qx + qy * qy + qz * qz;
        if (qn > 0.0) {
            const double ql = sqrt(qn);
            qw = qw / ql; qx = qx / ql; qy = qy / ql; qz = qz / ql;
        } else {
            qw = 1.0; qx = 0.0; qy = 0.0; qz = 0.0;
        }
        const double r00 = 1.0 - 2.0 * (qy * qy + qz * qz), r01 = 2.0 * (qx * qy - qw * qz),
                     r02 = 2.0 * (qx * qz + qw * qy);
        const double r10 = 2.0 * (qx * qy + qw * qz), r11 = 1.0 - 2.0 * (qx * qx + qz * qz),
                     r12 = 2.0 * (qy * qz - qw * qx);
        const double r20 = 2.0 * (qx * qz - qw * qy), r21 = 2.0 * (qy * qz + qw * qx),
                     r22 = 1.0 - 2.0 * (qx * qx + qy * qy);
        // M = R diag(s); Sigma3 = M M^T
        const double m00 = r00 * sx, m01 = r01 * sy, m02 = r02 * sz;
        const double m10 = r10 * sx, m11 = r11 * sy, m12 = r12 * sz;
        const double m20 = r20 * sx, m21 = r21 * sy, m22 = r22 * sz;
        const double s00 = m00 * m00 + m01 * m01 + m02 * m02;
        const double s01 = m00 * m10 + m01 * m11 + m02 * m12;
        const double s02 = m00 * m20 + m01 * m21 + m02 * m22;
        const double s11 = m10 * m10 + m11 * m11 + m12 * m12;
        const double s12 = m10 * m20 + m11 * m21 + m12 * m22;
        const double s22 = m20 * m20 + m21 * m21 + m22 * m22;

        // EWA: Jacobian of the perspective map at the clamped point, T = J W.
        // Divisions as the definitions are written (x / z, f / z, f x / z^2):
        // multiplying by a rounded 1/z instead moves the float32 record of
        // about one Gaussian in 10^5 by an ulp.
        const double pxz = px / pz, pyz = py / pz, zz = pz * pz;
        double txz = pxz, tyz = pyz;
        txz = txz < -a.limx ? -a.limx : (txz > a.limx ? a.limx : txz);
        tyz = tyz < -a.limy ? -a.limy : (tyz > a.limy ? a.limy : tyz);
        const double xc = txz * pz, yc = tyz * pz;
        const double j00 = a.fx / pz, j02 = -(a.fx * xc) / zz;
        const double j11 = a.fy / pz, j12 = -(a.fy * yc) / zz;
        const double t00 = j00 * a.R[0] + j02 * a.R[6];
        const double t01 = j00 * a.R[1] + j02 * a.R[7];
        const double t02 = j00 * a.R[2] + j02 * a.R[8];
        const double t10 = j11 * a.R[3] + j12 * a.R[6];
        const double t11 = j11 * a.R[4] + j12 * a.R[7];
        const double t12 = j11 * a.R[5] + j12 * a.R[8];
        // U = T Sigma3, Sigma2 = U T^T
        const double u00 = t00 * s00 + t01 * s01 + t02 * s02;
        const double u01 = t00 * s01 + t01 * s11 + t02 * s12;
        const double u02 = t00 * s02 + t01 * s12 + t02 * s22;
        const double u10 = t10 * s00 + t11 * s01 + t12 * s02;
        const double u11 = t10 * s01 + t11 * s11 + t12 * s12;
        const double u12 = t10 * s02 + t11 * s12 + t12 * s22;
        const double ca = (u00 * t00 + u01 * t01 + u02 * t02) + kDilation;
        const double cb = u00 * t10 + u01 * t11 + u02 * t12;
        const double cc = (u10 * t10 + u11 * t11 + u12 * t12) + kDilation;

        const double det = ca * cc - cb * cb;
        const double u = a.fx * pxz + a.cx;
        const double v = a.fy * pyz + a.cy;
        const bool finite = isfinite(u) && isfinite(v) && isfinite(ca) && isfinite(cb) && isfinite(cc);
        if (finite && det > 0.0) {
            const double sigma = 1.0 / (1.0 + exp(-(double)fop));
            // plain extent: 3 sqrt(lambda_max), discriminant floored
            const double mid = 0.5 * (ca + cc);
            double disc = mid * mid - det;
            if (disc < kLambdaFloor) disc = kLambdaFloor;
            double ext = 3.0 * sqrt(mid + sqrt(disc));
            double th = kTau, sc = 1.0;
            bool keep = true;
            if (a.adagscale) {
                // eq. (10): Th = K / (T_up(depth) 2 pi sqrt(det)) + tau
                const double f = (pz * kLutBins) / a.lut_depth_max;
                const int bin = f >= (double)(kLutBins - 1) ? kLutBins - 1 : (int)floor(f);
                const double tu = (double)a.lut[bin];
                if (!(tu > 0.0)) {
                    keep = false;
                } else {
                    const double denom = (tu * kTwoPi) * sqrt(det);
                    th = a.K / denom + kTau;
                    if (th >= sigma) {
                        keep = false;  // Sec. 3.3: negligible for this view
                    } else {
                        sc = a.force_unit_scale ? 1.0 : sqrt(log(sigma / th) / log(sigma / kTau));
                        if (a.extent_rule != 1) ext = ext * sc;  // rule 1: Th enters at pair generation
                    }
                }
            }
            double rd = ceil(ext);
            if (rd > kMaxRadius) rd = kMaxRadius;
            const int r = keep ? (int)rd : 0;
            if (r > 0) {
                double fx0 = floor((u - r) / kTile), fx1 = floor(((u + r) + (kTile - 1)) / kTile);
                double fy0 = floor((v - r) / kTile), fy1 = floor(((v + r) + (kTile - 1)) / kTile);
                const double TX = a.tiles_x, TY = a.tiles_y;
                fx0 = fx0 < 0.0 ? 0.0 : (fx0 > TX ? TX : fx0);
                fx1 = fx1 < 0.0 ? 0.0 : (fx1 > TX ? TX : fx1);
                fy0 = fy0 < 0.0 ? 0.0 : (fy0 > TY ? TY : fy0);
                fy1 = fy1 < 0.0 ? 0.0 : (fy1 > TY ? TY : fy1);
                const uint32_t x0 = (uint32_t)fx0, x1 = (uint32_t)fx1, y0 = (uint32_t)fy0,
                               y1 = (uint32_t)fy1;
                tiles = (x1 - x0) * (y1 - y0);
                if (tiles > 0) {
                    rect = (uint64_t)x0 | ((uint64_t)y0 << 16) | ((uint64_t)x1 << 32) |
                           ((uint64_t)y1 << 48);
                    // colour: SH along the unit view direction, +0.5, clamped at 0.  No
                    // discrete output depends on it, so it runs in float32 (the
                    // camera-to-mean difference is formed in double, then rounded).
                    const float ex = (float)(mx - a.campos[0]), ey = (float)(my - a.campos[1]),
                                ez = (float)(mz - a.campos[2]);
                    const float il = __builtin_amdgcn_rsqf(fmaf(ex, ex, fmaf(ey, ey, ez * ez)));
                    constexpr int nsh = (DEG + 1) * (DEG + 1);
                    float f[nsh * 3];
                    const float *shg = a.sh + (size_t)g * (nsh * 3);
                    if constexpr ((nsh * 3) % 4 == 0) {  // 16-byte aligned rows: vector loads
                        const float4 *s4 = reinterpret_cast<const float4 *>(shg);
#pragma unroll
                        for (int k = 0; k < nsh * 3 / 4; ++k) {
                            const float4 v = s4[k];
                            f[4 * k] = v.x; f[4 * k + 1] = v.y; f[4 * k + 2] = v.z; f[4 * k + 3] = v.w;
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < nsh * 3; ++k) f[k] = shg[k];
                    }
                    float Y[16];
                    sh_eval<float>(DEG, ex * il, ey * il, ez * il, a.shcf, Y);
                    float rgb[3];
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        float acc = 0.0f;
#pragma unroll
                        for (int k = 0; k < nsh; ++k) acc = fmaf(f[k * 3 + ch], Y[k], acc);
                        acc += 0.5f;
                        rgb[ch] = acc < 0.0f ? 0.0f : acc;
                    }
                    store_splat(a.splats + (size_t)g * 12,
                                make_float4((float)u, (float)v, (float)(cc / det), (float)(-cb / cc)),
                                make_float4((float)(1.0 / cc), (float)sigma, (float)pz, (float)th),
                                make_float4(rgb[0], rgb[1], rgb[2], (float)sc));
                }
            }
        }
    }
    a.rects[g] = rect;
    a.tiles_touched[g] = tiles;
}

// Threads per prefilter block: each takes kPreChunk / threads Gaussians, all
// their parameters requested at once.  Measured on the 6M city frame: 256
// (two per thread) 83 us, 128 (four) 87, 512 (one) 90.
#ifndef GSR_PRE_THREADS
#define GSR_PRE_THREADS 256
#endif
constexpr int kPreChunk = 512;                       // Gaussians per prefilter block and list
constexpr int kPreThreads = GSR_PRE_THREADS;         // threads per prefilter block
constexpr int kPreRounds = kPreChunk / kPreThreads;  // Gaussians per thread in the float32 pass
constexpr int kPreWaves = kPreThreads / kWave;
constexpr int kPreSub = kPreChunk / kWave;           // 64-Gaussian chunks per list
static_assert(kPreChunk % kPreThreads == 0 && kPreThreads % kWave == 0, "whole rounds of whole waves");

// List L holds the 64-Gaussian chunks c = L + k nlists (k = 0 .. kPreSub - 1,
// those below the chunk count): spread over the whole index range, so each
// list gets about the same share of the view's visible Gaussians however the
// scene orders them, while each wave still loads 64 consecutive floats per
// plane.  Slot i of a list is Gaussian i % 64 of its chunk k = i / 64; only
// the scene's last chunk can be partial, and it is its list's last.
__host__ __device__ __forceinline__ int64_t list_chunk(int64_t L, int k, int64_t nlists) {
    return L + (int64_t)k * nlists;
}

// A queued Gaussian: its id and its eleven parameters, 48 bytes.
struct PreEntry {
    float4 a, b, c;  // (id bits, mean x, y, z), (log-scales, q w), (q x, y, z, opacity logit)
};

// Appends this lane's entry when keep (wave ballot, one LDS atomic per wave).
__device__ __forceinline__ void queue_push(bool keep, const PreEntry &e, PreEntry *queue, uint32_t *qn) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t m = __ballot(keep);
    if (m) {  // wave-uniform: lane 0 reserves the wave's slots
        uint32_t old = 0u;
        if (lane == 0) old = atomicAdd(qn, (uint32_t)__popcll(m));
        const uint32_t wbase = (uint32_t)__builtin_amdgcn_readlane((int)old, 0);
        if (keep) queue[wbase + (uint32_t)__popcll(m & lanemask_lt())] = e;
    }
}

// The 48-byte splat record slot of list L's slot i (where its entries live).
__device__ __forceinline__ float4 *list_slot(const PreprocessArgs &a, int64_t L, uint32_t i, int64_t nlists) {
    const int64_t g = list_chunk(L, (int)(i / kWave), nlists) * kWave + (i % kWave);
    return reinterpret_cast<float4 *>(a.splats + g * 12);
}

// Pass 1: the float32 prefilter over one list per block, each parameter
// loaded once.  The cheap tier runs on every Gaussian; those it leaves
// undecided are queued in LDS with their parameters and the full tier runs on
// the queue (dense lanes), compacting it in place; a Gaussian either tier
// drops gets tiles_touched = 0.  The rest (candidates) are written, id and
// parameters, into the list's slots (the splat records of its own Gaussians,
// 48 bytes each, so they hold all of them), and their count into the rects
// entry of the list's first Gaussian; pass 2 reads a list in full before it
// writes any output.
__global__ __launch_bounds__(kPreThreads) void k_prefilter(const PreprocessArgs a, int64_t nlists) {
    __shared__ PreEntry q[kPreChunk];
    __shared__ uint32_t n1, n2;
    __shared__ float lut[kLutBins];
    if (threadIdx.x == 0) n1 = n2 = 0u;
    if (threadIdx.x < kLutBins) lut[threadIdx.x] = a.lut[threadIdx.x];
    __syncthreads();
    const int n = a.n;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int64_t L = blockIdx.x;
    // round r, wave w: chunk k = r * (waves per block) + w; every round's parameters are
    // requested before any is used
    float f[kPreRounds][11];
    int64_t gr[kPreRounds];
#pragma unroll
    for (int r = 0; r < kPreRounds; ++r) {
        gr[r] = list_chunk(L, r * kPreWaves + wid, nlists) * kWave + lane;
        const int g = gr[r] < n ? (int)gr[r] : 0;
        f[r][0] = a.means[g]; f[r][1] = a.means[plane_at(1, n, g)]; f[r][2] = a.means[plane_at(2, n, g)];
        f[r][3] = a.log_scales[g]; f[r][4] = a.log_scales[plane_at(1, n, g)];
        f[r][5] = a.log_scales[plane_at(2, n, g)];
        f[r][6] = a.quats[g]; f[r][7] = a.quats[plane_at(1, n, g)]; f[r][8] = a.quats[plane_at(2, n, g)];
        f[r][9] = a.quats[plane_at(3, n, g)];
        f[r][10] = a.opacity_logits[g];
    }
#pragma unroll
    for (int r = 0; r < kPreRounds; ++r) {
        const int64_t g64 = gr[r];
        bool undecided = false;
        if (g64 < n) {
            if (surely_no_tiles<1>(a, lut, f[r][0], f[r][1], f[r][2], f[r][3], f[r][4], f[r][5], f[r][6],
                                   f[r][7], f[r][8], f[r][9], f[r][10]))
                a.tiles_touched[g64] = 0u;
            else
                undecided = true;
        }
        const PreEntry e{make_float4(__uint_as_float((uint32_t)g64), f[r][0], f[r][1], f[r][2]),
                         make_float4(f[r][3], f[r][4], f[r][5], f[r][6]),
                         make_float4(f[r][7], f[r][8], f[r][9], f[r][10])};
        queue_push(undecided, e, q, &n1);
    }
    __syncthreads();
    const uint32_t c1 = n1;
    for (uint32_t i0 = 0; i0 < c1; i0 += kPreThreads) {  // block-uniform
        const uint32_t i = i0 + threadIdx.x;
        bool keep = false;
        PreEntry e{};
        if (i < c1) {
            e = q[i];
            const uint32_t g = __float_as_uint(e.a.x);
            if (surely_no_tiles<2>(a, lut, e.a.y, e.a.z, e.a.w, e.b.x, e.b.y, e.b.z, e.b.w, e.c.x, e.c.y,
                                   e.c.z, e.c.w))
                a.tiles_touched[g] = 0u;
            else
                keep = true;
        }
        // compaction in place: this round's kept entries land below i0 + kPreThreads,
        // after every entry of the round has been read
        __syncthreads();
        queue_push(keep, e, q, &n2);
        __syncthreads();
    }
    const uint32_t cnt = n2;
    for (uint32_t i = threadIdx.x; i < cnt; i += kPreThreads) {
        float4 *o = list_slot(a, L, i, nlists);
        o[0] = q[i].a;
        o[1] = q[i].b;
        o[2] = q[i].c;
    }
    if (threadIdx.x == 0) reinterpret_cast<uint32_t *>(a.rects + L * kWave)[0] = cnt;
}

// Pass 2: the double-precision path over `per` consecutive prefilter lists
// per block (at most kListsPerBlock).  A list is copied to LDS in full (every
// load has returned at the barrier) before any output overwrites it.  When
// the lists' candidates fit the LDS queue together (AdaGScale frames: few
// Gaussians of a view get tiles, and the lists share them evenly) they are
// staged at once and run as one dense set; otherwise list by list.
// 8 lists, about 200 candidates on AdaGScale frames: near one per thread, and
// twice the blocks of 16 lists (measured 40.7 against 41.5 us on the 6M city
// frame; the path is latency-bound)
constexpr int kListsPerBlock = 8;

template <int DEG>
__device__ __forceinline__ void run_staged(const PreprocessArgs &a, const PreEntry *q, uint32_t cnt) {
    for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
        const PreEntry e = q[i];
        preprocess_exact<DEG>(a, (int)__float_as_uint(e.a.x), e.a.y, e.a.z, e.a.w, e.b.x, e.b.y, e.b.z,
                              e.b.w, e.c.x, e.c.y, e.c.z, e.c.w);
    }
}

__device__ __forceinline__ void stage_list(const PreprocessArgs &a, int64_t L, uint32_t cnt, int64_t nlists,
                                           PreEntry *dst) {
    for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
        const float4 *in = list_slot(a, L, i, nlists);
        // three loads in flight, then three LDS stores (a PreEntry temporary
        // here went through scratch memory)
        const float4 e0 = in[0], e1 = in[1], e2 = in[2];
        dst[i].a = e0;
        dst[i].b = e1;
        dst[i].c = e2;
    }
}

// Block entry t (< total) of the lists staged together: entry t - off[l] of
// the list l with off[l] <= t < off[l + 1]; null past the total.
__device__ __forceinline__ const float4 *staged_slot(const PreprocessArgs &a, int64_t L0, const uint32_t *s_off,
                                                     uint32_t t, uint32_t total, int64_t nlists) {
    if (t >= total) return nullptr;
    int l = 0;
#pragma unroll
    for (int b = kListsPerBlock / 2; b > 0; b >>= 1)
        if (s_off[l + b] <= t) l += b;
    return list_slot(a, L0 + l, t - s_off[l], nlists);
}

template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess(const PreprocessArgs a, int64_t nlists, int per) {
    __shared__ PreEntry q[kPreChunk];
    __shared__ uint32_t s_cnt[kListsPerBlock], s_off[kListsPerBlock + 1];
    const int64_t L0 = (int64_t)blockIdx.x * per;
    if (threadIdx.x < kListsPerBlock) {
        const int64_t L = L0 + threadIdx.x;
        s_cnt[threadIdx.x] =
            (threadIdx.x < per && L < nlists) ? reinterpret_cast<const uint32_t *>(a.rects + L * kWave)[0] : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int l = 0; l < kListsPerBlock; ++l) {
            s_off[l] = acc;
            acc += s_cnt[l];
        }
        s_off[kListsPerBlock] = acc;
    }
    __syncthreads();
    const uint32_t total = s_off[kListsPerBlock];
    if (total <= (uint32_t)kPreChunk) {  // block-uniform
        // every list's entries in one pass: block entry t is entry t - off[l]
        // of the list l with off[l] <= t < off[l + 1]; both slots' loads are
        // in flight before either is stored
        static_assert(kPreChunk == 2 * 256, "two staging slots per thread");
        // (named registers: an array of the six here went through scratch)
        const uint32_t t0 = threadIdx.x, t1 = 256u + threadIdx.x;
        const float4 *in0 = staged_slot(a, L0, s_off, t0, total, nlists);
        const float4 *in1 = staged_slot(a, L0, s_off, t1, total, nlists);
        float4 e00{}, e01{}, e02{}, e10{}, e11{}, e12{};
        if (in0) { e00 = in0[0]; e01 = in0[1]; e02 = in0[2]; }
        if (in1) { e10 = in1[0]; e11 = in1[1]; e12 = in1[2]; }
        if (in0) { q[t0].a = e00; q[t0].b = e01; q[t0].c = e02; }
        if (in1) { q[t1].a = e10; q[t1].b = e11; q[t1].c = e12; }
        __syncthreads();
        run_staged<DEG>(a, q, total);
    } else {
        for (int l = 0; l < kListsPerBlock; ++l) {
            if (!s_cnt[l]) continue;  // block-uniform
            stage_list(a, L0 + l, s_cnt[l], nlists, q);
            __syncthreads();
            run_staged<DEG>(a, q, s_cnt[l]);
            __syncthreads();
        }
    }
}

// Plain 3D-GS: one thread per Gaussian straight through the double-precision
// path (no prefilter: without AdaGScale's cull most of a view's Gaussians in
// front of the camera get tiles, and queueing them costs more than the
// off-screen ones the prefilter would prove).  Every parameter is requested
// at once, before the near cull.
template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_direct(const PreprocessArgs a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int n = a.n;
    const float mx = a.means[g], my = a.means[plane_at(1, n, g)], mz = a.means[plane_at(2, n, g)];
    float l0 = a.log_scales[g], l1 = a.log_scales[plane_at(1, n, g)], l2 = a.log_scales[plane_at(2, n, g)];
    float qw = a.quats[g], qx = a.quats[plane_at(1, n, g)], qy = a.quats[plane_at(2, n, g)],
          qz = a.quats[plane_at(3, n, g)];
    float op = a.opacity_logits[g];
    // left alone, the compiler sinks these loads below the near cull, which
    // costs a second dependent trip to memory
    pin_vgpr(l0); pin_vgpr(l1); pin_vgpr(l2);
    pin_vgpr(qw); pin_vgpr(qx); pin_vgpr(qy); pin_vgpr(qz); pin_vgpr(op);
    preprocess_exact<DEG>(a, g, mx, my, mz, l0, l1, l2, qw, qx, qy, qz, op);
}

hipError_t launch_preprocess(const PreprocessArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (!a.adagscale) {
        const unsigned blocks = (unsigned)(((int64_t)a.n + 255) / 256);
        switch (a.sh_degree) {
            case 0: k_preprocess_direct<0><<<blocks, 256, 0, s>>>(a); break;
            case 1: k_preprocess_direct<1><<<blocks, 256, 0, s>>>(a); break;
            case 2: k_preprocess_direct<2><<<blocks, 256, 0, s>>>(a); break;
            default: k_preprocess_direct<3><<<blocks, 256, 0, s>>>(a); break;
        }
        return hipGetLastError();
    }
    const int64_t nchunks = ((int64_t)a.n + kWave - 1) / kWave;
    const int64_t nlists = (nchunks + kPreSub - 1) / kPreSub;
    const int per = kListsPerBlock;
    const unsigned blocks = (unsigned)((nlists + per - 1) / per);
    k_prefilter<<<(unsigned)nlists, kPreThreads, 0, s>>>(a, nlists);
    switch (a.sh_degree) {
        case 0: k_preprocess<0><<<blocks, 256, 0, s>>>(a, nlists, per); break;
        case 1: k_preprocess<1><<<blocks, 256, 0, s>>>(a, nlists, per); break;
        case 2: k_preprocess<2><<<blocks, 256, 0, s>>>(a, nlists, per); break;
        default: k_preprocess<3><<<blocks, 256, 0, s>>>(a, nlists, per); break;
    }
    return hipGetLastError();
}

}  // namespace gsr
