// Adjoints of stage 4 (blend, eq. 1-2) and stage 1 (preprocess).
//
// Raster backward: one wave per 16x16 tile with the forward's pixel layout
// (lane l owns column l % 16 of rows l / 16 + 4k, k = 0..3: four 16x4 strips).
// The tile's list is walked back to front, 64 records at a time, from the
// largest n_contrib of the tile; every lane gathers one record and decides,
// per strip, whether the Gaussian can reach alpha >= tau there (the forward's
// cull), and the wave visits the hits in reverse list order.  Each pixel
// recovers the transmittance in front of Gaussian i as T_i = T_{i+1} /
// (1 - alpha_i) starting from its final T, so no per-pixel list is stored;
// alpha and the blend decision are recomputed with exactly the forward's
// float32 operations, so a pixel differentiates precisely the Gaussians it
// blended.  Per Gaussian, each lane sums its four pixels' contributions and
// the wave's lanes are summed through LDS, a few Gaussians at a time (below).
//
// Preprocess backward: one thread per Gaussian, double precision, chaining the
// 2D record gradients (mean, A, beta, gamma, opacity, colour) back to the scene
// parameters.  The tile extent -- and with it AdaGScale's Th and s -- is a
// discrete choice of the forward pass and carries no gradient.
#include <math.h>

#include "gsr_internal.hpp"
#include "raster_cull.hpp"

namespace gsr {

namespace {
constexpr float kAlphaMaxF = 0.99f;

// v moved across lanes by the DPP pattern CTRL into the rows in ROW_MASK (0 elsewhere).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

}  // namespace

__global__ void k_zero_f32(float *p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0.0f;
}

__device__ __forceinline__ float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Per-Gaussian gradient sums go through LDS: for each contributing Gaussian
// the lanes add neighbour pairs with one DPP step and park the 32 pair sums
// of each of the 9 values in a row; every kRedG Gaussians, lane L < 9 kRedG
// sums row L and adds it to global memory, so one atomic instruction covers
// them all (in place of 9 wave-wide sums and 9 single-lane atomics each).
constexpr int kRedG = 5;
constexpr int kRedRows = 9 * kRedG;
constexpr int kRedPitch = 36;  // floats per row: 32 pair sums, 16-byte aligned rows

__global__ __launch_bounds__(256) void k_raster_backward(const RasterBwdArgs a) {
    __shared__ __align__(16) float s_red[4][kRedRows][kRedPitch];
    __shared__ uint32_t s_rgid[4][kRedG];
    const int tile = (int)blockIdx.x * 4 + (int)(threadIdx.x / kWave);
    if (tile >= a.tiles_x * a.tiles_y) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    int nred = 0;  // Gaussians parked (wave-uniform)
    // offsets of the 9 gradients in a 12-float splat record
    auto red_off = [](int q) { return q < 6 ? q : q + 2; };
    auto flush = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < 9 * nred) {
            const float4 *row = reinterpret_cast<const float4 *>(&s_red[wid][lane][0]);
            float sum = 0.0f;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float4 v = row[i];
                sum += (v.x + v.y) + (v.z + v.w);
            }
            const int slot = lane / 9, q = lane - 9 * slot;
            atomicAdd(a.grad_splats + (size_t)s_rgid[wid][slot] * 12 + red_off(q), sum);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        nred = 0;
    };
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int col = lane & 15, row0 = lane >> 4;
    const int px = tx * kTile + col;
    const float fpx = (float)px;
    const float x_lo = (float)(tx * kTile), x_hi = (float)(tx * kTile + kTile - 1);
    const size_t npix = (size_t)a.width * a.height;
    float fpy[4], T[4], G0[4], G1[4], G2[4], b0[4], b1[4], b2[4];
    uint32_t last[4];
    uint32_t max_last = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int py = ty * kTile + row0 + 4 * k;
        fpy[k] = (float)py;
        pin_vgpr(fpy[k]);
        last[k] = 0;
        T[k] = G0[k] = G1[k] = G2[k] = 0.0f;
        if (px < a.width && py < a.height) {
            const size_t pix = (size_t)py * a.width + px;
            last[k] = a.n_contrib[pix];
            T[k] = a.final_T[pix];
            G0[k] = a.dL_dimage[pix];
            G1[k] = a.dL_dimage[npix + pix];
            G2[k] = a.dL_dimage[2 * npix + pix];
        }
        // colour of everything behind the current Gaussian: starts with the background
        b0[k] = T[k] * a.bg[0];
        b1[k] = T[k] * a.bg[1];
        b2[k] = T[k] * a.bg[2];
        max_last = max_last > last[k] ? max_last : last[k];
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t other = (uint32_t)__shfl_xor((int)max_last, o, kWave);
        max_last = max_last > other ? max_last : other;
    }
    const uint32_t start = a.ranges[2 * tile];
    const float4 *spl = reinterpret_cast<const float4 *>(a.splats);

    for (int hi = (int)max_last; hi > 0; hi -= kWave) {
        const int lo = hi > kWave ? hi - kWave : 0;
        // a strip takes part while one of its pixels has blended list position >= lo
        uint32_t alive = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (__ballot(last[k] > (uint32_t)lo) != 0ull) alive |= 1u << k;
        const int j = lo + lane;
        float mx = 0.f, my = 0.f, A = 0.f, beta = 0.f, gam = 0.f, sig = 0.f, r = 0.f, g = 0.f, bl = 0.f;
        BlendCoef kc{0.f, 0.f, 0.f, 0.f};
        uint32_t gid = 0, hit = 0;
        if (j < hi) {
            gid = a.gids[start + j];
            const float4 g0 = spl[3 * (size_t)gid], g1 = spl[3 * (size_t)gid + 1], g2 = spl[3 * (size_t)gid + 2];
            mx = g0.x; my = g0.y; A = g0.z; beta = g0.w; gam = g1.x; sig = g1.y; r = g2.x; g = g2.y; bl = g2.z;
            // the forward's exponent coefficients and strip bound, computed identically
            kc = blend_coef(A, beta, gam, sig);
            hit = strip_hits(mx, my, A, beta, gam, kLog2Tau - kc.ls, x_lo, x_hi, (float)(ty * kTile),
                             (float)(ty * kTile) + 7.5f);
        }
        uint64_t m[4], any = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            m[k] = ((alive >> k) & 1u) ? __ballot((hit >> k) & 1u) : 0ull;
            any |= m[k];
        }
        while (any) {  // back to front: highest list position first
            const int jj = 63 - __clzll((long long)any);
            any &= ~(1ull << jj);
            const float smx = bcast(mx, jj), smy = bcast(my, jj), sA = bcast(A, jj);
            const float sbeta = bcast(beta, jj), sgam = bcast(gam, jj), ssig = bcast(sig, jj);
            const float sa = bcast(kc.a, jj), sab = bcast(kc.ab, jj), sc = bcast(kc.c, jj);
            const float sls = bcast(kc.ls, jj), isig = __builtin_amdgcn_rcpf(ssig);
            const float sr = bcast(r, jj), sg = bcast(g, jj), sb = bcast(bl, jj);
            const uint32_t pos = (uint32_t)(lo + jj);
            const float dx = smx - fpx;
            const float adx = sa * dx;
            float d[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) d[q] = 0.0f;
            bool contrib = false;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!((m[k] >> jj) & 1ull)) continue;  // uniform: strip k missed
                const float dy = smy - fpy[k];
                const float u = fmaf(sbeta, dy, dx);
                // the forward's exponent (log2 opacity included), term for term
                const float e2 = blend_exponent(adx, sab, sc, sls, dy);
                if (pos < last[k] && e2 >= kLog2Tau) {  // the forward blended it here
                    contrib = true;
                    const float raw = __builtin_amdgcn_exp2f(e2);  // opacity exp(power)
                    const float e = raw * isig;                    // exp(power)
                    const float alpha = fminf(kAlphaMaxF, raw);
                    const float iom = 1.0f / (1.0f - alpha);  // one division, four products
                    const float Tb = T[k] * iom;  // transmittance in front of this Gaussian
                    const float w = alpha * Tb;
                    d[6] = fmaf(w, G0[k], d[6]);
                    d[7] = fmaf(w, G1[k], d[7]);
                    d[8] = fmaf(w, G2[k], d[8]);
                    const float dLda = G0[k] * (Tb * sr - b0[k] * iom) + G1[k] * (Tb * sg - b1[k] * iom) +
                                       G2[k] * (Tb * sb - b2[k] * iom);
                    b0[k] = fmaf(w, sr, b0[k]);
                    b1[k] = fmaf(w, sg, b1[k]);
                    b2[k] = fmaf(w, sb, b2[k]);
                    T[k] = Tb;
                    if (!(raw > kAlphaMaxF)) {  // a clamped alpha does not depend on the Gaussian
                        d[5] = fmaf(dLda, e, d[5]);  // opacity
                        const float dLdp = dLda * alpha;  // d/d(power), power = -q/2
                        const float Au = sA * u;
                        d[2] = fmaf(dLdp, -0.5f * u * u, d[2]);           // A
                        d[3] = fmaf(dLdp, -Au * dy, d[3]);                // beta
                        d[4] = fmaf(dLdp, -0.5f * dy * dy, d[4]);         // gamma
                        d[0] = fmaf(dLdp, -Au, d[0]);                     // mean x
                        d[1] = fmaf(dLdp, -(Au * sbeta + sgam * dy), d[1]);  // mean y
                    }
                }
            }
            if (__ballot(contrib) != 0ull) {
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const float pr = d[q] + dpp<0xB1, 0xF>(d[q]);  // lanes 2i, 2i+1: their sum
                    if ((lane & 1) == 0) s_red[wid][9 * nred + q][lane >> 1] = pr;
                }
                if (lane == 0) s_rgid[wid][nred] = (uint32_t)__builtin_amdgcn_readlane((int)gid, jj);
                if (++nred == kRedG) flush();
            }
        }
    }
    if (nred > 0) flush();
}

hipError_t launch_raster_backward(const RasterBwdArgs &a, int64_t n, hipStream_t s) {
    const int64_t m = 12 * (n > 0 ? n : 0);
    if (m > 0) k_zero_f32<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(a.grad_splats, m);
    const unsigned tiles = (unsigned)a.tiles_x * (unsigned)a.tiles_y;
    k_raster_backward<<<(tiles + 3) / 4, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ------------------------------------------------------------ preprocess backward
namespace {
// Real SH basis (as in the forward's colour) in float32, DEG a compile-time
// degree so the polynomials stay in registers.
template <int DEG>
__device__ __forceinline__ void sh_basis_f(float x, float y, float z, const float *c, float *Y) {
    Y[0] = c[0];
    if (DEG < 1) return;
    Y[1] = -c[1] * y;
    Y[2] = c[1] * z;
    Y[3] = -c[1] * x;
    if (DEG < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c[2] * (x * y);
    Y[5] = -c[2] * (y * z);
    Y[6] = c[3] * (3.0f * zz - 1.0f);
    Y[7] = -c[2] * (x * z);
    Y[8] = c[4] * (xx - yy);
    if (DEG < 3) return;
    Y[9] = -c[5] * (y * (3.0f * xx - yy));
    Y[10] = c[6] * (x * y * z);
    Y[11] = -c[7] * (y * (5.0f * zz - 1.0f));
    Y[12] = c[8] * (z * (5.0f * zz - 3.0f));
    Y[13] = -c[7] * (x * (5.0f * zz - 1.0f));
    Y[14] = c[9] * (z * (xx - yy));
    Y[15] = -c[5] * (x * (xx - 3.0f * yy));
}

// g = sum_k w[k] grad Y_k at (x, y, z): the partials of the basis polynomials
// above (extended off the sphere; the caller keeps the tangential part).
template <int DEG>
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, const float *c, const float *w,
                                            float *g) {
    g[0] = g[1] = g[2] = 0.0f;
    if (DEG < 1) return;
    g[1] += w[1] * -c[1];
    g[2] += w[2] * c[1];
    g[0] += w[3] * -c[1];
    if (DEG < 2) return;
    g[0] += w[4] * (c[2] * y);         g[1] += w[4] * (c[2] * x);
    g[1] += w[5] * (-c[2] * z);        g[2] += w[5] * (-c[2] * y);
    g[2] += w[6] * (6.0f * c[3] * z);
    g[0] += w[7] * (-c[2] * z);        g[2] += w[7] * (-c[2] * x);
    g[0] += w[8] * (2.0f * c[4] * x);  g[1] += w[8] * (-2.0f * c[4] * y);
    if (DEG < 3) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    g[0] += w[9] * (-c[5] * 6.0f * x * y);
    g[1] += w[9] * (-c[5] * (3.0f * xx - 3.0f * yy));
    g[0] += w[10] * (c[6] * y * z);    g[1] += w[10] * (c[6] * x * z);  g[2] += w[10] * (c[6] * x * y);
    g[1] += w[11] * (-c[7] * (5.0f * zz - 1.0f));
    g[2] += w[11] * (-c[7] * 10.0f * y * z);
    g[2] += w[12] * (c[8] * (15.0f * zz - 3.0f));
    g[0] += w[13] * (-c[7] * (5.0f * zz - 1.0f));
    g[2] += w[13] * (-c[7] * 10.0f * x * z);
    g[0] += w[14] * (2.0f * c[9] * x * z);
    g[1] += w[14] * (-2.0f * c[9] * y * z);
    g[2] += w[14] * (c[9] * (xx - yy));
    g[0] += w[15] * (-c[5] * (3.0f * xx - 3.0f * yy));
    g[1] += w[15] * (c[5] * 6.0f * x * y);
}
}  // namespace

// One thread per Gaussian, 128 per block.  The geometry adjoint runs in FP64
// (one reciprocal per repeated denominator); the colour adjoint in float32.
// d_sh rows (Gaussian-major, 3 (DEG+1)^2 floats each) are assembled in LDS
// and the block's contiguous span of d_sh is written with consecutive
// threads on consecutive words.
template <int DEG>
__global__ __launch_bounds__(128) void k_preprocess_backward(const PreprocessBwdArgs a) {
    constexpr int NSH = (DEG + 1) * (DEG + 1), NC = NSH * 3, ROW = NC + 1;  // odd row pitch
    __shared__ float s_dsh[128 * ROW];
    const int g0 = blockIdx.x * 128;
    const int g = g0 + threadIdx.x;
    const int n = a.n;
    float *row = s_dsh + threadIdx.x * ROW;
#pragma unroll
    for (int k = 0; k < NC; ++k) row[k] = 0.0f;
    if (g < n) {
        double dmean[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dop = 0.0;
        if (a.tiles_touched[g] > 0) {
            const float *G = a.grad_splats + (size_t)g * 12;
            const double gmx = G[0], gmy = G[1], gA = G[2], gbeta = G[3], ggam = G[4], gsig = G[5];
            const float grgb[3] = {G[8], G[9], G[10]};
            const double mx = a.means[g], my = a.means[plane_at(1, n, g)],
                         mz = a.means[plane_at(2, n, g)];
            const double *R = a.R;
            const double p0 = R[0] * mx + R[1] * my + R[2] * mz + a.t[0];
            const double p1 = R[3] * mx + R[4] * my + R[5] * mz + a.t[1];
            const double p2 = R[6] * mx + R[7] * my + R[8] * mz + a.t[2];
            const double s[3] = {exp((double)a.log_scales[g]),
                                 exp((double)a.log_scales[plane_at(1, n, g)]),
                                 exp((double)a.log_scales[plane_at(2, n, g)])};
            const double q0[4] = {a.quats[g], a.quats[plane_at(1, n, g)],
                                  a.quats[plane_at(2, n, g)], a.quats[plane_at(3, n, g)]};
            const double qn = q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3];
            const bool qdeg = !(qn > 0.0);
            const double iqr = qdeg ? 1.0 : 1.0 / sqrt(qn);
            const double w = qdeg ? 1.0 : q0[0] * iqr, x = qdeg ? 0.0 : q0[1] * iqr,
                         y = qdeg ? 0.0 : q0[2] * iqr, z = qdeg ? 0.0 : q0[3] * iqr;
            const double Rq[3][3] = {
                {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
            double M[3][3], S3[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) M[i][j] = Rq[i][j] * s[j];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    S3[i][j] = M[i][0] * M[j][0] + M[i][1] * M[j][1] + M[i][2] * M[j][2];
            const double ip2 = 1.0 / p2, ip22 = ip2 * ip2;
            double txz = p0 * ip2, tyz = p1 * ip2;
            int clx = 0, cly = 0;
            if (txz < -a.limx) { txz = -a.limx; clx = -1; }
            if (txz > a.limx) { txz = a.limx; clx = 1; }
            if (tyz < -a.limy) { tyz = -a.limy; cly = -1; }
            if (tyz > a.limy) { tyz = a.limy; cly = 1; }
            const double xc = txz * p2, yc = tyz * p2;
            const double J00 = a.fx * ip2, J02 = -(a.fx * xc) * ip22, J11 = a.fy * ip2,
                         J12 = -(a.fy * yc) * ip22;
            double T[2][3];
            for (int j = 0; j < 3; ++j) {
                T[0][j] = J00 * R[j] + J02 * R[6 + j];
                T[1][j] = J11 * R[3 + j] + J12 * R[6 + j];
            }
            double U[2][3];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j)
                    U[i][j] = T[i][0] * S3[0][j] + T[i][1] * S3[1][j] + T[i][2] * S3[2][j];
            const double ca = U[0][0] * T[0][0] + U[0][1] * T[0][1] + U[0][2] * T[0][2] + 0.3;
            const double cb = U[0][0] * T[1][0] + U[0][1] * T[1][1] + U[0][2] * T[1][2];
            const double cc = U[1][0] * T[1][0] + U[1][1] * T[1][1] + U[1][2] * T[1][2] + 0.3;
            const double det = ca * cc - cb * cb, id2 = 1.0 / (det * det), icc = 1.0 / cc;
            (void)ca;

            // mean2d
            double dp[3] = {gmx * a.fx * ip2, gmy * a.fy * ip2,
                            -gmx * a.fx * p0 * ip22 - gmy * a.fy * p1 * ip22};
            // (A, beta, gamma) = (c/det, -b/c, 1/c)
            const double ga = gA * (-cc * cc * id2);
            const double gb = gA * (2.0 * cb * cc * id2) + gbeta * (-icc);
            const double gc = gA * (-cb * cb * id2) + gbeta * (cb * icc * icc) + ggam * (-icc * icc);
            const double G2[2][2] = {{ga, 0.5 * gb}, {0.5 * gb, gc}};
            // dL/dSigma3 = T^T G2 T ; dL/dT = 2 G2 T Sigma3
            double G3[3][3], GT[2][3], TS[2][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double acc = 0.0;
                    for (int k = 0; k < 2; ++k)
                        for (int l = 0; l < 2; ++l) acc += T[k][i] * G2[k][l] * T[l][j];
                    G3[i][j] = acc;
                }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j)
                    TS[i][j] = T[i][0] * S3[0][j] + T[i][1] * S3[1][j] + T[i][2] * S3[2][j];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j) GT[i][j] = 2.0 * (G2[i][0] * TS[0][j] + G2[i][1] * TS[1][j]);
            // T = J W -> dL/dJ = dL/dT W^T (only the four non-zero J entries matter)
            double GJ00 = 0, GJ02 = 0, GJ11 = 0, GJ12 = 0;
            for (int k = 0; k < 3; ++k) {
                GJ00 += GT[0][k] * R[k];
                GJ02 += GT[0][k] * R[6 + k];
                GJ11 += GT[1][k] * R[3 + k];
                GJ12 += GT[1][k] * R[6 + k];
            }
            dp[2] += GJ00 * (-a.fx * ip22) + GJ11 * (-a.fy * ip22);
            if (clx == 0) {
                dp[0] += GJ02 * (-a.fx * ip22);
                dp[2] += GJ02 * (2.0 * a.fx * p0 * (ip22 * ip2));
            } else {
                dp[2] += GJ02 * (a.fx * clx * a.limx * ip22);
            }
            if (cly == 0) {
                dp[1] += GJ12 * (-a.fy * ip22);
                dp[2] += GJ12 * (2.0 * a.fy * p1 * (ip22 * ip2));
            } else {
                dp[2] += GJ12 * (a.fy * cly * a.limy * ip22);
            }
            // Sigma3 = M M^T -> dL/dM = 2 G3 M; M = Rq diag(s)
            double GM[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    GM[i][j] = 2.0 * (G3[i][0] * M[0][j] + G3[i][1] * M[1][j] + G3[i][2] * M[2][j]);
            for (int j = 0; j < 3; ++j)
                dls[j] = (GM[0][j] * Rq[0][j] + GM[1][j] * Rq[1][j] + GM[2][j] * Rq[2][j]) * s[j];
            double GR[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) GR[i][j] = GM[i][j] * s[j];
            // dRq/dq for unit q = (w, x, y, z)
            double gq[4];
            gq[0] = GR[0][1] * (-2 * z) + GR[0][2] * (2 * y) + GR[1][0] * (2 * z) + GR[1][2] * (-2 * x) +
                    GR[2][0] * (-2 * y) + GR[2][1] * (2 * x);
            gq[1] = GR[0][1] * (2 * y) + GR[0][2] * (2 * z) + GR[1][0] * (2 * y) + GR[1][1] * (-4 * x) +
                    GR[1][2] * (-2 * w) + GR[2][0] * (2 * z) + GR[2][1] * (2 * w) + GR[2][2] * (-4 * x);
            gq[2] = GR[0][0] * (-4 * y) + GR[0][1] * (2 * x) + GR[0][2] * (2 * w) + GR[1][0] * (2 * x) +
                    GR[1][2] * (2 * z) + GR[2][0] * (-2 * w) + GR[2][1] * (2 * z) + GR[2][2] * (-4 * y);
            gq[3] = GR[0][0] * (-4 * z) + GR[0][1] * (-2 * w) + GR[0][2] * (2 * x) + GR[1][0] * (2 * w) +
                    GR[1][1] * (-4 * z) + GR[1][2] * (2 * y) + GR[2][0] * (2 * x) + GR[2][1] * (2 * y);
            if (!qdeg) {
                const double qv[4] = {w, x, y, z};
                const double qg = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
                for (int k = 0; k < 4; ++k) dq[k] = (gq[k] - qv[k] * qg) * iqr;
            }
            // opacity
            const double sg = 1.0 / (1.0 + exp(-(double)a.opacity_logits[g]));
            dop = gsig * sg * (1.0 - sg);
            // colour (float32): rgb = max(sum_k sh[k] Y_k(dir) + 0.5, 0) per channel
            const double dv[3] = {mx - a.campos[0], my - a.campos[1], mz - a.campos[2]};
            const double len = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]), ilen = 1.0 / len;
            const double dir[3] = {dv[0] * ilen, dv[1] * ilen, dv[2] * ilen};
            const float fx = (float)dir[0], fy = (float)dir[1], fz = (float)dir[2];
            float Y[16];
            sh_basis_f<DEG>(fx, fy, fz, a.shcf, Y);
            const float *shg = a.sh + (size_t)g * NC;
            float f[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) f[k] = shg[k];
            float gch[3];  // d rgb, zero for a clamped channel
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < NSH; ++k) acc = fmaf(f[k * 3 + ch], Y[k], acc);
                gch[ch] = acc + 0.5f < 0.0f ? 0.0f : grgb[ch];
            }
            float wk[16];
#pragma unroll
            for (int k = 0; k < NSH; ++k) {
                wk[k] = gch[0] * f[k * 3] + gch[1] * f[k * 3 + 1] + gch[2] * f[k * 3 + 2];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) row[k * 3 + ch] = gch[ch] * Y[k];
            }
            float gd3[3];
            sh_grad_dot<DEG>(fx, fy, fz, a.shcf, wk, gd3);
            const double gdir[3] = {gd3[0], gd3[1], gd3[2]};
            const double gd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
            for (int e = 0; e < 3; ++e)
                dmean[e] = (gdir[e] - dir[e] * gd) * ilen + R[e] * dp[0] + R[3 + e] * dp[1] +
                           R[6 + e] * dp[2];
        }
        for (int e = 0; e < 3; ++e) {
            a.d_means[plane_at(e, n, g)] = (float)dmean[e];
            a.d_log_scales[plane_at(e, n, g)] = (float)dls[e];
        }
        for (int e = 0; e < 4; ++e) a.d_quats[plane_at(e, n, g)] = (float)dq[e];
        a.d_opacity_logits[g] = (float)dop;
    }
    __syncthreads();
    const int cnt = min(128, n - g0);
    float *dst = a.d_sh + (size_t)g0 * NC;
    for (int i = threadIdx.x; i < cnt * NC; i += 128) dst[i] = s_dsh[(i / NC) * ROW + i % NC];
}

hipError_t launch_preprocess_backward(const PreprocessBwdArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.n + 127) / 128);
    switch (a.sh_degree) {
        case 0: k_preprocess_backward<0><<<blocks, 128, 0, s>>>(a); break;
        case 1: k_preprocess_backward<1><<<blocks, 128, 0, s>>>(a); break;
        case 2: k_preprocess_backward<2><<<blocks, 128, 0, s>>>(a); break;
        default: k_preprocess_backward<3><<<blocks, 128, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace gsr
