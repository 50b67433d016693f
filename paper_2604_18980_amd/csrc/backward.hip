// Adjoints of stage 4 (blend, eq. 1-2) and stage 1 (preprocess).
//
// Raster backward: one workgroup per 16x16 tile, one pixel per thread, the
// tile's list walked back to front in LDS batches from the largest n_contrib
// of the tile.  Each pixel recovers the transmittance before Gaussian i as
// T_i = T_{i+1} / (1 - alpha_i) starting from its final T, so no per-pixel
// list is stored.  alpha is recomputed with exactly the forward's float32
// operations, so the skip decisions (alpha < tau) and the clamp are the
// forward's.  Per Gaussian, the 9 gradients of a wave are summed with a
// butterfly reduction and added to global memory by one lane.
//
// Preprocess backward: one thread per Gaussian, double precision, chaining the
// 2D record gradients (mean, A, beta, gamma, opacity, colour) back to the scene
// parameters.  The tile extent -- and with it AdaGScale's Th and s -- is a
// discrete choice of the forward pass and carries no gradient.
#include <math.h>

#include "gsr_internal.hpp"

namespace gsr {

namespace {
constexpr float kTauF = 1.0f / 255.0f;
constexpr float kAlphaMaxF = 0.99f;
constexpr int kBatch = 256;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
}  // namespace

__global__ void k_zero_f32(float *p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0.0f;
}

__global__ __launch_bounds__(256) void k_raster_backward(const RasterBwdArgs a) {
    __shared__ float4 s_geo[kBatch];  // mean x, mean y, A, beta
    __shared__ float4 s_att[kBatch];  // gamma, opacity, red, green
    __shared__ float s_blue[kBatch];
    __shared__ uint32_t s_gid[kBatch];
    __shared__ uint32_t s_max_last;
    const int tile = blockIdx.x;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int px = tx * kTile + (threadIdx.x & (kTile - 1));
    const int py = ty * kTile + (threadIdx.x / kTile);
    const bool inside = px < a.width && py < a.height;
    const float fpx = (float)px, fpy = (float)py;
    const uint32_t start = a.ranges[2 * tile];
    const float4 *spl = reinterpret_cast<const float4 *>(a.splats);
    const size_t npix = (size_t)a.width * a.height, pix = (size_t)py * a.width + px;

    uint32_t last = 0;
    float T = 0.0f, G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;
    if (inside) {
        last = a.n_contrib[pix];
        T = a.final_T[pix];
        G0 = a.dL_dimage[pix];
        G1 = a.dL_dimage[npix + pix];
        G2 = a.dL_dimage[2 * npix + pix];
    }
    // colour of everything behind the current Gaussian: starts with the background
    float b0 = T * a.bg[0], b1 = T * a.bg[1], b2 = T * a.bg[2];
    if (threadIdx.x == 0) s_max_last = 0;
    __syncthreads();
    atomicMax(&s_max_last, last);
    __syncthreads();
    const int max_last = (int)s_max_last;

    for (int hi = max_last; hi > 0; hi -= kBatch) {
        const int lo = hi > kBatch ? hi - kBatch : 0;
        __syncthreads();
        const int j = lo + (int)threadIdx.x;
        if (j < hi) {
            const size_t g = a.gids[start + j];
            const float4 g0 = spl[3 * g], g1 = spl[3 * g + 1], g2 = spl[3 * g + 2];
            s_geo[threadIdx.x] = g0;
            s_att[threadIdx.x] = make_float4(g1.x, g1.y, g2.x, g2.y);
            s_blue[threadIdx.x] = g2.z;
            s_gid[threadIdx.x] = (uint32_t)g;
        }
        __syncthreads();
        for (int k = hi - lo - 1; k >= 0; --k) {
            float d[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) d[q] = 0.0f;
            bool contrib = false;
            if ((uint32_t)(lo + k) < last) {
                const float4 g = s_geo[k];
                const float4 c = s_att[k];
                const float dx = g.x - fpx, dy = g.y - fpy;
                const float u = fmaf(g.w, dy, dx);
                const float power = -0.5f * fmaf(g.z * u, u, c.x * (dy * dy));
                if (!(power > 0.0f)) {
                    const float e = __expf(power);
                    const float raw = c.y * e;
                    const float alpha = fminf(kAlphaMaxF, raw);
                    if (!(alpha < kTauF)) {
                        contrib = true;
                        const float om = 1.0f - alpha;
                        T = T / om;  // transmittance in front of this Gaussian
                        const float w = alpha * T;
                        const float cb = s_blue[k];
                        d[6] = w * G0;
                        d[7] = w * G1;
                        d[8] = w * G2;
                        const float dLda = G0 * (T * c.z - b0 / om) + G1 * (T * c.w - b1 / om) +
                                           G2 * (T * cb - b2 / om);
                        b0 = fmaf(w, c.z, b0);
                        b1 = fmaf(w, c.w, b1);
                        b2 = fmaf(w, cb, b2);
                        if (!(raw > kAlphaMaxF)) {
                            d[5] = dLda * e;  // d opacity
                            const float dLdp = dLda * alpha;
                            const float Au = g.z * u;
                            d[2] = dLdp * (-0.5f * u * u);        // d A
                            d[3] = dLdp * (-Au * dy);             // d beta
                            d[4] = dLdp * (-0.5f * dy * dy);      // d gamma
                            d[0] = dLdp * (-Au);                  // d mean x
                            d[1] = dLdp * (-(Au * g.w + c.x * dy)); // d mean y
                        }
                    }
                }
            }
            if (__ballot(contrib) != 0ull) {
#pragma unroll
                for (int q = 0; q < 9; ++q) d[q] = wave_sum(d[q]);
                if ((threadIdx.x & (kWave - 1)) == 0) {
                    float *dst = a.grad_splats + (size_t)s_gid[k] * 12;
                    atomicAdd(dst + 0, d[0]);
                    atomicAdd(dst + 1, d[1]);
                    atomicAdd(dst + 2, d[2]);
                    atomicAdd(dst + 3, d[3]);
                    atomicAdd(dst + 4, d[4]);
                    atomicAdd(dst + 5, d[5]);
                    atomicAdd(dst + 8, d[6]);
                    atomicAdd(dst + 9, d[7]);
                    atomicAdd(dst + 10, d[8]);
                }
            }
        }
    }
}

hipError_t launch_raster_backward(const RasterBwdArgs &a, int64_t n, hipStream_t s) {
    const int64_t m = 12 * (n > 0 ? n : 0);
    if (m > 0) k_zero_f32<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(a.grad_splats, m);
    const unsigned tiles = (unsigned)a.tiles_x * (unsigned)a.tiles_y;
    k_raster_backward<<<tiles, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ------------------------------------------------------------ preprocess backward
namespace {
// Real SH basis (as in the forward) and its partials in x, y, z (the
// polynomials extended off the sphere; only their tangential part is used).
__device__ void sh_eval_grad(int degree, double x, double y, double z, const double *c, double *Y,
                             double (*dY)[3]) {
    for (int k = 0; k < 16; ++k) { Y[k] = 0.0; dY[k][0] = dY[k][1] = dY[k][2] = 0.0; }
    Y[0] = c[0];
    if (degree < 1) return;
    Y[1] = -c[1] * y; dY[1][1] = -c[1];
    Y[2] = c[1] * z;  dY[2][2] = c[1];
    Y[3] = -c[1] * x; dY[3][0] = -c[1];
    if (degree < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c[2] * x * y;              dY[4][0] = c[2] * y;  dY[4][1] = c[2] * x;
    Y[5] = -c[2] * y * z;             dY[5][1] = -c[2] * z; dY[5][2] = -c[2] * y;
    Y[6] = c[3] * (3.0 * zz - 1.0);   dY[6][2] = 6.0 * c[3] * z;
    Y[7] = -c[2] * x * z;             dY[7][0] = -c[2] * z; dY[7][2] = -c[2] * x;
    Y[8] = c[4] * (xx - yy);          dY[8][0] = 2.0 * c[4] * x; dY[8][1] = -2.0 * c[4] * y;
    if (degree < 3) return;
    Y[9] = -c[5] * y * (3.0 * xx - yy);
    dY[9][0] = -c[5] * 6.0 * x * y;   dY[9][1] = -c[5] * (3.0 * xx - 3.0 * yy);
    Y[10] = c[6] * x * y * z;
    dY[10][0] = c[6] * y * z;         dY[10][1] = c[6] * x * z; dY[10][2] = c[6] * x * y;
    Y[11] = -c[7] * y * (5.0 * zz - 1.0);
    dY[11][1] = -c[7] * (5.0 * zz - 1.0); dY[11][2] = -c[7] * 10.0 * y * z;
    Y[12] = c[8] * z * (5.0 * zz - 3.0);
    dY[12][2] = c[8] * (15.0 * zz - 3.0);
    Y[13] = -c[7] * x * (5.0 * zz - 1.0);
    dY[13][0] = -c[7] * (5.0 * zz - 1.0); dY[13][2] = -c[7] * 10.0 * x * z;
    Y[14] = c[9] * z * (xx - yy);
    dY[14][0] = 2.0 * c[9] * x * z;   dY[14][1] = -2.0 * c[9] * y * z; dY[14][2] = c[9] * (xx - yy);
    Y[15] = -c[5] * x * (xx - 3.0 * yy);
    dY[15][0] = -c[5] * (3.0 * xx - 3.0 * yy); dY[15][1] = c[5] * 6.0 * x * y;
}
}  // namespace

__global__ __launch_bounds__(128) void k_preprocess_backward(const PreprocessBwdArgs a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int n = a.n;
    const int nsh = (a.sh_degree + 1) * (a.sh_degree + 1);
    double dmean[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dop = 0.0;
    double dsh[16][3];
    for (int k = 0; k < nsh; ++k) dsh[k][0] = dsh[k][1] = dsh[k][2] = 0.0;

    if (a.tiles_touched[g] > 0) {
        const float *G = a.grad_splats + (size_t)g * 12;
        const double gmx = G[0], gmy = G[1], gA = G[2], gbeta = G[3], ggam = G[4], gsig = G[5];
        const double grgb[3] = {G[8], G[9], G[10]};
        const double mx = a.means[g], my = a.means[n + g], mz = a.means[2 * n + g];
        const double *R = a.R;
        const double p0 = R[0] * mx + R[1] * my + R[2] * mz + a.t[0];
        const double p1 = R[3] * mx + R[4] * my + R[5] * mz + a.t[1];
        const double p2 = R[6] * mx + R[7] * my + R[8] * mz + a.t[2];
        const double s[3] = {exp((double)a.log_scales[g]), exp((double)a.log_scales[n + g]),
                             exp((double)a.log_scales[2 * n + g])};
        const double q0[4] = {a.quats[g], a.quats[n + g], a.quats[2 * n + g], a.quats[3 * n + g]};
        const double qn = q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3];
        const bool qdeg = !(qn > 0.0);
        const double qr = qdeg ? 1.0 : sqrt(qn);
        const double w = qdeg ? 1.0 : q0[0] / qr, x = qdeg ? 0.0 : q0[1] / qr,
                     y = qdeg ? 0.0 : q0[2] / qr, z = qdeg ? 0.0 : q0[3] / qr;
        const double Rq[3][3] = {
            {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
            {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
            {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
        double M[3][3], S3[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = Rq[i][j] * s[j];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) S3[i][j] = M[i][0] * M[j][0] + M[i][1] * M[j][1] + M[i][2] * M[j][2];
        double txz = p0 / p2, tyz = p1 / p2;
        int clx = 0, cly = 0;
        if (txz < -a.limx) { txz = -a.limx; clx = -1; }
        if (txz > a.limx) { txz = a.limx; clx = 1; }
        if (tyz < -a.limy) { tyz = -a.limy; cly = -1; }
        if (tyz > a.limy) { tyz = a.limy; cly = 1; }
        const double xc = txz * p2, yc = tyz * p2, p22 = p2 * p2;
        const double J00 = a.fx / p2, J02 = -(a.fx * xc) / p22, J11 = a.fy / p2, J12 = -(a.fy * yc) / p22;
        double T[2][3];
        for (int j = 0; j < 3; ++j) {
            T[0][j] = J00 * R[j] + J02 * R[6 + j];
            T[1][j] = J11 * R[3 + j] + J12 * R[6 + j];
        }
        double U[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) U[i][j] = T[i][0] * S3[0][j] + T[i][1] * S3[1][j] + T[i][2] * S3[2][j];
        const double ca = U[0][0] * T[0][0] + U[0][1] * T[0][1] + U[0][2] * T[0][2] + 0.3;
        const double cb = U[0][0] * T[1][0] + U[0][1] * T[1][1] + U[0][2] * T[1][2];
        const double cc = U[1][0] * T[1][0] + U[1][1] * T[1][1] + U[1][2] * T[1][2] + 0.3;
        const double det = ca * cc - cb * cb, d2 = det * det;

        // mean2d
        double dp[3] = {gmx * a.fx / p2, gmy * a.fy / p2, -gmx * a.fx * p0 / p22 - gmy * a.fy * p1 / p22};
        // (A, beta, gamma) = (c/det, -b/c, 1/c)
        const double ga = gA * (-cc * cc / d2);
        const double gb = gA * (2.0 * cb * cc / d2) + gbeta * (-1.0 / cc);
        const double gc = gA * (-cb * cb / d2) + gbeta * (cb / (cc * cc)) + ggam * (-1.0 / (cc * cc));
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
            for (int j = 0; j < 3; ++j) TS[i][j] = T[i][0] * S3[0][j] + T[i][1] * S3[1][j] + T[i][2] * S3[2][j];
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
        dp[2] += GJ00 * (-a.fx / p22) + GJ11 * (-a.fy / p22);
        if (clx == 0) {
            dp[0] += GJ02 * (-a.fx / p22);
            dp[2] += GJ02 * (2.0 * a.fx * p0 / (p22 * p2));
        } else {
            dp[2] += GJ02 * (a.fx * clx * a.limx / p22);
        }
        if (cly == 0) {
            dp[1] += GJ12 * (-a.fy / p22);
            dp[2] += GJ12 * (2.0 * a.fy * p1 / (p22 * p2));
        } else {
            dp[2] += GJ12 * (a.fy * cly * a.limy / p22);
        }
        // Sigma3 = M M^T -> dL/dM = 2 G3 M; M = Rq diag(s)
        double GM[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) GM[i][j] = 2.0 * (G3[i][0] * M[0][j] + G3[i][1] * M[1][j] + G3[i][2] * M[2][j]);
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
            for (int k = 0; k < 4; ++k) dq[k] = (gq[k] - qv[k] * qg) / qr;
        }
        // opacity
        const double sg = 1.0 / (1.0 + exp(-(double)a.opacity_logits[g]));
        dop = gsig * sg * (1.0 - sg);
        // colour
        const double dv[3] = {mx - a.campos[0], my - a.campos[1], mz - a.campos[2]};
        const double len = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        const double dir[3] = {dv[0] / len, dv[1] / len, dv[2] / len};
        double Y[16], dY[16][3];
        sh_eval_grad(a.sh_degree, dir[0], dir[1], dir[2], a.shc, Y, dY);
        double gdir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int k = 0; k < nsh; ++k) acc += (double)a.sh[((size_t)k * 3 + ch) * n + g] * Y[k];
            if (acc + 0.5 < 0.0) continue;  // clamped channel
            for (int k = 0; k < nsh; ++k) {
                dsh[k][ch] = grgb[ch] * Y[k];
                const double cf = grgb[ch] * (double)a.sh[((size_t)k * 3 + ch) * n + g];
                gdir[0] += cf * dY[k][0];
                gdir[1] += cf * dY[k][1];
                gdir[2] += cf * dY[k][2];
            }
        }
        const double gd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
        for (int e = 0; e < 3; ++e)
            dmean[e] = (gdir[e] - dir[e] * gd) / len + R[e] * dp[0] + R[3 + e] * dp[1] + R[6 + e] * dp[2];
    }
    for (int e = 0; e < 3; ++e) {
        a.d_means[(size_t)e * n + g] = (float)dmean[e];
        a.d_log_scales[(size_t)e * n + g] = (float)dls[e];
    }
    for (int e = 0; e < 4; ++e) a.d_quats[(size_t)e * n + g] = (float)dq[e];
    a.d_opacity_logits[g] = (float)dop;
    for (int k = 0; k < nsh; ++k)
        for (int ch = 0; ch < 3; ++ch) a.d_sh[((size_t)k * 3 + ch) * n + g] = (float)dsh[k][ch];
}

hipError_t launch_preprocess_backward(const PreprocessBwdArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    k_preprocess_backward<<<(a.n + 127) / 128, 128, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace gsr
