// The preprocess' float32 prefilter (preprocess.hip), in a header of its own
// so that host code can run the same test (it is __host__ __device__).
#pragma once
#include <math.h>

#include "gsr_internal.hpp"

namespace gsr {

// Hardware approximations on the device (reciprocal and square root within
// about one ulp, exponential through exp2 of the scaled argument); the
// libm functions on the host, which are at least as accurate.
__host__ __device__ __forceinline__ float gs_rcpf(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ float gs_sqrtf(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}
__host__ __device__ __forceinline__ float gs_expf(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __expf(x);
#else
    return expf(x);
#endif
}

// Float32 proof that the preprocess' double-precision path gives a Gaussian
// no tiles: true only when that is certain -- its depth is clearly behind the
// near plane, or its determinant clearly not positive, or (AdaGScale) its Th
// of eq. (10) clearly reaches its opacity, or a bound of its 3-sigma
// rectangle lies clearly outside the image.  Every bound below majorises the
// difference between the float32 value and the double path's value (U =
// 2^-24; hardware reciprocals, square roots and exponentials are charged a few
// U, the exponential also its argument's rounding; the double path's own
// rounding is far smaller than the slack); a NaN or infinity anywhere makes
// every test false.  Two tiers share the first part:
//   cheap: no rotation.  With M = J W Sigma3 W^T J^T (Sigma2 = M + 0.3 I),
//     tr M <= ||J||_F^2 lambda_1 and det M <= det(J J^T) lambda_1 lambda_2
//     (the compression of Sigma3 to a plane has eigenvalues at most its two
//     largest, lambda_i = s_i^2 sorted, by interlacing), and det Sigma2 =
//     det M + 0.3 tr M + 0.09 <= (tr Sigma2 / 2)^2.
//   full: Sigma3 from the rotation, Sigma2 and its determinant with bounds.
// lut: the T_up table (kLutBins floats).  Returns 0 when undecided, else the
// tier that proved it (1 cheap, 2 full); TIERS = 1 runs the cheap tier alone.
template <int TIERS = 2>
__host__ __device__ __forceinline__ int surely_no_tiles(const PreprocessArgs &a, const float *lut,
                                                        float mx, float my, float mz, float l0,
                                                        float l1, float l2, float qw, float qx,
                                                        float qy, float qz, float op) {
    constexpr float U = 5.9604645e-8f;
    const float *W = a.Rf, *t = a.tf;
    // camera-space position; e: absolute error bounds (the camera's float32
    // rounding, three products, three sums)
    float p[3], e[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float x0 = W[3 * i] * mx, x1 = W[3 * i + 1] * my, x2 = W[3 * i + 2] * mz;
        p[i] = ((x0 + x1) + x2) + t[i];
        e[i] = 16.0f * U * (((fabsf(x0) + fabsf(x1)) + fabsf(x2)) + fabsf(t[i]));
    }
    const float pz = p[2], ez = e[2];
    if (pz + ez < 0.19999f) return 1;  // near cull: the double path needs pz > 0.2
    if (!(pz - ez > 0.2f)) return 0;   // too close to the near plane to tell
    const float pzl = pz - ez;
    if (!(fabsf(l0) < 40.0f && fabsf(l1) < 40.0f && fabsf(l2) < 40.0f)) return 0;
    // projected mean (double path: u = fx px / pz + cx) and its error
    const float rz = gs_rcpf(pz), rzl = gs_rcpf(pzl) * (1.0f + 4.0f * U);
    const float txz = p[0] * rz, tyz = p[1] * rz;
    const float etx = (e[0] + fabsf(txz) * ez) * rzl + 8.0f * U * fabsf(txz);
    const float ety = (e[1] + fabsf(tyz) * ez) * rzl + 8.0f * U * fabsf(tyz);
    const float u = a.fxf * txz + a.cxf, v = a.fyf * tyz + a.cyf;
    const float eu = a.fxf * etx + 8.0f * U * (fabsf(a.fxf * txz) + fabsf(a.cxf));
    const float ev = a.fyf * ety + 8.0f * U * (fabsf(a.fyf * tyz) + fabsf(a.cyf));
    // Jacobian rows at the clamped point: (j00, 0, j02), (0, j11, j12), with
    // j02 = -j00 clamp(x / z) (the double path's -fx xc / z^2); d0, d1 bound
    // each row's error relative to j00, j11 (pz's and the ratios' errors)
    const float lx = a.limxf, ly = a.limyf;
    const float cxz = fminf(fmaxf(txz, -lx), lx), cyz = fminf(fmaxf(tyz, -ly), ly);
    const float j00 = a.fxf * rz, j11 = a.fyf * rz;
    const float dz = ez * rzl + 8.0f * U;
    const float d0 = dz * (1.0f + lx) + etx + 8.0f * U * (1.0f + lx);
    const float d1 = dz * (1.0f + ly) + ety + 8.0f * U * (1.0f + ly);
    // opacity from above, and the largest T_up over the depth bins pz may fall in
    float sig_hi = 0.0f, tu = 1.0f;
    bool ada = a.adagscale != 0;
    if (ada) {
        const float eo = gs_expf(-op);
        // exp(-op) to (2 |op| + 4) U (exp2 of the rounded scaled argument),
        // the reciprocal and the sum a few U more
        sig_hi = gs_rcpf(1.0f + eo) * (1.0f + (2.5f * fminf(fabsf(op), 200.0f) + 24.0f) * U);
        const float f_lo = (pzl * a.lut_scalef) * (1.0f - 8.0f * U);
        const float f_hi = ((pz + ez) * a.lut_scalef) * (1.0f + 8.0f * U);
        const int b_lo = f_lo >= (float)(kLutBins - 1) ? kLutBins - 1 : (int)floorf(fmaxf(f_lo, 0.0f));
        const int b_hi = f_hi >= (float)(kLutBins - 1) ? kLutBins - 1 : (int)floorf(fmaxf(f_hi, 0.0f));
        if (b_hi - b_lo <= 2) {
            tu = 0.0f;
            for (int b = b_lo; b <= b_hi; ++b) tu = fmaxf(tu, lut[b]);
            if (!(tu > 0.0f)) return 1;  // every possible bin drops it
        } else {
            ada = false;  // pz too uncertain to pick the bin: no AdaGScale test
        }
    }
    const float X = 16.0f * (float)a.tiles_x, Y = 16.0f * (float)a.tiles_y;
    {   // cheap tier
        const float lmax = fmaxf(fmaxf(l0, l1), l2);
        const float lmid = fmaxf(fminf(l0, l1), fminf(fmaxf(l0, l1), l2));  // the median, exactly
        // |2 lmax| < 80 (exact doubling): exp to 2 * 80 + 4 U; |2 (lmax +
        // lmid)| < 160 plus the sum's rounding (80 U in the argument)
        const float lam1 = gs_expf(2.0f * lmax) * (1.0f + 200.0f * U);
        const float lam12 = gs_expf(2.0f * (lmax + lmid)) * (1.0f + 600.0f * U);
        const float FJ = 1.0f + 4.0f * (d0 + d1) * (1.0f + lx + ly) + 64.0f * U;
        const float c2 = cxz * cxz, d2 = cyz * cyz;
        const float jr = (j00 * j00) * (1.0f + c2) + (j11 * j11) * (1.0f + d2);  // ||J||_F^2
        const float jd = (j00 * j11) * (j00 * j11) * ((1.0f + c2) + d2);       // det(J J^T)
        const float trM = jr * lam1 * FJ;
        const float detM = jd * lam12 * (FJ * FJ);
        const float tr_hi = trM + 0.6f * (1.0f + 4.0f * U);
        if (ada) {
            const float det_hi = fminf((0.5f * tr_hi) * (0.5f * tr_hi), (detM + 0.3f * trM) + 0.09f) *
                                 (1.0f + 16.0f * U);
            const float den = (tu * 6.2831855f) * gs_sqrtf(det_hi) * (1.0f + 16.0f * U);
            const float th_lo = (a.Kf * gs_rcpf(den)) * (1.0f - 8.0f * U) + 0.0039215642f;
            if (th_lo >= sig_hi) return 1;
        }
        const float r_hi = 3.0f * gs_sqrtf(tr_hi + 0.02f) * (1.0f + 8.0f * U) + 1.0f;
        const float sx = 8.0f * U * (fabsf(u) + eu + r_hi + X) + 1e-3f;
        const float sy = 8.0f * U * (fabsf(v) + ev + r_hi + Y) + 1e-3f;
        if (u + eu + r_hi + sx < 1.0f || u - eu - r_hi - sx >= X) return 1;
        if (v + ev + r_hi + sy < 1.0f || v - ev - r_hi - sy >= Y) return 1;
    }
    if (TIERS == 1) return 0;
    // full tier
    const float qn = qw * qw + qx * qx + qy * qy + qz * qz;
    if (!(qn > 1e-30f && qn < 1e30f)) return 0;  // the double path normalises any qn > 0
    // Sigma3 = M M^T, M = R(q) diag(s); every entry is at most S2 = tr Sigma3
    // in magnitude and within 40 U S2 of the double path's
    const float s0 = expf(l0), s1 = expf(l1), s2 = expf(l2);
    const float S2 = (s0 * s0 + s1 * s1) + s2 * s2;
    const float il = 1.0f / sqrtf(qn);
    const float w = qw * il, x = qx * il, y = qy * il, z = qz * il;
    const float r00 = 1.0f - 2.0f * (y * y + z * z), r01 = 2.0f * (x * y - w * z),
                r02 = 2.0f * (x * z + w * y);
    const float r10 = 2.0f * (x * y + w * z), r11 = 1.0f - 2.0f * (x * x + z * z),
                r12 = 2.0f * (y * z - w * x);
    const float r20 = 2.0f * (x * z - w * y), r21 = 2.0f * (y * z + w * x),
                r22 = 1.0f - 2.0f * (x * x + y * y);
    const float m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
    const float m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
    const float m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
    const float c00 = m00 * m00 + m01 * m01 + m02 * m02, c01 = m00 * m10 + m01 * m11 + m02 * m12,
                c02 = m00 * m20 + m01 * m21 + m02 * m22, c11 = m10 * m10 + m11 * m11 + m12 * m12,
                c12 = m10 * m20 + m11 * m21 + m12 * m22, c22 = m20 * m20 + m21 * m21 + m22 * m22;
    const float j02 = -j00 * cxz, j12 = -j11 * cyz;
    // T = J W: rows t0 = j00 W0 + j02 W2, t1 = j11 W1 + j12 W2; G_i bounds
    // sum_k |t_ik| and the errors sum_k |dt_ik| <= E_i = (d_i + 6U) G_i
    const float t00 = j00 * W[0] + j02 * W[6], t01 = j00 * W[1] + j02 * W[7], t02 = j00 * W[2] + j02 * W[8];
    const float t10 = j11 * W[3] + j12 * W[6], t11 = j11 * W[4] + j12 * W[7], t12 = j11 * W[5] + j12 * W[8];
    const float mlx = fmaxf(lx, 1.0f), mly = fmaxf(ly, 1.0f);
    const float G0 = j00 * ((fabsf(W[0]) + fabsf(W[1]) + fabsf(W[2])) + mlx * (fabsf(W[6]) + fabsf(W[7]) + fabsf(W[8])));
    const float G1 = j11 * ((fabsf(W[3]) + fabsf(W[4]) + fabsf(W[5])) + mly * (fabsf(W[6]) + fabsf(W[7]) + fabsf(W[8])));
    const float E0 = (d0 + 6.0f * U) * G0, E1 = (d1 + 6.0f * U) * G1;
    // Sigma2 = T Sigma3 T^T + 0.3 I and its error bounds
    const float v00 = t00 * c00 + t01 * c01 + t02 * c02, v01 = t00 * c01 + t01 * c11 + t02 * c12,
                v02 = t00 * c02 + t01 * c12 + t02 * c22;
    const float v10 = t10 * c00 + t11 * c01 + t12 * c02, v11 = t10 * c01 + t11 * c11 + t12 * c12,
                v12 = t10 * c02 + t11 * c12 + t12 * c22;
    const float ca = (v00 * t00 + v01 * t01 + v02 * t02) + 0.3f;
    const float cb = v00 * t10 + v01 * t11 + v02 * t12;
    const float cc = (v10 * t10 + v11 * t11 + v12 * t12) + 0.3f;
    const float ea = S2 * (2.0f * E0 * G0 + E0 * E0 + 64.0f * U * G0 * G0) + 2.0f * U;
    const float ec = S2 * (2.0f * E1 * G1 + E1 * E1 + 64.0f * U * G1 * G1) + 2.0f * U;
    const float eb = S2 * (E0 * G1 + G0 * E1 + E0 * E1 + 64.0f * U * G0 * G1);
    // det = a c - b^2 <= (a + ea)(c + ec) - max(|b| - eb, 0)^2, plus this
    // float32 expression's own rounding
    const float ah = ca + ea, ch = cc + ec, bl = fmaxf(fabsf(cb) - eb, 0.0f);
    const float det_hi = (ah * ch - bl * bl) + 4.0f * U * (ah * ch + bl * bl);
    if (det_hi <= 0.0f) return 2;  // the double path needs det > 0
    if (ada) {  // Th >= K / (T_up,max 2 pi sqrt(det_hi)) + tau
        const float den = (tu * 6.2831855f) * sqrtf(det_hi) * (1.0f + 8.0f * U);
        const float th_lo = (a.Kf / den) * (1.0f - 8.0f * U) + 0.0039215642f;
        if (th_lo >= sig_hi) return 2;  // Th >= sigma: dropped (Sec. 3.3)
    }
    // the rectangle of any radius r <= ceil(3 sqrt(a + c + 0.3163)) is empty
    // when u + r < 1 or u - r >= 16 TX (and likewise in y)
    const float r_hi = 3.0f * sqrtf((ah + ch) + 0.32f) * (1.0f + 8.0f * U) + 1.0f;
    const float sx = 8.0f * U * (fabsf(u) + eu + r_hi + X) + 1e-3f;
    const float sy = 8.0f * U * (fabsf(v) + ev + r_hi + Y) + 1e-3f;
    if (u + eu + r_hi + sx < 1.0f || u - eu - r_hi - sx >= X) return 2;
    if (v + ev + r_hi + sy < 1.0f || v - ev - r_hi - sy >= Y) return 2;
    return 0;
}

}  // namespace gsr
