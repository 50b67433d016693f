// Per-Gaussian quantities shared by the wave rasterizer and its adjoint, so
// both take the same alpha >= tau decision and bound the same strips.
#pragma once
#include "gsr_internal.hpp"

namespace gsr {

constexpr float kLog2Tau = -7.9943534368588578f;       // log2(1/255)
constexpr float kNeg2Ln2 = -1.3862943611198906f;       // -2 ln 2

constexpr float kHalfLog2e = 0.72134752044448170368f;  // log2(e) / 2

// The blend's exponent in base 2 with the opacity folded in.  Per Gaussian
// a = sqrt(A log2(e)/2), ab = a beta, c = sqrt(gamma log2(e)/2) and
// ls = log2(opacity) (BlendCoef); per pixel adx = a dx, then
//   e = -(adx + ab dy)^2 - (c dy)^2 + ls = log2(opacity) - q log2(e) / 2
// with q = A (dx + beta dy)^2 + gamma dy^2, so alpha = min(0.99, 2^e) and
// alpha >= tau  <=>  e >= log2(tau).  Both squares are non-negative terms
// (no cancellation); a NaN offset gives a NaN exponent, which fails the test.
struct BlendCoef {
    float a, ab, c, ls;
};
__device__ __forceinline__ BlendCoef blend_coef(float A, float beta, float gam, float sig) {
    BlendCoef k;
    k.a = __builtin_amdgcn_sqrtf(A * kHalfLog2e);
    k.ab = k.a * beta;
    k.c = __builtin_amdgcn_sqrtf(gam * kHalfLog2e);
    k.ls = __builtin_amdgcn_logf(sig);
    return k;
}
__device__ __forceinline__ float blend_exponent(float adx, float ab, float c, float ls, float dy) {
    const float u = fmaf(ab, dy, adx);
    const float t = c * dy;
    return fmaf(-u, u, fmaf(-t, t, ls));
}

// Which of the NS 16x4 strips from row y0 of a 16x16 tile (columns [x_lo,
// x_hi], strip k = rows y0 + 4k .. y0 + 4k + 3) can hold a pixel with
// alpha >= tau: bit k is set unless the exponent's minimum over the strip,
// taken per row over the continuous column interval, exceeds the cut.  With
// u = dx + beta dy the quadratic form is A u^2 + gamma dy^2; over a row u
// spans [mx - x_hi + beta dy, mx - x_lo + beta dy], whose distance from 0 is
// max(lo, -hi, 0).  alpha >= tau  <=>  q <= qlim = -2 ln2 elim; the cut adds
// a margin above the float32 rounding of this test and of the per-pixel
// evaluation: relative 1e-3, plus a term growing with the distance of the
// centre from the tile's centre row yc (dx and dy lose digits there).
template <int NS = 4>
__device__ __forceinline__ uint32_t strip_hits(float mx, float my, float A, float beta, float gam,
                                               float elim, float x_lo, float x_hi, float y0,
                                               float yc) {
    const float qlim = kNeg2Ln2 * elim;
    if (!(qlim > -1e-3f)) return 0u;
    const float ql = fmaxf(qlim, 0.0f);
    const float far = fabsf(mx - (x_lo + 7.5f)) + fabsf(my - yc);
    const float qcut = ql + 1e-3f * (1.0f + ql) +
                       1e-5f * far * (1.0f + __builtin_amdgcn_sqrtf((A + gam) * ql));
    const float clo = mx - x_hi, chi = x_lo - mx;  // lo = clo + beta dy, -hi = chi - beta dy
    const float dy0 = my - y0;
    uint32_t hit = 0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        float qmin = 3.0e38f;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const float dy = dy0 - (float)(4 * k + rr);
            const float lo = fmaf(beta, dy, clo), nhi = fmaf(-beta, dy, chi);
            const float um = fmaxf(fmaxf(lo, nhi), 0.0f);
            qmin = fminf(qmin, fmaf(A * um, um, (gam * dy) * dy));
        }
        if (qmin <= qcut) hit |= 1u << k;
    }
    return hit;
}

}  // namespace gsr
