// Per-Gaussian quantities shared by the wave rasterizer and its adjoint, so
// both take the same alpha >= tau decision and bound the same strips.
#pragma once
#include "gsr_internal.hpp"

namespace gsr {

constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2
constexpr float kLog2Tau = -7.9943534368588578f;           // log2(1/255)
constexpr float kNeg2Ln2 = -1.3862943611198906f;           // -2 ln 2

// alpha = opacity 2^e2 >= tau  <=>  e2 >= elim = log2(tau) - log2(opacity).
// The hardware log2 (about one ulp); an opacity at or below the smallest
// normal float gives elim = +inf (never blended: its alpha is far below tau).
__device__ __forceinline__ float alpha_tau_elim(float sig) {
    return kLog2Tau - __builtin_amdgcn_logf(sig);
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
