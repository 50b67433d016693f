// Ellipse tile test (extent rule 1): the ellipse boundary of the prior work
// the paper builds on (Sec. 2.3, Fig. 3(c); Sec. 4.1), with AdaGScale's
// threshold Th as the alpha level (Sec. 3.3) and tau for plain 3D-GS.
//
// A Gaussian reaches alpha >= t only where
//     q(X, Y) = A (X + beta Y)^2 + gamma Y^2 <= c,   c = 2 ln(opacity / t),
// (X, Y) being the pixel's offset from the projected mean.  Tile (tx, ty) is
// kept when its pixel box [16 tx, 16 tx + 15] x [16 ty, 16 ty + 15] meets that
// ellipse.  Per tile row: the ellipse's slice at height Y spans
// X in [-beta Y - S(Y), -beta Y + S(Y)], S(Y) = sqrt((c - gamma Y^2) / A), for
// |Y| <= R = sqrt(c / gamma).  The left end is convex and the right end
// concave in Y, so over the row's band they peak at the clamp of the
// unconstrained extremes Y = w (leftmost point) and Y = -w (rightmost),
// w = beta sqrt(A c / (gamma (gamma + A beta^2))); the band's x-range
// [xl, xr] then meets columns ceil((xl - 15) / 16) .. floor(xr / 16).
//
// Everything is evaluated in double precision from the float32 record values
// (the same record the rasterizer blends), with a fixed operation order, so
// the preprocess (which counts the tiles) and the emission (which writes
// them) get the same spans, and so does an IEEE FP64 reimplementation.  The
// build disables FP contraction.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace gsr {

struct Ellipse {
    double u, v, A, beta, gamma, c, R, w;
};

__device__ __forceinline__ bool finite_d(double x) { return x == x && fabs(x) <= 1.79769313486231570815e308; }

// False (no tiles) unless every value is finite, A, gamma > 0 and c > 0.
__device__ __forceinline__ bool ellipse_setup(float fu, float fv, float fA, float fbeta, float fgamma,
                                              float fsigma, float ft, Ellipse &e) {
    const double u = fu, v = fv, A = fA, beta = fbeta, gamma = fgamma;
    if (!(finite_d(u) && finite_d(v) && finite_d(A) && finite_d(beta) && finite_d(gamma))) return false;
    if (!(A > 0.0 && gamma > 0.0)) return false;
    const double c = 2.0 * log((double)fsigma / (double)ft);
    if (!(c > 0.0 && finite_d(c))) return false;
    const double R = sqrt(c / gamma);
    const double w = beta * sqrt((A * c) / (gamma * (gamma + A * (beta * beta))));
    if (!(finite_d(R) && finite_d(w))) return false;
    e.u = u; e.v = v; e.A = A; e.beta = beta; e.gamma = gamma; e.c = c; e.R = R; e.w = w;
    return true;
}

__device__ __forceinline__ double ellipse_half_width(const Ellipse &e, double Y) {
    double r = e.c - e.gamma * (Y * Y);
    if (!(r > 0.0)) r = 0.0;
    return sqrt(r / e.A);
}

// Inclusive tile columns [a, b] of row ty that meet the ellipse, clipped to
// [cx0, cx1]; false (empty) otherwise.  A NaN bound clips to the range.
__device__ __forceinline__ bool ellipse_row_span(const Ellipse &e, int ty, int cx0, int cx1, int &a,
                                                 int &b) {
    const double y0 = (double)(16 * ty) - e.v, y1 = y0 + 15.0;
    if (y1 < -e.R || y0 > e.R) return false;
    const double lo = y0 < -e.R ? -e.R : y0, hi = y1 > e.R ? e.R : y1;
    const double wl = e.w < lo ? lo : (e.w > hi ? hi : e.w);
    const double wr = -e.w < lo ? lo : (-e.w > hi ? hi : -e.w);
    const double xl = (e.u - e.beta * wl) - ellipse_half_width(e, wl);
    const double xr = (e.u - e.beta * wr) + ellipse_half_width(e, wr);
    double fa = ceil((xl - 15.0) / 16.0);
    double fb = floor(xr / 16.0);
    fa = fa >= (double)cx0 ? fa : (double)cx0;
    fb = fb <= (double)cx1 ? fb : (double)cx1;
    if (fa > (double)cx1 || fb < (double)cx0 || fb < fa) return false;
    a = (int)fa;
    b = (int)fb;
    return true;
}

}  // namespace gsr
