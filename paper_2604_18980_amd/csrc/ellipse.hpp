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
// the pair count and the emission get the same spans; so does any FP64
// reimplementation with the same operation order whose log agrees to the last
// bit (the other operations are correctly rounded).  The build disables FP
// contraction.  The test runs inside the preprocess's plain tile rectangle and
// only removes tiles from it.
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
    // when the band holds both extremes, wr = -wl and the half widths are the
    // same number (Y * Y is exact under negation): evaluate it once
    const double sl = ellipse_half_width(e, wl);
    const double sr = wr == -wl ? sl : ellipse_half_width(e, wr);
    const double xl = (e.u - e.beta * wl) - sl;
    const double xr = (e.u - e.beta * wr) + sr;
    double fa = ceil((xl - 15.0) / 16.0);
    double fb = floor(xr / 16.0);
    fa = fa >= (double)cx0 ? fa : (double)cx0;
    fb = fb <= (double)cx1 ? fb : (double)cx1;
    if (fa > (double)cx1 || fb < (double)cx0 || fb < fa) return false;
    a = (int)fa;
    b = (int)fb;
    return true;
}

// The rows of [y0, y1) that can meet the band |Y| <= R: row ty meets it when
// 16 ty - v + 15 >= -R and 16 ty - v <= R, i.e. ceil((v - R - 15) / 16) <= ty
// <= floor((v + R) / 16); one row to spare on each side absorbs the rounding
// of these bounds (far below a pixel).  The rows left out have empty spans, so
// walking [ra, rb) instead of [y0, y1) gives the same result.
__device__ __forceinline__ void ellipse_row_band(const Ellipse &e, int y0, int y1, int &ra, int &rb) {
    const double flo = ceil((e.v - e.R - 15.0) / 16.0) - 1.0;
    const double fhi = floor((e.v + e.R) / 16.0) + 2.0;
    ra = flo > (double)y0 ? (flo < (double)y1 ? (int)flo : y1) : y0;
    rb = fhi < (double)y1 ? (fhi > (double)ra ? (int)fhi : ra) : y1;
}

// Number of tiles of the rectangle [x0, x1) x [y0, y1) that meet the ellipse.
__device__ __forceinline__ uint32_t ellipse_tile_count(const Ellipse &e, int x0, int y0, int x1, int y1) {
    int ra, rb;
    ellipse_row_band(e, y0, y1, ra, rb);
    uint32_t cnt = 0;
    for (int ty = ra; ty < rb; ++ty) {
        int a, b;
        if (ellipse_row_span(e, ty, x0, x1 - 1, a, b)) cnt += (uint32_t)(b - a + 1);
    }
    return cnt;
}

}  // namespace gsr
