// Tile tests of the extent rules beyond the rectangle, evaluated per tile row
// in double precision from the float32 splat record (the values the
// rasterizer blends), with a fixed operation order, so the pair count and the
// emission get the same spans; so does any FP64 reimplementation with the same
// operation order (the ellipse's one log per Gaussian aside, the operations
// are correctly rounded).  The build disables FP contraction.  Both tests run
// inside the preprocess's tile rectangle and only remove tiles from it.
//
// Ellipse (extent rule 1): the ellipse boundary of the prior work the paper
// builds on (Sec. 2.3, Fig. 3(c); Sec. 4.1), with AdaGScale's threshold Th as
// the alpha level (Sec. 3.3) and tau for plain 3D-GS.  A Gaussian reaches
// alpha >= t only where
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
// Oriented box (extent rule 2): the OBB test of the prior work (GSCore,
// Sec. 2.3 Fig. 3(b)) -- the box on the projected mean along the eigenvectors
// of the 2D covariance (recovered from the record: a = 1/A + beta^2/gamma,
// b = -beta/gamma, c = 1/gamma), half-lengths 3 sqrt(lambda_i) times the
// AdaGScale scale s (the rectangle rule's 3-sigma extent, oriented).  Per tile
// row the box's x-range inside the row's band comes from the vertices in the
// band and the edges' crossings of the band's two lines.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace gsr {

// Reads lane `src` (wave-uniform) of a register: v_readlane, a scalar read,
// instead of a cross-lane permute through the LDS crossbar.
__device__ __forceinline__ uint32_t lane_u32(uint32_t x, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, src);
}
__device__ __forceinline__ int lane_i32(int x, int src) { return __builtin_amdgcn_readlane(x, src); }
__device__ __forceinline__ uint64_t lane_u64(uint64_t x, int src) {
    return (uint64_t)lane_u32((uint32_t)x, src) | ((uint64_t)lane_u32((uint32_t)(x >> 32), src) << 32);
}
__device__ __forceinline__ double lane_f64(double x, int src) {
    return __longlong_as_double((long long)lane_u64((uint64_t)__double_as_longlong(x), src));
}

__device__ __forceinline__ bool finite_d(double x) { return x == x && fabs(x) <= 1.79769313486231570815e308; }

// Columns ceil((xl - 15) / 16) .. floor(xr / 16) clipped to [cx0, cx1]; false
// when empty.  A NaN bound clips to the range.
__device__ __forceinline__ bool tile_columns(double xl, double xr, int cx0, int cx1, int &a, int &b) {
    double fa = ceil((xl - 15.0) / 16.0);
    double fb = floor(xr / 16.0);
    fa = fa >= (double)cx0 ? fa : (double)cx0;
    fb = fb <= (double)cx1 ? fb : (double)cx1;
    if (fa > (double)cx1 || fb < (double)cx0 || fb < fa) return false;
    a = (int)fa;
    b = (int)fb;
    return true;
}

// Rows of [y0, y1) whose band [16 ty, 16 ty + 15] can meet [ylo, yhi] (the
// shape's row extent), one row to spare on each side against the rounding of
// these bounds; the rows left out have empty spans.
__device__ __forceinline__ void rows_meeting(double ylo, double yhi, int y0, int y1, int &ra, int &rb) {
    const double flo = ceil((ylo - 15.0) / 16.0) - 1.0;
    const double fhi = floor(yhi / 16.0) + 2.0;
    ra = flo > (double)y0 ? (flo < (double)y1 ? (int)flo : y1) : y0;
    rb = fhi < (double)y1 ? (fhi > (double)ra ? (int)fhi : ra) : y1;
}

// The fields of a 48-byte splat record a shape reads, requested together:
// left alone, the compiler splits them over the setup's early exits and
// sinks them below the caller's conditions, one memory trip each.  `pin`
// (an empty asm claiming to modify every field) makes them all arrive at one
// point, after the caller's other loads of the same Gaussian are issued.
struct SplatRec {
    float4 q0, q1, q2;  // (u, v, A, beta), (gamma, opacity, depth, threshold), (r, g, b, scale)
    __device__ __forceinline__ static SplatRec load(const float *rec, bool third) {
        const float4 *p = reinterpret_cast<const float4 *>(rec);
        SplatRec r;
        r.q0 = p[0];
        r.q1 = p[1];
        r.q2 = third ? p[2] : make_float4(0.f, 0.f, 0.f, 0.f);
        return r;
    }
    __device__ __forceinline__ void pin(bool third) {
        __asm__ volatile("" : "+v"(q0.x), "+v"(q0.y), "+v"(q0.z), "+v"(q0.w));
        __asm__ volatile("" : "+v"(q1.x), "+v"(q1.y), "+v"(q1.w));
        if (third) __asm__ volatile("" : "+v"(q2.w));
    }
};

struct Ellipse {
    double u, v, A, beta, gamma, c, R, w;
    static constexpr bool kThird = false;  // reads record words 0-7

    // False (no tiles) unless every value is finite, A, gamma > 0 and c > 0.
    __device__ __forceinline__ bool setup(const SplatRec &rec) {
        const double u_ = rec.q0.x, v_ = rec.q0.y, A_ = rec.q0.z, beta_ = rec.q0.w, gamma_ = rec.q1.x;
        if (!(finite_d(u_) && finite_d(v_) && finite_d(A_) && finite_d(beta_) && finite_d(gamma_)))
            return false;
        if (!(A_ > 0.0 && gamma_ > 0.0)) return false;
        const double c_ = 2.0 * log((double)rec.q1.y / (double)rec.q1.w);
        if (!(c_ > 0.0 && finite_d(c_))) return false;
        const double R_ = sqrt(c_ / gamma_);
        const double w_ = beta_ * sqrt((A_ * c_) / (gamma_ * (gamma_ + A_ * (beta_ * beta_))));
        if (!(finite_d(R_) && finite_d(w_))) return false;
        u = u_; v = v_; A = A_; beta = beta_; gamma = gamma_; c = c_; R = R_; w = w_;
        return true;
    }

    __device__ __forceinline__ double half_width(double Y) const {
        double r = c - gamma * (Y * Y);
        if (!(r > 0.0)) r = 0.0;
        return sqrt(r / A);
    }

    // Rows where |Y| <= R can hold: 16 ty - v + 15 >= -R and 16 ty - v <= R.
    __device__ __forceinline__ void row_band(int y0, int y1, int &ra, int &rb) const {
        rows_meeting(v - R, v + R, y0, y1, ra, rb);
    }

    // Inclusive tile columns [a, b] of row ty that meet the ellipse, clipped
    // to [cx0, cx1]; false (empty) otherwise.
    __device__ __forceinline__ bool row_span(int ty, int cx0, int cx1, int &a, int &b) const {
        const double y0 = (double)(16 * ty) - v, y1 = y0 + 15.0;
        if (y1 < -R || y0 > R) return false;
        const double lo = y0 < -R ? -R : y0, hi = y1 > R ? R : y1;
        const double wl = w < lo ? lo : (w > hi ? hi : w);
        const double wr = -w < lo ? lo : (-w > hi ? hi : -w);
        // when the band holds both extremes, wr = -wl and the half widths are
        // the same number (Y * Y is exact under negation): evaluate it once
        const double sl = half_width(wl);
        const double sr = wr == -wl ? sl : half_width(wr);
        const double xl = (u - beta * wl) - sl;
        const double xr = (u - beta * wr) + sr;
        return tile_columns(xl, xr, cx0, cx1, a, b);
    }

    __device__ __forceinline__ void broadcast(int src) {
        u = lane_f64(u, src); v = lane_f64(v, src); A = lane_f64(A, src);
        beta = lane_f64(beta, src); gamma = lane_f64(gamma, src); c = lane_f64(c, src);
        R = lane_f64(R, src); w = lane_f64(w, src);
    }
};

struct OrientedBox {
    double vx[4], vy[4], k[4], ymin, ymax;
    static constexpr bool kThird = true;  // also reads word 11 (the scale)

    __device__ __forceinline__ bool setup(const SplatRec &rec) {
        const double u = rec.q0.x, v = rec.q0.y, A = rec.q0.z, beta = rec.q0.w, gamma = rec.q1.x,
                     s = rec.q2.w;
        if (!(finite_d(u) && finite_d(v) && finite_d(A) && finite_d(beta) && finite_d(gamma) &&
              finite_d(s)))
            return false;
        if (!(A > 0.0 && gamma > 0.0 && s > 0.0)) return false;
        const double a = 1.0 / A + (beta * beta) / gamma, b = -(beta / gamma), c = 1.0 / gamma;
        const double mid = 0.5 * (a + c), det = a * c - b * b;
        double disc = mid * mid - det;
        if (!(disc > 0.0)) disc = 0.0;
        const double sq = sqrt(disc), l1 = mid + sq;
        double l2 = mid - sq;
        if (!(l2 > 0.0)) l2 = 0.0;
        // major eigenvector: (b, l1 - a) or (l1 - c, b), whichever is longer
        const double px = b, py = l1 - a, qx = l1 - c, qy = b;
        const double np = px * px + py * py, nq = qx * qx + qy * qy;
        double ex = np >= nq ? px : qx, ey = np >= nq ? py : qy;
        const double nn = np >= nq ? np : nq;
        if (nn > 0.0) {
            const double r = sqrt(nn);
            ex = ex / r;
            ey = ey / r;
        } else {
            ex = 1.0;
            ey = 0.0;
        }
        const double h1 = (3.0 * sqrt(l1)) * s, h2 = (3.0 * sqrt(l2)) * s;
        const double ax = h1 * ex, ay = h1 * ey, bx = -(h2 * ey), by = h2 * ex;
        // vertices in order around the box: +a+b, +a-b, -a-b, -a+b
        vx[0] = (u + ax) + bx; vy[0] = (v + ay) + by;
        vx[1] = (u + ax) - bx; vy[1] = (v + ay) - by;
        vx[2] = (u - ax) - bx; vy[2] = (v - ay) - by;
        vx[3] = (u - ax) + bx; vy[3] = (v - ay) + by;
        ymin = vy[0];
        ymax = vy[0];
        bool ok = true;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = (i + 1) & 3;
            const double dy = vy[j] - vy[i];
            k[i] = dy != 0.0 ? (vx[j] - vx[i]) / dy : 0.0;
            ymin = vy[i] < ymin ? vy[i] : ymin;
            ymax = vy[i] > ymax ? vy[i] : ymax;
            ok = ok && finite_d(vx[i]) && finite_d(k[i]);
        }
        return ok && finite_d(ymin) && finite_d(ymax);
    }

    __device__ __forceinline__ void row_band(int y0, int y1, int &ra, int &rb) const {
        rows_meeting(ymin, ymax, y0, y1, ra, rb);
    }

    __device__ __forceinline__ bool row_span(int ty, int cx0, int cx1, int &a, int &b) const {
        const double y0 = (double)(16 * ty), y1 = y0 + 15.0;
        if (y1 < ymin || y0 > ymax) return false;
        double xmin = INFINITY, xmax = -INFINITY;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (vy[i] >= y0 && vy[i] <= y1) {
                xmin = vx[i] < xmin ? vx[i] : xmin;
                xmax = vx[i] > xmax ? vx[i] : xmax;
            }
            const int j = (i + 1) & 3;
            const double ya = vy[i], yb = vy[j];
            if (ya == yb) continue;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const double yl = e ? y1 : y0;
                if ((yl - ya) * (yl - yb) <= 0.0) {
                    const double x = vx[i] + (yl - ya) * k[i];
                    xmin = x < xmin ? x : xmin;
                    xmax = x > xmax ? x : xmax;
                }
            }
        }
        if (!(xmin <= xmax)) return false;
        return tile_columns(xmin, xmax, cx0, cx1, a, b);
    }

    __device__ __forceinline__ void broadcast(int src) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            vx[i] = lane_f64(vx[i], src);
            vy[i] = lane_f64(vy[i], src);
            k[i] = lane_f64(k[i], src);
        }
        ymin = lane_f64(ymin, src);
        ymax = lane_f64(ymax, src);
    }
};

}  // namespace gsr
