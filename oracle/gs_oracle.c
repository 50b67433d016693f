/*
 * gs_oracle.c -- plain FP64 CPU oracle of the 3D-GS tile-rendering path with
 * AdaGScale (Jo et al., "AdaGScale: Viewpoint-Adaptive Gaussian Scaling in 3D
 * Gaussian Splatting to Reduce Gaussian-Tile Pairs").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP path; it is slow on purpose and written so that each step can be
 * checked against the paper by eye:
 *
 *   preprocess   Sec. 2.1 (cull, EWA projection, colour, depth) and, for
 *                AdaGScale, eq. (10) for Th, the Th > opacity cull of Sec. 3.3
 *                and the reduced extent used by the tile test (Sec. 3.1, 3.3)
 *   emit         Sec. 2.1: one (tile, depth, Gaussian) pair per intersected tile
 *   sort         Sec. 2.1: pairs ordered by depth inside each tile
 *   ranges       start/end of every tile's run in the sorted list
 *   blend        eq. (1) and eq. (2) with tau = 1/255 and the 1e-4 early exit,
 *                original covariance and tau in both modes (dual size, Sec. 3.3);
 *                optionally skipping blends of low contribution (eq. 3 and its
 *                max(T) and T_up(depth) approximations, Sec. 2.4, 3.2)
 *   backward     analytic adjoint of the above with every discrete decision
 *                frozen (pair set, skips, stop, clamps)
 *
 * Every floating-point value is double.  Compile with -ffp-contract=off so each
 * expression is rounded exactly as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TILE 16
#define TAU (1.0 / 255.0)        /* alpha threshold, Sec. 2.1 */
#define T_STOP 1e-4              /* early-exit transmittance, Sec. 2.1 */
#define ALPHA_MAX 0.99           /* alpha clamp */
#define NEAR_Z 0.2               /* near-plane cull */
#define DILATION 0.3             /* low-pass added to the 2D covariance */
#define FRUSTUM_SLACK 1.3        /* clamp of x/z and y/z in the EWA Jacobian */
#define LAMBDA_FLOOR 0.1         /* floor of the eigenvalue discriminant */
#define LUT_BINS 20              /* T_upper depth bins, Sec. 3.4 */
#define TWO_PI 6.283185307179586 /* 2*pi rounded to double */

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, written from their definition.                  */
/*                                                                           */
/*   Y_l^0      = N_l0 P_l(z)                                                */
/*   Y_l^{+m}   = sqrt(2) N_lm (-1)^m P_l^(m)(z) Re((x+iy)^m)                 */
/*   Y_l^{-m}   = sqrt(2) N_lm (-1)^m P_l^(m)(z) Im((x+iy)^m)                 */
/*                                                                           */
/* with N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l the Legendre           */
/* polynomial, P_l^(m) its m-th derivative (so (-1)^m sin^m(theta) P_l^(m)   */
/* is the associated Legendre function with the Condon-Shortley phase) and   */
/* (x, y, z) a unit direction.  Coefficient k = l*l + l + m.                  */
/* ------------------------------------------------------------------------ */
#define SH_LMAX 3

static double factorial(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* Coefficients (ascending powers of z) of P_l, from Bonnet's recurrence
 * (n+1) P_{n+1} = (2n+1) z P_n - n P_{n-1}. */
static void legendre_coeffs(int l, double c[SH_LMAX + 1]) {
    double p0[SH_LMAX + 2] = {1.0}, p1[SH_LMAX + 2] = {0.0, 1.0}, p2[SH_LMAX + 2];
    memset(c, 0, sizeof(double) * (SH_LMAX + 1));
    if (l == 0) { c[0] = 1.0; return; }
    for (int n = 1; n < l; ++n) {
        memset(p2, 0, sizeof(p2));
        for (int i = 0; i <= n; ++i) p2[i + 1] += (2.0 * n + 1.0) * p1[i];
        for (int i = 0; i <= n; ++i) p2[i] -= n * p0[i];
        for (int i = 0; i <= n + 1; ++i) p2[i] /= (n + 1.0);
        memcpy(p0, p1, sizeof(p0));
        memcpy(p1, p2, sizeof(p1));
    }
    for (int i = 0; i <= l; ++i) c[i] = p1[i];
}

/* value of d^m/dz^m of P_l at z, and (if dval) of d^{m+1}/dz^{m+1} */
static double legendre_deriv(int l, int m, double z, double *dval) {
    double c[SH_LMAX + 1];
    legendre_coeffs(l, c);
    for (int k = 0; k < m; ++k) {             /* differentiate m times */
        for (int i = 0; i < l; ++i) c[i] = c[i + 1] * (i + 1);
        c[l] = 0.0;
    }
    double v = 0.0, dv = 0.0, zp = 1.0;
    for (int i = 0; i <= l; ++i) { v += c[i] * zp; zp *= z; }
    zp = 1.0;
    for (int i = 1; i <= l; ++i) { dv += c[i] * i * zp; zp *= z; }
    if (dval) *dval = dv;
    return v;
}

/* Re and Im of (x + i y)^m, and their partials in x and y. */
static void zpow(int m, double x, double y, double *re, double *im) {
    double r = 1.0, i = 0.0;
    for (int k = 0; k < m; ++k) { double nr = r * x - i * y; i = r * y + i * x; r = nr; }
    *re = r; *im = i;
}

/* Basis values Y[k] and (optionally) gradients dY[k][3] with respect to the
 * Cartesian components, for the unit direction d. */
void orc_sh_basis(int degree, const double d[3], double *Y, double *dY) {
    for (int l = 0; l <= degree; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m, k = l * l + l + m;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double dq, q = legendre_deriv(l, am, d[2], &dq);
            double re, im, re1 = 0.0, im1 = 0.0;
            zpow(am, d[0], d[1], &re, &im);
            if (am > 0) zpow(am - 1, d[0], d[1], &re1, &im1);
            double sgn = (am % 2) ? -1.0 : 1.0;
            double f = (m == 0) ? N : sqrt(2.0) * N * sgn;
            double ang = (m >= 0) ? re : im;
            /* d/dx (x+iy)^m = m (x+iy)^(m-1); d/dy = i m (x+iy)^(m-1) */
            double dang_dx = (m >= 0) ? am * re1 : am * im1;
            double dang_dy = (m >= 0) ? -am * im1 : am * re1;
            Y[k] = f * q * ang;
            if (dY) {
                dY[3 * k + 0] = f * q * dang_dx;
                dY[3 * k + 1] = f * q * dang_dy;
                dY[3 * k + 2] = f * dq * ang;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* AdaGScale threshold and extent (Sec. 3.2 eq. (10), Sec. 3.3).             */
/*                                                                           */
/* The approximated peripheral score of eq. (9) grows linearly in x, so the  */
/* largest x with PS(x) <= K (eq. (5)) is eq. (10):                          */
/*     Th = K / (T_up(depth) * 2 pi * sqrt(det(G_cov))) + tau.               */
/* A Gaussian whose Th reaches its opacity is dropped for this view.  The     */
/* tile test then uses the region alpha >= Th instead of alpha >= tau.  For   */
/* a 2D Gaussian, alpha >= t is the ellipse of Mahalanobis radius            */
/* sqrt(2 ln(sigma/t)), so raising the threshold from tau to Th shrinks every */
/* axis by s = sqrt(ln(sigma/Th) / ln(sigma/tau)); the plain extent v is      */
/* scaled by s.                                                              */
/* ------------------------------------------------------------------------ */

/* Plain extent: 3 standard deviations along the major axis of the 2D
 * covariance (a, b; b, c), with the discriminant floored as in the original
 * 3D-GS rasterizer. */
double orc_plain_extent(double a, double b, double c) {
    double det = a * c - b * b;
    double mid = 0.5 * (a + c);
    double disc = mid * mid - det;
    if (disc < LAMBDA_FLOOR) disc = LAMBDA_FLOOR;
    double lam = mid + sqrt(disc);
    return 3.0 * sqrt(lam);
}

/* Returns 1 if the Gaussian survives.  Outputs Th (eq. 10) and s. */
int orc_adagscale(double det, double sigma, double depth, double K, const float *t_upper,
                  double lut_depth_max, int force_unit_scale, double *th, double *s) {
    double f = (depth * LUT_BINS) / lut_depth_max;
    int bin = (f >= LUT_BINS - 1) ? LUT_BINS - 1 : (int)floor(f);
    double tu = (double)t_upper[bin];
    if (!(tu > 0.0)) { *th = INFINITY; *s = 0.0; return 0; }
    double denom = (tu * TWO_PI) * sqrt(det);
    *th = K / denom + TAU;
    if (*th >= sigma) { *s = 0.0; return 0; }
    *s = force_unit_scale ? 1.0 : sqrt(log(sigma / *th) / log(sigma / TAU));
    return 1;
}

static int is_finite(double x) { return x == x && fabs(x) <= 1.79769313486231570815e308; }

/* ------------------------------------------------------------------------ */
/* Ellipse tile test (extent rule 1): the ellipse boundary of the prior work */
/* the paper builds on (Sec. 2.3, Fig. 3(c); Sec. 4.1), with the alpha       */
/* threshold t = Th of Sec. 3.3 under AdaGScale and t = tau otherwise.       */
/*                                                                           */
/* Pixel (px, py) can reach alpha >= t only inside the ellipse               */
/*     q(X, Y) = A (X + beta Y)^2 + gamma Y^2 <= c,  c = 2 ln(sigma / t),     */
/* with (X, Y) = (px - u, py - v).  A tile (tx, ty) is kept when its pixel   */
/* box [16 tx, 16 tx + 15] x [16 ty, 16 ty + 15] meets the ellipse.  For the  */
/* row band Y in [Y0, Y1] the ellipse's slice at Y spans                      */
/*     X in [-beta Y - S(Y), -beta Y + S(Y)],  S(Y) = sqrt((c - gamma Y^2)/A), */
/* for |Y| <= R = sqrt(c / gamma).  The left end is convex in Y and the right */
/* end concave, so over the band they reach their extremes at the clamp of    */
/* the unconstrained extremes Y = w (leftmost point of the ellipse) and       */
/* Y = -w (rightmost), w = beta sqrt(A c / (gamma (gamma + A beta^2))).       */
/* The band's pixel x-range [xl, xr] then meets tile column tx exactly when   */
/* ceil((xl - 15) / 16) <= tx <= floor(xr / 16).                             */
/*                                                                           */
/* Every value is the float32 record value widened to double (the renderer   */
/* blends the same record).  The test runs inside the plain tile rectangle   */
/* and only removes tiles from it.                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    double u, v, A, beta, gamma, c, R, w;
    int ok;
} ellipse_t;

static double f32r(double x) { return (double)(float)x; }

/* ok = 0 (no tiles) unless every value is finite, A, gamma > 0 and c > 0. */
static void ellipse_setup(double u, double v, double A, double beta, double gamma, double sigma,
                          double t, ellipse_t *e) {
    e->ok = 0;
    if (!(is_finite(u) && is_finite(v) && is_finite(A) && is_finite(beta) && is_finite(gamma)))
        return;
    if (!(A > 0.0 && gamma > 0.0)) return;
    double c = 2.0 * log(sigma / t);
    if (!(c > 0.0 && is_finite(c))) return;
    double R = sqrt(c / gamma);
    double w = beta * sqrt((A * c) / (gamma * (gamma + A * (beta * beta))));
    if (!(is_finite(R) && is_finite(w))) return;
    e->u = u; e->v = v; e->A = A; e->beta = beta; e->gamma = gamma; e->c = c; e->R = R; e->w = w;
    e->ok = 1;
}

static double ellipse_half_width(const ellipse_t *e, double Y) {
    double r = e->c - e->gamma * (Y * Y);
    if (!(r > 0.0)) r = 0.0;
    return sqrt(r / e->A);
}

/* Tile columns [*a, *b] of row ty that meet the ellipse, clipped to
 * [cx0, cx1]; empty when *b < *a.  A NaN bound clips to the column range. */
static void ellipse_row_span(const ellipse_t *e, int ty, int cx0, int cx1, int *a, int *b) {
    double y0 = (double)(TILE * ty) - e->v, y1 = y0 + (double)(TILE - 1);
    *a = 1; *b = 0;
    if (y1 < -e->R || y0 > e->R) return;
    double lo = y0 < -e->R ? -e->R : y0, hi = y1 > e->R ? e->R : y1;
    double wl = e->w < lo ? lo : (e->w > hi ? hi : e->w);
    double wr = -e->w < lo ? lo : (-e->w > hi ? hi : -e->w);
    double xl = (e->u - e->beta * wl) - ellipse_half_width(e, wl);
    double xr = (e->u - e->beta * wr) + ellipse_half_width(e, wr);
    double fa = ceil((xl - (double)(TILE - 1)) / (double)TILE);
    double fb = floor(xr / (double)TILE);
    fa = fa >= (double)cx0 ? fa : (double)cx0;
    fb = fb <= (double)cx1 ? fb : (double)cx1;
    if (fa > (double)cx1 || fb < (double)cx0 || fb < fa) return;
    *a = (int)fa; *b = (int)fb;
}

/* ------------------------------------------------------------------------ */
/* Oriented-box tile test (extent rule 2): the OBB test of the prior work    */
/* (GSCore, Sec. 2.3 Fig. 3(b)).  The box is centred on the projected mean,  */
/* along the eigenvectors of the 2D covariance, with half-lengths 3 sqrt of  */
/* the eigenvalues times the AdaGScale scale s (1 plain): the same 3-sigma   */
/* extent as the rectangle rule, oriented.  A tile is kept when its pixel    */
/* box [16 tx, 16 tx + 15] x [16 ty, 16 ty + 15] meets the OBB: per tile row, */
/* the x-range of the OBB inside the row's band is spanned by the vertices   */
/* in the band and the edges' crossings of the band's two lines.  The        */
/* covariance is recovered from the float32 record (A, beta, gamma):         */
/* a = 1/A + beta^2/gamma, b = -beta/gamma, c = 1/gamma.  Candidates are the  */
/* rectangle rule's tiles, so the test only removes tiles.                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double vx[4], vy[4], k[4], ymin, ymax;
    int ok;
} obb_t;

static void obb_setup(double u, double v, double A, double beta, double gamma, double s, obb_t *o) {
    o->ok = 0;
    if (!(is_finite(u) && is_finite(v) && is_finite(A) && is_finite(beta) && is_finite(gamma) &&
          is_finite(s)))
        return;
    if (!(A > 0.0 && gamma > 0.0 && s > 0.0)) return;
    double a = 1.0 / A + (beta * beta) / gamma, b = -(beta / gamma), c = 1.0 / gamma;
    double mid = 0.5 * (a + c), det = a * c - b * b;
    double disc = mid * mid - det;
    if (!(disc > 0.0)) disc = 0.0;
    double sq = sqrt(disc), l1 = mid + sq, l2 = mid - sq;
    if (!(l2 > 0.0)) l2 = 0.0;
    /* major eigenvector: (b, l1 - a) or (l1 - c, b), whichever is longer */
    double px = b, py = l1 - a, qx = l1 - c, qy = b;
    double np = px * px + py * py, nq = qx * qx + qy * qy;
    double ex = np >= nq ? px : qx, ey = np >= nq ? py : qy, nn = np >= nq ? np : nq;
    if (nn > 0.0) {
        double r = sqrt(nn);
        ex = ex / r;
        ey = ey / r;
    } else {
        ex = 1.0;
        ey = 0.0;
    }
    double h1 = (3.0 * sqrt(l1)) * s, h2 = (3.0 * sqrt(l2)) * s;
    double ax = h1 * ex, ay = h1 * ey, bx = -(h2 * ey), by = h2 * ex;
    /* vertices in order around the box: +a+b, +a-b, -a-b, -a+b */
    o->vx[0] = (u + ax) + bx; o->vy[0] = (v + ay) + by;
    o->vx[1] = (u + ax) - bx; o->vy[1] = (v + ay) - by;
    o->vx[2] = (u - ax) - bx; o->vy[2] = (v - ay) - by;
    o->vx[3] = (u - ax) + bx; o->vy[3] = (v - ay) + by;
    o->ymin = o->vy[0]; o->ymax = o->vy[0];
    for (int i = 0; i < 4; ++i) {
        int j = (i + 1) & 3;
        double dy = o->vy[j] - o->vy[i];
        o->k[i] = dy != 0.0 ? (o->vx[j] - o->vx[i]) / dy : 0.0;
        if (o->vy[i] < o->ymin) o->ymin = o->vy[i];
        if (o->vy[i] > o->ymax) o->ymax = o->vy[i];
    }
    if (!(is_finite(o->ymin) && is_finite(o->ymax))) return;
    for (int i = 0; i < 4; ++i)
        if (!(is_finite(o->vx[i]) && is_finite(o->k[i]))) return;
    o->ok = 1;
}

/* Tile columns [*a, *b] of row ty that meet the box, clipped to [cx0, cx1]. */
static void obb_row_span(const obb_t *o, int ty, int cx0, int cx1, int *a, int *b) {
    double y0 = (double)(TILE * ty), y1 = y0 + (double)(TILE - 1);
    *a = 1; *b = 0;
    if (y1 < o->ymin || y0 > o->ymax) return;
    double xmin = INFINITY, xmax = -INFINITY;
    for (int i = 0; i < 4; ++i) {
        if (o->vy[i] >= y0 && o->vy[i] <= y1) {
            if (o->vx[i] < xmin) xmin = o->vx[i];
            if (o->vx[i] > xmax) xmax = o->vx[i];
        }
        int j = (i + 1) & 3;
        double ya = o->vy[i], yb = o->vy[j];
        if (ya == yb) continue;
        for (int e = 0; e < 2; ++e) {
            double yl = e ? y1 : y0;
            if ((yl - ya) * (yl - yb) <= 0.0) {
                double x = o->vx[i] + (yl - ya) * o->k[i];
                if (x < xmin) xmin = x;
                if (x > xmax) xmax = x;
            }
        }
    }
    if (!(xmin <= xmax)) return;
    double fa = ceil((xmin - (double)(TILE - 1)) / (double)TILE);
    double fb = floor(xmax / (double)TILE);
    fa = fa >= (double)cx0 ? fa : (double)cx0;
    fb = fb <= (double)cx1 ? fb : (double)cx1;
    if (fa > (double)cx1 || fb < (double)cx0 || fb < fa) return;
    *a = (int)fa; *b = (int)fb;
}

int orc_obb_spans(double u, double v, double A, double beta, double gamma, double s, int ty0,
                  int ty1, int cx0, int cx1, int32_t *spans, double *verts) {
    obb_t o;
    obb_setup(u, v, A, beta, gamma, s, &o);
    for (int ty = ty0; ty < ty1; ++ty) {
        int a = 1, b = 0;
        if (o.ok) obb_row_span(&o, ty, cx0, cx1, &a, &b);
        spans[2 * (ty - ty0)] = a;
        spans[2 * (ty - ty0) + 1] = b;
    }
    if (verts)
        for (int i = 0; i < 4; ++i) { verts[2 * i] = o.vx[i]; verts[2 * i + 1] = o.vy[i]; }
    return o.ok;
}

/* Python-facing form of the row test for the pins: spans[2 * (ty - ty0)]. */
int orc_ellipse_spans(double u, double v, double A, double beta, double gamma, double sigma,
                      double t, int ty0, int ty1, int cx0, int cx1, int32_t *spans) {
    ellipse_t e;
    ellipse_setup(u, v, A, beta, gamma, sigma, t, &e);
    for (int ty = ty0; ty < ty1; ++ty) {
        int a = 1, b = 0;
        if (e.ok) ellipse_row_span(&e, ty, cx0, cx1, &a, &b);
        spans[2 * (ty - ty0)] = a;
        spans[2 * (ty - ty0) + 1] = b;
    }
    return e.ok;
}

/* ------------------------------------------------------------------------ */
/* Preprocess (Sec. 2.1; AdaGScale additions Sec. 3.3).                      */
/*                                                                           */
/* Inputs are float32 structure-of-arrays, [C][N]; cam[0..11] is the          */
/* row-major [R|t] world-to-camera matrix, cam[12..15] = fx, fy, cx, cy.      */
/* Outputs (double, [N][k]): mean2d[2], conic[3] (inverse 2D covariance      */
/* entries Cxx, Cxy, Cyy: d^T Sigma2^-1 d = Cxx dx^2 + 2 Cxy dx dy + Cyy dy^2, */
/* what the blend of eq. (1) evaluates), quad[3] (the same form as a sum of   */
/* squares, A (dx + beta dy)^2 + gamma dy^2 with A = c/det, beta = -b/c,      */
/* gamma = 1/c: the parametrisation the ellipse and oriented-box tile tests   */
/* take, and the splat record's storage form), opacity, rgb[3], depth, cov2d[3] */
/* (dilated a, b, c), extent (plain v), th, scale, rect[4] (x0, y0, x1, y1    */
/* half-open, tiles), tiles_touched, radius (int).                           */
/* flags: 0 culled, 1 projected (finite, in front), 2 projected with tiles.   */
/* extent_rule 0 (and 2, whose oriented box pair generation then tests):    */
/* the rectangle of radius ceil(v s) (s = 1 when plain) and                  */
/* tiles_touched = its area.  extent_rule 1: the plain radius-ceil(v)         */
/* rectangle and its area, the candidates that pair generation then tests    */
/* against the alpha >= th ellipse (Sec. 3.3 applies Th in that stage).      */
/* ------------------------------------------------------------------------ */
void orc_preprocess(int64_t n, const float *means, const float *log_scales, const float *quats,
                    const float *opacity_logits, const float *sh, int sh_degree,
                    const float *cam, int width, int height,
                    int adagscale, double K, const float *t_upper, double lut_depth_max,
                    int force_unit_scale, int extent_rule,
                    double *mean2d, double *conic, double *quad, double *opacity, double *rgb,
                    double *depth,
                    double *cov2d, double *extent, double *th, double *scale,
                    int32_t *rect, int64_t *tiles_touched, int32_t *radius, int32_t *flags) {
    double W[3][3], t[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) W[i][j] = cam[4 * i + j];
        t[i] = cam[4 * i + 3];
    }
    double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    int TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    int nsh = (sh_degree + 1) * (sh_degree + 1);
    /* camera centre in world coordinates: -R^T t */
    double campos[3];
    for (int j = 0; j < 3; ++j) campos[j] = -(W[0][j] * t[0] + W[1][j] * t[1] + W[2][j] * t[2]);

    /* Gaussians are independent: the OpenMP build (timing only) splits them
       over threads; each iteration writes only its own entries. */
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        flags[g] = 0; tiles_touched[g] = 0; radius[g] = 0;
        for (int k = 0; k < 4; ++k) rect[4 * g + k] = 0;
        double mu[3] = {means[g], means[n + g], means[2 * n + g]};

        /* view transform and near cull */
        double p[3];
        for (int i = 0; i < 3; ++i) p[i] = W[i][0] * mu[0] + W[i][1] * mu[1] + W[i][2] * mu[2] + t[i];
        if (!(p[2] > NEAR_Z)) continue;

        /* 3D covariance  Sigma3 = R S S^T R^T  from scale = exp(log_scale) and the
           normalised quaternion (w, x, y, z) */
        double s3[3] = {exp((double)log_scales[g]), exp((double)log_scales[n + g]),
                        exp((double)log_scales[2 * n + g])};
        double q[4] = {quats[g], quats[n + g], quats[2 * n + g], quats[3 * n + g]};
        double qn = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        if (qn > 0.0) {
            double qlen = sqrt(qn);
            for (int k = 0; k < 4; ++k) q[k] = q[k] / qlen;
        } else {
            q[0] = 1.0; q[1] = q[2] = q[3] = 0.0;
        }
        double w = q[0], x = q[1], y = q[2], z = q[3];
        double R[3][3] = {
            {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
            {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
            {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
        double M[3][3], S3[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = R[i][j] * s3[j];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += M[i][k] * M[j][k];
                S3[i][j] = acc;
            }

        /* EWA projection: Sigma2 = J W Sigma3 W^T J^T + 0.3 I (the J of the
           perspective map at the clamped point) */
        double limx = FRUSTUM_SLACK * ((0.5 * width) / fx);
        double limy = FRUSTUM_SLACK * ((0.5 * height) / fy);
        double txz = p[0] / p[2], tyz = p[1] / p[2];
        if (txz < -limx) txz = -limx;
        if (txz > limx) txz = limx;
        if (tyz < -limy) tyz = -limy;
        if (tyz > limy) tyz = limy;
        double xc = txz * p[2], yc = tyz * p[2];
        double zz = p[2] * p[2];
        double J[2][3] = {{fx / p[2], 0.0, -(fx * xc) / zz},
                          {0.0, fy / p[2], -(fy * yc) / zz}};
        double T[2][3], U[2][3], S2[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += J[i][k] * W[k][j];
                T[i][j] = acc;
            }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += T[i][k] * S3[k][j];
                U[i][j] = acc;
            }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += U[i][k] * T[j][k];
                S2[i][j] = acc;
            }
        double a = S2[0][0] + DILATION, b = S2[0][1], c = S2[1][1] + DILATION;

        /* determinant, conic (eq. 1 uses the inverse of G_cov), mean, depth */
        double det = a * c - b * b;
        double u = fx * (p[0] / p[2]) + cx;
        double v = fy * (p[1] / p[2]) + cy;
        if (!(is_finite(u) && is_finite(v) && is_finite(a) && is_finite(b) && is_finite(c))) continue;
        if (!(det > 0.0)) continue;
        double sigma = 1.0 / (1.0 + exp(-(double)opacity_logits[g]));
        mean2d[2 * g] = u;
        mean2d[2 * g + 1] = v;
        conic[3 * g] = c / det;
        conic[3 * g + 1] = -b / det;
        conic[3 * g + 2] = a / det;
        quad[3 * g] = c / det;
        quad[3 * g + 1] = -b / c;
        quad[3 * g + 2] = 1.0 / c;
        cov2d[3 * g] = a; cov2d[3 * g + 1] = b; cov2d[3 * g + 2] = c;
        opacity[g] = sigma;
        depth[g] = p[2];
        flags[g] = 1;

        /* tile extent: plain 3-sigma, or scaled by AdaGScale */
        double ext = orc_plain_extent(a, b, c);
        extent[g] = ext;
        th[g] = TAU;
        scale[g] = 1.0;
        if (adagscale) {
            double thv, sv;
            int keep = orc_adagscale(det, sigma, p[2], K, t_upper, lut_depth_max, force_unit_scale,
                                     &thv, &sv);
            th[g] = thv;
            scale[g] = sv;
            if (!keep) continue;
            if (extent_rule != 1) ext = ext * sv;  /* rule 1: Th enters at pair generation */
        }
        double rd = ceil(ext);
        if (rd > 1073741824.0) rd = 1073741824.0; /* 2^30 px: covers any image */
        int r = (int)rd;
        radius[g] = r;
        if (r <= 0) continue;

        /* axis-aligned rectangle of 16x16 tiles, half-open */
        double fx0 = floor((u - r) / TILE), fx1 = floor(((u + r) + (TILE - 1)) / TILE);
        double fy0 = floor((v - r) / TILE), fy1 = floor(((v + r) + (TILE - 1)) / TILE);
        fx0 = fx0 < 0 ? 0 : (fx0 > TX ? TX : fx0);
        fx1 = fx1 < 0 ? 0 : (fx1 > TX ? TX : fx1);
        fy0 = fy0 < 0 ? 0 : (fy0 > TY ? TY : fy0);
        fy1 = fy1 < 0 ? 0 : (fy1 > TY ? TY : fy1);
        int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
        int64_t tiles = (int64_t)(x1 - x0) * (int64_t)(y1 - y0);
        if (tiles <= 0) continue;
        rect[4 * g] = x0; rect[4 * g + 1] = y0; rect[4 * g + 2] = x1; rect[4 * g + 3] = y1;
        tiles_touched[g] = tiles;
        flags[g] = 2;

        /* view-dependent colour: SH evaluated along the unit direction from the
           camera centre, offset by 0.5 and clamped at 0 */
        double dir[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
        double len = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        for (int k = 0; k < 3; ++k) dir[k] /= len;
        double Y[(SH_LMAX + 1) * (SH_LMAX + 1)];
        orc_sh_basis(sh_degree, dir, Y, NULL);
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int k = 0; k < nsh; ++k) acc += (double)sh[((int64_t)k * 3 + ch) * n + g] * Y[k];
            acc += 0.5;
            rgb[3 * g + ch] = acc < 0.0 ? 0.0 : acc;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Pair emission (Sec. 2.1): Gaussians in index order, tile rows outer,       */
/* columns inner.  key = tile << 32 | bits(float32 depth), value = index.    */
/* Rule 0 emits the whole rectangle; rule 1 each row's ellipse span and      */
/* rule 2 each row's oriented-box span, from the float32 record values the   */
/* renderer blends.                                                          */
/* ------------------------------------------------------------------------ */
int64_t orc_emit(int64_t n, const int32_t *rect, const int64_t *tiles_touched, const float *depth_f32,
                 int width, int extent_rule, const double *mean2d, const double *quad,
                 const double *opacity, const double *th, const double *scale, uint64_t *keys,
                 uint32_t *vals) {
    int TX = (width + TILE - 1) / TILE;
    int64_t p = 0;
    for (int64_t g = 0; g < n; ++g) {
        if (tiles_touched[g] <= 0) continue;
        uint32_t dbits;
        memcpy(&dbits, &depth_f32[g], 4);
        ellipse_t e;
        obb_t ob;
        if (extent_rule == 1) {
            ellipse_setup(f32r(mean2d[2 * g]), f32r(mean2d[2 * g + 1]), f32r(quad[3 * g]),
                          f32r(quad[3 * g + 1]), f32r(quad[3 * g + 2]), f32r(opacity[g]),
                          f32r(th[g]), &e);
            if (!e.ok) continue;
        } else if (extent_rule == 2) {
            obb_setup(f32r(mean2d[2 * g]), f32r(mean2d[2 * g + 1]), f32r(quad[3 * g]),
                      f32r(quad[3 * g + 1]), f32r(quad[3 * g + 2]), f32r(scale[g]), &ob);
            if (!ob.ok) continue;
        }
        for (int ty = rect[4 * g + 1]; ty < rect[4 * g + 3]; ++ty) {
            int a = rect[4 * g], b = rect[4 * g + 2] - 1;
            if (extent_rule == 1) ellipse_row_span(&e, ty, a, b, &a, &b);
            if (extent_rule == 2) obb_row_span(&ob, ty, a, b, &a, &b);
            for (int tx = a; tx <= b; ++tx) {
                if (keys) {
                    keys[p] = ((uint64_t)(uint32_t)(ty * TX + tx) << 32) | dbits;
                    vals[p] = (uint32_t)g;
                }
                ++p;
            }
        }
    }
    return p;
}

/* Sort (Sec. 2.1): ascending (key, value).  Equal keys keep index order,
 * which is the emission order, so this equals a stable sort by key. */
typedef struct { uint64_t k; uint32_t v; } kv_t;
static int kv_cmp(const void *a, const void *b) {
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return 0;
}
void orc_sort(int64_t np, uint64_t *keys, uint32_t *vals) {
    kv_t *a = (kv_t *)malloc(sizeof(kv_t) * (size_t)(np > 0 ? np : 1));
    for (int64_t i = 0; i < np; ++i) { a[i].k = keys[i]; a[i].v = vals[i]; }
    qsort(a, (size_t)np, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < np; ++i) { keys[i] = a[i].k; vals[i] = a[i].v; }
    free(a);
}

/* ranges[2t], ranges[2t+1] = first and one-past-last index of tile t. */
void orc_ranges(int64_t np, const uint64_t *keys, int num_tiles, int64_t *ranges) {
    for (int t = 0; t < num_tiles; ++t) ranges[2 * t] = ranges[2 * t + 1] = 0;
    for (int64_t i = 0; i < np; ++i) {
        int t = (int)(keys[i] >> 32);
        if (i == 0 || (int)(keys[i - 1] >> 32) != t) ranges[2 * t] = i;
        if (i == np - 1 || (int)(keys[i + 1] >> 32) != t) ranges[2 * t + 1] = i + 1;
    }
}

/* ------------------------------------------------------------------------ */
/* Blending of one pixel, eq. (1)-(2), front to back.                        */
/*                                                                           */
/* rec[g*9 .. g*9+8] = mean x, mean y, the inverse 2D covariance (conic) as  */
/* Cxx, Cxy, Cyy, opacity, r, g, b.  For each listed Gaussian, with          */
/* dx = mean x - px, dy = mean y - py, eq. (1) as written:                   */
/*   power = -(Cxx dx^2 + 2 Cxy dx dy + Cyy dy^2)/2 = -d^T Sigma2^-1 d / 2;   */
/*   skipped if power > 0 (the original 3D-GS guard);                        */
/*   alpha = min(0.99, opacity * exp(power)); skipped if alpha < tau;        */
/*   if T (1 - alpha) < 1e-4 the pixel stops before adding this Gaussian;    */
/*   otherwise colour += alpha T rgb and T *= 1 - alpha.                     */
/*                                                                           */
/* Decision margins.  A float32 renderer may take the other branch of a     */
/* decision when the double value lies within float32 rounding of its       */
/* threshold.  Model of such a renderer: mean, inverse covariance, opacity   */
/* and colour stored in float32 (unit roundoff U = 2^-24), the offset (dx,   */
/* dy) formed in float32 and the quadratic form evaluated as a sum of        */
/* non-negative terms (no cancellation).  To first order its alpha then has  */
/* relative error at most                                                     */
/*   e_alpha = U (32 + 6 q + 2 sqrt(q) G),  q = d^T Sigma2^-1 d,             */
/*   G = sqrt(Cxx) |dx| + sqrt(Cyy) |dy|                                     */
/* (the offset's rounding moves q by 2 sqrt(q) G U at most; stored values,   */
/* products and the exponential by a few U each), and the relative error of */
/* T after blends j = 1..k is at most sum_j (alpha_j e_alpha,j + U) /        */
/* (1 - alpha_j) (each factor 1 - alpha_j and each product).  A relative    */
/* error e moves the logarithm of a value by e (to first order), so the      */
/* distance of a decision to its threshold is taken in logarithms:           */
/* |ln(alpha / tau)|, |ln(T' / 1e-4)|, |ln(c / theta)|, each over its bound.  */
/* (The log form stays valid where the bound itself is large: far out on a   */
/* thin Gaussian q, and with it e_alpha, grows without limit while alpha is  */
/* vanishingly small, and ln(alpha / tau) = ln(opacity / tau) - q / 2 grows  */
/* with it.)  A pixel's margin is the smallest such ratio over its           */
/* decisions; below 1 a float32 renderer may legitimately decide otherwise. */
/* ------------------------------------------------------------------------ */
#define U32 5.9604644775390625e-08 /* 2^-24, the float32 unit roundoff */

/* |ln(v / th)| / e: the distance of v >= 0 to the threshold th > 0 in units of
 * the relative error bound e (infinite for v = 0, which no rounding lifts). */
static double log_margin(double v, double th, double e) {
    return v > 0.0 ? fabs(log(v / th)) / e : INFINITY;
}

static double quad_form(const double *g, double dx, double dy) {
    return g[2] * dx * dx + 2.0 * g[3] * dx * dy + g[4] * dy * dy;
}

static double alpha_err(const double *g, double dx, double dy, double q) {
    double G = sqrt(g[2]) * fabs(dx) + sqrt(g[4]) * fabs(dy);
    double sq = q > 0.0 ? sqrt(q) : 0.0;
    return U32 * (32.0 + 6.0 * q + 2.0 * sq * G);
}

typedef struct {
    double color[3];
    double T;
    int64_t last;      /* 1 + list position of the last blended Gaussian, 0 if none */
    int64_t blended;   /* number of blended Gaussians */
    int64_t evaluated; /* list entries evaluated before the stop */
    double margin;
    uint64_t sig;      /* hash of the blended positions */
} pix_t;

/* Contribution-skip rule of the analysis experiments (Sec. 2.4, Sec. 3.2):
 * a blend operation of Gaussian i at a pixel is skipped -- no colour, no
 * transmittance update -- when its contribution is below theta.  The
 * contribution is alpha T (eq. 3, kind 0, with the pixel's running T), alpha
 * max(T^i) (kind 1, weight[i] = the Gaussian's largest T over the pixels where
 * it blends, Sec. 3.2) or alpha T_up(depth_i) (kind 2, the depth-binned table
 * of Sec. 3.2-3.4, bin = min(floor(20 depth / lut_depth_max), 19)). */
typedef struct {
    int kind;
    double theta;
    const double *weight;   /* kind 1: [n] */
    const float *depth_f32; /* kind 2: [n] */
    const double *lut;      /* kind 2: [20] */
    double lut_depth_max;
} skip_t;

static double skip_weight(const skip_t *sk, uint32_t g, double T) {
    if (sk->kind == 0) return T;
    if (sk->kind == 1) return sk->weight[g];
    double f = ((double)sk->depth_f32[g] * LUT_BINS) / sk->lut_depth_max;
    int bin = (f >= LUT_BINS - 1) ? LUT_BINS - 1 : (int)floor(f);
    return sk->lut[bin];
}

/* Contribution profile (Sec. 2.4, Fig. 4(b)): per bin of the Mahalanobis
 * distance m = sqrt(d^T Sigma2^-1 d) between the pixel and the Gaussian's
 * mean, bin = min(floor(m / bin_width), nbins - 1), the sum and the number of
 * the contributions alpha T of the blends made. */
typedef struct {
    int nbins;
    double bin_width;
    double *sums;
    int64_t *counts;
} profile_t;

/* First-order bound on the image error of a float32 renderer of the model
 * above (orc_blend's `bound` output).  Per channel, the alpha errors move
 * the colour by sum_k |dC/dalpha_k| alpha_k e_alpha,k with
 *   dC/dalpha_k = T_k c_k - B_k / (1 - alpha_k),
 *   B_k = sum_{j>k} alpha_j T_j c_j + T_final bg   (the colour behind k),
 * the rounding of each product T (1 - alpha) by B_{k} U / (1 - alpha_k), and
 * the colour sum's own roundings by U (blends + 2) (sum_k alpha_k T_k |c_k| +
 * T_final |bg|).  Scratch arrays hold the blended entries of the pixel. */
typedef struct {
    const double *bg;
    double *al, *Tk, *ea;
    int64_t *gid;
    double out[3];
} bound_t;

static void pixel_bound(const double *rec, int64_t nb, double T, bound_t *b) {
    double behind[3], absum[3];
    for (int ch = 0; ch < 3; ++ch) {
        behind[ch] = T * b->bg[ch];
        absum[ch] = T * fabs(b->bg[ch]);
        b->out[ch] = 0.0;
    }
    for (int64_t k = nb - 1; k >= 0; --k) {
        const double *g = rec + 9 * b->gid[k];
        double a = b->al[k], Ti = b->Tk[k];
        for (int ch = 0; ch < 3; ++ch) {
            double dCda = Ti * g[6 + ch] - behind[ch] / (1.0 - a);
            b->out[ch] += fabs(dCda) * a * b->ea[k] + fabs(behind[ch]) * U32 / (1.0 - a);
            behind[ch] += a * Ti * g[6 + ch];
            absum[ch] += a * Ti * fabs(g[6 + ch]);
        }
    }
    for (int ch = 0; ch < 3; ++ch) b->out[ch] += U32 * (double)(nb + 2) * absum[ch];
}

/* max_t (nullable, [n]): per Gaussian, the largest transmittance in front of
 * it at a pixel where it is blended (the max(T^i) of Sec. 3.2).  sk
 * (nullable): the contribution-skip rule above; skipped blends count in
 * *skipped (nullable).  pf (nullable): the contribution profile.  bd
 * (nullable): the error bound above. */
static void blend_pixel_prof(double px, double py, const uint32_t *list, int64_t len,
                             const double *rec, pix_t *o, double *max_t, const skip_t *sk,
                             int64_t *skipped, const profile_t *pf, bound_t *bd) {
    double T = 1.0, C[3] = {0.0, 0.0, 0.0}, margin = INFINITY;
    double eT = 0.0; /* relative error bound of T so far */
    int64_t last = 0, blended = 0, ev = 0;
    uint64_t sig = 1469598103934665603ull;
    for (int64_t j = 0; j < len; ++j) {
        const double *g = rec + 9 * (int64_t)list[j];
        ++ev;
        double dx = g[0] - px, dy = g[1] - py;
        double q = quad_form(g, dx, dy);
        double power = -0.5 * q;
        if (power > 0.0) continue;
        double alpha = g[5] * exp(power);
        if (alpha > ALPHA_MAX) alpha = ALPHA_MAX;
        double ea = alpha_err(g, dx, dy, q);
        double ma = log_margin(alpha, TAU, ea);
        if (ma < margin) margin = ma;
        if (alpha < TAU) continue;
        if (sk && sk->theta > 0.0) {
            double c = alpha * skip_weight(sk, list[j], T);
            double ec = ea + (sk->kind == 0 ? eT : 0.0) + U32;
            double mc = log_margin(c, sk->theta, ec);
            if (mc < margin) margin = mc;
            if (c < sk->theta) {
                if (skipped) ++*skipped;
                continue;
            }
        }
        double Tn = T * (1.0 - alpha);
        double eTn = eT + (alpha * ea + U32) / (1.0 - alpha) + U32;
        double mt = log_margin(Tn, T_STOP, eTn);
        if (mt < margin) margin = mt;
        if (Tn < T_STOP) break;
        for (int ch = 0; ch < 3; ++ch) C[ch] += alpha * T * g[6 + ch];
        if (max_t && T > max_t[list[j]]) max_t[list[j]] = T;
        if (pf) {
            double m = sqrt(q);
            double fb = floor(m / pf->bin_width);
            int bin = fb >= (double)(pf->nbins - 1) ? pf->nbins - 1 : (int)fb;
            pf->sums[bin] += alpha * T;
            pf->counts[bin] += 1;
        }
        if (bd) {
            bd->al[blended] = alpha;
            bd->Tk[blended] = T;
            bd->ea[blended] = ea;
            bd->gid[blended] = list[j];
        }
        T = Tn;
        eT = eTn - U32;
        last = j + 1;
        ++blended;
        sig = (sig ^ (uint64_t)j) * 1099511628211ull;
    }
    for (int ch = 0; ch < 3; ++ch) o->color[ch] = C[ch];
    o->T = T; o->last = last; o->blended = blended; o->evaluated = ev; o->margin = margin; o->sig = sig;
    if (bd) pixel_bound(rec, blended, T, bd);
}

static void blend_pixel(double px, double py, const uint32_t *list, int64_t len, const double *rec,
                        pix_t *o, double *max_t) {
    blend_pixel_prof(px, py, list, len, rec, o, max_t, NULL, NULL, NULL, NULL);
}

static void store_pixel(const pix_t *o, int64_t idx, int64_t npix, const double *bg, double *image,
                        double *final_T, int64_t *n_contrib, double *margin, int64_t *evals,
                        uint64_t *sig, int64_t *blended) {
    for (int ch = 0; ch < 3; ++ch) image[ch * npix + idx] = o->color[ch] + o->T * bg[ch];
    final_T[idx] = o->T;
    n_contrib[idx] = o->last;
    if (margin) margin[idx] = o->margin;
    if (evals) evals[idx] = o->evaluated;
    if (sig) sig[idx] = o->sig ^ (uint64_t)o->blended;
    if (blended) blended[idx] = o->blended;
}

static int64_t longest_list(const int64_t *ranges, int num_tiles) {
    int64_t cap = 0;
    for (int t = 0; t < num_tiles; ++t) {
        int64_t len = ranges[2 * t + 1] - ranges[2 * t];
        if (len > cap) cap = len;
    }
    return cap;
}

/* Tile-list rasterizer: pixel (px, py) lies in tile (px/16, py/16) and blends
 * that tile's sorted list.  tiles: optional subset of tile ids (n_sel >= 0);
 * n_sel < 0 blends every tile.  Outputs are [3][H][W] and [H][W]; margin,
 * evals, sig, blended (Gaussians blended per pixel), max_t (per Gaussian,
 * raised to the transmittance in front of it where it blends; caller
 * initialises) and bound ([3][H][W], the first-order float32 error bound
 * above) may be NULL. */
void orc_blend(int width, int height, const int64_t *ranges, const uint32_t *sorted_vals,
               const double *rec, const double *bg, const int32_t *tiles, int64_t n_sel,
               double *image, double *final_T, int64_t *n_contrib, double *margin, int64_t *evals,
               uint64_t *sig, int64_t *blended, double *max_t, double *bound) {
    int TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    int64_t npix = (int64_t)width * height;
    int64_t count = n_sel >= 0 ? n_sel : (int64_t)TX * TY;
    bound_t bd, *pbd = NULL;
    if (bound) {
        int64_t cap = longest_list(ranges, TX * TY) + 1;
        bd.bg = bg;
        bd.al = (double *)malloc(sizeof(double) * (size_t)cap);
        bd.Tk = (double *)malloc(sizeof(double) * (size_t)cap);
        bd.ea = (double *)malloc(sizeof(double) * (size_t)cap);
        bd.gid = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        pbd = &bd;
    }
    /* Pixels are independent: the OpenMP build (timing only) splits the
       tiles over threads when nothing is shared between pixels (no max_t, no
       bound scratch). */
#pragma omp parallel for schedule(dynamic, 4) if (!max_t && !bound)
    for (int64_t s = 0; s < count; ++s) {
        int t = n_sel >= 0 ? tiles[s] : (int)s;
        int tx = t % TX, ty = t / TX;
        for (int py = ty * TILE; py < (ty + 1) * TILE && py < height; ++py)
            for (int px = tx * TILE; px < (tx + 1) * TILE && px < width; ++px) {
                pix_t o;
                blend_pixel_prof((double)px, (double)py, sorted_vals + ranges[2 * t],
                                 ranges[2 * t + 1] - ranges[2 * t], rec, &o, max_t, NULL, NULL,
                                 NULL, pbd);
                int64_t idx = (int64_t)py * width + px;
                store_pixel(&o, idx, npix, bg, image, final_T, n_contrib, margin, evals, sig,
                            blended);
                if (bound)
                    for (int ch = 0; ch < 3; ++ch) bound[ch * npix + idx] = bd.out[ch];
            }
    }
    if (bound) { free(bd.al); free(bd.Tk); free(bd.ea); free(bd.gid); }
}

/* orc_blend with the contribution-skip rule (kind, theta, weight / depth and
 * table as in skip_t); skipped[0] receives the number of skipped blends and
 * blended (nullable, [H][W]) the blends kept per pixel. */
void orc_blend_skip(int width, int height, const int64_t *ranges, const uint32_t *sorted_vals,
                    const double *rec, const double *bg, const int32_t *tiles, int64_t n_sel,
                    int kind, double theta, const double *weight, const float *depth_f32,
                    const double *lut, double lut_depth_max, double *image, double *final_T,
                    int64_t *n_contrib, double *margin, int64_t *blended, int64_t *skipped) {
    skip_t sk = {kind, theta, weight, depth_f32, lut, lut_depth_max};
    int TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    int64_t npix = (int64_t)width * height;
    int64_t count = n_sel >= 0 ? n_sel : (int64_t)TX * TY;
    skipped[0] = 0;
    for (int64_t s = 0; s < count; ++s) {
        int t = n_sel >= 0 ? tiles[s] : (int)s;
        int tx = t % TX, ty = t / TX;
        for (int py = ty * TILE; py < (ty + 1) * TILE && py < height; ++py)
            for (int px = tx * TILE; px < (tx + 1) * TILE && px < width; ++px) {
                pix_t o;
                blend_pixel_prof((double)px, (double)py, sorted_vals + ranges[2 * t],
                                 ranges[2 * t + 1] - ranges[2 * t], rec, &o, NULL, &sk, skipped,
                                 NULL, NULL);
                store_pixel(&o, (int64_t)py * width + px, npix, bg, image, final_T, n_contrib,
                            margin, NULL, NULL, blended);
            }
    }
}

/* Contribution profile of the whole frame (orc_blend's walk): sums[nbins]
 * and counts[nbins] are overwritten. */
void orc_contrib_profile(int width, int height, const int64_t *ranges, const uint32_t *sorted_vals,
                         const double *rec, int nbins, double bin_width, double *sums,
                         int64_t *counts) {
    profile_t pf = {nbins, bin_width, sums, counts};
    for (int b = 0; b < nbins; ++b) { sums[b] = 0.0; counts[b] = 0; }
    int TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    for (int t = 0; t < TX * TY; ++t) {
        int tx = t % TX, ty = t / TX;
        for (int py = ty * TILE; py < (ty + 1) * TILE && py < height; ++py)
            for (int px = tx * TILE; px < (tx + 1) * TILE && px < width; ++px) {
                pix_t o;
                blend_pixel_prof((double)px, (double)py, sorted_vals + ranges[2 * t],
                                 ranges[2 * t + 1] - ranges[2 * t], rec, &o, NULL, NULL, NULL, &pf,
                                 NULL);
            }
    }
}

/* Brute-force blenders on small scenes.
 * mode 1 (tile-restricted): every Gaussian whose tile rectangle contains the
 *   pixel's tile, ordered by (float32 depth, index) -- must equal orc_blend.
 * mode 2 (unrestricted): every projected Gaussian (flags >= 1) in the same
 *   order, whatever its rectangle -- a diagnostic of the mass outside the
 *   extent. */
typedef struct { float d; uint32_t i; } di_t;
static int di_cmp(const void *a, const void *b) {
    const di_t *x = (const di_t *)a, *y = (const di_t *)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}
void orc_blend_bruteforce(int mode, int64_t n, int width, int height, const int32_t *rect,
                          const int32_t *flags, const float *depth_f32, const double *rec,
                          const double *bg, double *image, double *final_T, int64_t *n_contrib) {
    int64_t npix = (int64_t)width * height;
    di_t *cand = (di_t *)malloc(sizeof(di_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    for (int py = 0; py < height; ++py)
        for (int px = 0; px < width; ++px) {
            int tx = px / TILE, ty = py / TILE;
            int64_t m = 0;
            for (int64_t g = 0; g < n; ++g) {
                int in;
                if (mode == 1)
                    in = flags[g] == 2 && rect[4 * g] <= tx && tx < rect[4 * g + 2] &&
                         rect[4 * g + 1] <= ty && ty < rect[4 * g + 3];
                else
                    in = flags[g] >= 1;
                if (in) { cand[m].d = depth_f32[g]; cand[m].i = (uint32_t)g; ++m; }
            }
            qsort(cand, (size_t)m, sizeof(di_t), di_cmp);
            for (int64_t k = 0; k < m; ++k) list[k] = cand[k].i;
            pix_t o;
            blend_pixel((double)px, (double)py, list, m, rec, &o, NULL);
            store_pixel(&o, (int64_t)py * width + px, npix, bg, image, final_T, n_contrib, NULL,
                        NULL, NULL, NULL);
        }
    free(cand);
    free(list);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the blend with the discrete decisions of the forward pass      */
/* frozen.  For the blended Gaussians i = 1..n of a pixel, with T_1 = 1,      */
/* T_{i+1} = T_i (1 - alpha_i) and C = sum alpha_i T_i c_i + T_{n+1} bg:       */
/*   dC/dc_i     = alpha_i T_i                                               */
/*   dC/dalpha_i = T_i c_i - (sum_{j>i} alpha_j T_j c_j + T_{n+1} bg)/(1-alpha_i) */
/* alpha = min(0.99, sigma e^power): a clamped alpha has zero derivative;     */
/* otherwise dalpha/dsigma = e^power and dalpha/dpower = alpha, with          */
/* power = -(Cxx dx^2 + 2 Cxy dx dy + Cyy dy^2)/2 and dx = mean x - px:       */
/*   dpower/dCxx = -dx^2/2, dpower/dCxy = -dx dy, dpower/dCyy = -dy^2/2,     */
/*   dpower/d(mean x) = -(Cxx dx + Cxy dy), dpower/d(mean y) = -(Cxy dx + Cyy dy). */
/* Outputs accumulate into g2d[g*9 + (mx, my, Cxx, Cxy, Cyy, sigma, r, g, b)].  */
/* tiles (n_sel >= 0): only those tiles' pixels are differentiated (the others  */
/* are taken to have zero dL/dimage).                                          */
/* ------------------------------------------------------------------------ */
void orc_blend_backward(int width, int height, const int64_t *ranges, const uint32_t *sorted_vals,
                        const double *rec, const double *bg, const double *dL_dimage, double *g2d,
                        const int32_t *tiles, int64_t n_sel) {
    int TX = (width + TILE - 1) / TILE, TY = (height + TILE - 1) / TILE;
    int64_t npix = (int64_t)width * height;
    int64_t cap = longest_list(ranges, TX * TY);
    int64_t count = n_sel >= 0 ? n_sel : (int64_t)TX * TY;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap + 1));
    double *al = (double *)malloc(sizeof(double) * (size_t)(cap + 1));
    double *ex = (double *)malloc(sizeof(double) * (size_t)(cap + 1));
    int *cl = (int *)malloc(sizeof(int) * (size_t)(cap + 1));
    double *Ts = (double *)malloc(sizeof(double) * (size_t)(cap + 2));
    for (int64_t sidx = 0; sidx < count; ++sidx) {
        int t = n_sel >= 0 ? tiles[sidx] : (int)sidx;
        int tx = t % TX, ty = t / TX;
        const uint32_t *list = sorted_vals + ranges[2 * t];
        int64_t len = ranges[2 * t + 1] - ranges[2 * t];
        for (int py = ty * TILE; py < (ty + 1) * TILE && py < height; ++py)
            for (int px = tx * TILE; px < (tx + 1) * TILE && px < width; ++px) {
                /* forward, recording the blended entries */
                double T = 1.0;
                int64_t nb = 0;
                for (int64_t j = 0; j < len; ++j) {
                    const double *g = rec + 9 * (int64_t)list[j];
                    double dx = g[0] - px, dy = g[1] - py;
                    double power = -0.5 * quad_form(g, dx, dy);
                    if (power > 0.0) continue;
                    double e = exp(power);
                    double alpha = g[5] * e;
                    int clamped = 0;
                    if (alpha > ALPHA_MAX) { alpha = ALPHA_MAX; clamped = 1; }
                    if (alpha < TAU) continue;
                    double Tn = T * (1.0 - alpha);
                    if (Tn < T_STOP) break;
                    idx[nb] = j; al[nb] = alpha; ex[nb] = e; cl[nb] = clamped; Ts[nb] = T;
                    ++nb;
                    T = Tn;
                }
                Ts[nb] = T;
                int64_t pix = (int64_t)py * width + px;
                double G[3] = {dL_dimage[pix], dL_dimage[npix + pix], dL_dimage[2 * npix + pix]};
                /* back to front */
                double behind[3] = {T * bg[0], T * bg[1], T * bg[2]};
                for (int64_t k = nb - 1; k >= 0; --k) {
                    int64_t gid = list[idx[k]];
                    const double *g = rec + 9 * gid;
                    double *o = g2d + 9 * gid;
                    double a = al[k], Ti = Ts[k];
                    double dLda = 0.0;
                    for (int ch = 0; ch < 3; ++ch) {
                        o[6 + ch] += a * Ti * G[ch];
                        dLda += G[ch] * (Ti * g[6 + ch] - behind[ch] / (1.0 - a));
                    }
                    for (int ch = 0; ch < 3; ++ch) behind[ch] += a * Ti * g[6 + ch];
                    if (cl[k]) continue;
                    double dx = g[0] - px, dy = g[1] - py;
                    o[5] += dLda * ex[k];
                    double dLdp = dLda * a;
                    o[2] += dLdp * (-0.5 * dx * dx);
                    o[3] += dLdp * (-dx * dy);
                    o[4] += dLdp * (-0.5 * dy * dy);
                    o[0] += dLdp * (-(g[2] * dx + g[3] * dy));
                    o[1] += dLdp * (-(g[3] * dx + g[4] * dy));
                }
            }
    }
    free(idx); free(al); free(ex); free(cl); free(Ts);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the preprocess (per Gaussian), from g2d (gradients of mean x, */
/* mean y, Cxx, Cxy, Cyy, opacity, r, g, b) to the scene parameters.        */
/* Frozen: the tile extent (no gradient through Th, s or the rectangle), the */
/* EWA clamp branch and the colour clamp at 0.                               */
/* Outputs are [C][N] like the inputs; d_sh is [(d+1)^2][3][N].               */
/* ------------------------------------------------------------------------ */
static void rot_partials(const double q[4], double dR[4][3][3]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double Rw[3][3] = {{0, -2 * z, 2 * y}, {2 * z, 0, -2 * x}, {-2 * y, 2 * x, 0}};
    double Rx[3][3] = {{0, 2 * y, 2 * z}, {2 * y, -4 * x, -2 * w}, {2 * z, 2 * w, -4 * x}};
    double Ry[3][3] = {{-4 * y, 2 * x, 2 * w}, {2 * x, 0, 2 * z}, {-2 * w, 2 * z, -4 * y}};
    double Rz[3][3] = {{-4 * z, -2 * w, 2 * x}, {2 * w, -4 * z, 2 * y}, {2 * x, 2 * y, 0}};
    memcpy(dR[0], Rw, sizeof(Rw));
    memcpy(dR[1], Rx, sizeof(Rx));
    memcpy(dR[2], Ry, sizeof(Ry));
    memcpy(dR[3], Rz, sizeof(Rz));
}

void orc_preprocess_backward(int64_t n, const float *means, const float *log_scales,
                             const float *quats, const float *opacity_logits, const float *sh,
                             int sh_degree, const float *cam, int width, int height,
                             const int32_t *flags, const double *g2d, double *d_means,
                             double *d_log_scales, double *d_quats, double *d_opacity_logits,
                             double *d_sh) {
    double W[3][3], t[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) W[i][j] = cam[4 * i + j];
        t[i] = cam[4 * i + 3];
    }
    double fx = cam[12], fy = cam[13];
    int nsh = (sh_degree + 1) * (sh_degree + 1);
    double campos[3];
    for (int j = 0; j < 3; ++j) campos[j] = -(W[0][j] * t[0] + W[1][j] * t[1] + W[2][j] * t[2]);

    for (int64_t g = 0; g < n; ++g) {
        for (int k = 0; k < 3; ++k) d_means[k * n + g] = d_log_scales[k * n + g] = 0.0;
        for (int k = 0; k < 4; ++k) d_quats[k * n + g] = 0.0;
        d_opacity_logits[g] = 0.0;
        for (int k = 0; k < nsh * 3; ++k) d_sh[(int64_t)k * n + g] = 0.0;
        if (flags[g] != 2) continue;
        const double *G = g2d + 9 * g;
        double mu[3] = {means[g], means[n + g], means[2 * n + g]};
        double p[3];
        for (int i = 0; i < 3; ++i) p[i] = W[i][0] * mu[0] + W[i][1] * mu[1] + W[i][2] * mu[2] + t[i];

        /* forward quantities again */
        double s3[3] = {exp((double)log_scales[g]), exp((double)log_scales[n + g]),
                        exp((double)log_scales[2 * n + g])};
        double q0[4] = {quats[g], quats[n + g], quats[2 * n + g], quats[3 * n + g]};
        double qn = q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3], qr = sqrt(qn);
        double q[4];
        int qdegenerate = !(qn > 0.0);
        for (int k = 0; k < 4; ++k) q[k] = qdegenerate ? (k == 0) : q0[k] / qr;
        double w = q[0], x = q[1], y = q[2], z = q[3];
        double R[3][3] = {
            {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
            {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
            {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
        double M[3][3], S3[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = R[i][j] * s3[j];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                S3[i][j] = 0.0;
                for (int k = 0; k < 3; ++k) S3[i][j] += M[i][k] * M[j][k];
            }
        double limx = FRUSTUM_SLACK * ((0.5 * width) / fx), limy = FRUSTUM_SLACK * ((0.5 * height) / fy);
        double txz = p[0] / p[2], tyz = p[1] / p[2];
        int clx = 0, cly = 0;
        if (txz < -limx) { txz = -limx; clx = -1; }
        if (txz > limx) { txz = limx; clx = 1; }
        if (tyz < -limy) { tyz = -limy; cly = -1; }
        if (tyz > limy) { tyz = limy; cly = 1; }
        double xc = txz * p[2], yc = tyz * p[2];
        double J[2][3] = {{fx / p[2], 0.0, -(fx * xc) / (p[2] * p[2])},
                          {0.0, fy / p[2], -(fy * yc) / (p[2] * p[2])}};
        double T[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) {
                T[i][j] = 0.0;
                for (int k = 0; k < 3; ++k) T[i][j] += J[i][k] * W[k][j];
            }
        double S2[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                S2[i][j] = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) S2[i][j] += T[i][k] * S3[k][l] * T[j][l];
            }
        double a = S2[0][0] + DILATION, b = S2[0][1], c = S2[1][1] + DILATION;
        double det = a * c - b * b, d2 = det * det;

        double dp[3] = {0.0, 0.0, 0.0};
        /* mean2d: u = fx p0/p2 + cx, v = fy p1/p2 + cy */
        dp[0] += G[0] * fx / p[2];
        dp[1] += G[1] * fy / p[2];
        dp[2] += -G[0] * fx * p[0] / (p[2] * p[2]) - G[1] * fy * p[1] / (p[2] * p[2]);

        /* conic = (Cxx, Cxy, Cyy) = (c, -b, a) / det, det = a c - b^2  ->  dL/d(a, b, c) */
        double gxx = G[2], gxy = G[3], gyy = G[4];
        double ga = gxx * (-c * c / d2) + gxy * (b * c / d2) + gyy * (-b * b / d2);
        double gb = gxx * (2.0 * b * c / d2) + gxy * (-(det + 2.0 * b * b) / d2) +
                    gyy * (2.0 * a * b / d2);
        double gc = gxx * (-b * b / d2) + gxy * (a * b / d2) + gyy * (-a * a / d2);
        /* symmetric matrix gradient of Sigma2 (b occupies both off-diagonals) */
        double G2[2][2] = {{ga, 0.5 * gb}, {0.5 * gb, gc}};
        /* dL/dSigma3 = T^T G2 T ; dL/dT = 2 G2 T Sigma3 */
        double G3[3][3], GT[2][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                G3[i][j] = 0.0;
                for (int k = 0; k < 2; ++k)
                    for (int l = 0; l < 2; ++l) G3[i][j] += T[k][i] * G2[k][l] * T[l][j];
            }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) {
                GT[i][j] = 0.0;
                for (int k = 0; k < 2; ++k)
                    for (int l = 0; l < 3; ++l) GT[i][j] += 2.0 * G2[i][k] * T[k][l] * S3[l][j];
            }
        /* T = J W  ->  dL/dJ = dL/dT W^T */
        double GJ[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) {
                GJ[i][j] = 0.0;
                for (int k = 0; k < 3; ++k) GJ[i][j] += GT[i][k] * W[j][k];
            }
        /* J00 = fx/p2, J11 = fy/p2; J02 = -fx xc/p2^2 with xc = p0 (unclamped) or
           +-limx p2 (clamped); likewise J12 */
        dp[2] += GJ[0][0] * (-fx / (p[2] * p[2])) + GJ[1][1] * (-fy / (p[2] * p[2]));
        if (clx == 0) {
            dp[0] += GJ[0][2] * (-fx / (p[2] * p[2]));
            dp[2] += GJ[0][2] * (2.0 * fx * p[0] / (p[2] * p[2] * p[2]));
        } else {
            dp[2] += GJ[0][2] * (fx * clx * limx / (p[2] * p[2]));
        }
        if (cly == 0) {
            dp[1] += GJ[1][2] * (-fy / (p[2] * p[2]));
            dp[2] += GJ[1][2] * (2.0 * fy * p[1] / (p[2] * p[2] * p[2]));
        } else {
            dp[2] += GJ[1][2] * (fy * cly * limy / (p[2] * p[2]));
        }
        /* Sigma3 = M M^T -> dL/dM = 2 G3 M ; M = R diag(s) */
        double GM[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                GM[i][j] = 0.0;
                for (int k = 0; k < 3; ++k) GM[i][j] += 2.0 * G3[i][k] * M[k][j];
            }
        for (int j = 0; j < 3; ++j) {
            double gs = 0.0;
            for (int i = 0; i < 3; ++i) gs += GM[i][j] * R[i][j];
            d_log_scales[j * n + g] = gs * s3[j];
        }
        double GR[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) GR[i][j] = GM[i][j] * s3[j];
        double dR[4][3][3], gq[4];
        rot_partials(q, dR);
        for (int k = 0; k < 4; ++k) {
            gq[k] = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) gq[k] += GR[i][j] * dR[k][i][j];
        }
        /* normalisation q = q0/|q0|: dq/dq0 = (I - q q^T)/|q0| */
        if (!qdegenerate) {
            double qg = gq[0] * q[0] + gq[1] * q[1] + gq[2] * q[2] + gq[3] * q[3];
            for (int k = 0; k < 4; ++k) d_quats[k * n + g] = (gq[k] - q[k] * qg) / qr;
        }

        /* opacity: sigma = 1/(1+exp(-o)) */
        double sg = 1.0 / (1.0 + exp(-(double)opacity_logits[g]));
        d_opacity_logits[g] = G[5] * sg * (1.0 - sg);

        /* colour */
        double dv[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
        double len = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        double dir[3] = {dv[0] / len, dv[1] / len, dv[2] / len};
        double Y[(SH_LMAX + 1) * (SH_LMAX + 1)], dY[3 * (SH_LMAX + 1) * (SH_LMAX + 1)];
        orc_sh_basis(sh_degree, dir, Y, dY);
        double gdir[3] = {0.0, 0.0, 0.0};
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int k = 0; k < nsh; ++k) acc += (double)sh[((int64_t)k * 3 + ch) * n + g] * Y[k];
            if (acc + 0.5 < 0.0) continue; /* clamped channel */
            double gc_ = G[6 + ch];
            for (int k = 0; k < nsh; ++k) {
                d_sh[((int64_t)k * 3 + ch) * n + g] = gc_ * Y[k];
                for (int e = 0; e < 3; ++e)
                    gdir[e] += gc_ * (double)sh[((int64_t)k * 3 + ch) * n + g] * dY[3 * k + e];
            }
        }
        /* dir = dv/|dv|: d dir/d dv = (I - dir dir^T)/|dv| */
        double gd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
        double gmu[3];
        for (int e = 0; e < 3; ++e) gmu[e] = (gdir[e] - dir[e] * gd) / len;
        /* p = W mu + t */
        for (int j = 0; j < 3; ++j)
            d_means[j * n + g] = gmu[j] + W[0][j] * dp[0] + W[1][j] * dp[1] + W[2][j] * dp[2];
    }
}

/* The oracle's constants, for comparison with the values printed in the paper:
 * tau, early-exit T, LUT bins, 2 pi, alpha clamp, near plane, dilation,
 * frustum slack, discriminant floor, tile size. */
/* T_upper look-up table (Sec. 3.4): LUT_BINS uniform depth bins over
 * [0, lut_depth_max); bin = min(floor(LUT_BINS depth / lut_depth_max),
 * LUT_BINS - 1) of the float32 depth; each bin takes the largest max_t of the
 * Gaussians in it that were blended somewhere (max_t > 0), raising lut[]
 * (the caller initialises it, 0 for a first view).  Several views accumulate
 * by calling once per view. */
void orc_t_upper_accumulate(int64_t n, const float *depth, const double *max_t, double lut_depth_max,
                            double *lut) {
    for (int64_t i = 0; i < n; ++i) {
        if (!(max_t[i] > 0.0)) continue;
        const double f = ((double)depth[i] * LUT_BINS) / lut_depth_max;
        const int bin = f >= LUT_BINS - 1 ? LUT_BINS - 1 : (int)floor(f);
        if (max_t[i] > lut[bin]) lut[bin] = max_t[i];
    }
}

/* Threads the blend and preprocess loops run on: 1 in the plain build, the
   OpenMP team size in the OpenMP build used for timing. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_constants(double *out) {
    out[0] = TAU; out[1] = T_STOP; out[2] = LUT_BINS; out[3] = TWO_PI; out[4] = ALPHA_MAX;
    out[5] = NEAR_Z; out[6] = DILATION; out[7] = FRUSTUM_SLACK; out[8] = LAMBDA_FLOOR; out[9] = TILE;
}
