"""Pins of the FP64 oracle against things other than itself: values printed in
the paper, closed forms, library routines, quadrature and brute force.

None of these tests touches the GPU."""
import json
import math
import os

import numpy as np
import pytest

from paper_2604_18980_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


# --------------------------------------------------------------------------- constants
def test_constants_match_paper(O):
    """tau = 1/255 and the 1e-4 early exit (Sec. 2.1), 20 LUT bins over
    [0, 100] (Sec. 3.4) and the 2 pi of eq. (9)-(10), as printed."""
    gold = json.load(open(GOLDEN))
    c = O.constants()
    assert c["tau"] == gold["tau"]["value"] == 1.0 / 255.0
    assert c["t_stop"] == gold["early_exit_T"]["value"]
    assert c["lut_bins"] == gold["t_upper_bins"]["value"]
    assert c["two_pi"] == gold["eq9_factor"]["value"] == 2 * math.pi
    assert O.Mode().lut_depth_max == gold["t_upper_depth_range"]["value"][1]
    assert c["tile"] == 16


# --------------------------------------------------------------------------- SH colour basis
def test_sh_basis_matches_scipy(O):
    """Real SH with the Condon-Shortley phase: Y_l^{+m} = sqrt2 Re Y_l^m,
    Y_l^{-m} = sqrt2 Im Y_l^m of scipy's complex harmonics."""
    import scipy.special as sp
    rng = np.random.default_rng(1)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        Y = O.sh_basis(3, d)
        th, ph = np.arccos(d[2]), np.arctan2(d[1], d[0])
        for l in range(4):
            for m in range(-l, l + 1):
                c = sp.sph_harm_y(l, abs(m), th, ph)
                ref = c.real if m == 0 else np.sqrt(2) * (c.real if m > 0 else c.imag)
                assert abs(Y[l * l + l + m] - ref) < 1e-12


def test_sh_basis_orthonormal(O):
    """Gram matrix over the sphere is the identity (Gauss-Legendre in cos(theta)
    x uniform phi: exact for these polynomial degrees)."""
    x, w = np.polynomial.legendre.leggauss(12)
    nphi = 16
    G = np.zeros((16, 16))
    for z, wz in zip(x, w):
        for k in range(nphi):
            ph = 2 * np.pi * k / nphi
            s = np.sqrt(1 - z * z)
            Y = O.sh_basis(3, np.array([s * np.cos(ph), s * np.sin(ph), z]))
            G += np.outer(Y, Y) * wz * (2 * np.pi / nphi)
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_gradient_tangential_fd(O):
    rng = np.random.default_rng(2)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        Y, dY = O.sh_basis(3, d, with_grad=True)
        t = rng.normal(size=3)
        t -= d * (t @ d)
        t /= np.linalg.norm(t)
        h = 1e-6
        yp = O.sh_basis(3, (d + h * t) / np.linalg.norm(d + h * t))
        ym = O.sh_basis(3, (d - h * t) / np.linalg.norm(d - h * t))
        assert np.abs((yp - ym) / (2 * h) - dY @ t).max() < 1e-8


# --------------------------------------------------------------------------- projection
def _single(mu, log_scale, quat, logit=3.0, sh_dc=(0.0, 0.0, 0.0)):
    sc = scenes.Scene(np.array(mu, np.float32).reshape(3, 1),
                      np.array(log_scale, np.float32).reshape(3, 1),
                      np.array(quat, np.float32).reshape(4, 1),
                      np.array([logit], np.float32),
                      np.array(sh_dc, np.float32).reshape(1, 3, 1), 0)
    return sc


def test_isotropic_on_axis_closed_form(O):
    """A sphere of radius s at depth z on the optical axis projects to
    (fx s / z)^2 I + 0.3 I, centred on the principal point."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 256, 256)
    for z, ls in [(5.0, -2.0), (3.0, -3.5), (10.0, 0.0)]:
        pre = O.preprocess(_single([0, 0, z], [ls] * 3, [1, 0, 0, 0]), cam)
        s = math.exp(np.float32(ls))
        fx = float(cam["fx"])
        var = (fx * s / z) ** 2 + 0.3
        assert pre.flags[0] >= 1
        np.testing.assert_allclose(pre.cov2d[0], [var, 0, var], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(pre.conic[0], [1 / var, 0, 1 / var], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(pre.mean2d[0], [float(cam["cx"]), float(cam["cy"])], atol=1e-12)
        assert pre.depth[0] == pytest.approx(z, rel=1e-15)
        assert pre.extent[0] == pytest.approx(3 * math.sqrt(var + math.sqrt(0.1)), rel=1e-12)


def test_ewa_matches_monte_carlo_projection(O):
    """Sample the 3D Gaussian built from scipy's rotation convention, push the
    samples through the pinhole camera, and compare the sample covariance of
    the image points with the oracle's 2D covariance (minus the 0.3 dilation).
    Small s/z makes the first-order (EWA) projection accurate."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(3)
    cam = scenes.look_camera((0.3, -0.2, -6.0), (0.05, 0.02, 1.0), (0, -1, 0), 320, 240)
    vm = np.asarray(cam["viewmat"], np.float64).reshape(3, 4)
    Rc, tc = vm[:, :3], vm[:, 3]
    fx, fy, cx, cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    for trial in range(3):
        mu = rng.uniform(-0.5, 0.5, 3)
        ls = rng.uniform(-4.5, -3.0, 3)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        sc = _single(mu, ls, q)
        pre = O.preprocess(sc, cam)
        mu64 = sc.means[:, 0].astype(np.float64)
        s64 = np.exp(sc.log_scales[:, 0].astype(np.float64))
        q64 = sc.quats[:, 0].astype(np.float64)
        R = Rotation.from_quat([q64[1], q64[2], q64[3], q64[0]]).as_matrix()
        S3 = R @ np.diag(s64 ** 2) @ R.T
        pts = rng.multivariate_normal(mu64, S3, size=400_000)
        pc = pts @ Rc.T + tc
        uv = np.stack([fx * pc[:, 0] / pc[:, 2] + cx, fy * pc[:, 1] / pc[:, 2] + cy])
        emp = np.cov(uv)
        ora = np.array([[pre.cov2d[0, 0] - 0.3, pre.cov2d[0, 1]],
                        [pre.cov2d[0, 1], pre.cov2d[0, 2] - 0.3]])
        scale = np.sqrt(np.diag(ora)).max() ** 2
        assert np.abs(emp - ora).max() / scale < 0.02
        pc0 = Rc @ mu64 + tc
        np.testing.assert_allclose(pre.mean2d[0], [fx * pc0[0] / pc0[2] + cx, fy * pc0[1] / pc0[2] + cy],
                                   rtol=1e-12)


def test_near_cull_and_degenerate_quaternion(O):
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 64, 64)
    assert O.preprocess(_single([0, 0, 0.1999], [-2] * 3, [1, 0, 0, 0]), cam).flags[0] == 0
    assert O.preprocess(_single([0, 0, 0.2001], [-2] * 3, [1, 0, 0, 0]), cam).flags[0] >= 1
    a = O.preprocess(_single([0.1, 0.2, 4], [-2, -3, -2.5], [0, 0, 0, 0]), cam)
    b = O.preprocess(_single([0.1, 0.2, 4], [-2, -3, -2.5], [1, 0, 0, 0]), cam)
    np.testing.assert_array_equal(a.cov2d, b.cov2d)
    nan = O.preprocess(_single([np.nan, 0, 4], [-2] * 3, [1, 0, 0, 0]), cam)
    assert nan.flags[0] == 0


# --------------------------------------------------------------------------- eq. (9)-(10)
def _annulus_integral(a, b, c, sigma, x, h_frac=0.004):
    """Quadrature of alpha over {tau <= alpha < x} on a fine pixel-free grid
    (the integral of eq. (8), evaluated numerically)."""
    cov = np.array([[a, b], [b, c]])
    inv = np.linalg.inv(cov)
    lam = np.linalg.eigvalsh(cov)
    R = math.sqrt(2 * math.log(sigma / O_TAU)) * math.sqrt(lam.max()) * 1.02
    h = h_frac * math.sqrt(lam.min())
    g = np.arange(-R, R + h, h)
    X, Y = np.meshgrid(g, g, indexing="ij")
    q = inv[0, 0] * X * X + 2 * inv[0, 1] * X * Y + inv[1, 1] * Y * Y
    al = sigma * np.exp(-0.5 * q)
    m = (al >= O_TAU) & (al < x)
    return float(al[m].sum() * h * h)


O_TAU = 1.0 / 255.0


@pytest.mark.parametrize("a,b,c,sigma,K,Tu", [
    (4.3, 0.0, 1.3, 0.5, 0.1, 1.0),
    (9.3, 2.0, 4.3, 0.8, 1.0, 1.0),
    (0.9, 0.1, 0.7, 0.3, 0.1, 1.0),
    (25.3, -6.0, 16.3, 0.9, 3.0, 0.4),
])
def test_threshold_solves_eq5_with_quadrature(O, a, b, c, sigma, K, Tu):
    """Th of eq. (10) is the largest x with T_up * integral_{tau <= alpha < x} alpha <= K
    (eq. (5) with the integral of eq. (8)); found here by bisection on a
    numerically integrated score."""
    det = a * c - b * b
    lut = np.full(20, Tu, np.float32)
    keep, th, s = O.adagscale(det, sigma, 5.0, K, lut)
    assert keep
    lo, hi = O_TAU, sigma
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if np.float32(Tu) * _annulus_integral(a, b, c, sigma, mid) <= K:
            lo = mid
        else:
            hi = mid
    assert th == pytest.approx(lo, rel=2e-3)
    # closed-form annulus integral of eq. (9) against the quadrature, at a few x
    for x in (0.02, 0.5 * sigma, sigma):
        quad = _annulus_integral(a, b, c, sigma, x)
        assert quad == pytest.approx(2 * math.pi * math.sqrt(det) * (x - O_TAU), rel=2e-3)


def test_scale_factor_is_contour_ratio(O):
    """s shrinks the alpha = tau contour onto the alpha = Th contour: along any
    direction the radius where alpha drops to Th, over the radius where it
    drops to tau, equals s (bisection on alpha along the ray)."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        L = rng.normal(size=(2, 2))
        cov = L @ L.T + np.eye(2) * 0.5
        a, b, c = cov[0, 0], cov[0, 1], cov[1, 1]
        sigma = rng.uniform(0.05, 0.99)
        K = rng.uniform(0.01, 2.0)
        keep, th, s = O.adagscale(a * c - b * b, sigma, 3.0, K)
        if not keep:
            assert th >= sigma
            continue
        u = rng.normal(size=2)
        u /= np.linalg.norm(u)
        inv = np.linalg.inv(cov)

        def radius(t):
            lo, hi = 0.0, 1e3
            for _ in range(200):
                m = 0.5 * (lo + hi)
                if sigma * math.exp(-0.5 * m * m * (u @ inv @ u)) >= t:
                    lo = m
                else:
                    hi = m
            return lo
        assert radius(th) / radius(O_TAU) == pytest.approx(s, rel=1e-9)


def test_threshold_special_cases(O):
    """Th >= tau always; K = 0 gives Th = tau and s = 1 exactly; Th >= opacity
    drops the Gaussian (Sec. 3.3); an empty LUT bin (T_up = 0) drops it too."""
    keep, th, s = O.adagscale(4.0, 0.5, 3.0, 0.0)
    assert keep and th == O_TAU and s == 1.0
    rng = np.random.default_rng(5)
    for _ in range(200):
        det = rng.uniform(0.1, 1e4)
        sigma = rng.uniform(0.0, 1.0)
        K = rng.uniform(0, 10)
        keep, th, s = O.adagscale(det, sigma, 3.0, K)
        assert th >= O_TAU
        assert keep == (th < sigma)
        if keep:
            assert 0.0 < s <= 1.0
    assert not O.adagscale(4.0, 0.5, 3.0, 0.1, np.zeros(20, np.float32))[0]


def test_lut_bin_lookup(O):
    """T_up is piecewise constant over 20 uniform depth bins of [0, D_max]
    (Sec. 3.4); depths beyond D_max use the last bin."""
    lut = np.arange(1, 21, dtype=np.float32) / 20
    det, sigma, K = 9.0, 0.9, 0.05
    for depth, b in [(0.3, 0), (4.99, 0), (5.0, 1), (52.0, 10), (99.9, 19), (150.0, 19)]:
        _, th, _ = O.adagscale(det, sigma, depth, K, lut, 100.0)
        expect_tu = float(lut[b])
        assert th == pytest.approx(K / (expect_tu * 2 * math.pi * 3.0) + O_TAU, rel=1e-14)
    _, th, _ = O.adagscale(det, sigma, 52.0, K, lut, 1000.0)
    assert th == pytest.approx(K / (float(lut[1]) * 2 * math.pi * 3.0) + O_TAU, rel=1e-14)


# --------------------------------------------------------------------------- blend closed forms
def _pipeline_single(O, gaussians, cam, bg=(0, 0, 0)):
    """Build a Frame from explicit 2D records (mean x, mean y, A, beta, gamma,
    opacity, r, g, b), rounded to float32, where the inverse covariance is
    [[A, A beta], [A beta, A beta^2 + gamma]]; the blend reads it as the conic
    (Cxx, Cxy, Cyy) of that matrix."""
    n = len(gaussians)
    rec = np.zeros((n, 9))
    for i, g in enumerate(gaussians):
        rec[i] = g
    rec = rec.astype(np.float32).astype(np.float64)
    A, beta, gamma = rec[:, 2].copy(), rec[:, 3].copy(), rec[:, 4].copy()
    rec[:, 2], rec[:, 3], rec[:, 4] = A, A * beta, A * beta * beta + gamma
    ntiles = O.num_tiles(cam)
    sv = np.arange(n, dtype=np.uint32)
    rg = np.zeros((ntiles, 2), np.int64)
    rg[:, 1] = n
    fr = O.Frame(None, None, None, None, sv, rg)
    return O.blend(fr, cam, bg, rec=rec)


def test_blend_single_gaussian_at_centre(O):
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 16, 16)
    for sigma in (0.2, 0.7, 0.995):
        img, T, nc, *_ = _pipeline_single(O, [(5, 7, 0.5, 0.1, 0.3, sigma, 0.2, 0.5, 0.9)], cam)
        a = min(0.99, float(np.float32(sigma)))
        np.testing.assert_allclose(img[:, 7, 5], a * np.float32([0.2, 0.5, 0.9]).astype(np.float64),
                                   rtol=1e-14)
        assert T[7, 5] == pytest.approx(1 - a, rel=1e-14)
        assert nc[7, 5] == 1


def test_blend_two_gaussians_closed_form(O):
    """C = a1 c1 + a2 (1 - a1) c2 + (1 - a1)(1 - a2) bg with a_i = s_i exp(power_i),
    power_i = -d^T M_i d / 2 evaluated as a plain matrix product."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 16, 16)
    g1 = (3.0, 4.0, 0.2, 0.05, 0.1, 0.6, 1.0, 0.0, 0.2)
    g2 = (6.0, 2.0, 0.1, -0.02, 0.3, 0.8, 0.0, 1.0, 0.4)
    bg = (0.1, 0.2, 0.3)
    img, T, nc, *_ = _pipeline_single(O, [g1, g2], cam, bg)
    for py, px in [(4, 3), (2, 6), (5, 5), (0, 0)]:
        col = np.zeros(3)
        Tt = 1.0
        for g in (g1, g2):
            g = np.float32(g).astype(np.float64)
            d = np.array([g[0] - px, g[1] - py])
            M = np.array([[g[2], g[2] * g[3]], [g[2] * g[3], g[2] * g[3] ** 2 + g[4]]])
            a = min(0.99, g[5] * math.exp(-0.5 * d @ M @ d))
            if a < O_TAU:
                continue
            col += a * Tt * g[6:9]
            Tt *= 1 - a
        np.testing.assert_allclose(img[:, py, px], col + Tt * np.array(bg), rtol=1e-13, atol=1e-15)


def test_blend_early_exit_and_clamp(O):
    """Stacked opaque Gaussians: alpha clamps to 0.99, T goes 1 -> 0.01 -> 1e-4;
    the third would push T below 1e-4, so the pixel stops with two blended."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 16, 16)
    g = (8.0, 8.0, 0.5, 0.0, 0.5, 0.999, 1.0, 1.0, 1.0)
    img, T, nc, *_ = _pipeline_single(O, [g, g, g, g], cam)
    assert nc[8, 8] == 2
    assert T[8, 8] == pytest.approx(1e-4, rel=1e-10)
    assert T[8, 8] >= 1e-4
    assert img[0, 8, 8] == pytest.approx(0.99 + 0.99 * 0.01, rel=1e-12)


def test_blend_counts_stacked(O):
    """Work counts on the stacked case: at the centre four entries are
    evaluated (two blended, the third stops the pixel, the fourth is never
    reached -> 3 evaluated); far from the centre every alpha is below tau, so
    all four are evaluated and none blended."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 16, 16)
    g = (8.0, 8.0, 0.5, 0.0, 0.5, 0.999, 1.0, 1.0, 1.0)
    rec = np.asarray([g] * 4, np.float64).astype(np.float32).astype(np.float64)
    rg = np.zeros((O.num_tiles(cam), 2), np.int64)
    rg[:, 1] = 4
    fr = O.Frame(None, None, None, None, np.arange(4, dtype=np.uint32), rg)
    ev, bl, mg = O.blend_counts(fr, cam, rec=rec)
    assert ev[8, 8] == 3 and bl[8, 8] == 2
    assert ev[0, 0] == 4 and bl[0, 0] == 0


def test_blend_counts_invariants_tiny(O):
    """blended <= n_contrib <= evaluated per pixel; blended > 0 iff n_contrib > 0;
    evaluated equals the blend's own count."""
    sc, cam = scenes.tiny_scene(seed=5)
    fr = O.render(sc, cam, O.Mode(adagscale=True, K=0.1))
    ev, bl, mg = O.blend_counts(fr, cam)
    np.testing.assert_array_equal(ev, fr.evals)
    assert np.all(bl <= fr.n_contrib) and np.all(fr.n_contrib <= ev)
    np.testing.assert_array_equal(bl > 0, fr.n_contrib > 0)
    assert bl.sum() > 0


def test_blend_skips_below_tau(O):
    """A Gaussian whose alpha stays below 1/255 everywhere contributes nothing."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 16, 16)
    img, T, nc, *_ = _pipeline_single(O, [(8, 8, 0.5, 0, 0.5, 1.0 / 256, 1, 1, 1)], cam)
    assert np.all(img == 0) and np.all(T == 1) and np.all(nc == 0)


# --------------------------------------------------------------------------- pipeline vs brute force
@pytest.mark.parametrize("adagscale,K", [(False, 0.0), (True, 0.1), (True, 1.0)])
def test_tile_pipeline_equals_bruteforce(O, adagscale, K):
    """Emit + sort + ranges + blend equals blending, per pixel, every Gaussian
    whose tile rectangle holds the pixel's tile, ordered by (depth, index)."""
    sc, cam = scenes.tiny_scene(n=400, seed=11)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 64, 48)
    fr = O.render(sc, cam, O.Mode(adagscale=adagscale, K=K), bg=(0.1, 0.0, 0.3))
    img, T, nc = O.blend_bruteforce(fr.pre, cam, 1, bg=(0.1, 0.0, 0.3))
    np.testing.assert_array_equal(fr.image, img)
    np.testing.assert_array_equal(fr.final_T, T)
    np.testing.assert_array_equal(fr.n_contrib, nc)


def test_emit_sort_ranges_against_numpy(O):
    sc, cam = scenes.tiny_scene(seed=3)
    pre = O.preprocess(sc, cam, O.Mode(adagscale=True, K=0.3))
    keys, vals = O.emit(pre, cam)
    assert keys.size == pre.tiles_touched.sum()
    # emitted multiset: every tile of every rectangle exactly once
    TX = (cam["width"] + 15) // 16
    exp = []
    for g in np.nonzero(pre.tiles_touched)[0]:
        x0, y0, x1, y1 = pre.rect[g]
        d = np.float32(pre.depth[g]).view(np.uint32)
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                exp.append(((ty * TX + tx) << 32) | int(d))
    np.testing.assert_array_equal(keys, np.array(exp, np.uint64))
    sk, sv = O.sort(keys, vals)
    order = np.lexsort((vals, keys))
    np.testing.assert_array_equal(sk, keys[order])
    np.testing.assert_array_equal(sv, vals[order])
    rg = O.ranges(sk, O.num_tiles(cam))
    tiles = (sk >> np.uint64(32)).astype(np.int64)
    for t in range(O.num_tiles(cam)):
        assert rg[t, 0] == np.searchsorted(tiles, t, "left") or rg[t, 0] == rg[t, 1] == 0
        assert rg[t, 1] - rg[t, 0] == np.count_nonzero(tiles == t)


def test_blend_invariants_tiny(O):
    sc, cam = scenes.tiny_scene()
    fr = O.render(sc, cam)
    assert np.all(fr.final_T >= 1e-4) and np.all(fr.final_T <= 1)
    lens = fr.ranges[:, 1] - fr.ranges[:, 0]
    TX = 8
    for py in range(0, 128, 7):
        for px in range(0, 128, 5):
            t = (py // 16) * TX + px // 16
            assert fr.n_contrib[py, px] <= lens[t]
            assert fr.evals[py, px] <= lens[t]
    assert np.all(fr.image >= 0)


def test_unrestricted_blend_is_close(O):
    """Diagnostic: blending every Gaussian (no tile rectangles) differs from the
    tile pipeline only by the alpha mass outside the 3-sigma extent."""
    sc, cam = scenes.tiny_scene(n=300, seed=2)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 48, 48)
    fr = O.render(sc, cam)
    img2, _, _ = O.blend_bruteforce(fr.pre, cam, 2)
    assert np.abs(img2 - fr.image).max() < 0.05


# --------------------------------------------------------------------------- metrics
def test_psnr_ssim_definitions(O):
    rng = np.random.default_rng(6)
    a = rng.uniform(0, 1, (3, 40, 40))
    b = np.clip(a + 0.01, 0, 1)
    assert O.psnr(a, b) == pytest.approx(10 * np.log10(1 / np.mean((a - b) ** 2)))
    assert O.ssim(a, a) == pytest.approx(1.0, abs=1e-12)
    c1, c2 = np.full((3, 20, 20), 0.3), np.full((3, 20, 20), 0.6)
    C1 = 0.01 ** 2
    assert O.ssim(c1, c2) == pytest.approx((2 * 0.18 + C1) / (0.09 + 0.36 + C1), rel=1e-9)


def test_conic_inverts_covariance(O):
    """conic is Sigma2^-1, and the sum-of-squares record (A, beta, gamma) gives
    the same quadratic form d^T Sigma2^-1 d (numpy's matrix inverse)."""
    sc, cam = scenes.tiny_scene(seed=9)
    pre = O.preprocess(sc, cam)
    m = pre.flags >= 1
    A, B, Cc = pre.conic[m].T
    a, b, c = pre.cov2d[m].T
    np.testing.assert_allclose(A * a + B * b, 1, atol=1e-12)
    np.testing.assert_allclose(A * b + B * c, 0, atol=1e-12)
    np.testing.assert_allclose(B * b + Cc * c, 1, atol=1e-12)
    rng = np.random.default_rng(0)
    for i in np.nonzero(m)[0][:200]:
        inv = np.linalg.inv(np.array([[pre.cov2d[i, 0], pre.cov2d[i, 1]],
                                      [pre.cov2d[i, 1], pre.cov2d[i, 2]]]))
        d = rng.normal(size=2) * 10
        qa, qb, qg = pre.quad[i]
        q = qa * (d[0] + qb * d[1]) ** 2 + qg * d[1] ** 2
        assert q == pytest.approx(d @ inv @ d, rel=1e-10)


@pytest.mark.parametrize("adagscale", [False, True])
def test_rect_covers_extent_disc(O, adagscale):
    """Every pixel within the (scaled) extent of the centre, less one pixel (the
    rectangle rule rounds the centre's far edge to whole pixels), lies in a tile
    of the Gaussian's rectangle, and no rectangle tile lies farther than one
    tile beyond the extent (brute force over pixels)."""
    sc, _ = scenes.tiny_scene(n=150, seed=4)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 100, 70)
    pre = O.preprocess(sc, cam, O.Mode(adagscale=adagscale, K=0.5))
    py, px = np.mgrid[0:70, 0:100]
    for g in np.nonzero(pre.flags == 2)[0]:
        u, v = pre.mean2d[g]
        r = pre.radius[g]
        assert r == math.ceil(pre.extent[g] * pre.scale[g])
        x0, y0, x1, y1 = pre.rect[g]
        e = pre.extent[g] * pre.scale[g] - 1.0
        inside = (np.abs(px - u) <= e) & (np.abs(py - v) <= e)
        tx, ty = px[inside] // 16, py[inside] // 16
        assert np.all((tx >= x0) & (tx < x1) & (ty >= y0) & (ty < y1))
        for t_y in range(y0, y1):
            for t_x in range(x0, x1):
                nx = min(max(u, 16 * t_x), 16 * t_x + 15)
                ny = min(max(v, 16 * t_y), 16 * t_y + 15)
                assert max(abs(nx - u), abs(ny - v)) <= r + 16


# --------------------------------------------------------------------------- T_upper calibration (Sec. 3.4)
def _frame_of(O, gaussians, cam):
    n = len(gaussians)
    rec = np.asarray(gaussians, np.float64).astype(np.float32).astype(np.float64)
    rg = np.zeros((O.num_tiles(cam), 2), np.int64)
    rg[:, 1] = n
    return O.Frame(None, None, None, None, np.arange(n, dtype=np.uint32), rg), rec


def test_max_transmittance_stacked_closed_form(O):
    """Two narrow Gaussians on pixel (5, 5) (alpha < tau one pixel away) and a
    wide one behind: the front one sees T = 1, the second 1 - 0.5 = 0.5 (it
    blends only behind the first), the wide one T = 1 at pixels the narrow
    ones do not reach; a Gaussian below tau everywhere gets 0."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 16, 16)
    g1 = (5.0, 5.0, 20.0, 0.0, 20.0, 0.5, 1, 0, 0)
    g2 = (5.0, 5.0, 20.0, 0.0, 20.0, 0.75, 0, 1, 0)
    g3 = (8.0, 8.0, 0.01, 0.0, 0.01, 0.5, 0, 0, 1)
    g4 = (8.0, 8.0, 0.5, 0.0, 0.5, 1.0 / 256, 1, 1, 1)
    fr, rec = _frame_of(O, [g1, g2, g3, g4], cam)
    mt, _ = O.max_transmittance(fr, cam, rec=rec)
    assert mt[0] == 1.0
    assert mt[1] == 0.5
    assert mt[2] == 1.0
    assert mt[3] == 0.0
    # T after g1 and g2 at (5, 5) is 0.5 * 0.25; g3 there sees at most 1 elsewhere
    img, T, nc, *_ = O.blend(fr, cam, rec=rec)
    a32 = float(np.float32(0.01))  # records hold float32 values
    assert T[5, 5] == pytest.approx(0.5 * 0.25 * (1 - 0.5 * math.exp(-0.5 * a32 * 18)), rel=1e-12)


def test_t_upper_table_bins_and_empty_bins(O):
    """Binning by float32 depth into 20 bins over [0, D_max) with the last bin
    open-ended; the table keeps the largest max T per bin across views, and
    bins no Gaussian reached become 1."""
    depth = np.float32([0.5, 4.9, 5.0, 52.0, 99.0, 250.0, 10.0])
    mt1 = np.array([0.3, 0.9, 0.2, 0.4, 0.6, 0.7, 0.0])
    lut = O.t_upper_accumulate(depth, mt1, 100.0)
    expect = np.zeros(20)
    expect[0], expect[1], expect[10], expect[19] = 0.9, 0.2, 0.4, 0.7
    np.testing.assert_array_equal(lut, expect)
    # a second view raises bins, never lowers them
    lut = O.t_upper_accumulate(np.float32([5.5, 60.0]), np.array([0.1, 0.8]), 100.0, lut)
    expect[12] = 0.8
    np.testing.assert_array_equal(lut, expect)
    fin = O.t_upper_finish(lut)
    assert fin[0] == 0.9 and fin[12] == 0.8 and fin[2] == 1.0 and np.sum(fin == 1.0) == 15


def test_max_transmittance_invariants_tiny(O):
    """On a tiny scene: 0 <= max T <= 1; positive exactly for the Gaussians that
    blend somewhere (brute force over the tile lists); the table built from it
    is an upper bound of every blended Gaussian's max T in its bin."""
    sc, cam = scenes.tiny_scene(seed=7)
    fr = O.render(sc, cam)
    mt, mg = O.max_transmittance(fr, cam)
    assert np.all(mt >= 0) and np.all(mt <= 1)
    # a Gaussian blends somewhere iff some pixel's blend signature includes it:
    # re-blend with that Gaussian's opacity zeroed and look for a change
    rec = fr.pre.record()
    img0 = fr.image
    rng = np.random.default_rng(3)
    for i in rng.choice(np.flatnonzero(fr.pre.tiles_touched > 0), 12, replace=False):
        r2 = rec.copy()
        r2[i, 5] = 0.0
        img, *_ = O.blend(fr, cam, rec=r2)
        changed = bool(np.any(img != img0))
        assert changed == (mt[i] > 0), (i, mt[i])
    d32 = fr.pre.depth_f32
    lut = O.t_upper_finish(O.t_upper_accumulate(d32, mt, 20.0))
    f = d32.astype(np.float64) * 20 / 20.0
    b = np.minimum(np.floor(f), 19).astype(int)
    ok = mt > 0
    assert np.all(mt[ok] <= lut[b[ok]])


# --------------------------------------------------------------------------- ellipse tile test (rule 1)
def _box_min_q(A, beta, gamma, X0, X1, Y0, Y1):
    """Minimum of q(X, Y) = A (X + beta Y)^2 + gamma Y^2 over the box
    [X0, X1] x [Y0, Y1]: 0 if the box holds the centre, else the smallest of
    the four edge minima (each a 1-D quadratic, minimised in closed form and
    clamped into the edge)."""
    q = lambda X, Y: A * (X + beta * Y) ** 2 + gamma * Y * Y
    if X0 <= 0.0 <= X1 and Y0 <= 0.0 <= Y1:
        return 0.0
    best = math.inf
    for X in (X0, X1):  # vertical edges: dq/dY = 0 at Y = -A beta X / (A beta^2 + gamma)
        Y = min(max(-A * beta * X / (A * beta * beta + gamma), Y0), Y1)
        best = min(best, q(X, Y))
    for Y in (Y0, Y1):  # horizontal edges: minimum at X = -beta Y
        X = min(max(-beta * Y, X0), X1)
        best = min(best, q(X, Y))
    return best


def test_ellipse_spans_match_box_minimum(O):
    """The row spans are exactly the tiles whose pixel box [16 tx, 16 tx + 15]
    x [16 ty, 16 ty + 15] holds a point with q <= 2 ln(sigma / t) (a convex
    minimum over the box, computed edge by edge), on random ellipses of every
    orientation and size; tiles within 1e-9 of tangency are not judged."""
    rng = np.random.default_rng(21)
    checked = 0
    for it in range(300):
        sx, sy = np.exp(rng.uniform(-0.5, 3.5, 2))
        th = rng.uniform(0, np.pi)
        cth, sth = np.cos(th), np.sin(th)
        a = cth * cth * sx * sx + sth * sth * sy * sy
        b = cth * sth * (sx * sx - sy * sy)
        c = sth * sth * sx * sx + cth * cth * sy * sy
        det = a * c - b * b
        A, beta, gamma = c / det, -b / c, 1.0 / c
        u, v = rng.uniform(-40, 200, 2)
        sigma = rng.uniform(0.01, 1.0)
        t = rng.choice([1 / 255, rng.uniform(1 / 255, sigma)])
        cc = 2 * math.log(sigma / t)
        ok, spans = O.ellipse_spans(u, v, A, beta, gamma, sigma, t, 0, 12, 0, 11)
        assert ok == (cc > 0)
        for ty in range(12):
            for tx in range(12):
                m = _box_min_q(A, beta, gamma, 16 * tx - u, 16 * tx + 15 - u,
                               16 * ty - v, 16 * ty + 15 - v)
                if ok and abs(m - cc) <= 1e-9 * cc:
                    continue
                want = ok and m <= cc
                got = spans[ty, 0] <= tx <= spans[ty, 1]
                assert got == want, (it, ty, tx, m, cc, spans[ty])
                checked += 1
    assert checked > 40000


def test_ellipse_spans_axis_aligned_closed_form(O):
    """beta = 0: the ellipse X^2/rx^2 + Y^2/ry^2 <= 1, rx = sqrt(c/A), ry =
    sqrt(c/gamma).  A row band meets it over |X| <= rx sqrt(1 - Y*^2/ry^2)
    with Y* the band's point nearest the centre; the span is the tiles that
    range touches.  Also: t >= sigma (c <= 0) has no tiles."""
    A, gamma, sigma, t = 1 / 400.0, 1 / 100.0, 0.8, 1 / 255
    cc = 2 * math.log(sigma / t)
    rx, ry = math.sqrt(cc / A), math.sqrt(cc / gamma)
    u, v = 100.5, 70.25
    ok, spans = O.ellipse_spans(u, v, A, 0.0, gamma, sigma, t, 0, 10, 0, 14)
    assert ok
    for ty in range(10):
        Y0, Y1 = 16 * ty - v, 16 * ty + 15 - v
        if Y1 < -ry or Y0 > ry:
            assert spans[ty, 1] < spans[ty, 0]
            continue
        Ys = min(max(0.0, Y0), Y1)
        hw = rx * math.sqrt(max(0.0, 1 - (Ys / ry) ** 2))
        lo, hi = u - hw, u + hw
        want = [tx for tx in range(15) if 16 * tx <= hi and 16 * tx + 15 >= lo]
        assert list(range(spans[ty, 0], spans[ty, 1] + 1)) == want
    ok, spans = O.ellipse_spans(u, v, A, 0.0, gamma, 0.5, 0.5, 0, 10, 0, 14)
    assert not ok and np.all(spans[:, 1] < spans[:, 0])


def _pair_sets(keys, vals):
    return set(zip((keys >> np.uint64(32)).tolist(), vals.tolist()))


@pytest.mark.parametrize("adagscale,K", [(False, 0.0), (True, 0.3)])
def test_rule1_tiles_are_the_ellipse_tiles(O, adagscale, K):
    """Rule 1 on a tiny scene: the preprocess keeps the plain rectangle (and
    its area) as the candidates, and each Gaussian's emitted tiles are the
    candidates whose box meets the alpha >= th ellipse (box minimum, from the
    float32 record values); every pixel of the plain rectangle that the blend
    would give alpha >= th lies in one of them."""
    sc, _ = scenes.tiny_scene(n=300, seed=5)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 100, 70)
    m0 = O.Mode(adagscale=adagscale, K=K)
    m1 = O.Mode(adagscale=adagscale, K=K, extent_rule=1)
    p0, p1 = O.preprocess(sc, cam, m0), O.preprocess(sc, cam, m1)
    k1, v1 = O.emit(p1, cam)
    TX = (cam["width"] + 15) // 16
    f32 = lambda x: float(np.float32(x))
    py, px = np.mgrid[0:70, 0:100]
    n_dropped = 0
    for g in np.nonzero(p0.flags >= 1)[0]:
        mine = k1[v1 == g] >> np.uint64(32)
        tiles = sorted(int(t) for t in mine)
        u, v = f32(p1.mean2d[g, 0]), f32(p1.mean2d[g, 1])
        A, beta, gamma = (f32(x) for x in p1.quad[g])
        sigma, t = f32(p1.opacity[g]), f32(p1.th[g])
        cc = 2 * math.log(sigma / t) if sigma > t else -1.0
        if p1.radius[g] > 0:
            # the plain rectangle: radius ceil(v), not the scaled one
            assert p1.radius[g] == math.ceil(p1.extent[g])
        x0, y0, x1, y1 = O_plain_rect(p1, g, cam)
        if p1.tiles_touched[g] > 0:
            assert tuple(p1.rect[g]) == (x0, y0, x1, y1)
        assert p1.tiles_touched[g] == (x1 - x0) * (y1 - y0)
        want = []
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                m = _box_min_q(A, beta, gamma, 16 * tx - u, 16 * tx + 15 - u,
                               16 * ty - v, 16 * ty + 15 - v)
                if cc > 0 and m <= cc:
                    want.append(ty * TX + tx)
        assert tiles == sorted(want)
        if tiles:
            # pixels reaching alpha >= t lie in the emitted tiles
            X, Y = px - u, py - v
            alpha = sigma * np.exp(-0.5 * (A * (X + beta * Y) ** 2 + gamma * Y * Y))
            inrect = (px // 16 >= x0) & (px // 16 < x1) & (py // 16 >= y0) & (py // 16 < y1)
            hit = (alpha >= t * (1 + 1e-9)) & inrect
            assert set(((py[hit] // 16) * TX + px[hit] // 16).tolist()) <= set(tiles)
        n_dropped += (x1 - x0) * (y1 - y0) - len(tiles)
    assert n_dropped > 0


def O_plain_rect(pre, g, cam):
    """The plain rectangle of radius pre.radius[g] around the double mean, in
    tiles (the rule both extent rules start from)."""
    TX, TY = (cam["width"] + 15) // 16, (cam["height"] + 15) // 16
    u, v = pre.mean2d[g]
    r = int(pre.radius[g])
    if r <= 0:
        return 0, 0, 0, 0
    cl = lambda x, hi: int(min(max(x, 0), hi))
    return (cl(math.floor((u - r) / 16), TX), cl(math.floor((v - r) / 16), TY),
            cl(math.floor((u + r + 15) / 16), TX), cl(math.floor((v + r + 15) / 16), TY))


def test_rule1_plain_renders_the_same_image(O):
    """Plain 3D-GS with the ellipse test drops only pairs whose every pixel has
    alpha < tau, which the blend skips without effect: image, final T and the
    per-pixel blended count equal the rectangle rule's, with fewer pairs."""
    sc, _ = scenes.tiny_scene(n=400, seed=12)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 96, 64)
    f0 = O.render(sc, cam, O.Mode(), bg=(0.2, 0.1, 0.0))
    f1 = O.render(sc, cam, O.Mode(extent_rule=1), bg=(0.2, 0.1, 0.0))
    assert f1.keys.size < 0.9 * f0.keys.size
    assert _pair_sets(f1.keys, f1.vals) <= _pair_sets(f0.keys, f0.vals)
    np.testing.assert_array_equal(f1.image, f0.image)
    np.testing.assert_array_equal(f1.final_T, f0.final_T)
    ev1, bl1, _ = O.blend_counts(f1, cam)
    ev0, bl0, _ = O.blend_counts(f0, cam)
    np.testing.assert_array_equal(bl1, bl0)
    assert ev1.sum() < ev0.sum()


def test_rule1_adagscale_pairs_within_plain(O):
    """Th >= tau shrinks the ellipse: AdaGScale's rule-1 pairs are a subset of
    plain rule-1 pairs, and K = 0 (Th = tau) gives the same pairs."""
    sc, cam = scenes.tiny_scene(n=1000, seed=8)
    kp, vp = O.emit(O.preprocess(sc, cam, O.Mode(extent_rule=1)), cam)
    ka, va = O.emit(O.preprocess(sc, cam, O.Mode(adagscale=True, K=0.5, extent_rule=1)), cam)
    k0, v0 = O.emit(O.preprocess(sc, cam, O.Mode(adagscale=True, K=0.0, extent_rule=1)), cam)
    assert ka.size < kp.size
    assert _pair_sets(ka, va) <= _pair_sets(kp, vp)
    assert _pair_sets(k0, v0) == _pair_sets(kp, vp)


# --------------------------------------------------------------------------- contribution-skip blend (Sec. 2.4, 3.2)
def test_skip_blend_theta_zero_is_the_blend(O):
    """theta = 0 skips nothing: every kind equals the plain blend bit for bit."""
    sc, cam = scenes.tiny_scene(n=500, seed=31)
    fr = O.render(sc, cam, bg=(0.1, 0.2, 0.3))
    mt, _ = O.max_transmittance(fr, cam)
    for kind, kw in ((0, {}), (1, dict(weight=mt)), (2, dict(lut=np.linspace(1, 0.2, 20)))):
        img, T, nc, _, _, skipped = O.blend_skip(fr, cam, kind, 0.0, bg=(0.1, 0.2, 0.3), **kw)
        assert skipped == 0
        np.testing.assert_array_equal(img, fr.image)
        np.testing.assert_array_equal(T, fr.final_T)
        np.testing.assert_array_equal(nc, fr.n_contrib)


def test_skip_blend_stacked_closed_form(O):
    """Two Gaussians on pixel (5, 5), front alpha 0.3 (red), back alpha 0.5
    (green), black background.  Exact contributions 0.3 and 0.5 x 0.7 = 0.35.
    theta = 0.2 keeps both: colour (0.3, 0.35, 0), T = 0.35.  theta = 0.32
    drops the front one, after which the back one contributes 0.5 x 1 and is
    kept: colour (0, 0.5, 0), T = 0.5.  theta = 0.4: exact (kind 0) still keeps
    the back one (0.5), while with max(T) weights (1 and 0.7, kind 1) it
    contributes 0.35 and is dropped too.  theta = 0.6 drops both."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 16, 16)
    g1 = (5.0, 5.0, 20.0, 0.0, 20.0, 0.3, 1, 0, 0)
    g2 = (5.0, 5.0, 20.0, 0.0, 20.0, 0.5, 0, 1, 0)
    fr, rec = _frame_of(O, [g1, g2], cam)
    a1, a2 = float(np.float32(0.3)), float(np.float32(0.5))  # records hold float32 values
    img, T, nc, _, bl, sk = O.blend_skip(fr, cam, 0, 0.2, rec=rec)
    np.testing.assert_allclose(img[:, 5, 5], [a1, a2 * (1 - a1), 0.0], rtol=1e-15, atol=0)
    assert T[5, 5] == pytest.approx((1 - a1) * (1 - a2), rel=1e-15) and nc[5, 5] == 2
    img, T, nc, _, bl, sk = O.blend_skip(fr, cam, 0, 0.32, rec=rec)
    np.testing.assert_allclose(img[:, 5, 5], [0.0, a2, 0.0], rtol=1e-15, atol=0)
    assert T[5, 5] == 1 - a2 and nc[5, 5] == 2 and bl[5, 5] == 1
    img, T, nc, _, bl, sk = O.blend_skip(fr, cam, 0, 0.4, rec=rec)
    assert T[5, 5] == 1 - a2 and bl[5, 5] == 1
    w = np.array([1.0, 1 - a1])
    img, T, nc, _, bl, sk = O.blend_skip(fr, cam, 1, 0.32, weight=w, rec=rec)
    assert T[5, 5] == 1 - a2 and bl[5, 5] == 1
    img, T, nc, _, bl, sk = O.blend_skip(fr, cam, 1, 0.4, weight=w, rec=rec)
    assert T[5, 5] == 1.0 and nc[5, 5] == 0 and not img[:, 5, 5].any()
    img, T, nc, _, bl, sk = O.blend_skip(fr, cam, 0, 0.6, rec=rec)
    assert T[5, 5] == 1.0 and nc[5, 5] == 0 and not img[:, 5, 5].any()


def _numpy_skip_blend(pre, fr, cam, thr_of):
    """Per pixel, the tile's sorted list walked front to back in plain numpy:
    alpha = min(0.99, opacity exp(-q/2)); skipped if alpha < tau or
    thr_of(i, alpha) (a T-independent rule); stop before T(1 - alpha) < 1e-4."""
    W, H = cam["width"], cam["height"]
    rec = pre.record()
    TX = (W + 15) // 16
    img = np.zeros((3, H, W))
    Tm = np.ones((H, W))
    for py in range(H):
        for px in range(W):
            t = (py // 16) * TX + px // 16
            T = 1.0
            col = np.zeros(3)
            for i in fr.sorted_vals[fr.ranges[t, 0]:fr.ranges[t, 1]]:
                mx, my, cxx, cxy, cyy, op = rec[i, :6]
                dx, dy = mx - px, my - py
                q = np.array([dx, dy]) @ np.array([[cxx, cxy], [cxy, cyy]]) @ np.array([dx, dy])
                alpha = min(0.99, op * math.exp(-0.5 * q))
                if alpha < 1 / 255 or thr_of(i, alpha):
                    continue
                if T * (1 - alpha) < 1e-4:
                    break
                col += alpha * T * rec[i, 6:9]
                T *= 1 - alpha
            img[:, py, px] = col
            Tm[py, px] = T
    return img, Tm


def test_skip_blend_t_independent_kinds_against_numpy(O):
    """Kinds 1 and 2 do not depend on the running T: their skip is a fixed
    per-(Gaussian, alpha) test, so a plain numpy walk of the same lists with
    that test reproduces them (max(T) weights from the oracle's own walk,
    a decreasing depth table)."""
    sc, _ = scenes.tiny_scene(n=150, seed=33)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 40, 28)
    fr = O.render(sc, cam)
    pre = fr.pre
    mt, _ = O.max_transmittance(fr, cam)
    lut = np.linspace(1.0, 0.3, 20)
    d32 = pre.depth.astype(np.float32).astype(np.float64)
    binw = lambda i: lut[min(int(np.floor(d32[i] * 20 / 8.0)), 19)]
    for kind, theta, kw, rule in (
            (1, 0.05, dict(weight=mt), lambda i, a: a * mt[i] < 0.05),
            (2, 0.08, dict(lut=lut, lut_depth_max=8.0), lambda i, a: a * binw(i) < 0.08)):
        img, T, nc, mg, bl, sk = O.blend_skip(fr, cam, kind, theta, **kw)
        want_img, want_T = _numpy_skip_blend(pre, fr, cam, rule)
        assert sk > 0
        ok = mg >= 1e-9
        assert np.abs(img - want_img)[:, ok].max() < 1e-12
        assert np.abs(T - want_T)[ok].max() < 1e-12


def test_skip_blend_huge_theta_and_monotone(O):
    """theta above any contribution skips every blend (background, T = 1);
    for the T-independent kinds the skipped count grows with theta."""
    sc, cam = scenes.tiny_scene(n=400, seed=34)
    fr = O.render(sc, cam, bg=(0.2, 0.4, 0.6))
    img, T, nc, _, bl, sk = O.blend_skip(fr, cam, 0, 2.0, bg=(0.2, 0.4, 0.6))
    assert np.all(T == 1.0) and not nc.any() and not bl.any() and sk > 0
    np.testing.assert_array_equal(img[1], np.full_like(img[1], 0.4))
    mt, _ = O.max_transmittance(fr, cam)
    for kind, kw in ((1, dict(weight=mt)), (2, dict(lut=np.linspace(1, 0.1, 20)))):
        counts = [O.blend_skip(fr, cam, kind, th, **kw)[5] for th in (0.0, 0.01, 0.05, 0.2, 0.5)]
        assert counts == sorted(counts) and counts[0] == 0 and counts[-1] > counts[1]


# --------------------------------------------------------------------------- oriented-box tile test (rule 2)
def _box_meets_polygon(verts, X0, X1, Y0, Y1, eps=0.0):
    """Separating-axis test of an axis-aligned box against a convex polygon:
    returns the largest separation gap over the candidate axes (<= 0: they
    meet)."""
    box = np.array([[X0, Y0], [X1, Y0], [X1, Y1], [X0, Y1]])
    axes = [np.array([1.0, 0.0]), np.array([0.0, 1.0])]
    for i in range(len(verts)):
        e = verts[(i + 1) % len(verts)] - verts[i]
        nrm = np.array([-e[1], e[0]])
        if np.linalg.norm(nrm) > 0:
            axes.append(nrm / np.linalg.norm(nrm))
    gap = -np.inf
    for ax in axes:
        p, q = verts @ ax, box @ ax
        gap = max(gap, max(q.min() - p.max(), p.min() - q.max()))
    return gap


def test_obb_vertices_are_the_scaled_eigenbox(O):
    """The box's vertices are the mean +- 3 s sqrt(lambda_i) e_i of the
    covariance recovered from (A, beta, gamma), against numpy's eigh."""
    rng = np.random.default_rng(61)
    for _ in range(100):
        sx, sy = np.exp(rng.uniform(-0.5, 3.0, 2))
        th = rng.uniform(0, np.pi)
        c_, s_ = np.cos(th), np.sin(th)
        S = np.array([[c_ * c_ * sx * sx + s_ * s_ * sy * sy, c_ * s_ * (sx * sx - sy * sy)],
                      [c_ * s_ * (sx * sx - sy * sy), s_ * s_ * sx * sx + c_ * c_ * sy * sy]])
        a, b, c = S[0, 0], S[0, 1], S[1, 1]
        det = a * c - b * b
        A, beta, gamma = c / det, -b / c, 1.0 / c
        u, v, sc = rng.uniform(0, 100, 2).tolist() + [rng.uniform(0.2, 1.0)]
        ok, _, verts = O.obb_spans(u, v, A, beta, gamma, sc, 0, 1, 0, 10)
        assert ok
        lam, vec = np.linalg.eigh(S)
        h = 3 * np.sqrt(lam) * sc
        want = [np.array([u, v]) + s1 * h[1] * vec[:, 1] + s2 * h[0] * vec[:, 0]
                for s1 in (1, -1) for s2 in (1, -1)]
        for w in want:  # every eigen-box corner is one of the vertices
            assert np.min(np.linalg.norm(verts - w, axis=1)) < 1e-9 * (1 + h.max())


def test_obb_spans_match_separating_axis_test(O):
    """The row spans are exactly the tiles whose pixel box meets the oriented
    box (separating-axis test), on random boxes; tiles within 1e-9 px of
    touching are not judged."""
    rng = np.random.default_rng(62)
    checked = 0
    for it in range(300):
        sx, sy = np.exp(rng.uniform(-0.5, 3.5, 2))
        th = rng.uniform(0, np.pi)
        c_, s_ = np.cos(th), np.sin(th)
        a = c_ * c_ * sx * sx + s_ * s_ * sy * sy
        b = c_ * s_ * (sx * sx - sy * sy)
        c = s_ * s_ * sx * sx + c_ * c_ * sy * sy
        det = a * c - b * b
        A, beta, gamma = c / det, -b / c, 1.0 / c
        u, v = rng.uniform(-40, 200, 2)
        sc = rng.choice([1.0, rng.uniform(0.1, 1.0)])
        ok, spans, verts = O.obb_spans(u, v, A, beta, gamma, sc, 0, 12, 0, 11)
        assert ok
        for ty in range(12):
            for tx in range(12):
                gap = _box_meets_polygon(verts, 16 * tx, 16 * tx + 15, 16 * ty, 16 * ty + 15)
                if abs(gap) <= 1e-9:
                    continue
                got = spans[ty, 0] <= tx <= spans[ty, 1]
                assert got == (gap < 0), (it, ty, tx, gap, spans[ty])
                checked += 1
    assert checked > 40000


@pytest.mark.parametrize("adagscale,K", [(False, 0.0), (True, 0.3)])
def test_rule2_pairs_cover_the_extent_ellipse(O, adagscale, K):
    """Rule 2 on a tiny scene: the rectangle and tile count are rule 0's (the
    candidates), the pairs are a subset of rule 0's, and every pixel of the
    rectangle within the 3 s sigma ellipse (Mahalanobis distance <= 3 s,
    which the oriented box contains) lies in an emitted tile."""
    sc, _ = scenes.tiny_scene(n=300, seed=63)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 100, 70)
    p0 = O.preprocess(sc, cam, O.Mode(adagscale=adagscale, K=K))
    p2 = O.preprocess(sc, cam, O.Mode(adagscale=adagscale, K=K, extent_rule=2))
    np.testing.assert_array_equal(p2.rect, p0.rect)
    np.testing.assert_array_equal(p2.tiles_touched, p0.tiles_touched)
    k0, v0 = O.emit(p0, cam)
    k2, v2 = O.emit(p2, cam)
    assert _pair_sets(k2, v2) <= _pair_sets(k0, v0) and k2.size < k0.size
    TX = (cam["width"] + 15) // 16
    py, px = np.mgrid[0:70, 0:100]
    f32 = lambda x: float(np.float32(x))
    for g in np.nonzero(p2.tiles_touched > 0)[0]:
        tiles = set(int(t) for t in (k2[v2 == g] >> np.uint64(32)))
        u, v = f32(p2.mean2d[g, 0]), f32(p2.mean2d[g, 1])
        A, beta, gamma = (f32(x) for x in p2.quad[g])
        s = f32(p2.scale[g])
        X, Y = px - u, py - v
        q = A * (X + beta * Y) ** 2 + gamma * Y * Y
        x0, y0, x1, y1 = p2.rect[g]
        inrect = (px // 16 >= x0) & (px // 16 < x1) & (py // 16 >= y0) & (py // 16 < y1)
        inside = (q <= (3 * s) ** 2 * (1 - 1e-9)) & inrect
        assert set(((py[inside] // 16) * TX + px[inside] // 16).tolist()) <= tiles


def test_contrib_profile_single_gaussian_closed_form(O):
    """One Gaussian alone (T = 1 in front of it): every blend's contribution is
    alpha = opacity exp(-m^2 / 2), so each bin's mean lies between the values
    at its edges, the total count is the number of pixels with alpha >= tau,
    and the counts sum to the blends of the frame."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 48, 48)
    g = (20.3, 22.7, 1 / 36.0, 0.3, 1 / 25.0, 0.8, 1, 1, 1)
    fr, rec = _frame_of(O, [g], cam)
    sums, counts = O.contrib_profile(fr, cam, rec=rec)
    _, bl, _ = O.blend_counts(fr, cam, rec=rec)
    assert counts.sum() == bl.sum() > 100
    op = float(np.float32(0.8))
    for b in np.nonzero(counts)[0]:
        lo, hi = 0.1 * b, 0.1 * (b + 1)
        mean = sums[b] / counts[b]
        assert op * math.exp(-hi * hi / 2) - 1e-12 <= mean <= op * math.exp(-lo * lo / 2) + 1e-12
    # alpha >= 1/255 ends at m = sqrt(2 ln(255 opacity))
    assert counts[int(math.floor(10 * math.sqrt(2 * math.log(255 * op)))) + 1:].sum() == 0
