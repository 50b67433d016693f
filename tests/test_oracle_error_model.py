"""Pins of the oracle's decision margins and per-pixel float32 error bound
(eq. 1-2 evaluated by a float32 renderer) against an actual float32
computation: a numpy renderer that stores the record in float32 (mean, the
sum-of-squares inverse covariance A, beta, gamma, opacity, colour), forms the
pixel offset in float32 and evaluates eq. (1) as A (dx + beta dy)^2 +
gamma dy^2 with float32 exponentials -- the model the margins and the bound
describe.  Wherever the oracle's margin is at least 1, that renderer must
take every decision the double-precision blend takes (same n_contrib), and
its image must lie within the oracle's bound of the double-precision blend of
the unrounded record.  A needle case checks that far out on a thin Gaussian,
where the first-order relative error of alpha is large but alpha vanishes, the
margin stays large."""
import numpy as np
import pytest

from paper_2604_18980_amd import scenes

TILE = 16
F = np.float32


def _f32_render(pre, fr, cam, tiles, bg):
    """Float32 numpy renderer of the listed tiles: image [3][H][W], final T and
    n_contrib [H][W] (zero outside the tiles)."""
    W, H = cam["width"], cam["height"]
    TX = (W + TILE - 1) // TILE
    mean = pre.mean2d.astype(F)
    A, beta, gamma = (pre.quad[:, k].astype(F) for k in range(3))
    op = pre.opacity.astype(F)
    rgb = pre.rgb.astype(F)
    tau, t_stop, amax, half = F(1.0 / 255.0), F(1e-4), F(0.99), F(0.5)
    bgv = np.asarray(bg, F)
    img = np.zeros((3, H, W), F)
    Tout = np.zeros((H, W), F)
    nc = np.zeros((H, W), np.int64)
    for t in tiles:
        ty, tx = divmod(int(t), TX)
        ys, xs = np.arange(ty * TILE, min((ty + 1) * TILE, H)), np.arange(tx * TILE, min((tx + 1) * TILE, W))
        PY, PX = np.meshgrid(ys.astype(F), xs.astype(F), indexing="ij")
        T = np.ones(PX.shape, F)
        C = np.zeros((3,) + PX.shape, F)
        done = np.zeros(PX.shape, bool)
        last = np.zeros(PX.shape, np.int64)
        s, e = fr.ranges[int(t)]
        for j in range(int(s), int(e)):
            g = int(fr.sorted_vals[j])
            dx = mean[g, 0] - PX
            dy = mean[g, 1] - PY
            u = dx + beta[g] * dy
            q = A[g] * (u * u) + gamma[g] * (dy * dy)
            alpha = np.minimum(amax, op[g] * np.exp(-half * q))
            live = ~done & (alpha >= tau)
            Tn = T * (F(1) - alpha)
            stop = live & (Tn < t_stop)
            done |= stop
            blend = live & ~stop
            w = alpha * T
            for ch in range(3):
                C[ch] = np.where(blend, C[ch] + w * rgb[g, ch], C[ch])
            T = np.where(blend, Tn, T)
            last = np.where(blend, j - int(s) + 1, last)
        for ch in range(3):
            img[ch][np.ix_(ys, xs)] = C[ch] + T * bgv[ch]
        Tout[np.ix_(ys, xs)] = T
        nc[np.ix_(ys, xs)] = last
    return img, Tout, nc


def _check(O, sc, cam, mode, tiles=None, bg=(0.0, 0.0, 0.0)):
    fr = O.render(sc, cam, mode)
    ntiles = O.num_tiles(cam)
    tiles = np.arange(ntiles) if tiles is None else np.asarray(tiles)
    img32, T32, nc32 = _f32_render(fr.pre, fr, cam, tiles, bg)
    img, T, nc, mg, _, _, bd = O.blend(fr, cam, bg, tiles=tiles, rec=fr.pre.record("exact"),
                                       bound=True)
    mask = np.zeros(mg.shape, bool)
    TX = (cam["width"] + TILE - 1) // TILE
    for t in tiles:
        ty, tx = divmod(int(t), TX)
        mask[ty * TILE:(ty + 1) * TILE, tx * TILE:(tx + 1) * TILE] = True
    ok = (mg >= 1.0) & mask
    np.testing.assert_array_equal(nc32[ok], nc[ok])
    diff = np.abs(img32.astype(np.float64) - img)
    ratio = (diff / (bd + 1e-9))[:, ok]
    # the bound is first order; the float32 image must sit inside it
    assert ratio.max(initial=0.0) <= 1.0, ratio.max()
    return int((mask & ~ok).sum()), float(ratio.max(initial=0.0)), int(mask.sum())


@pytest.mark.parametrize("sh_degree", [0, 3])
@pytest.mark.parametrize("adagscale", [False, True])
def test_float32_renderer_within_bound_tiny(O, sh_degree, adagscale):
    sc, cam = scenes.tiny_scene(n=2000, seed=7, sh_degree=sh_degree)
    mode = O.Mode(adagscale=adagscale, K=0.1 if adagscale else 0.0)
    n_amb, worst, n = _check(O, sc, cam, mode, bg=(0.2, 0.1, 0.3))
    print(f"ambiguous {n_amb} of {n}, largest |f32 - f64| / bound {worst:.3f}")


def test_float32_renderer_within_bound_mid_tiles(O):
    """A denser clustered scene (thin and large Gaussians, SH degree 3); the
    longest lists plus a spread of tiles."""
    sc, cam = scenes.mid_scene(n=30_000, seed=4, width=320, height=192)
    mode = O.Mode()
    pre = O.preprocess(sc, cam, mode)
    ntiles = O.num_tiles(cam)
    tiles = np.unique(np.concatenate([np.arange(0, ntiles, 9), [ntiles // 2]]))
    n_amb, worst, n = _check(O, sc, cam, mode, tiles=tiles)
    assert n_amb <= 0.01 * n
    print(f"ambiguous {n_amb} of {n}, largest |f32 - f64| / bound {worst:.3f}")


def _needle_scene(aspect, s_short_px=0.7, size=1024):
    """One thin Gaussian in front of a size x size camera: short axis
    s_short_px pixels, long axis aspect times that, rotated 30 degrees in the
    image plane."""
    sc, _ = scenes.tiny_scene(n=1, seed=0)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), size, size)
    z = 5.0
    sc.means[:, 0] = (0.0, 0.0, z)
    s_short = s_short_px * z / cam["fx"]
    sc.log_scales[:, 0] = (np.log(s_short * aspect), np.log(s_short), np.log(s_short))
    th = np.deg2rad(30.0) / 2
    sc.quats[:, 0] = (np.cos(th), 0.0, 0.0, np.sin(th))
    sc.opacity_logits[0] = 3.0
    return sc, cam


def test_needle_far_pixels_have_large_margins(O):
    """Far out on a needle's short axis (hundreds of short-axis sigmas, q up
    to about 5e5) the first-order relative error of alpha reaches tenths,
    yet alpha is vanishingly small and no float32 rounding brings it near
    tau: those pixels are not decision-ambiguous (a margin taken as the
    linear distance |alpha - tau| / tau over that error would be a few
    units there), and the float32 renderer agrees with the blend."""
    sc, cam = _needle_scene(aspect=300.0)
    fr = O.render(sc, cam, O.Mode())
    assert fr.pre.tiles_touched[0] > 0
    _, _, _, mg, ev, _ = O.blend(fr, cam)
    rec = fr.pre.record("exact")
    H, W = mg.shape
    PY, PX = np.mgrid[0:H, 0:W].astype(np.float64)
    dx, dy = rec[0, 0] - PX, rec[0, 1] - PY
    q = rec[0, 2] * dx * dx + 2 * rec[0, 3] * dx * dy + rec[0, 4] * dy * dy
    far = (q > 1e5) & (ev > 0)  # evaluated pixels (inside the rectangle's tiles)
    assert far.sum() > 10_000
    assert mg[far].min() > 1e3
    n_amb, worst, n = _check(O, sc, cam, O.Mode())
    assert n_amb <= 4


def test_margin_small_at_the_tau_contour(O):
    """A pixel whose alpha equals tau to within float32 resolution has a
    margin below 1, one a hair further out a margin above it."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 32, 16)
    # isotropic unit-variance splat centred at x = 0.5 + c: at pixel x = 0.5 + c
    # - r alpha = sigma exp(-r^2 / 2); choose the centre so pixel (16, 8) sits
    # at the tau contour, then shift by a tiny amount
    sigma = 0.8
    r_tau = np.sqrt(2.0 * np.log(sigma * 255.0))
    out = []
    for eps in (0.0, 1e-3):
        mx = 16.0 + r_tau + eps
        rec = np.array([[mx, 8.0, 1.0, 0.0, 1.0, sigma, 1.0, 1.0, 1.0]])
        sv = np.zeros(1, np.uint32)
        rg = np.zeros((O.num_tiles(cam), 2), np.int64)
        rg[:, 1] = 1
        fr = O.Frame(None, None, None, None, sv, rg)
        _, _, _, mg, _, _ = O.blend(fr, cam, rec=rec)
        out.append(mg[8, 16])
    assert out[0] < 1.0 < out[1]
