"""Helpers shared by the GPU tests: run the HIP path through the C-ABI and
fetch its outputs; compare with the oracle."""
import numpy as np
import torch

from paper_2604_18980_amd import render as R
from paper_2604_18980_amd import gsr

# A pixel is exempt from the image comparison when one of its blend decisions
# (alpha >= tau, T (1 - alpha) >= 1e-4, a skip threshold) lies within
# EXEMPT_MARGIN first-order float32 error bounds of its threshold: the oracle's
# margin is the distance in units of that bound, so below 1 a float32 renderer
# may legitimately take the other branch; 2 leaves room for the second-order
# terms the bound drops.
EXEMPT_MARGIN = 2.0
# At most this fraction of the compared pixels may be exempt (plus a floor of a
# few pixels for tiny images).  The exempt set is the oracle's alone (no kernel
# output enters it); the cap keeps at least 99.5% of the pixels compared.  Each
# pixel makes one decision per evaluated list entry, so pixels of long lists
# hold more near-threshold decisions: 0 on the tiny scenes, up to 2.4e-3 on the
# heaviest sampled tiles of the plain 6M city (thousands of entries per pixel).
EXEMPT_MAX_FRAC = 5e-3
EXEMPT_MAX_FLOOR = 4
IMAGE_TOL = 2e-5       # max-abs per channel outside exempt pixels


def to_np(t):
    return t.detach().cpu().numpy()


def decode_rects(r):
    r = r.astype(np.uint64)
    return np.stack([(r >> np.uint64(s)) & np.uint64(0xFFFF) for s in (0, 16, 32, 48)], 1).astype(np.int64)


def gpu_frame(scene, cam, mode=None, bg=(0.0, 0.0, 0.0), capacity=None, staged=True):
    """Full frame through the C-ABI.  Returns a dict of numpy outputs.  The
    staged path (gs_emit_pairs + gs_sort) also yields the emission-order pairs;
    otherwise gs_bin_pairs runs, with sorted tiles requested, and the
    emission-order arrays are absent."""
    mode = mode or {}
    ds = R.DeviceScene.from_host(scene)
    fb = None
    if capacity is not None:
        fb = R.FrameBuffers(ds.n, cam["width"], cam["height"], capacity)
    fb = R.render(ds, cam, bg=bg, fb=fb, staged=staged, with_tiles=not staged, **mode)
    torch.cuda.synchronize()
    P = int(fb.num_pairs.item())
    m = min(P, fb.capacity)
    out = dict(
        n=ds.n, num_pairs=P, capacity=fb.capacity,
        splats=to_np(fb.splats)[: ds.n],
        rects=decode_rects(to_np(fb.rects)[: ds.n]),
        tiles=to_np(fb.tiles_touched)[: ds.n].astype(np.uint32).astype(np.int64),
        pair_tiles=to_np(fb.pair_tiles)[:m].astype(np.uint32).astype(np.int64) if staged else None,
        pair_gids=to_np(fb.pair_gids)[:m].astype(np.uint32).astype(np.int64) if staged else None,
        sorted_tiles=to_np(fb.sorted_tiles)[:m].astype(np.uint32).astype(np.int64),
        sorted_gids=to_np(fb.sorted_gids)[:m].astype(np.uint32).astype(np.int64),
        ranges=to_np(fb.ranges).astype(np.uint32).astype(np.int64),
        image=to_np(fb.image), final_T=to_np(fb.final_T),
        n_contrib=to_np(fb.n_contrib).astype(np.uint32).astype(np.int64),
    )
    return out


def oracle_mode(O, mode):
    mode = mode or {}
    return O.Mode(adagscale=mode.get("adagscale", False), K=mode.get("K", 0.0),
                  t_upper=mode.get("t_upper"), lut_depth_max=mode.get("lut_depth_max", 100.0),
                  force_unit_scale=mode.get("force_unit_scale", False),
                  extent_rule=mode.get("extent_rule", 0))


def record_conic(splats):
    """The inverse covariance of eq. (1) held by float32 splat records [n][12]
    (sum-of-squares fields A, beta, gamma): (Cxx, Cxy, Cyy) = (A, A beta,
    A beta^2 + gamma), in double."""
    s = np.asarray(splats, np.float64)
    A, beta, gamma = s[:, 2], s[:, 3], s[:, 4]
    return np.stack([A, A * beta, (A * beta) * beta + gamma], axis=1)


def conic_grads(g, splats):
    """GPU splat-record gradients [n][12] (slots: mean x, mean y, A, beta,
    gamma, opacity, -, -, r, g, b) -> gradients of the oracle's record [n][9]
    (mean x, mean y, Cxx, Cxy, Cyy, opacity, r, g, b).  The record stores
    (A, beta, gamma) = (Cxx, Cxy / Cxx, Cyy - Cxy^2 / Cxx), so by the chain
    rule dCxx = dA - dbeta beta / A + dgamma beta^2, dCxy = dbeta / A -
    2 beta dgamma, dCyy = dgamma."""
    g = np.asarray(g, np.float64)
    A, beta = np.asarray(splats, np.float64)[:, 2], np.asarray(splats, np.float64)[:, 3]
    A = np.where(A != 0, A, 1.0)
    dA, db, dgm = g[:, 2], g[:, 3], g[:, 4]
    out = np.zeros((g.shape[0], 9))
    out[:, 0:2] = g[:, 0:2]
    out[:, 2] = dA - db * beta / A + dgm * beta * beta
    out[:, 3] = db / A - 2.0 * beta * dgm
    out[:, 4] = dgm
    out[:, 5] = g[:, 5]
    out[:, 6:9] = g[:, 8:11]
    return out


def check_preprocess(pre, g):
    """Bit-exact discrete outputs and float32 records; colour within 1e-6; the
    record's inverse covariance against the oracle's conic of eq. (1) in
    double (within float32 rounding of the stored fields)."""
    np.testing.assert_array_equal(g["tiles"], pre.tiles_touched)
    vis = pre.tiles_touched > 0
    np.testing.assert_array_equal(g["rects"][vis], pre.rect[vis])
    s = g["splats"][vis]
    f32 = lambda a: np.asarray(a, np.float64).astype(np.float32)
    np.testing.assert_array_equal(s[:, 0], f32(pre.mean2d[vis, 0]))
    np.testing.assert_array_equal(s[:, 1], f32(pre.mean2d[vis, 1]))
    np.testing.assert_array_equal(s[:, 2:5], f32(pre.quad[vis]))
    np.testing.assert_array_equal(s[:, 5], f32(pre.opacity[vis]))
    np.testing.assert_array_equal(s[:, 6], f32(pre.depth[vis]))
    np.testing.assert_array_equal(s[:, 7], f32(pre.th[vis]))
    np.testing.assert_array_equal(s[:, 11], f32(pre.scale[vis]))
    assert np.abs(s[:, 8:11] - pre.rgb[vis]).max(initial=0) < 1e-6
    check_record_conic(pre, s, vis)


def check_record_conic(pre, s, vis):
    """Each stored field carries a relative rounding of at most 2^-24, so the
    conic formed from them is within a few 2^-24 of the oracle's, relative to
    sqrt(Cxx Cyy) (which bounds |Cxy|)."""
    c = record_conic(s)
    o = pre.conic[vis]
    scale = np.sqrt(np.abs(o[:, 0] * o[:, 2]))
    u = 2.0 ** -24
    err = np.abs(c - o)
    assert np.all(err[:, 0] <= 2 * u * np.abs(o[:, 0]))
    assert np.all(err[:, 1] <= 4 * u * scale)
    assert np.all(err[:, 2] <= 8 * u * np.maximum(np.abs(o[:, 2]), scale))


def check_pairs(fr, g, cam):
    assert g["num_pairs"] == fr.keys.size
    o_tiles = (fr.keys >> np.uint64(32)).astype(np.int64)
    o_gids = fr.vals.astype(np.int64)
    a = np.lexsort((g["pair_gids"], g["pair_tiles"]))
    b = np.lexsort((o_gids, o_tiles))
    np.testing.assert_array_equal(g["pair_tiles"][a], o_tiles[b])
    np.testing.assert_array_equal(g["pair_gids"][a], o_gids[b])


def check_emission_order(g):
    """Emitted list is depth-major: (float32 depth bits, Gaussian id) never decreases."""
    gid = g["pair_gids"]
    if gid.size < 2:
        return
    d = g["splats"][gid, 6].view(np.uint32).astype(np.int64)
    key = d * (1 << 32) + gid
    assert np.all(np.diff(key) >= 0)


def check_sorted(fr, g, ntiles):
    np.testing.assert_array_equal(g["sorted_tiles"], (fr.sorted_keys >> np.uint64(32)).astype(np.int64))
    np.testing.assert_array_equal(g["sorted_gids"], fr.sorted_vals.astype(np.int64))
    np.testing.assert_array_equal(g["ranges"], fr.ranges)


def max_exempt(checked, frac=EXEMPT_MAX_FRAC):
    return EXEMPT_MAX_FLOOR + int(frac * checked)


def check_image(fr, g, tol=IMAGE_TOL, margin=EXEMPT_MARGIN, mask=None, max_frac=EXEMPT_MAX_FRAC):
    """Images within tol outside pixels whose blend decisions sit within
    `margin` float32 error bounds of a threshold (exempt pixels, at most
    max_frac of the compared ones); n_contrib exact and final T within tol
    there too.  Returns the number of exempt pixels."""
    ex = fr.margin < margin
    sel = np.ones_like(ex) if mask is None else mask
    ok = ~ex & sel
    n_ex = int((ex & sel).sum())
    checked = int(sel.sum())
    assert n_ex <= max_exempt(checked, max_frac), (n_ex, checked)
    diff = np.abs(g["image"] - fr.image)
    assert diff[:, ok].max(initial=0) <= tol, diff[:, ok].max()
    np.testing.assert_array_equal(g["n_contrib"][ok], fr.n_contrib[ok])
    assert np.abs(g["final_T"] - fr.final_T)[ok].max(initial=0) <= tol
    return n_ex


def check_image_exact(O, fr, g, cam, bg=(0.0, 0.0, 0.0), tiles=None, mask=None):
    """The GPU image against the oracle's blend of eq. (1) on the unrounded
    double-precision record (only the pixel mean rounded to float32, as the
    interface stores it; Preproc.record("exact")): within the oracle's
    per-pixel first-order float32 error bound of that blend (plus 1e-7),
    outside exempt pixels.  This measures the float32 storage form of the
    inverse covariance and the float32 blend against eq. (1) itself.
    Returns (exempt pixels, largest |diff| / bound)."""
    rec = fr.pre.record("exact")
    img, T, nc, mg, _, _, bd = O.blend(fr, cam, bg, tiles=tiles, rec=rec, bound=True)
    ex = mg < EXEMPT_MARGIN
    sel = np.ones_like(ex) if mask is None else mask
    ok = ~ex & sel
    n_ex = int((ex & sel).sum())
    assert n_ex <= max_exempt(int(sel.sum())), n_ex
    diff = np.abs(g["image"] - img)
    lim = bd + 1e-7
    worst = float((diff / lim)[:, ok].max(initial=0.0))
    assert worst <= 1.0, (worst, float(diff[:, ok].max(initial=0.0)))
    np.testing.assert_array_equal(g["n_contrib"][ok], nc[ok])
    return n_ex, worst
