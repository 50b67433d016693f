"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (wave-per-tile raster, pair buffers sized from the count),
on what the oracle can compute at that size:

* every Gaussian's rectangle, tile count and float32 record, bit for bit;
* the pair total and every tile's list length;
* the sorted lists and the pixels of sampled tiles (the longest lists plus
  uniformly drawn ones);
* the adjoint of the differentiable workload with dL/dimage supported on
  sampled tiles;
* sampled tiles of sampled views of the batched workload.
"""
import functools

import numpy as np
import pytest

from paper_2604_18980_amd import scenes

from gpu_util import (EXEMPT_MARGIN, check_image, check_image_exact, check_record_conic,
                      conic_grads, decode_rects, to_np)
from sampled import pick_tiles, tile_counts, tile_frame, tile_mask

pytestmark = pytest.mark.gpu

# The K at which the 6M city frame reaches 29.8 dB against plain 3D-GS with
# the rectangle rule, and the measured (headline) configuration: the ellipse
# test at its own 29.8 dB K, with the 16-view calibrated T_up table over
# [0, 1200) m (every bin of which calibrates to 1 on this scene).
CITY_K = 459.1846
HEADLINE = dict(adagscale=True, K=400.4415, extent_rule=1, lut_depth_max=1200.0,
                t_upper=np.ones(20, np.float32))
# pair counts up to which the whole sorted list and every range are compared
FULL_LIST_MAX_PAIRS = 60_000_000


@functools.lru_cache(maxsize=1)
def _city():
    return scenes.city_scene()


def _gpu_frame(sc, cam, mode):
    import torch
    from paper_2604_18980_amd import render as R
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam, slack=1.05, **mode)
    torch.cuda.synchronize()
    return ds, fb


def _omode(O, mode):
    return O.Mode(adagscale=mode.get("adagscale", False), K=mode.get("K", 0.0),
                  t_upper=mode.get("t_upper"), lut_depth_max=mode.get("lut_depth_max", 100.0),
                  extent_rule=mode.get("extent_rule", 0))


def _pairs(O, pre, cam):
    """The oracle's emitted pairs under the ellipse and oriented-box rules
    (None under the rectangle rule, whose lists follow from the rectangles)."""
    return O.emit(pre, cam) if pre.extent_rule != 0 else None


def check_full_lists(O, pre, cam, fb, pairs):
    """The whole sorted list and every tile's range, bit for bit, against the
    oracle's own emission, sort and ranges."""
    keys, vals = pairs if pairs is not None else O.emit(pre, cam)
    sk, sv = O.sort(keys, vals)
    rg = O.ranges(sk, O.num_tiles(cam))
    P = sv.size
    gids = to_np(fb.sorted_gids)[:P].astype(np.uint32)
    np.testing.assert_array_equal(gids, sv)
    np.testing.assert_array_equal(to_np(fb.ranges).astype(np.uint32).astype(np.int64), rg)
    return sk, sv, rg


def check_sampled(O, pre, cam, fb, tiles, n, check_records=True, pairs=None, full_image=False):
    """Everything of one view that the oracle can check at full size: records,
    counts, every list length; every list in full when the pair count allows
    (else the sampled tiles' lists); the pixels of the sampled tiles (or of
    the whole image with full_image), against both the stored-record blend
    (2e-5) and the exact-record blend (its float32 error bound)."""
    if check_records:
        tt = to_np(fb.tiles_touched)[:n].astype(np.uint32).astype(np.int64)
        np.testing.assert_array_equal(tt, pre.tiles_touched)
        vis = pre.tiles_touched > 0
        np.testing.assert_array_equal(decode_rects(to_np(fb.rects)[:n])[vis], pre.rect[vis])
        s = to_np(fb.splats)[:n][vis]
        f32 = lambda a: np.asarray(a, np.float64).astype(np.float32)
        np.testing.assert_array_equal(s[:, 0:2], f32(pre.mean2d[vis]))
        np.testing.assert_array_equal(s[:, 2:5], f32(pre.quad[vis]))
        np.testing.assert_array_equal(s[:, 5], f32(pre.opacity[vis]))
        np.testing.assert_array_equal(s[:, 6], f32(pre.depth[vis]))
        np.testing.assert_array_equal(s[:, 7], f32(pre.th[vis]))
        np.testing.assert_array_equal(s[:, 11], f32(pre.scale[vis]))
        assert np.abs(s[:, 8:11] - pre.rgb[vis]).max(initial=0) < 1e-6
        check_record_conic(pre, s, vis)
        P = int(fb.num_pairs.item())
        want = int(pre.tiles_touched.sum()) if pairs is None else int(pairs[0].size)
        assert P == want and P <= fb.capacity
    rg = to_np(fb.ranges).astype(np.uint32).astype(np.int64)
    counts = tile_counts(pre, cam, pairs)
    np.testing.assert_array_equal(rg[:, 1] - rg[:, 0], counts)
    nz = counts > 0
    if nz.any():
        st = np.sort(rg[nz, 0])
        en = np.sort(rg[nz, 1])
        assert st[0] == 0 and np.all(st[1:] == en[:-1]) and en[-1] == counts.sum()
    full = int(counts.sum()) <= FULL_LIST_MAX_PAIRS
    if full:
        sk, sv, orng = check_full_lists(O, pre, cam, fb, pairs)
        fr = O.Frame(pre, None, None, sk, sv, orng)
    else:
        fr, lists = tile_frame(O, pre, cam, tiles, pairs)
        gids = to_np(fb.sorted_gids).astype(np.uint32)
        for t, lst in zip(tiles, lists):
            np.testing.assert_array_equal(gids[rg[t, 0]:rg[t, 1]], lst)
    sel = None if full_image else tiles
    fr.image, fr.final_T, fr.n_contrib, fr.margin, _, _ = O.blend(fr, cam, tiles=sel)
    g = dict(image=to_np(fb.image), final_T=to_np(fb.final_T),
             n_contrib=to_np(fb.n_contrib).astype(np.uint32).astype(np.int64))
    mask = None if full_image else tile_mask(cam, tiles)
    n_ex = check_image(fr, g, mask=mask)
    n_ex2, worst = check_image_exact(O, fr, g, cam, tiles=sel, mask=mask)
    print(f"  lists compared {'in full' if full else 'on sampled tiles'}; pixels compared "
          f"{'all' if full_image else int(mask.sum())}; exempt {n_ex} (exact record {n_ex2}, "
          f"largest diff / bound {worst:.2f})", flush=True)
    return int(counts.sum()), n_ex


@pytest.mark.parametrize("mode", [{}, dict(adagscale=True, K=CITY_K), dict(extent_rule=1),
                                  dict(adagscale=True, K=CITY_K, extent_rule=1),
                                  dict(adagscale=True, K=CITY_K, extent_rule=2), HEADLINE],
                         ids=["plain", "ada", "plain_ellipse", "ada_ellipse", "ada_obb",
                              "headline"])
def test_city_6M_4608x3456(O, mode):
    import torch
    sc, cam = _city()
    print(f"city 6M 4608x3456 {mode}", flush=True)
    ds, fb = _gpu_frame(sc, cam, mode)
    pre = O.preprocess(sc, cam, _omode(O, mode))
    pairs = _pairs(O, pre, cam)
    tiles = pick_tiles(tile_counts(pre, cam, pairs), 40, 8, 0)
    P, n_ex = check_sampled(O, pre, cam, fb, tiles, sc.n, pairs=pairs,
                            full_image=mode is HEADLINE)
    print(f"  pairs {P}, {tiles.size} tiles checked, {n_ex} exempt pixels", flush=True)
    del ds, fb
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", [{}, dict(adagscale=True, K=1.0)], ids=["plain", "ada"])
def test_mid_500k_1920x1080(O, mode):
    sc, cam = scenes.mid_scene()
    print(f"mid 500K 1920x1080 {mode}", flush=True)
    ds, fb = _gpu_frame(sc, cam, mode)
    pre = O.preprocess(sc, cam, _omode(O, mode))
    tiles = pick_tiles(tile_counts(pre, cam), 60, 8, 1)
    P, n_ex = check_sampled(O, pre, cam, fb, tiles, sc.n)
    print(f"  pairs {P}, {tiles.size} tiles checked, {n_ex} exempt pixels", flush=True)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_diff_1M_1280x720_adjoint(O):
    """dL/dimage drawn on sampled tiles (zero elsewhere and on float32-ambiguous
    pixels); the GPU adjoint against the oracle adjoint over the same tiles."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    sc, cam, _ = scenes.diff_workload()
    mode = dict(adagscale=True, K=0.1)
    print("diff 1M 1280x720 adjoint", flush=True)
    ds, fb = _gpu_frame(sc, cam, mode)
    pre = O.preprocess(sc, cam, _omode(O, mode))
    tiles = pick_tiles(tile_counts(pre, cam), 24, 6, 3)
    fr, _ = tile_frame(O, pre, cam, tiles)
    img, T, nc, mg, _, _ = O.blend(fr, cam, tiles=tiles)
    rng = np.random.default_rng(5)
    dL = (rng.normal(size=(3, cam["height"], cam["width"])) * tile_mask(cam, tiles)).astype(np.float32)
    dL[:, mg < EXEMPT_MARGIN] = 0.0
    grad = torch.empty_like(fb.splats)
    gsr.gs_rasterize_backward(fb.splats, fb.n, fb.sorted_gids, fb.ranges, gsr.camera_struct(cam),
                              (0.0, 0.0, 0.0), fb.final_T, fb.n_contrib,
                              torch.from_numpy(dL).cuda(), grad)
    out = [torch.empty_like(t) for t in (ds.means, ds.log_scales, ds.quats, ds.opacity_logits, ds.sh)]
    gsr.gs_preprocess_backward(ds.struct(), gsr.camera_struct(cam), fb.tiles_touched, grad,
                               gsr.GsSceneGrads(*[t.data_ptr() for t in out]))
    torch.cuda.synchronize()
    g2d = O.blend_backward(fr, cam, dL.astype(np.float64), tiles=tiles)
    g = conic_grads(to_np(grad), to_np(fb.splats)[:sc.n])
    for name, cols in [("mean", [0, 1]), ("conic", [2, 3, 4]), ("opacity", [5]),
                       ("rgb", [6, 7, 8])]:
        r = _rel(g[:, cols], g2d[:, cols])
        print(f"  splat {name}: rel {r:.2e}", flush=True)
        assert r < 1e-4, (name, r)
    ref = O.preprocess_backward(sc, cam, pre, g2d)
    for name, t in zip(("means", "log_scales", "quats", "opacity_logits", "sh"), out):
        h = R.sh_to_host_layout(t) if name == "sh" else to_np(t)
        r = _rel(h.astype(np.float64), ref[name])
        print(f"  {name}: rel {r:.2e}", flush=True)
        assert r < 1e-4, (name, r)


def test_batched_64_views_2M(O):
    """All 64 views of the 2M scene through the persistent multi-view raster;
    list lengths of every tile and sampled tiles' lists and pixels of four
    views (one per resolution) against the oracle."""
    import torch
    from paper_2604_18980_amd import render as R
    from paper_2604_18980_amd.views import MultiView
    sc, cams = scenes.batched_workload()
    mode = dict(adagscale=True, K=3.0)
    print("batched 64 views 2M", flush=True)
    ds = R.DeviceScene.from_host(sc)
    mv = MultiView(ds, cams, mode=mode)
    mv.enqueue()
    torch.cuda.synchronize()
    assert not mv.overflowed()
    for v in (0, 17, 38, 63):
        cam = cams[v]
        pre = O.preprocess(sc, cam, _omode(O, mode))
        tiles = pick_tiles(tile_counts(pre, cam), 12, 4, v)
        P, n_ex = check_sampled(O, pre, cam, mv.fbs[v], tiles, sc.n, check_records=(v == 17))
        print(f"  view {v} {cam['width']}x{cam['height']}: pairs {P}, {n_ex} exempt", flush=True)
