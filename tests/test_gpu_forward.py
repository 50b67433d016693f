"""GPU parity of the forward path (preprocess, emit, sort, ranges, raster)
against the FP64 oracle, through the C-ABI.  Discrete outputs must match
bit for bit; images within 2e-5 outside decision-ambiguous pixels."""
import math

import numpy as np
import pytest

from paper_2604_18980_amd import scenes

from gpu_util import (EXEMPT_MARGIN, check_emission_order, check_image, check_image_exact, max_exempt,
                      check_pairs, check_preprocess, check_sorted, gpu_frame, oracle_mode)

pytestmark = pytest.mark.gpu

MODES = [
    ("plain", {}),
    ("ada_K0", dict(adagscale=True, K=0.0)),
    ("ada_K0.1", dict(adagscale=True, K=0.1)),
    ("ada_K1", dict(adagscale=True, K=1.0)),
    ("ada_unit", dict(adagscale=True, K=1.0, force_unit_scale=True)),
    ("ada_lut", dict(adagscale=True, K=0.3, t_upper=np.linspace(1.0, 0.05, 20), lut_depth_max=8.0)),
    # the ellipse tile test (extent rule 1)
    ("plain_ell", dict(extent_rule=1)),
    ("ada_ell_K0.1", dict(adagscale=True, K=0.1, extent_rule=1)),
    ("ada_ell_K1", dict(adagscale=True, K=1.0, extent_rule=1)),
    ("ada_ell_lut", dict(adagscale=True, K=0.3, t_upper=np.linspace(1.0, 0.05, 20),
                         lut_depth_max=8.0, extent_rule=1)),
    # the oriented-box tile test (extent rule 2)
    ("plain_obb", dict(extent_rule=2)),
    ("ada_obb_K0.1", dict(adagscale=True, K=0.1, extent_rule=2)),
    ("ada_obb_unit", dict(adagscale=True, K=1.0, force_unit_scale=True, extent_rule=2)),
]


def _full_check(O, sc, cam, mode, bg=(0.0, 0.0, 0.0)):
    print(f"case n={sc.n} {cam['width']}x{cam['height']} mode={mode}", flush=True)
    g = gpu_frame(sc, cam, mode, bg)
    fr = O.render(sc, cam, oracle_mode(O, mode), bg)
    check_preprocess(fr.pre, g)
    check_pairs(fr, g, cam)
    check_emission_order(g)
    check_sorted(fr, g, O.num_tiles(cam))
    n_ex = check_image(fr, g)
    n_ex2, worst = check_image_exact(O, fr, g, cam, bg)
    print(f"  pairs={g['num_pairs']} exempt_pixels={n_ex} (exact record: {n_ex2}, "
          f"largest diff / bound {worst:.2f})", flush=True)
    return g, fr


@pytest.mark.parametrize("name,mode", MODES, ids=[m[0] for m in MODES])
def test_tiny_scene_parity(O, name, mode):
    sc, cam = scenes.tiny_scene()
    _full_check(O, sc, cam, mode)


def test_tiny_scene_sh3_background(O):
    sc, cam = scenes.tiny_scene(seed=4, sh_degree=3)
    _full_check(O, sc, cam, dict(adagscale=True, K=0.2), bg=(0.3, 0.6, 0.1))


@pytest.mark.parametrize("w,h", [(100, 37), (17, 16), (1, 1), (16, 300), (257, 129)])
def test_ragged_image_sizes(O, w, h):
    sc, _ = scenes.tiny_scene(n=1500, seed=7)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), w, h)
    _full_check(O, sc, cam, dict(adagscale=True, K=0.1))
    _full_check(O, sc, cam, {})
    _full_check(O, sc, cam, dict(adagscale=True, K=0.1, extent_rule=1))


def test_mid_scene_subsample(O):
    """Mid-scene generator (clustered, SH degree 3, far shell), 60K Gaussians at
    1920x1080: spans thousands of tiles, several sort blocks and ragged tails."""
    sc, cam = scenes.mid_scene(n=60_000, seed=1)
    for mode in ({}, dict(adagscale=True, K=1.0), dict(extent_rule=1),
                 dict(adagscale=True, K=1.0, extent_rule=1), dict(adagscale=True, K=1.0, extent_rule=2)):
        g = gpu_frame(sc, cam, mode)
        fr = O.render(sc, cam, oracle_mode(O, mode),
                      tiles=np.arange(0, O.num_tiles(cam), 37, dtype=np.int32))
        check_preprocess(fr.pre, g)
        check_pairs(fr, g, cam)
        check_emission_order(g)
        check_sorted(fr, g, O.num_tiles(cam))
        TX = (cam["width"] + 15) // 16
        mask = np.zeros((cam["height"], cam["width"]), bool)
        for t in range(0, O.num_tiles(cam), 37):
            ty, tx = divmod(t, TX)
            mask[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = True
        n_ex = check_image(fr, g, mask=mask)
        n_ex2, worst = check_image_exact(O, fr, g, cam,
                                         tiles=np.arange(0, O.num_tiles(cam), 37, dtype=np.int32),
                                         mask=mask)
        print(f"  mid {mode}: exempt {n_ex} / {int(mask.sum())} (exact record: {n_ex2}, "
              f"largest diff / bound {worst:.2f})", flush=True)


def test_empty_and_culled_scenes(O):
    sc, cam = scenes.tiny_scene(n=300)
    behind = scenes.make_camera(np.diag([1.0, -1.0, -1.0]), np.zeros(3), 64, 48)  # looks away
    g = gpu_frame(sc, behind)
    assert g["num_pairs"] == 0 and np.all(g["tiles"] == 0)
    assert np.all(g["image"] == 0) and np.all(g["final_T"] == 1) and np.all(g["n_contrib"] == 0)
    empty = sc.subset(np.array([], dtype=np.int64))
    g = gpu_frame(empty, cam)
    assert g["num_pairs"] == 0 and np.all(g["final_T"] == 1)


def test_non_finite_and_degenerate_inputs(O):
    sc, cam = scenes.tiny_scene(n=400, seed=8)
    sc.means[0, :5] = np.nan
    sc.means[2, 5:10] = np.inf
    sc.quats[:, 10:20] = 0.0
    sc.log_scales[:, 20:25] = 8.0        # giant: covers every tile
    sc.log_scales[:, 25:30] = -30.0      # sub-pixel: dilation dominates
    sc.opacity_logits[30:40] = -30.0     # opacity ~ 0
    sc.opacity_logits[40:50] = 30.0      # opacity ~ 1, alpha clamps at 0.99
    for mode in ({}, dict(adagscale=True, K=0.5), dict(extent_rule=1),
                 dict(adagscale=True, K=0.5, extent_rule=1), dict(extent_rule=2)):
        _full_check(O, sc, cam, mode)


@pytest.mark.parametrize("staged", [False, True], ids=["bin", "staged"])
@pytest.mark.parametrize("rule", [0, 1, 2], ids=["rect", "ellipse", "obb"])
def test_capacity_overflow_reports_required_count(O, rule, staged):
    """An undersized pair buffer: emit reports the required count, the stages
    after it stay in bounds, and a regrown buffer gives the full result."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    sc, cam = scenes.tiny_scene()
    full = gpu_frame(sc, cam, dict(extent_rule=rule))
    ds = R.DeviceScene.from_host(sc)
    cam_s, mode_s = gsr.camera_struct(cam), gsr.mode_struct(extent_rule=rule)
    fb = R.FrameBuffers(ds.n, cam["width"], cam["height"], full["num_pairs"] // 3)
    R.enqueue_frame(ds, cam_s, mode_s, fb, staged=staged)
    torch.cuda.synchronize()
    assert int(fb.num_pairs.item()) == full["num_pairs"]
    assert fb.capacity == full["num_pairs"] // 3
    fb.set_capacity(full["num_pairs"])
    R.enqueue_frame(ds, cam_s, mode_s, fb, staged=staged)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(fb.image.cpu().numpy(), full["image"])


def test_ellipse_rule_on_gpu_drops_only_empty_pairs(O):
    """Plain 3D-GS with the ellipse test: a subset of the rectangle rule's
    pairs, markedly fewer, and the same image within the parity tolerance."""
    sc, cam = scenes.tiny_scene(seed=14)
    rect = gpu_frame(sc, cam, {})
    ell = gpu_frame(sc, cam, dict(extent_rule=1))
    assert ell["num_pairs"] < 0.9 * rect["num_pairs"]
    pr = set(zip(rect["pair_tiles"].tolist(), rect["pair_gids"].tolist()))
    pe = set(zip(ell["pair_tiles"].tolist(), ell["pair_gids"].tolist()))
    assert pe <= pr
    ok = O.render(sc, cam).margin >= EXEMPT_MARGIN  # no blend decision near a threshold
    assert int((~ok).sum()) <= max_exempt(ok.size)
    assert np.abs(ell["image"] - rect["image"])[:, ok].max() <= 2e-5
    print(f"  pairs rect {rect['num_pairs']} ellipse {ell['num_pairs']}", flush=True)


def test_deterministic(O):
    sc, cam = scenes.tiny_scene(seed=12)
    a = gpu_frame(sc, cam, dict(adagscale=True, K=0.2))
    b = gpu_frame(sc, cam, dict(adagscale=True, K=0.2))
    for k in ("tiles", "pair_tiles", "pair_gids", "sorted_gids", "ranges", "image", "final_T",
              "n_contrib"):
        np.testing.assert_array_equal(a[k], b[k])
    # records and rectangles are specified for the Gaussians with tiles
    vis = a["tiles"] > 0
    np.testing.assert_array_equal(a["splats"][vis], b["splats"][vis])
    np.testing.assert_array_equal(a["rects"][vis], b["rects"][vis])


def test_adagscale_subset_on_gpu(O):
    sc, cam = scenes.tiny_scene(seed=13)
    plain = gpu_frame(sc, cam)
    prev = None
    for K in (0.0, 0.1, 0.5, 2.0):
        g = gpu_frame(sc, cam, dict(adagscale=True, K=K))
        s = set(zip(g["pair_tiles"].tolist(), g["pair_gids"].tolist()))
        assert s <= set(zip(plain["pair_tiles"].tolist(), plain["pair_gids"].tolist()))
        if prev is not None:
            assert s <= prev
        prev = s


def test_evaluation_counts_match_oracle(O):
    """n_evaluated (list entries a pixel evaluates before its stop) equals the
    oracle's count outside decision-ambiguous pixels."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    sc, cam = scenes.tiny_scene(seed=21)
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam, adagscale=True, K=0.1)
    ne = torch.empty((cam["height"], cam["width"]), dtype=torch.int32, device="cuda")
    R.run_raster(fb, gsr.camera_struct(cam), (0.0, 0.0, 0.0), n_evaluated=ne)
    torch.cuda.synchronize()
    fr = O.render(sc, cam, O.Mode(adagscale=True, K=0.1))
    ok = fr.margin >= EXEMPT_MARGIN
    assert int((~ok).sum()) <= max_exempt(ok.size)
    np.testing.assert_array_equal(ne.cpu().numpy()[ok], fr.evals[ok])


@pytest.mark.parametrize("which", ["tiny", "mid"])
def test_raster_work_counts(O, which):
    """gs_raster_work: its list-evaluation total equals the n_evaluated sum,
    its blended count equals the oracle's (up to decision-ambiguous pixels),
    and the strip and load counts are consistent with both."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    if which == "tiny":
        sc, cam = scenes.tiny_scene(seed=21)
    else:
        sc, cam = scenes.mid_scene(n=40_000, seed=6, width=640, height=360)
    mode = O.Mode(adagscale=True, K=0.1)
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam, adagscale=True, K=0.1)
    cam_s = gsr.camera_struct(cam)
    ne = torch.empty((cam["height"], cam["width"]), dtype=torch.int32, device="cuda")
    R.run_raster(fb, cam_s, (0.0, 0.0, 0.0), n_evaluated=ne)
    w = R.raster_work(fb, cam_s)
    w2 = R.raster_work(fb, cam_s)
    assert w == w2
    P = int(fb.num_pairs.item())
    print(which, P, w, flush=True)
    assert w["list_evaluations"] == int(ne.to(torch.int64).sum().item())
    fr = O.render(sc, cam, mode)
    ev, bl, mg = O.blend_counts(fr, cam)
    amb = mg < EXEMPT_MARGIN
    lens = (fr.ranges[:, 1] - fr.ranges[:, 0]).max()
    slack = int(amb.sum()) * int(lens)
    assert abs(w["list_evaluations"] - int(ev.sum())) <= slack
    assert abs(w["blended"] - int(bl.sum())) <= slack
    assert w["blended"] > 0
    assert w["blended"] <= 64 * w["strip_evaluations"]
    assert w["strip_evaluations"] <= 4 * w["loaded"]
    nonempty = int((fr.ranges[:, 1] > fr.ranges[:, 0]).sum())
    assert nonempty <= w["loaded"] <= P


@pytest.mark.parametrize("geom", [(256, 1, 256), (128, 2, 64), (64, 4, 64)], ids=["block", "half", "wave"])
@pytest.mark.parametrize("which", ["tiny", "mid"])
def test_raster_geometries_match_oracle(O, geom, which):
    """Every built raster geometry (workgroup per tile, two waves per tile,
    wave per tile; the wave programs with strip culling) against the oracle on
    the same sorted lists."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    if which == "tiny":
        sc, cam = scenes.tiny_scene(seed=31, sh_degree=3)
        tiles = None
    else:
        sc, cam = scenes.mid_scene(n=60_000, seed=2)
        tiles = np.arange(5, O.num_tiles(cam), 41, dtype=np.int32)
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam, adagscale=True, K=0.3)
    ne = torch.empty((cam["height"], cam["width"]), dtype=torch.int32, device="cuda")
    R.run_raster(fb, gsr.camera_struct(cam), (0.2, 0.1, 0.0), cfg=gsr.GsRasterCfg(*geom),
                 n_evaluated=ne)
    torch.cuda.synchronize()
    fr = O.render(sc, cam, O.Mode(adagscale=True, K=0.3), bg=(0.2, 0.1, 0.0), tiles=tiles)
    g = dict(image=fb.image.cpu().numpy(), final_T=fb.final_T.cpu().numpy(),
             n_contrib=fb.n_contrib.cpu().numpy().astype(np.int64))
    mask = None
    if tiles is not None:
        TX = (cam["width"] + 15) // 16
        mask = np.zeros((cam["height"], cam["width"]), bool)
        for t in tiles:
            ty, tx = divmod(int(t), TX)
            mask[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = True
    n_ex = check_image(fr, g, mask=mask)
    ok = (fr.margin >= EXEMPT_MARGIN) & (mask if mask is not None else True)
    np.testing.assert_array_equal(ne.cpu().numpy()[ok], fr.evals[ok])
    print(f"geometry {geom}: exempt {n_ex}")


def test_half_tile_geometry_equals_wave():
    """Two waves per tile (2 pixels per lane) run the same per-pixel
    arithmetic in the same list order as one wave per tile, so every output
    is bit-identical, at a ragged 1000x600 frame of the mid scene."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    sc, cam = scenes.mid_scene(n=60_000, seed=9, width=1000, height=600)
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam, adagscale=True, K=0.3, extent_rule=1)
    out = []
    for geom in ((64, 4, 64), (128, 2, 64)):
        ne = torch.empty((cam["height"], cam["width"]), dtype=torch.int32, device="cuda")
        R.run_raster(fb, gsr.camera_struct(cam), (0.2, 0.1, 0.0), cfg=gsr.GsRasterCfg(*geom),
                     n_evaluated=ne)
        torch.cuda.synchronize()
        out.append([fb.image.cpu().numpy().copy(), fb.final_T.cpu().numpy().copy(),
                    fb.n_contrib.cpu().numpy().copy(), ne.cpu().numpy()])
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_single_view_graph_replay(O):
    """A whole frame (all four C-ABI stages) captured in a HIP graph: replays
    with eager work and host syncs in between reproduce the eager frame."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    sc, cam = scenes.tiny_scene(seed=41, sh_degree=3)
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam, adagscale=True, K=0.2, slack=1.1)
    ref = fb.image.cpu().numpy().copy()
    cam_s, mode_s = gsr.camera_struct(cam), gsr.mode_struct(adagscale=True, K=0.2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        R.enqueue_frame(ds, cam_s, mode_s, fb, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        R.enqueue_frame(ds, cam_s, mode_s, fb, stream=torch.cuda.current_stream())
    for rep in range(3):
        fb.image.fill_(-1.0)
        fb.sorted_gids.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(fb.image.cpu().numpy(), ref)
        _ = (torch.arange(100, device="cuda") * 2).sum().item()
