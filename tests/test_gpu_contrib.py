"""gs_rasterize_skip (the contribution analysis of Sec. 2.4 and its max(T^i)
and T_up(depth) approximations, Sec. 3.2) against the oracle's
contribution-skip blend: theta = 0 equals gs_rasterize bit for bit, and for
every contribution kind the image, final T and n_contrib match the oracle
outside decision-ambiguous pixels, with the same skipped and kept blend
counts."""
import numpy as np
import pytest

from paper_2604_18980_amd import scenes

from gpu_util import EXEMPT_MARGIN, check_image, to_np

pytestmark = pytest.mark.gpu

SKIP_EXEMPT_FRAC = 1e-2


def _case(name):
    if name == "tiny":
        sc, cam = scenes.tiny_scene(n=2000, seed=51)
        return sc, cam, None
    sc, cam = scenes.mid_scene(n=40_000, seed=12, width=640, height=360)
    return sc, cam, None


def _gpu_skip(ds, fb, cam, kind, theta, weight=None, lut=None, dmax=100.0, bg=(0.0, 0.0, 0.0)):
    import torch
    from paper_2604_18980_amd import gsr
    img = torch.empty_like(fb.image)
    T = torch.empty_like(fb.final_T)
    nc = torch.empty_like(fb.n_contrib)
    counts = torch.zeros(2, dtype=torch.int64, device=img.device)
    w = None if weight is None else torch.from_numpy(np.asarray(weight, np.float32)).to(img.device)
    gsr.gs_rasterize_skip(fb.splats, fb.n, fb.sorted_gids, fb.ranges, gsr.camera_struct(cam), bg,
                          kind, theta, w, lut, dmax, img, T, nc, counts)
    torch.cuda.synchronize()
    return (to_np(img), to_np(T), to_np(nc).astype(np.uint32).astype(np.int64),
            [int(x) for x in counts.cpu().tolist()])


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_theta_zero_is_the_renderer(O, name):
    from paper_2604_18980_amd import render as R
    sc, cam, _ = _case(name)
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam, bg=(0.1, 0.2, 0.3))
    ref = (to_np(fb.image), to_np(fb.final_T), to_np(fb.n_contrib).astype(np.int64))
    for kind, kw in ((0, {}), (1, dict(weight=np.ones(ds.n))), (2, dict(lut=np.ones(20)))):
        img, T, nc, counts = _gpu_skip(ds, fb, cam, kind, 0.0, bg=(0.1, 0.2, 0.3), **kw)
        np.testing.assert_array_equal(img, ref[0])
        np.testing.assert_array_equal(T, ref[1])
        np.testing.assert_array_equal(nc, ref[2])
        assert counts[0] == 0


@pytest.mark.parametrize("name", ["tiny", "mid"])
@pytest.mark.parametrize("kind,theta", [(0, 0.02), (0, 0.1), (1, 0.02), (1, 0.1), (2, 0.05)])
def test_skip_matches_oracle(O, name, kind, theta):
    """The max(T^i) weights come from the oracle's walk of the same view
    (rounded to float32 on both sides); the depth table decreases over
    [0, D_max)."""
    from paper_2604_18980_amd import render as R
    sc, cam, _ = _case(name)
    print(f"skip case {name} kind {kind} theta {theta}", flush=True)
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam)
    fr = O.render(sc, cam, O.Mode())
    kw, okw = {}, {}
    dmax = 20.0 if name == "tiny" else 80.0
    if kind == 1:
        mt, _ = O.max_transmittance(fr, cam)
        w32 = mt.astype(np.float32)
        kw = dict(weight=w32)
        okw = dict(weight=w32.astype(np.float64))
    elif kind == 2:
        lut = np.linspace(1.0, 0.2, 20).astype(np.float32)
        kw = dict(lut=lut, dmax=dmax)
        okw = dict(lut=lut.astype(np.float64), lut_depth_max=float(np.float32(dmax)))
    img, T, nc, counts = _gpu_skip(ds, fb, cam, kind, theta, **kw)
    o_img, o_T, o_nc, o_mg, o_bl, o_sk = O.blend_skip(fr, cam, kind, float(np.float32(theta)), **okw)
    ofr = O.Frame(fr.pre, None, None, None, None, None)
    ofr.image, ofr.final_T, ofr.n_contrib, ofr.margin = o_img, o_T, o_nc, o_mg
    # the skip rule adds a decision per blend (alpha x weight against theta),
    # and under kind 0 its weight is the running T with the walk's accumulated
    # error bound, so more pixels hold a decision near a threshold than in a
    # plain blend: up to 1e-2 of them may be exempt
    n_ex = check_image(ofr, dict(image=img, final_T=T, n_contrib=nc), max_frac=SKIP_EXEMPT_FRAC)
    kept = int(o_bl.sum())
    print(f"  skipped {counts[0]} (oracle {o_sk}), kept {counts[1]} (oracle {kept}), "
          f"exempt pixels {n_ex}", flush=True)
    assert o_sk > 0
    if n_ex == 0:
        assert counts == [o_sk, kept]
    else:  # an ambiguous pixel moves at most its own list's decisions
        assert abs(counts[0] - o_sk) <= 64 * n_ex and abs(counts[1] - kept) <= 64 * n_ex


def test_skip_rejects_bad_arguments(O):
    import ctypes as C
    from paper_2604_18980_amd import gsr
    L = gsr.load()
    cam = gsr.camera_struct(scenes.tiny_scene(n=10)[1])
    P = C.c_void_p
    bg = (C.c_float * 3)()
    assert L.gs_rasterize_skip(P(1), 1, P(1), P(1), C.byref(cam), bg, 3, 0.1, P(1), None, 1.0,
                               P(1), P(1), P(1), None, None) == 1
    assert b"kind" in L.gs_last_error()
    assert L.gs_rasterize_skip(P(1), 1, P(1), P(1), C.byref(cam), bg, 0, -1.0, None, None, 1.0,
                               P(1), P(1), P(1), None, None) == 1
    assert L.gs_rasterize_skip(P(1), 1, P(1), P(1), C.byref(cam), bg, 1, 0.1, None, None, 1.0,
                               P(1), P(1), P(1), None, None) == 1
    assert L.gs_rasterize_skip(P(1), 1, P(1), P(1), C.byref(cam), bg, 2, 0.1, None, None, 1.0,
                               P(1), P(1), P(1), None, None) == 1


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_contribution_profile_matches_oracle(O, name):
    """Fig. 4(b) profile: the same blends in total as the oracle's walk, each
    distance bin's count and contribution sum equal up to the blends whose
    distance sits at a bin edge in float32 (and the float sums' rounding)."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    sc, cam, _ = _case(name)
    ds = R.DeviceScene.from_host(sc)
    fb = R.render(ds, cam)
    sums = torch.zeros(34, dtype=torch.float32, device="cuda")
    counts = torch.zeros(34, dtype=torch.int64, device="cuda")
    gsr.gs_contribution_profile(fb.splats, fb.n, fb.sorted_gids, fb.ranges, gsr.camera_struct(cam),
                                34, 0.1, sums, counts)
    torch.cuda.synchronize()
    fr = O.render(sc, cam)
    o_sums, o_counts = O.contrib_profile(fr, cam, nbins=34, bin_width=float(np.float32(0.1)))
    g_counts = counts.cpu().numpy()
    g_sums = sums.cpu().numpy().astype(np.float64)
    n_amb = int((fr.margin < EXEMPT_MARGIN).sum())
    total = int(o_counts.sum())
    print(f"  blends {int(g_counts.sum())} (oracle {total}), ambiguous pixels {n_amb}", flush=True)
    assert abs(int(g_counts.sum()) - total) <= 4 * n_amb
    assert np.abs(g_counts - o_counts).max() <= max(8, total * 1e-4)
    np.testing.assert_allclose(g_sums, o_sums, rtol=1e-3, atol=1e-3 * o_sums.max())
    # contributions fall off with distance (Fig. 4(b)): mean per blend in the
    # first bins well above the last populated ones
    mean = o_sums / np.maximum(o_counts, 1)
    live = np.nonzero(o_counts)[0]
    assert mean[live[:3]].mean() > 5 * mean[live[-3:]].mean()
