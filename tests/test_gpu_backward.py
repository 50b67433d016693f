"""GPU parity of the adjoint path against the FP64 oracle's analytic adjoint
(itself checked against central differences on the CPU).  Gradients are
compared normwise per parameter group: float32 atomics make the summation
order vary, so agreement is to a tolerance, not bitwise."""
import numpy as np
import pytest

from paper_2604_18980_amd import scenes

from gpu_util import EXEMPT_MARGIN, conic_grads

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _host(name, t):
    """A parameter gradient in the host scene layout (SH back to [(d+1)^2][3][n])."""
    from paper_2604_18980_amd.render import sh_to_host_layout
    return sh_to_host_layout(t) if name == "sh" else t.cpu().numpy()


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _setup(sh_degree=3, seed=5, n=2000, mode=None):
    import torch
    from paper_2604_18980_amd import render as R
    sc, cam = scenes.tiny_scene(n=n, seed=seed, sh_degree=sh_degree)
    ds = R.DeviceScene.from_host(sc)
    mode = mode or {}
    fb = R.render(ds, cam, bg=(0.1, 0.2, 0.3), **mode)
    torch.cuda.synchronize()
    return sc, cam, ds, fb, mode


@pytest.mark.parametrize("mode", [{}, dict(adagscale=True, K=0.2)], ids=["plain", "ada"])
def test_raster_backward_matches_oracle(O, mode):
    import torch
    from paper_2604_18980_amd import gsr
    sc, cam, ds, fb, mode = _setup(mode=mode)
    rng = np.random.default_rng(1)
    dL = rng.normal(size=(3, cam["height"], cam["width"])).astype(np.float32)
    grad = torch.empty_like(fb.splats)
    gsr.gs_rasterize_backward(fb.splats, fb.n, fb.sorted_gids, fb.ranges, gsr.camera_struct(cam),
                              (0.1, 0.2, 0.3), fb.final_T, fb.n_contrib, torch.from_numpy(dL).cuda(),
                              grad)
    torch.cuda.synchronize()
    g = grad.cpu().numpy()
    fr = O.render(sc, cam, O.Mode(adagscale=mode.get("adagscale", False), K=mode.get("K", 0.0)),
                  bg=(0.1, 0.2, 0.3))
    # skip the (rare) pixels whose forward decisions are ambiguous in float32
    amb = fr.margin < EXEMPT_MARGIN
    dLo = dL.astype(np.float64).copy()
    dLo[:, amb] = 0.0
    if amb.any():
        dLg = dL.copy()
        dLg[:, amb] = 0.0
        gsr.gs_rasterize_backward(fb.splats, fb.n, fb.sorted_gids, fb.ranges,
                                  gsr.camera_struct(cam), (0.1, 0.2, 0.3), fb.final_T, fb.n_contrib,
                                  torch.from_numpy(dLg).cuda(), grad)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
    g2d = O.blend_backward(fr, cam, dLo, bg=(0.1, 0.2, 0.3))
    gc = conic_grads(g, fb.splats.cpu().numpy())
    for name, cols in [("mean", [0, 1]), ("conic", [2, 3, 4]), ("opacity", [5]),
                       ("rgb", [6, 7, 8])]:
        r = _rel(gc[:, cols], g2d[:, cols])
        print(f"{name}: rel {r:.2e}")
        assert r < TOL, (name, r)
    assert np.all(g[:, [6, 7, 11]] == 0)


def test_preprocess_backward_matches_oracle(O):
    """Same 2D gradients in, scene gradients out: isolates the preprocess adjoint."""
    import torch
    from paper_2604_18980_amd import gsr
    sc, cam, ds, fb, mode = _setup(sh_degree=3, seed=8)
    fr = O.render(sc, cam, O.Mode(), bg=(0.1, 0.2, 0.3))
    rng = np.random.default_rng(2)
    g2d = rng.normal(size=(sc.n, 9))
    g2d[fr.pre.tiles_touched == 0] = 0
    g2d32 = g2d.astype(np.float32)
    gs = np.zeros((sc.n, 12), np.float32)
    gs[:, [0, 1, 2, 3, 4, 5, 8, 9, 10]] = g2d32
    out = [torch.empty_like(t) for t in (ds.means, ds.log_scales, ds.quats, ds.opacity_logits, ds.sh)]
    gsr.gs_preprocess_backward(ds.struct(), gsr.camera_struct(cam), fb.tiles_touched,
                               torch.from_numpy(gs).cuda(), gsr.GsSceneGrads(*[t.data_ptr() for t in out]))
    torch.cuda.synchronize()
    # the same gradients on the oracle's record (Cxx, Cxy, Cyy), by the chain
    # rule at the double-precision (A, beta)
    sp = np.zeros((sc.n, 12))
    sp[:, 2:4] = fr.pre.quad[:, 0:2]
    ref = O.preprocess_backward(sc, cam, fr.pre, conic_grads(gs, sp))
    for name, t in zip(("means", "log_scales", "quats", "opacity_logits", "sh"), out):
        r = _rel(_host(name, t), ref[name])
        print(f"{name}: rel {r:.2e}")
        assert r < 1e-5, (name, r)


@pytest.mark.parametrize("mode", [{}, dict(adagscale=True, K=0.1)], ids=["plain", "ada"])
def test_autograd_end_to_end(O, mode):
    """L1 loss to a seeded random target through RasterizeFn; every parameter
    group against the oracle's adjoint."""
    import torch
    from paper_2604_18980_amd.autograd import rasterize
    sc, cam = scenes.tiny_scene(n=1500, seed=9, sh_degree=3)
    target = scenes.target_image(cam["width"], cam["height"], seed=7)
    from paper_2604_18980_amd.render import sh_to_device_layout
    params = [torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True)
              for a in (sc.means, sc.log_scales, sc.quats, sc.opacity_logits,
                        sh_to_device_layout(sc.sh))]
    fr = O.render(sc, cam, O.Mode(adagscale=mode.get("adagscale", False), K=mode.get("K", 0.0)))
    keep = (fr.margin >= EXEMPT_MARGIN).astype(np.float32)  # drop float32-ambiguous pixels
    img = rasterize(*params, sc.sh_degree, cam, bg=(0.0, 0.0, 0.0), **mode)
    loss = ((img - torch.from_numpy(target).cuda()).abs() * torch.from_numpy(keep).cuda()).sum() / img.numel()
    loss.backward()
    torch.cuda.synchronize()
    dL = np.sign(fr.image - target) * keep / fr.image.size
    g2d = O.blend_backward(fr, cam, dL)
    ref = O.preprocess_backward(sc, cam, fr.pre, g2d)
    for name, p in zip(("means", "log_scales", "quats", "opacity_logits", "sh"), params):
        r = _rel(_host(name, p.grad), ref[name])
        print(f"{name}: rel {r:.2e}")
        assert r < TOL, (name, r)
