"""The oracle's analytic adjoint against FP64 central finite differences of
the oracle's own forward pass, with the pair lists frozen at the unperturbed
point and every blend decision checked unchanged (a sample whose decisions
flip is discarded).  Parameters are float32, so each difference uses the
perturbation actually represented after rounding."""
import numpy as np
import pytest

from paper_2604_18980_amd import scenes

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _scene(n, seed, sh_degree):
    sc, _ = scenes.tiny_scene(n=n, seed=seed, sh_degree=sh_degree)
    # larger, fewer Gaussians so every parameter matters
    sc.log_scales += np.float32(1.2)
    cam = scenes.look_camera((0.2, -0.1, 0.0), (0.02, 0.01, 1.0), (0, -1, 0), 40, 32)
    return sc, cam


def _forward(O, sc, cam, frame, mode, w, bg):
    pre = O.preprocess(sc, cam, mode)
    rec = pre.record("double")
    img, T, nc, mg, ev, sig = O.blend(frame, cam, bg, rec=rec)
    return float((w * img).sum()), sig, pre.flags


@pytest.mark.parametrize("sh_degree,adagscale", [(0, False), (3, False), (3, True)])
def test_adjoint_matches_central_differences(O, sh_degree, adagscale):
    sc, cam = _scene(50, 7 + sh_degree, sh_degree)
    mode = O.Mode(adagscale=adagscale, K=0.05)
    bg = (0.2, 0.1, 0.05)
    frame = O.render(sc, cam, mode, bg)
    rng = np.random.default_rng(0)
    w = rng.normal(size=frame.image.shape)
    rec = frame.pre.record("double")
    g2d = O.blend_backward(frame, cam, w, bg, rec=rec)
    grads = O.preprocess_backward(sc, cam, frame.pre, g2d)
    L0, sig0, flags0 = _forward(O, sc, cam, frame, mode, w, bg)
    live = np.nonzero(frame.pre.flags == 2)[0]
    checked = 0
    worst = 0.0
    gscale = max(np.abs(grads[k]).max() for k in GROUPS)
    for group in GROUPS:
        arr = getattr(sc, group)
        for trial in range(10):
            g = int(rng.choice(live))
            if group == "opacity_logits":
                idx = (g,)
            elif group == "sh":
                idx = (int(rng.integers(arr.shape[0])), int(rng.integers(3)), g)
            else:
                idx = (int(rng.integers(arr.shape[0])), g)
            base = arr[idx]
            h = 1e-4 * max(1.0, abs(float(base)))
            arr[idx] = np.float32(base + h)
            hp = float(arr[idx]) - float(base)
            Lp, sigp, fp = _forward(O, sc, cam, frame, mode, w, bg)
            arr[idx] = np.float32(base - h)
            hm = float(base) - float(arr[idx])
            Lm, sigm, fm = _forward(O, sc, cam, frame, mode, w, bg)
            arr[idx] = base
            if not (np.array_equal(sigp, sig0) and np.array_equal(sigm, sig0)):
                continue
            if not (np.array_equal(fp, flags0) and np.array_equal(fm, flags0)):
                continue
            fd = (Lp - Lm) / (hp + hm)
            an = grads[group][idx]
            err = abs(fd - an) / (abs(an) + 1e-3 * gscale)
            worst = max(worst, err)
            checked += 1
            assert err < 1e-4, (group, idx, fd, an)
    assert checked >= 35
    # random directions over every parameter of every live Gaussian
    for trial in range(5):
        saved = {k: getattr(sc, k).copy() for k in GROUPS}
        vs = {k: rng.normal(size=getattr(sc, k).shape) for k in GROUPS}
        eps = 1e-4
        for k in GROUPS:
            getattr(sc, k)[...] = (saved[k] + eps * vs[k]).astype(np.float32)
        Lp, sigp, _ = _forward(O, sc, cam, frame, mode, w, bg)
        dp = {k: getattr(sc, k).astype(np.float64) - saved[k] for k in GROUPS}
        for k in GROUPS:
            getattr(sc, k)[...] = (saved[k] - eps * vs[k]).astype(np.float32)
        Lm, sigm, _ = _forward(O, sc, cam, frame, mode, w, bg)
        dm = {k: saved[k] - getattr(sc, k).astype(np.float64) for k in GROUPS}
        for k in GROUPS:
            getattr(sc, k)[...] = saved[k]
        if not (np.array_equal(sigp, sig0) and np.array_equal(sigm, sig0)):
            continue
        pred = sum((grads[k] * (dp[k] + dm[k])).sum() for k in GROUPS)
        assert (Lp - Lm) == pytest.approx(pred, rel=1e-4)
