"""The preprocess' float32 prefilter (csrc/prefilter.hpp), run on the host:
every Gaussian it drops must be one the double-precision preprocess gives no
tiles (the oracle's tiles_touched is 0), on the workloads' scenes in the
benchmarked modes and on an adversarial scene (Gaussians at the near plane,
extreme scales, degenerate quaternions, opacities at the threshold, depth-bin
edges, empty lookup-table bins).  It must also drop most of the Gaussians
AdaGScale culls on the city frame (that is what it is for)."""
import os
import subprocess

import numpy as np
import pytest

from paper_2604_18980_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r'''
#include "prefilter.hpp"
#include <stdio.h>
#include <stdlib.h>
#include <vector>
// stdin: n, then camera viewmat[12] fx fy cx cy (float32), width height
// (int32), adagscale (int32), K, lut_depth_max (float32), lut[20] (float32),
// then means [3][n], log_scales [3][n], quats [4][n], opacity_logits [n]
// (float32); stdout: one byte per Gaussian, the tier that drops it (0: kept).
int main() {
    long long n;
    float cam[16], K, dmax, lut[20];
    int wh[2], ada;
    if (fread(&n, 8, 1, stdin) != 1 || fread(cam, 4, 16, stdin) != 16 || fread(wh, 4, 2, stdin) != 2 ||
        fread(&ada, 4, 1, stdin) != 1 || fread(&K, 4, 1, stdin) != 1 || fread(&dmax, 4, 1, stdin) != 1 ||
        fread(lut, 4, 20, stdin) != 20) return 2;
    std::vector<float> d(11 * (size_t)n);
    if (fread(d.data(), 4, d.size(), stdin) != d.size()) return 3;
    gsr::PreprocessArgs a{};
    double R[9], t[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) R[3 * i + j] = cam[4 * i + j];
        t[i] = cam[4 * i + 3];
    }
    const double fx = cam[12], fy = cam[13];
    for (int i = 0; i < 9; ++i) a.Rf[i] = (float)R[i];
    for (int i = 0; i < 3; ++i) a.tf[i] = (float)t[i];
    a.fxf = (float)fx; a.fyf = (float)fy; a.cxf = cam[14]; a.cyf = cam[15];
    a.limxf = (float)(1.3 * ((0.5 * wh[0]) / fx));
    a.limyf = (float)(1.3 * ((0.5 * wh[1]) / fy));
    a.tiles_x = (wh[0] + 15) / 16;
    a.tiles_y = (wh[1] + 15) / 16;
    a.adagscale = ada;
    a.Kf = K;
    a.lut_scalef = (float)(20.0 / (double)dmax);
    for (int i = 0; i < 20; ++i) a.lut[i] = lut[i];
    std::vector<unsigned char> out((size_t)n);
    const float *m = d.data(), *l = m + 3 * n, *q = l + 3 * n, *o = q + 4 * n;
    for (long long g = 0; g < n; ++g)
        out[g] = gsr::surely_no_tiles(a, a.lut, m[g], m[n + g], m[2 * n + g], l[g], l[n + g], l[2 * n + g],
                                      q[g], q[n + g], q[2 * n + g], q[3 * n + g], o[g]);
    fwrite(out.data(), 1, out.size(), stdout);
    return 0;
}
'''


@pytest.fixture(scope="module")
def prefilter(tmp_path_factory):
    d = tmp_path_factory.mktemp("prefilter")
    src = d / "prefilter_host.cpp"
    src.write_text(PROG)
    exe = d / "prefilter_host"
    cmd = ["/opt/rocm/bin/hipcc", "-std=c++17", "-O2", "-ffp-contract=off",
           "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2604_18980_amd", "csrc"), str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

    def run(sc, cam, adagscale=False, K=0.0, lut=None, dmax=100.0, extent_rule=0):
        # the prefilter's culls do not depend on the extent rule
        lut = np.ones(20, np.float32) if lut is None else np.asarray(lut, np.float32)
        camv = np.concatenate([np.asarray(cam["viewmat"], np.float32).reshape(-1),
                               np.float32([cam["fx"], cam["fy"], cam["cx"], cam["cy"]])])
        buf = b"".join([np.int64(sc.n).tobytes(), camv.astype(np.float32).tobytes(),
                        np.int32([cam["width"], cam["height"], int(adagscale)]).tobytes(),
                        np.float32([K, dmax]).tobytes(), lut.tobytes(),
                        np.ascontiguousarray(sc.means, np.float32).tobytes(),
                        np.ascontiguousarray(sc.log_scales, np.float32).tobytes(),
                        np.ascontiguousarray(sc.quats, np.float32).tobytes(),
                        np.ascontiguousarray(sc.opacity_logits, np.float32).tobytes()])
        r = subprocess.run([str(exe)], input=buf, capture_output=True)
        assert r.returncode == 0, r.stderr
        return np.frombuffer(r.stdout, np.uint8)
    return run


def _check(O, run, sc, cam, **mode):
    tier = run(sc, cam, **mode)
    drop = tier > 0
    om = O.Mode(adagscale=mode.get("adagscale", False), K=mode.get("K", 0.0),
                t_upper=mode.get("lut"), lut_depth_max=mode.get("dmax", 100.0),
                extent_rule=mode.get("extent_rule", 0))
    pre = O.preprocess(sc, cam, om)
    none = pre.tiles_touched == 0
    bad = np.nonzero(drop & ~none)[0]
    assert bad.size == 0, f"prefilter dropped {bad.size} Gaussians with tiles, e.g. {bad[:5]}"
    frac = drop.sum() / max(int(none.sum()), 1)
    print(f"  dropped {int(drop.sum())} of {int(none.sum())} tile-less ({frac:.3f}; cheap tier "
          f"{int((tier == 1).sum())}), n={sc.n}")
    return frac


@pytest.mark.slow
def test_prefilter_sound_on_city(O, prefilter):
    sc, cam = scenes.city_scene()
    sub = sc.subset(np.arange(0, sc.n, 6))
    f = _check(O, prefilter, sub, cam, adagscale=True, K=400.4415, dmax=1200.0, extent_rule=1)
    assert f > 0.9  # most of AdaGScale's culls are proven in float32
    _check(O, prefilter, sub, cam, adagscale=True, K=459.1846)
    _check(O, prefilter, sub, cam)


def test_prefilter_sound_on_mid_and_tiny(O, prefilter):
    sc, cam = scenes.mid_scene(n=100_000, seed=3)
    _check(O, prefilter, sc, cam)
    _check(O, prefilter, sc, cam, adagscale=True, K=1.0)
    lut = np.linspace(1.0, 0.1, 20).astype(np.float32)
    lut[7] = 0.0
    _check(O, prefilter, sc, cam, adagscale=True, K=30.0, lut=lut, dmax=80.0)
    sc, cam = scenes.tiny_scene(n=2000, seed=5)
    _check(O, prefilter, sc, cam)
    _check(O, prefilter, sc, cam, adagscale=True, K=0.1)


def _adversarial(n=200_000, seed=11):
    """Gaussians in front of a 640x480 camera chosen to sit on every decision
    boundary: depths straddling the near plane, positions around the image
    border and far outside it, log-scales from -12 to 8 (needles and giants),
    quaternions with norms from 1e-20 to 1e6, opacity logits near the
    AdaGScale cut."""
    rng = np.random.default_rng(seed)
    sc, _ = scenes.tiny_scene(n=n, seed=seed)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 640, 480)
    z = np.where(rng.random(n) < 0.3, rng.uniform(0.15, 0.3, n), np.exp(rng.uniform(-1, 5, n)))
    half = 1.3 * np.tan(np.deg2rad(30.0))
    x = rng.uniform(-2.5 * half, 2.5 * half, n) * z
    y = rng.uniform(-2.0 * half, 2.0 * half, n) * z
    sc.means[:] = np.stack([x, y, z]).astype(np.float32)
    sc.log_scales[:] = rng.uniform(-12.0, 8.0, (3, n)).astype(np.float32)
    q = rng.normal(size=(4, n)) * np.exp(rng.uniform(np.log(1e-20), np.log(1e6), n))
    sc.quats[:] = q.astype(np.float32)
    sc.opacity_logits[:] = rng.normal(0.0, 4.0, n).astype(np.float32)
    return sc, cam


@pytest.mark.parametrize("K", [0.0, 1e-3, 1.0, 1e3])
def test_prefilter_sound_adversarial(O, prefilter, K):
    sc, cam = _adversarial()
    lut = np.exp(np.linspace(0.0, -3.0, 20)).astype(np.float32)
    lut[3] = 0.0
    _check(O, prefilter, sc, cam, adagscale=True, K=K, lut=lut, dmax=20.0)
    if K == 0.0:
        _check(O, prefilter, sc, cam)
