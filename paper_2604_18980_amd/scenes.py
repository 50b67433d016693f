"""Seeded synthetic scenes and cameras for the 3D-GS tile-rendering hot path.

This module only draws inputs. It holds none of the rendering method's
arithmetic (no projection, no blending, no AdaGScale threshold), so both the
HIP path and the CPU oracle can consume its arrays without sharing code.

Layouts (all float32, structure-of-arrays, ``[C][N]`` contiguous):

* ``means``          ``[3][N]``            world-space centres
* ``log_scales``     ``[3][N]``            per-axis log standard deviations
* ``quats``          ``[4][N]``            rotation quaternion, order (w, x, y, z)
* ``opacity_logits`` ``[N]``               opacity before the sigmoid
* ``sh``             ``[(d+1)^2][3][N]``   spherical-harmonic colour coefficients

A camera is a dict with ``viewmat`` (12 float32, row-major ``[R | t]`` mapping
world to camera coordinates, OpenCV axes: x right, y down, z forward), the
pinhole intrinsics ``fx, fy, cx, cy`` and the image ``width, height``.

The recipes stand in for the paper's datasets (Tanks&Temples, DeepBlending,
Mip-NeRF360, Mill-19, UrbanScene3D; Sec. 4.1 and Table I), which are not
available: shapes, sizes and distributions follow the five workloads the
build targets (tiny 2K / mid 500K / city 6M at 4608x3456 / differentiable 1M /
64 batched views of mixed resolution).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Scene", "make_camera", "look_camera", "tiny_scene", "mid_scene", "city_scene",
    "diff_workload", "batched_workload", "workload", "target_image", "WORKLOADS",
]


_CHUNK = 1 << 20
_POOL = ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1))


class Rand:
    """Seeded random arrays, filled in parallel.

    Every call takes the next child of a SeedSequence and splits the array into
    fixed 2^20-element chunks, each with its own PCG64 stream; the result
    depends only on the seed and the order of calls, not on the thread count."""

    def __init__(self, seed):
        self.ss = np.random.SeedSequence(seed)

    def _fill(self, shape, fn, out=None):
        if out is None:
            out = np.empty(shape, dtype=np.float32)
        flat = out.reshape(-1)
        nch = max(1, -(-flat.size // _CHUNK))
        seeds = self.ss.spawn(1)[0].spawn(nch)

        def work(i):
            g = np.random.Generator(np.random.PCG64(seeds[i]))
            seg = flat[i * _CHUNK:(i + 1) * _CHUNK]
            if seg.size:
                fn(g, seg)
        list(_POOL.map(work, range(nch)))
        return out

    def normal(self, shape, mean=0.0, std=1.0, out=None):
        """N(mean, std^2); ``out`` (contiguous float32) is filled in place."""
        m, sd = np.float32(mean), np.float32(std)

        def fn(g, seg):
            g.standard_normal(out=seg, dtype=np.float32)
            if sd != 1:
                seg *= sd
            if m != 0:
                seg += m
        return self._fill(shape, fn, out)

    def uniform(self, shape, lo=0.0, hi=1.0, out=None):
        w, l0 = np.float32(hi - lo), np.float32(lo)

        def fn(g, seg):
            g.random(out=seg, dtype=np.float32)
            seg *= w
            seg += l0
        return self._fill(shape, fn, out)

    def uniform64(self, size, lo=0.0, hi=1.0):
        """Small double-precision draws (building layouts, cluster centres)."""
        g = np.random.Generator(np.random.PCG64(self.ss.spawn(1)[0]))
        return g.uniform(lo, hi, size)

    def integers(self, size, hi):
        return np.minimum((self.uniform(size) * hi).astype(np.int64), hi - 1)

    def choice(self, size, p):
        cdf = np.cumsum(p)
        cdf = (cdf / cdf[-1]).astype(np.float32)
        return np.minimum(np.searchsorted(cdf, self.uniform(size), side="right"), len(p) - 1)

    def student_t(self, shape, dof):
        z = self.normal(shape)
        chi2 = np.zeros(shape, np.float32)
        for _ in range(dof):
            chi2 += self.normal(shape) ** 2
        return z / np.sqrt(chi2 / np.float32(dof))


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.means[:, idx]),
                     np.ascontiguousarray(self.log_scales[:, idx]),
                     np.ascontiguousarray(self.quats[:, idx]),
                     np.ascontiguousarray(self.opacity_logits[idx]),
                     np.ascontiguousarray(self.sh[:, :, idx]),
                     self.sh_degree)


def make_camera(R, t, width, height, fovx_deg=60.0):
    """Pinhole camera with square pixels and the principal point at the image centre.

    fx = (W/2) / tan(fovx/2), fy = fx, cx = (W-1)/2, cy = (H-1)/2 (pixel centres at
    integer coordinates)."""
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    t = np.asarray(t, dtype=np.float64).reshape(3)
    fx = (width / 2.0) / math.tan(math.radians(fovx_deg) / 2.0)
    vm = np.concatenate([R, t[:, None]], axis=1).astype(np.float32).reshape(12)
    return {"viewmat": vm, "fx": np.float32(fx), "fy": np.float32(fx),
            "cx": np.float32((width - 1) / 2.0), "cy": np.float32((height - 1) / 2.0),
            "width": int(width), "height": int(height)}


def look_camera(eye, forward, up, width, height, fovx_deg=60.0):
    """Camera at ``eye`` looking along ``forward``; ``up`` fixes the roll.

    Rows of R are the camera axes in world coordinates: right = f x up,
    down = f x right, forward = f; t = -R eye."""
    f = np.asarray(forward, dtype=np.float64)
    f = f / np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r = r / np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ np.asarray(eye, dtype=np.float64)
    return make_camera(R, t, width, height, fovx_deg)


def _quats(rng, n):
    q = rng.normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _sh(rng, n, degree, dc_std, rest_std):
    k = (degree + 1) ** 2
    sh = np.empty((k, 3, n), dtype=np.float32)
    rng.normal(None, std=dc_std, out=sh[:1])
    if k > 1:
        rng.normal(None, std=rest_std, out=sh[1:])
    return sh


def tiny_scene(n=2000, seed=0, sh_degree=0):
    """2K Gaussians in a 4x4x4 box 3-7 units in front of an identity-pose camera.

    means: x, y ~ U[-2, 2], z ~ U[3, 7]; log-scales ~ N(-3.5, 0.5) per axis;
    quaternions normalised N(0, I); opacity logits ~ N(0, 1.5); SH DC ~ N(0, 0.5)
    (higher bands, if asked for, ~ N(0, 0.1)). Camera: 128x128, fov 60 deg."""
    rng = Rand(seed)
    means = np.empty((3, n), dtype=np.float32)
    means[0] = rng.uniform(n, -2, 2)
    means[1] = rng.uniform(n, -2, 2)
    means[2] = rng.uniform(n, 3, 7)
    ls = rng.normal((3, n), -3.5, 0.5)
    q = _quats(rng, n)
    op = rng.normal(n, 0.0, 1.5)
    sh = _sh(rng, n, sh_degree, 0.5, 0.1)
    cam = make_camera(np.eye(3), np.zeros(3), 128, 128)
    return Scene(means, ls, q, op, sh, sh_degree), cam


def mid_scene(n=500_000, seed=0, sh_degree=3, width=1920, height=1080):
    """Clustered mid-size scene.

    95% of the Gaussians sit in 200 isotropic clusters (centres uniform in
    [-20,20]x[-5,5]x[-20,20], offsets N(0, 0.5^2 I)) with heavy-tailed log-scales
    -4 + t_3 (Student t, 3 dof) clipped to [-9, 0]; 5% are large background
    Gaussians on a far shell of radius 100 with log-scales ~ N(1, 0.5).
    Opacity logits ~ N(0, 2); SH degree 3 with DC ~ N(0, 0.5) and higher bands
    ~ N(0, 0.1). Camera at (0, 0, -35) looking at the origin, fovx 60 deg."""
    rng = Rand(seed)
    n_shell = n // 20
    n_cl = n - n_shell
    centres = np.stack([rng.uniform64(200, -20, 20), rng.uniform64(200, -5, 5),
                        rng.uniform64(200, -20, 20)]).astype(np.float32)
    which = rng.integers(n_cl, 200)
    means = np.empty((3, n), dtype=np.float32)
    means[:, :n_cl] = centres[:, which] + rng.normal((3, n_cl), std=0.5)
    d = rng.normal((3, n_shell)).astype(np.float64)
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    means[:, n_cl:] = (d * 100.0).astype(np.float32)
    ls = np.empty((3, n), dtype=np.float32)
    ls[:, :n_cl] = np.clip(np.float32(-4.0) + rng.student_t((3, n_cl), 3), -9.0, 0.0)
    ls[:, n_cl:] = rng.normal((3, n_shell), 1.0, 0.5)
    q = _quats(rng, n)
    op = rng.normal(n, 0.0, 2.0)
    sh = _sh(rng, n, sh_degree, 0.5, 0.1)
    cam = look_camera((0, 0, -35), (0, 0, 1), (0, -1, 0), width, height)
    return Scene(means, ls, q, op, sh, sh_degree), cam


def _city_points(rng, n, n_buildings):
    """City layout on a 1000 x 1000 m ground plane (z up).

    30% of the Gaussians lie on the ground (x, y ~ U[-500, 500], z ~ N(0, 0.2)).
    70% lie on the surfaces (four walls and the roof) of ``n_buildings`` box
    buildings with footprint sides ~ U[10, 40] m and heights lognormal with mean
    20 m and log-sigma 0.6; each building receives Gaussians in proportion to its
    surface area, and each face in proportion to its area."""
    n_ground = int(round(0.3 * n))
    n_b = n - n_ground
    means = np.empty((3, n), dtype=np.float32)
    means[0, :n_ground] = rng.uniform(n_ground, -500, 500)
    means[1, :n_ground] = rng.uniform(n_ground, -500, 500)
    means[2, :n_ground] = rng.normal(n_ground, std=0.2)
    bx = rng.uniform64(n_buildings, -500, 500)
    by = rng.uniform64(n_buildings, -500, 500)
    sx = rng.uniform64(n_buildings, 10, 40)
    sy = rng.uniform64(n_buildings, 10, 40)
    mu = math.log(20.0) - 0.5 * 0.6 ** 2
    h = np.exp(np.random.Generator(np.random.PCG64(rng.ss.spawn(1)[0])).standard_normal(n_buildings) * 0.6 + mu)
    # face areas: 0,1 walls normal to x (sy*h); 2,3 walls normal to y (sx*h); 4 roof (sx*sy)
    areas = np.stack([sy * h, sy * h, sx * h, sx * h, sx * sy], axis=1)
    tot = areas.sum(axis=1)
    b = rng.choice(n_b, tot / tot.sum())
    # face within the building, in proportion to its area
    cum = (np.cumsum(areas, axis=1) / tot[:, None]).astype(np.float32)
    r = rng.uniform(n_b)
    face = np.zeros(n_b, np.int8)
    for f in range(4):
        face += (r > cum[b, f]).astype(np.int8)
    u = rng.uniform(n_b, -0.5, 0.5).astype(np.float64)
    v = rng.uniform(n_b, 0.0, 1.0).astype(np.float64)
    sxb, syb, hb = sx[b], sy[b], h[b]
    wall_x = face <= 1
    wall_y = (face == 2) | (face == 3)
    sign = np.where((face == 0) | (face == 2), -0.5, 0.5)
    x = np.where(wall_x, sign * sxb, u * sxb)
    y = np.where(wall_y, sign * syb, np.where(wall_x, u * syb, (v - 0.5) * syb))
    z = np.where(face == 4, hb, v * hb)
    means[0, n_ground:] = bx[b] + x
    means[1, n_ground:] = by[b] + y
    means[2, n_ground:] = z
    return means


def _aerial_camera(eye, yaw, width, height, pitch_deg=30.0):
    p = math.radians(pitch_deg)
    f = (math.cos(yaw) * math.cos(p), math.sin(yaw) * math.cos(p), -math.sin(p))
    return look_camera(eye, f, (0, 0, 1), width, height)


def city_scene(n=6_000_000, seed=0, sh_degree=3, n_buildings=3000, width=4608, height=3456,
               progress=None):
    """City-scale scene: ground plane plus box buildings, log-scales ~ N(-1, 1.2),
    opacity logits ~ N(0, 2), SH degree 3 (DC ~ N(0, 0.5), bands ~ N(0, 0.1)).
    Oblique aerial camera at (0, -600, 150) looking along +y, pitched 30 deg down,
    fovx 60 deg, 4608x3456 (the Mill-19 resolution of Table I)."""
    say = progress or (lambda *_: None)
    rng = Rand(seed)
    means = _city_points(rng, n, n_buildings)
    say("city scene: positions drawn")
    ls = rng.normal((3, n), -1.0, 1.2)
    q = _quats(rng, n)
    op = rng.normal(n, 0.0, 2.0)
    say("city scene: shapes drawn")
    sh = _sh(rng, n, sh_degree, 0.5, 0.1)
    say("city scene: colours drawn")
    cam = _aerial_camera((0.0, -600.0, 150.0), math.pi / 2, width, height)
    return Scene(means, ls, q, op, sh, sh_degree), cam


def city_calibration_cameras(n_views=16, seed=99, width=4608, height=3456):
    """Calibration viewpoints for the city scene (the paper's 16 sampled
    training views, Sec. 3.4): aerial cameras around the measured one --
    eye (U(-150, 150), -600 + U(-150, 150), 150 + U(-30, 30)) m, yaw
    pi/2 + U(-0.3, 0.3), pitch 30 + U(-5, 5) deg -- none equal to it."""
    rng = np.random.Generator(np.random.PCG64(seed))  # 16 x 5 draws: sequential is fine
    cams = []
    for _ in range(n_views):
        eye = (rng.uniform(-150, 150), -600.0 + rng.uniform(-150, 150), 150.0 + rng.uniform(-30, 30))
        yaw = math.pi / 2 + rng.uniform(-0.3, 0.3)
        cams.append(_aerial_camera(eye, yaw, width, height, pitch_deg=30.0 + rng.uniform(-5, 5)))
    return cams


def mid_calibration_cameras(n_views=16, seed=98, width=1920, height=1080):
    """Calibration viewpoints for the mid scene: eye (U(-8, 8), U(-4, 4),
    -35 + U(-5, 5)) looking at the origin, none equal to the measured view."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cams = []
    for _ in range(n_views):
        eye = np.array([rng.uniform(-8, 8), rng.uniform(-4, 4), -35.0 + rng.uniform(-5, 5)])
        cams.append(look_camera(tuple(eye), tuple(-eye / np.linalg.norm(eye)), (0, -1, 0), width, height))
    return cams


def diff_workload(n=1_000_000, seed=0, target_seed=7):
    """Differentiable-render workload: the mid-scene generator at N=1M viewed at
    1280x720, with a seeded random target image U[0,1)^(3xHxW)."""
    scene, cam = mid_scene(n=n, seed=seed, sh_degree=3, width=1280, height=720)
    return scene, cam, target_image(cam["width"], cam["height"], target_seed)


def target_image(width, height, seed=7):
    return Rand(seed).uniform((3, height, width))


BATCH_RESOLUTIONS = ((640, 480), (1920, 1080), (3840, 2160), (3660, 3200))


def batched_workload(n=2_000_000, seed=0, n_views=64, orbit_seed=1234, n_buildings=1000):
    """Batched multi-view workload: a city-style scene of ``n`` Gaussians and
    ``n_views`` cameras at 150 m altitude on a radius-600 m orbit, azimuth
    2 pi k / n_views + U(-pi/n_views, pi/n_views), pitched 30 deg down toward the
    centre; view k has resolution ``BATCH_RESOLUTIONS[k % 4]``."""
    scene, _ = city_scene(n=n, seed=seed, n_buildings=n_buildings)
    rng = np.random.Generator(np.random.PCG64(orbit_seed))  # 64 draws: sequential is fine
    cams = []
    for k in range(n_views):
        az = 2 * math.pi * k / n_views + rng.uniform(-math.pi / n_views, math.pi / n_views)
        eye = (600 * math.cos(az), 600 * math.sin(az), 150.0)
        w, h = BATCH_RESOLUTIONS[k % 4]
        cams.append(_aerial_camera(eye, az + math.pi, w, h))
    return scene, cams


WORKLOADS = {
    "tiny": "2,000 Gaussians, 128x128, SH degree 0",
    "mid": "500K clustered Gaussians, 1920x1080, SH degree 3",
    "city": "6M-Gaussian synthetic city, 4608x3456, SH degree 3",
    "diff": "1M mid-style Gaussians, 1280x720, SH degree 3, L1 to a random target",
    "batched": "2M-Gaussian city, 64 views of mixed resolution",
}


def workload(name, **kw):
    if name == "tiny":
        return tiny_scene(**kw)
    if name == "mid":
        return mid_scene(**kw)
    if name == "city":
        return city_scene(**kw)
    if name == "diff":
        return diff_workload(**kw)
    if name == "batched":
        return batched_workload(**kw)
    raise KeyError(name)
