"""Offline calibration of AdaGScale's transmittance bound and peripheral-loss
budget (paper Sec. 3.2 and 3.4), done once per scene before rendering.

T_upper: each calibration view is rendered in plain mode and
gs_calibrate_t_upper takes, for every Gaussian blended there, the largest
transmittance in front of it over its pixels (max(T^i)) and raises the depth
bin of the Gaussian; the table is the per-bin maximum over all views, 1.0 for
bins no Gaussian reached (the trivial bound).

K: binary search (in log K) for the largest K whose AdaGScale renders keep the
mean PSNR against the plain renders of the same views at or above a target;
PSNR falls as K grows.

Everything runs through the C-ABI; this module only sequences calls."""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gsr
from . import render as R


def t_upper_table(scene: "R.DeviceScene", cams, lut_depth_max: float):
    """20-bin T_upper table over [0, lut_depth_max) from plain renders of
    ``cams``; returns (table float32[20], raw per-bin float bits, uint32)."""
    dev = scene.means.device
    bits = torch.zeros(gsr.LUT_BINS, dtype=torch.int32, device=dev)
    fb = None
    for cam in cams:
        if fb is not None and (fb.width, fb.height) != (cam["width"], cam["height"]):
            fb = None
        fb = R.render(scene, cam, fb=fb, slack=1.1)
        gsr.gs_calibrate_t_upper(fb.splats, fb.n, fb.sorted_gids, fb.ranges, gsr.camera_struct(cam),
                                 lut_depth_max, bits, None)
    raw = bits.cpu().numpy().astype(np.uint32)
    table = raw.view(np.float32).copy()
    table[raw == 0] = 1.0
    return table, raw


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    mse = torch.mean((a.clamp(0, 1) - b.clamp(0, 1)) ** 2).item()
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def search_k(scene: "R.DeviceScene", cams, target_psnr_db: float, t_upper=None,
             lut_depth_max: float = 100.0, lo: float = 1e-3, hi: float = 1e3, iters: int = 14,
             extent_rule: int = 0):
    """Largest K (to float32) with mean PSNR(AdaGScale vs plain) over ``cams``
    at or above the target (Sec. 3.4's offline binary search on calibration
    views); returns (K, mean PSNR at K).  The plain references use the tile
    rectangle; the AdaGScale renders use ``extent_rule``."""
    refs, fb = [], None
    for cam in cams:  # plain references
        if fb is not None and (fb.width, fb.height) != (cam["width"], cam["height"]):
            fb = None
        fb = R.render(scene, cam, fb=fb, slack=1.05)
        refs.append(fb.image.clone())
    mode = dict(adagscale=True, t_upper=t_upper, lut_depth_max=lut_depth_max,
                extent_rule=extent_rule)
    # AdaGScale pairs never exceed plain ones: the last plain buffers serve
    # every view of the same size (grown if a larger view needs it)

    def mean_psnr(K):
        out = []
        for cam, ref in zip(cams, refs):
            f = fb if (fb.width, fb.height) == (cam["width"], cam["height"]) else None
            out.append(psnr(R.render(scene, cam, K=K, fb=f, slack=1.2, **mode).image, ref))
        return float(np.mean(out))

    best, best_p = lo, mean_psnr(lo)
    for _ in range(iters):
        mid = math.sqrt(lo * hi)
        p = mean_psnr(mid)
        if p >= target_psnr_db:
            best, best_p, lo = mid, p, mid
        else:
            hi = mid
    K = float(np.float32(best))
    return K, mean_psnr(K)
