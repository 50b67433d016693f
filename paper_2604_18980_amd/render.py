"""Frame driver over the C-ABI: device buffers (torch allocations) and the
four stage calls of one frame, preprocess -> emit -> sort -> rasterize.

Every stage runs in libgsr's HIP kernels; this module only allocates and
enqueues.  ``FrameBuffers`` keeps the buffers of one view so repeated frames
(benchmarks, HIP-graph capture) allocate nothing.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import gsr


def sh_to_device_layout(sh):
    """Host SH [(d+1)^2][3][n] -> the library's Gaussian-major [n][(d+1)^2][3]."""
    return np.ascontiguousarray(np.asarray(sh, np.float32).transpose(2, 0, 1))


def sh_to_host_layout(sh):
    """The library's [n][(d+1)^2][3] (numpy or tensor) -> host [(d+1)^2][3][n]."""
    if isinstance(sh, torch.Tensor):
        sh = sh.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(sh).transpose(1, 2, 0))


@dataclass
class DeviceScene:
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @staticmethod
    def from_host(scene, device="cuda") -> "DeviceScene":
        """Upload a host scene (numpy, SH as [(d+1)^2][3][n]); SH goes to the
        library's Gaussian-major layout [n][(d+1)^2][3]."""
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return DeviceScene(f(scene.means), f(scene.log_scales), f(scene.quats),
                           f(scene.opacity_logits), f(sh_to_device_layout(scene.sh)),
                           int(scene.sh_degree))

    def struct(self) -> gsr.GsScene:
        return gsr.scene_struct(self.means, self.log_scales, self.quats, self.opacity_logits,
                                self.sh, self.sh_degree)


def num_tiles(width, height):
    return ((width + 15) // 16) * ((height + 15) // 16)


class FrameBuffers:
    """All device buffers of one (scene size, image size, pair capacity)."""

    def __init__(self, n, width, height, capacity, device="cuda"):
        self.n, self.width, self.height, self.device = int(n), int(width), int(height), device
        self.splats = torch.empty((max(self.n, 1), 12), dtype=torch.float32, device=device)
        self.rects = torch.empty(max(self.n, 1), dtype=torch.int64, device=device)
        self.tiles_touched = torch.empty(max(self.n, 1), dtype=torch.int32, device=device)
        self.num_pairs = torch.zeros(1, dtype=torch.int64, device=device)
        npix = self.width * self.height
        self.ranges = torch.empty((num_tiles(width, height), 2), dtype=torch.int32, device=device)
        self.image = torch.empty((3, self.height, self.width), dtype=torch.float32, device=device)
        self.final_T = torch.empty((self.height, self.width), dtype=torch.float32, device=device)
        self.n_contrib = torch.empty((self.height, self.width), dtype=torch.int32, device=device)
        assert npix == self.final_T.numel()
        self.capacity = -1
        self.extent_rule = 0  # the rule of the last preprocess; emission must match it
        self.set_capacity(capacity)

    def set_capacity(self, capacity):
        capacity = int(capacity)
        if capacity == self.capacity:
            return
        self.capacity = capacity
        c = max(capacity, 1)
        d = self.device
        self.pair_tiles = torch.empty(c, dtype=torch.int32, device=d)
        self.pair_gids = torch.empty(c, dtype=torch.int32, device=d)
        self.sorted_tiles = torch.empty(c, dtype=torch.int32, device=d)
        self.sorted_gids = torch.empty(c, dtype=torch.int32, device=d)
        ws_bytes = gsr.gs_workspace_size(self.n, capacity, self.width, self.height)
        self.ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=d)


def run_preprocess(scene: DeviceScene, cam_s, mode_s, fb: FrameBuffers, stream=None):
    gsr.gs_preprocess(scene.struct(), cam_s, mode_s, fb.splats, fb.rects, fb.tiles_touched, stream)
    fb.extent_rule = int(mode_s.extent_rule)


def run_emit(fb: FrameBuffers, cam_s, stream=None):
    gsr.gs_emit_pairs(fb.splats, fb.rects, fb.tiles_touched, fb.n, cam_s, fb.extent_rule,
                      fb.pair_tiles, fb.pair_gids, fb.capacity, fb.num_pairs, fb.ws, stream)


def run_sort(fb: FrameBuffers, cam_s, stream=None):
    gsr.gs_sort(fb.pair_tiles, fb.pair_gids, fb.num_pairs, fb.capacity, cam_s, fb.sorted_tiles,
                fb.sorted_gids, fb.ranges, fb.ws, stream)


def run_bin(fb: FrameBuffers, cam_s, stream=None, with_tiles=False):
    """Emission + sort + ranges in one call (gs_bin_pairs); pair_tiles and
    pair_gids are not written, sorted_tiles only with with_tiles."""
    gsr.gs_bin_pairs(fb.splats, fb.rects, fb.tiles_touched, fb.n, cam_s, fb.extent_rule,
                     fb.sorted_gids, fb.sorted_tiles if with_tiles else None, fb.ranges,
                     fb.capacity, fb.num_pairs, fb.ws, stream)


def run_raster(fb: FrameBuffers, cam_s, bg, stream=None, cfg=None, n_evaluated=None):
    gsr.gs_rasterize(fb.splats, fb.n, fb.sorted_gids, fb.ranges, cam_s, bg, cfg, fb.image,
                     fb.final_T, fb.n_contrib, n_evaluated, stream)


def raster_work(fb: FrameBuffers, cam_s, stream=None):
    """The default rasterizer's work on fb's lists (gs_raster_work), as a dict
    of Python ints; synchronises."""
    import torch
    w = torch.zeros(4, dtype=torch.int64, device=fb.image.device)
    gsr.gs_raster_work(fb.splats, fb.n, fb.sorted_gids, fb.ranges, cam_s, w, stream)
    v = w.cpu().tolist()
    return dict(list_evaluations=v[0], strip_evaluations=v[1], blended=v[2], loaded=v[3])


def enqueue_frame(scene: DeviceScene, cam_s, mode_s, fb: FrameBuffers, bg=(0.0, 0.0, 0.0),
                  stream=None, cfg=None, staged=False):
    """Enqueue one whole frame on the stream; no host synchronisation.  The
    default path bins the pairs with gs_bin_pairs; staged=True runs the
    separate emission and sort entry points instead (same lists)."""
    run_preprocess(scene, cam_s, mode_s, fb, stream)
    if staged:
        run_emit(fb, cam_s, stream)
        run_sort(fb, cam_s, stream)
    else:
        run_bin(fb, cam_s, stream)
    run_raster(fb, cam_s, bg, stream, cfg)


def render(scene: DeviceScene, cam, adagscale=False, K=0.0, t_upper=None, lut_depth_max=100.0,
           force_unit_scale=False, bg=(0.0, 0.0, 0.0), fb: FrameBuffers = None, slack=1.0,
           staged=False, with_tiles=False, extent_rule=0):
    """Render one frame.  Sizes the pair buffers from a counting pass (one host
    read of the pair count) unless ``fb`` already has enough capacity.
    staged=True uses gs_emit_pairs + gs_sort (emission-order pairs kept in
    fb.pair_tiles / fb.pair_gids); otherwise gs_bin_pairs, which also writes
    fb.sorted_tiles when with_tiles."""
    cam_s = gsr.camera_struct(cam)
    mode_s = gsr.mode_struct(adagscale, K, t_upper, lut_depth_max, force_unit_scale, extent_rule)
    if fb is None:
        fb = FrameBuffers(scene.n, cam["width"], cam["height"], 0, scene.means.device)
    run_preprocess(scene, cam_s, mode_s, fb)
    if staged:
        run_emit(fb, cam_s)
        need = int(fb.num_pairs.item())
        if need > fb.capacity:
            fb.set_capacity(int(need * slack))
            run_emit(fb, cam_s)
        run_sort(fb, cam_s)
    else:
        run_bin(fb, cam_s, with_tiles=with_tiles)
        need = int(fb.num_pairs.item())
        if need > fb.capacity:
            fb.set_capacity(int(need * slack))
            run_bin(fb, cam_s, with_tiles=with_tiles)
    run_raster(fb, cam_s, bg)
    return fb
