"""Many views of one scene per frame through one C-ABI call, gs_render_views:
every view's preprocess and binning (spread over the library's lane streams),
then every view's tiles rasterized by one persistent launch over a
longest-first (view, tile) queue.  After one eager frame sizes the pair
buffers, the whole frame can be captured in a HIP graph and replayed with no
host work."""
from __future__ import annotations

import numpy as np
import torch

from . import gsr
from . import render as R


class MultiView:
    """lanes: number of library streams the per-view preprocess and binning
    chains are spread over (views are independent until the shared raster
    launch, so their many small kernels overlap); 1 keeps everything on the
    caller's stream."""

    def __init__(self, scene: R.DeviceScene, cams, mode=None, bg=(0.0, 0.0, 0.0), cfg=None,
                 slack=1.02, lanes=4):
        self.scene, self.cams, self.bg = scene, list(cams), tuple(bg)
        self.lanes = max(1, int(lanes))
        self.mode = gsr.mode_struct(**(mode or {}))
        self.cam_s = [gsr.camera_struct(c) for c in self.cams]
        self.cfg = cfg
        dev = scene.means.device
        self.n_views = len(self.cams)
        self.total_tiles = sum(R.num_tiles(c["width"], c["height"]) for c in self.cams)
        self.fbs = [R.FrameBuffers(scene.n, c["width"], c["height"], 0, dev) for c in self.cams]
        self.ws = torch.empty(gsr.gs_render_views_workspace_size(self.n_views, self.total_tiles),
                              dtype=torch.uint8, device=dev)
        self.clock = torch.zeros(1 + self.n_views, dtype=torch.int64, device=dev)
        # size every view's pair buffers from one counting frame (capacity 0)
        self._frames()
        self.enqueue()
        torch.cuda.synchronize()
        for fb in self.fbs:
            fb.set_capacity(int(int(fb.num_pairs.item()) * slack) + 256)
            fb.extent_rule = int(self.mode.extent_rule)
        self._frames()
        self.graph = None

    def _frames(self):
        """The host table of gs_view_frame (rebuilt whenever a buffer moves)."""
        self.frames = (gsr.GsViewFrame * self.n_views)()
        for v, (fb, cs) in enumerate(zip(self.fbs, self.cam_s)):
            f = self.frames[v]
            f.cam = cs
            f.splats, f.rects = fb.splats.data_ptr(), fb.rects.data_ptr()
            f.tiles_touched = fb.tiles_touched.data_ptr()
            f.sorted_gids, f.ranges = fb.sorted_gids.data_ptr(), fb.ranges.data_ptr()
            f.pair_capacity = fb.capacity
            f.num_pairs = fb.num_pairs.data_ptr()
            f.ws, f.ws_bytes = fb.ws.data_ptr(), fb.ws.numel()
            f.image, f.final_T = fb.image.data_ptr(), fb.final_T.data_ptr()
            f.n_contrib = fb.n_contrib.data_ptr()
        # the raster targets alone (host table and a device copy), for timing
        # the persistent raster launch by itself (gs_rasterize_views)
        self.targets = (gsr.GsViewTarget * self.n_views)()
        for v, fb in enumerate(self.fbs):
            self.targets[v] = gsr.GsViewTarget(fb.splats.data_ptr(), fb.sorted_gids.data_ptr(),
                                               fb.ranges.data_ptr(), fb.image.data_ptr(),
                                               fb.final_T.data_ptr(), fb.n_contrib.data_ptr(),
                                               fb.width, fb.height)
        raw = np.frombuffer(bytes(self.targets), dtype=np.uint8)
        self.d_targets = torch.from_numpy(raw.copy()).to(self.scene.means.device)
        self.raster_ws = torch.empty(gsr.gs_views_workspace_size(self.n_views, self.total_tiles),
                                     dtype=torch.uint8, device=self.scene.means.device)

    def enqueue(self, stream=None):
        main = stream if stream is not None else torch.cuda.current_stream()
        gsr.gs_render_views(self.scene.struct(), self.mode, self.frames, self.n_views, self.bg,
                            self.cfg, self.lanes, self.clock, self.ws, main)

    def rasterize(self, cfg=None, stream=None):
        """Only the persistent raster launch over the current lists."""
        gsr.gs_rasterize_views(self.targets, self.d_targets, self.n_views, self.bg,
                               cfg if cfg is not None else self.cfg, self.clock, self.raster_ws,
                               stream)

    def overflowed(self):
        return any(int(fb.num_pairs.item()) > fb.capacity for fb in self.fbs)

    def capture(self):
        """Capture one frame in a HIP graph (after an eager warm-up frame)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.enqueue(s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.enqueue(torch.cuda.current_stream())
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def view_latency_ms(self):
        """Per-view completion time after the launch start, from device clocks."""
        clk = self.clock.cpu().numpy().astype(np.int64)
        dev = self.scene.means.device.index or 0
        return (clk[1:] - clk[0]) / float(gsr.gs_wall_clock_khz(dev))
