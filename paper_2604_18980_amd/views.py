"""Many views of one scene per frame: per-view preprocess and binning,
then every view's tiles rasterized by one persistent launch over a
longest-first (view, tile) queue (gs_rasterize_views).  After one eager frame
sizes the pair buffers, the whole frame can be captured in a HIP graph and
replayed with no host work."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import gsr
from . import render as R


class MultiView:
    """lanes: number of streams the per-view preprocess and binning chains are
    spread over (views are independent until the shared raster launch, so
    their many small kernels overlap); 1 keeps everything on one stream."""

    def __init__(self, scene: R.DeviceScene, cams, mode=None, bg=(0.0, 0.0, 0.0), cfg=None,
                 slack=1.02, lanes=4):
        self.scene, self.cams, self.bg = scene, list(cams), tuple(bg)
        self.lanes = max(1, int(lanes))
        self.mode = gsr.mode_struct(**(mode or {}))
        self.cam_s = [gsr.camera_struct(c) for c in self.cams]
        self.cfg = cfg
        dev = scene.means.device
        self.fbs = [R.FrameBuffers(scene.n, c["width"], c["height"], 0, dev) for c in self.cams]
        # size every view's pair buffers from one counting pass
        for fb, cs in zip(self.fbs, self.cam_s):
            R.run_preprocess(scene, cs, self.mode, fb)
            R.run_bin(fb, cs)
        torch.cuda.synchronize()
        for fb in self.fbs:
            fb.set_capacity(int(int(fb.num_pairs.item()) * slack) + 256)
        self.n_views = len(self.cams)
        self.total_tiles = sum(R.num_tiles(c["width"], c["height"]) for c in self.cams)
        self.views = (gsr.GsViewTarget * self.n_views)()
        for v, fb in enumerate(self.fbs):
            self.views[v] = gsr.GsViewTarget(fb.splats.data_ptr(), fb.sorted_gids.data_ptr(),
                                             fb.ranges.data_ptr(), fb.image.data_ptr(),
                                             fb.final_T.data_ptr(), fb.n_contrib.data_ptr(),
                                             fb.width, fb.height)
        raw = np.frombuffer(bytes(self.views), dtype=np.uint8)
        self.d_views = torch.from_numpy(raw.copy()).to(dev)
        self.ws = torch.empty(gsr.gs_views_workspace_size(self.n_views, self.total_tiles),
                              dtype=torch.uint8, device=dev)
        self.clock = torch.zeros(1 + self.n_views, dtype=torch.int64, device=dev)
        self.side = [torch.cuda.Stream(device=dev) for _ in range(self.lanes)] if self.lanes > 1 else []
        self.graph = None

    def enqueue(self, stream=None):
        main = stream if stream is not None else torch.cuda.current_stream()
        if not self.side:
            for fb, cs in zip(self.fbs, self.cam_s):
                R.run_preprocess(self.scene, cs, self.mode, fb, main)
                R.run_bin(fb, cs, main)
        else:
            # fork: every lane starts after the work already on the main stream;
            # view v runs on lane v % lanes; join before the shared raster launch
            for s in self.side:
                s.wait_stream(main)
            for v, (fb, cs) in enumerate(zip(self.fbs, self.cam_s)):
                s = self.side[v % len(self.side)]
                R.run_preprocess(self.scene, cs, self.mode, fb, s)
                R.run_bin(fb, cs, s)
            for s in self.side:
                main.wait_stream(s)
        gsr.gs_rasterize_views(self.views, self.d_views, self.n_views, self.bg, self.cfg,
                               self.clock, self.ws, main)

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
