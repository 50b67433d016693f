"""Raster-geometry autotuner.

Tiles stay 16x16 (so pair sets stay comparable); what varies is how a tile is
mapped to the machine: threads per tile, pixels per thread and the number of
Gaussian records staged per round.  The built geometries are

    (64, 4, 64)    one wave per tile, 4 pixels per lane, strip culling
    (128, 2, 64)   two waves per tile, 2 pixels per lane (each wave a 16x8 half,
                   walking the list for its own strips)
    (256, 1, B)    one workgroup per tile, 1 pixel per thread, B in {64, 128, 256}

which is every way to cover a 16x16 tile with 64, 128 or 256 threads at 4, 2
or 1 pixels each.

The tuner times every candidate on the caller's actual work (same sorted
lists, same views) with HIP events, keeps the fastest, and caches the choice
in a JSON file keyed by (GPU architecture, resolutions, pairs-per-tile bucket).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import gsr

CANDIDATES = ((64, 4, 64), (128, 2, 64), (256, 1, 64), (256, 1, 128), (256, 1, 256))


def cache_path() -> str:
    return os.environ.get("GSR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gsr", "autotune.json"))


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p + ".tmp", "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(p + ".tmp", p)
    except OSError:
        pass  # a read-only home only loses the cache


def cache_key(resolutions, pairs, tiles) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    res = sorted({(int(w), int(h)) for (w, h) in resolutions})
    ppt = pairs / max(tiles, 1)
    bucket = int(math.floor(math.log2(ppt))) if ppt >= 1 else 0
    return f"{arch}|{res}|ppt2^{bucket}"


def _time(fn, reps):
    fn()  # warm-up (also builds the grid-size cache)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(run, resolutions, pairs, tiles, reps=3, force=False):
    """run(cfg) enqueues the raster work once with geometry cfg.  Returns
    (GsRasterCfg, {candidate: ms}); cached unless force."""
    key = cache_key(resolutions, pairs, tiles)
    db = _load()
    if not force and key in db:
        return gsr.GsRasterCfg(*db[key]["cfg"]), db[key].get("ms", {})
    times = {}
    for c in CANDIDATES:
        cfg = gsr.GsRasterCfg(*c)
        times["x".join(map(str, c))] = _time(lambda: run(cfg), reps)
    best = min(CANDIDATES, key=lambda c: times["x".join(map(str, c))])
    db[key] = {"cfg": list(best), "ms": times}
    _store(db)
    return gsr.GsRasterCfg(*best), times


def tune_views(mv, reps=3, force=False):
    """Pick the geometry of a MultiView's persistent raster launch."""
    pairs = sum(int(fb.num_pairs.item()) for fb in mv.fbs)

    def run(cfg):
        mv.rasterize(cfg)

    cfg, times = tune(run, [(c["width"], c["height"]) for c in mv.cams], pairs, mv.total_tiles,
                      reps, force)
    mv.cfg = cfg
    return cfg, times


def tune_single(fb, cam, bg=(0.0, 0.0, 0.0), reps=3, force=False):
    """Pick the geometry of a one-view gs_rasterize over FrameBuffers fb."""
    from . import render as R
    cam_s = gsr.camera_struct(cam)

    def run(cfg):
        R.run_raster(fb, cam_s, bg, cfg=cfg)

    return tune(run, [(cam["width"], cam["height"])], int(fb.num_pairs.item()),
                R.num_tiles(cam["width"], cam["height"]), reps, force)
