"""Helpers shared by the GPU tests: run the HIP path through the C-ABI and
fetch its outputs; compare with the oracle."""
import numpy as np
import torch

from paper_2604_18980_amd import render as R
from paper_2604_18980_amd import gsr

EXEMPT_MARGIN = 1e-4   # relative distance of a blend decision to its threshold
IMAGE_TOL = 2e-5       # max-abs per channel outside exempt pixels


def to_np(t):
    return t.detach().cpu().numpy()


def decode_rects(r):
    r = r.astype(np.uint64)
    return np.stack([(r >> np.uint64(s)) & np.uint64(0xFFFF) for s in (0, 16, 32, 48)], 1).astype(np.int64)


def gpu_frame(scene, cam, mode=None, bg=(0.0, 0.0, 0.0), capacity=None, staged=True):
    """Full frame through the C-ABI.  Returns a dict of numpy outputs.  The
    staged path (gs_emit_pairs + gs_sort) also yields the emission-order pairs;
    otherwise gs_bin_pairs runs, with sorted tiles requested, and the
    emission-order arrays are absent."""
    mode = mode or {}
    ds = R.DeviceScene.from_host(scene)
    fb = None
    if capacity is not None:
        fb = R.FrameBuffers(ds.n, cam["width"], cam["height"], capacity)
    fb = R.render(ds, cam, bg=bg, fb=fb, staged=staged, with_tiles=not staged, **mode)
    torch.cuda.synchronize()
    P = int(fb.num_pairs.item())
    m = min(P, fb.capacity)
    out = dict(
        n=ds.n, num_pairs=P, capacity=fb.capacity,
        splats=to_np(fb.splats)[: ds.n],
        rects=decode_rects(to_np(fb.rects)[: ds.n]),
        tiles=to_np(fb.tiles_touched)[: ds.n].astype(np.uint32).astype(np.int64),
        pair_tiles=to_np(fb.pair_tiles)[:m].astype(np.uint32).astype(np.int64) if staged else None,
        pair_gids=to_np(fb.pair_gids)[:m].astype(np.uint32).astype(np.int64) if staged else None,
        sorted_tiles=to_np(fb.sorted_tiles)[:m].astype(np.uint32).astype(np.int64),
        sorted_gids=to_np(fb.sorted_gids)[:m].astype(np.uint32).astype(np.int64),
        ranges=to_np(fb.ranges).astype(np.uint32).astype(np.int64),
        image=to_np(fb.image), final_T=to_np(fb.final_T),
        n_contrib=to_np(fb.n_contrib).astype(np.uint32).astype(np.int64),
    )
    return out


def oracle_mode(O, mode):
    mode = mode or {}
    return O.Mode(adagscale=mode.get("adagscale", False), K=mode.get("K", 0.0),
                  t_upper=mode.get("t_upper"), lut_depth_max=mode.get("lut_depth_max", 100.0),
                  force_unit_scale=mode.get("force_unit_scale", False),
                  extent_rule=mode.get("extent_rule", 0))


def check_preprocess(pre, g):
    """Bit-exact discrete outputs and float32 records; colour within 1e-6."""
    np.testing.assert_array_equal(g["tiles"], pre.tiles_touched)
    vis = pre.tiles_touched > 0
    np.testing.assert_array_equal(g["rects"][vis], pre.rect[vis])
    s = g["splats"][vis]
    f32 = lambda a: np.asarray(a, np.float64).astype(np.float32)
    np.testing.assert_array_equal(s[:, 0], f32(pre.mean2d[vis, 0]))
    np.testing.assert_array_equal(s[:, 1], f32(pre.mean2d[vis, 1]))
    np.testing.assert_array_equal(s[:, 2:5], f32(pre.quad[vis]))
    np.testing.assert_array_equal(s[:, 5], f32(pre.opacity[vis]))
    np.testing.assert_array_equal(s[:, 6], f32(pre.depth[vis]))
    np.testing.assert_array_equal(s[:, 7], f32(pre.th[vis]))
    np.testing.assert_array_equal(s[:, 11], f32(pre.scale[vis]))
    assert np.abs(s[:, 8:11] - pre.rgb[vis]).max(initial=0) < 1e-6


def check_pairs(fr, g, cam):
    assert g["num_pairs"] == fr.keys.size
    o_tiles = (fr.keys >> np.uint64(32)).astype(np.int64)
    o_gids = fr.vals.astype(np.int64)
    a = np.lexsort((g["pair_gids"], g["pair_tiles"]))
    b = np.lexsort((o_gids, o_tiles))
    np.testing.assert_array_equal(g["pair_tiles"][a], o_tiles[b])
    np.testing.assert_array_equal(g["pair_gids"][a], o_gids[b])


def check_emission_order(g):
    """Emitted list is depth-major: (float32 depth bits, Gaussian id) never decreases."""
    gid = g["pair_gids"]
    if gid.size < 2:
        return
    d = g["splats"][gid, 6].view(np.uint32).astype(np.int64)
    key = d * (1 << 32) + gid
    assert np.all(np.diff(key) >= 0)


def check_sorted(fr, g, ntiles):
    np.testing.assert_array_equal(g["sorted_tiles"], (fr.sorted_keys >> np.uint64(32)).astype(np.int64))
    np.testing.assert_array_equal(g["sorted_gids"], fr.sorted_vals.astype(np.int64))
    np.testing.assert_array_equal(g["ranges"], fr.ranges)


def check_image(fr, g, tol=IMAGE_TOL, margin=EXEMPT_MARGIN, mask=None):
    """Images within tol outside pixels whose blend decisions sit within
    `margin` of a threshold; returns the number of exempt pixels."""
    ex = fr.margin < margin
    ok = ~ex if mask is None else (~ex & mask)
    diff = np.abs(g["image"] - fr.image)
    assert diff[:, ok].max(initial=0) <= tol, diff[:, ok].max()
    np.testing.assert_array_equal(g["n_contrib"][ok], fr.n_contrib[ok])
    assert np.abs(g["final_T"] - fr.final_T)[ok].max(initial=0) <= tol
    return int((ex if mask is None else (ex & mask)).sum())
