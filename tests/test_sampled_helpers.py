"""The per-tile shortcuts used at full size agree with the oracle's whole
emit -> sort -> ranges -> blend pipeline where both can run."""
import numpy as np
import pytest

from paper_2604_18980_amd import scenes

from sampled import pick_tiles, tile_counts, tile_frame, tile_mask


@pytest.mark.parametrize("case", ["tiny", "mid_subset", "ragged", "tiny_ellipse",
                                  "mid_subset_ellipse"])
def test_tile_shortcuts_match_full_pipeline(O, case):
    pairs = None
    if case == "tiny_ellipse":
        sc, cam = scenes.tiny_scene(n=2000, seed=3)
        mode = O.Mode(extent_rule=1)
    elif case == "mid_subset_ellipse":
        sc, cam = scenes.mid_scene(n=20_000, seed=2, width=480, height=270)
        mode = O.Mode(adagscale=True, K=1.0, extent_rule=1)
    elif case == "tiny":
        sc, cam = scenes.tiny_scene(n=2000, seed=3)
        mode = O.Mode()
    elif case == "mid_subset":
        sc, cam = scenes.mid_scene(n=20_000, seed=2, width=480, height=270)
        mode = O.Mode(adagscale=True, K=1.0)
    else:
        sc, cam = scenes.tiny_scene(n=1500, seed=4)
        cam = dict(cam, width=100, height=37)
        mode = O.Mode()
    fr = O.render(sc, cam, mode)
    if mode.extent_rule != 0:
        pairs = O.emit(fr.pre, cam)
    counts = tile_counts(fr.pre, cam, pairs)
    np.testing.assert_array_equal(counts, fr.ranges[:, 1] - fr.ranges[:, 0])
    tiles = pick_tiles(counts, 12, 4, 0)
    sub, lists = tile_frame(O, fr.pre, cam, tiles, pairs)
    for t, lst in zip(tiles, lists):
        np.testing.assert_array_equal(fr.sorted_vals[fr.ranges[t, 0]:fr.ranges[t, 1]], lst)
    img, T, nc, mg, ev, sg = O.blend(sub, cam, tiles=tiles)
    m = tile_mask(cam, tiles)
    np.testing.assert_array_equal(img[:, m], fr.image[:, m])
    np.testing.assert_array_equal(T[m], fr.final_T[m])
    np.testing.assert_array_equal(nc[m], fr.n_contrib[m])
    # the adjoint over a tile subset equals the full adjoint of a dL/dimage
    # that vanishes outside those tiles
    rng = np.random.default_rng(1)
    dL = rng.normal(size=(3, cam["height"], cam["width"])) * m
    g_sub = O.blend_backward(sub, cam, dL, tiles=tiles)
    g_full = O.blend_backward(fr, cam, dL)
    np.testing.assert_allclose(g_sub, g_full, rtol=1e-12, atol=1e-12)
