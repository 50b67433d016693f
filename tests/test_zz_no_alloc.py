"""gs_sort_noalloc (the sort on the library's fixed scratch array, no
workspace argument) against gs_sort with a caller workspace, through the
C-ABI: sorted tile ids, sorted Gaussian ids and tile ranges bit for bit, on two
calls in a row -- the second with fewer pairs and fewer tiles, so it runs on
what the first left in the scratch -- plus the capacity limit, checked on the
host before anything is enqueued."""
import numpy as np
import pytest

from paper_2604_18980_amd import scenes

pytestmark = pytest.mark.gpu


def _pairs(n_pairs, width, height, seed):
    """Pairs in emission order: Gaussian ids ascending, tile ids drawn with a
    skewed (clustered) distribution over the tile grid, so runs of equal tiles
    are long and a stable sort has ties to keep in order."""
    rng = np.random.default_rng(seed)
    TX, TY = (width + 15) // 16, (height + 15) // 16
    nt = TX * TY
    centres = rng.integers(0, nt, size=64)
    tiles = (centres[rng.integers(0, 64, size=n_pairs)] +
             rng.geometric(0.02, size=n_pairs)) % nt
    gids = np.sort(rng.integers(0, 1 << 24, size=n_pairs)).astype(np.uint32)
    return tiles.astype(np.uint32), gids, nt


def _run(torch, gsr, tiles, gids, nt, cap, cam, noalloc):
    dev = torch.device("cuda:0")
    t = torch.from_numpy(tiles.view(np.int32)).to(dev)
    g = torch.from_numpy(gids.view(np.int32)).to(dev)
    pt = torch.zeros(cap, dtype=torch.int32, device=dev)
    pg = torch.zeros(cap, dtype=torch.int32, device=dev)
    pt[: t.numel()] = t
    pg[: g.numel()] = g
    num = torch.tensor([tiles.size], dtype=torch.int64, device=dev)
    st = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    sg = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    rg = torch.full((nt, 2), -1, dtype=torch.int32, device=dev)
    cs = gsr.camera_struct(cam)
    if noalloc:
        gsr.gs_sort_noalloc(pt, pg, num, cap, cs, st, sg, rg)
    else:
        wsb = gsr.load().gs_workspace_size(0, cap, 0, 0)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        gsr.gs_sort(pt, pg, num, cap, cs, st, sg, rg, ws)
    torch.cuda.synchronize()
    m = tiles.size
    return (st.cpu().numpy().view(np.uint32)[:m], sg.cpu().numpy().view(np.uint32)[:m],
            rg.cpu().numpy().view(np.uint32))


def test_noalloc_sort_equals_workspace_sort():
    import torch
    from paper_2604_18980_amd import gsr
    cases = [(6_200_000, 4608, 3456, 6_500_000, 1), (300_000, 1920, 1080, 310_000, 2)]
    for n_pairs, w, h, cap, seed in cases:
        print(f"noalloc sort case: {n_pairs} pairs, {w}x{h}, capacity {cap}", flush=True)
        tiles, gids, nt = _pairs(n_pairs, w, h, seed)
        cam = scenes.make_camera(np.eye(3), np.zeros(3), w, h)
        a = _run(torch, gsr, tiles, gids, nt, cap, cam, noalloc=True)
        b = _run(torch, gsr, tiles, gids, nt, cap, cam, noalloc=False)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
        # and both are the stable sort by tile (numpy), with its ranges
        order = np.argsort(tiles, kind="stable")
        np.testing.assert_array_equal(a[0], tiles[order])
        np.testing.assert_array_equal(a[1], gids[order])
        starts = np.searchsorted(a[0], np.arange(nt), side="left")
        ends = np.searchsorted(a[0], np.arange(nt), side="right")
        want = np.where((ends > starts)[:, None], np.stack([starts, ends], 1), 0)
        np.testing.assert_array_equal(a[2].astype(np.int64), want)
