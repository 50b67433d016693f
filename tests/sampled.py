"""Per-tile views of the oracle's frame for checks at full size, where the
oracle's whole sort/blend would take too long: list lengths of every tile,
and the sorted lists of a few sampled tiles, derived from the oracle's
rectangles and float32 depths (rectangle rule) or from the oracle's emitted
pairs (ellipse rule, whose pairs are not whole rectangles)."""
import numpy as np

TILE = 16


def tile_counts(pre, cam, pairs=None):
    """Length of every tile's list: how many visible rectangles hold the tile
    (2D difference array over the tile grid), or, given the oracle's emitted
    (keys, vals), how many pairs name it."""
    TX, TY = (cam["width"] + TILE - 1) // TILE, (cam["height"] + TILE - 1) // TILE
    if pairs is not None:
        return np.bincount((pairs[0] >> np.uint64(32)).astype(np.int64), minlength=TX * TY)
    r = pre.rect[pre.tiles_touched > 0].astype(np.int64)
    W1 = TX + 1
    m = (TY + 1) * W1
    b = lambda y, x: np.bincount(y * W1 + x, minlength=m)
    D = b(r[:, 1], r[:, 0]) - b(r[:, 1], r[:, 2]) - b(r[:, 3], r[:, 0]) + b(r[:, 3], r[:, 2])
    return D.reshape(TY + 1, W1).cumsum(0).cumsum(1)[:TY, :TX].reshape(-1)


def tile_lists(pre, cam, tiles, pairs=None):
    """Sorted list of each tile in `tiles`: the visible Gaussians whose
    rectangle holds it (or, given the oracle's emitted (keys, vals), that are
    paired with it), by float32 depth, ties by index."""
    TX = (cam["width"] + TILE - 1) // TILE
    if pairs is not None:
        t_of = (pairs[0] >> np.uint64(32)).astype(np.int64)
        d32 = pre.depth.astype(np.float32)
        out = []
        for t in tiles:
            ids = pairs[1][t_of == int(t)].astype(np.int64)
            out.append(ids[np.lexsort((ids, d32[ids]))].astype(np.uint32))
        return out
    vis = np.nonzero(pre.tiles_touched > 0)[0]
    r = pre.rect[vis]
    d32 = pre.depth[vis].astype(np.float32)
    out = []
    for t in tiles:
        ty, tx = divmod(int(t), TX)
        m = (r[:, 0] <= tx) & (tx < r[:, 2]) & (r[:, 1] <= ty) & (ty < r[:, 3])
        ids = vis[m]
        out.append(ids[np.lexsort((ids, d32[m]))].astype(np.uint32))
    return out


def tile_frame(O, pre, cam, tiles, pairs=None):
    """Oracle Frame whose ranges cover only `tiles` (the other tiles empty),
    for blending or differentiating those tiles alone."""
    lists = tile_lists(pre, cam, tiles, pairs)
    ranges = np.zeros((O.num_tiles(cam), 2), np.int64)
    off = 0
    for t, lst in zip(tiles, lists):
        ranges[int(t)] = (off, off + lst.size)
        off += lst.size
    sv = np.concatenate(lists) if lists else np.zeros(0, np.uint32)
    return O.Frame(pre, None, None, None, sv, ranges), lists


def pick_tiles(counts, n_random, n_heavy, seed):
    """The n_heavy longest lists plus n_random tiles drawn uniformly."""
    rng = np.random.default_rng(seed)
    heavy = np.argsort(counts, kind="stable")[::-1][:n_heavy]
    rand = rng.choice(counts.size, size=min(n_random, counts.size), replace=False)
    return np.unique(np.concatenate([heavy, rand])).astype(np.int32)


def tile_mask(cam, tiles):
    TX = (cam["width"] + TILE - 1) // TILE
    mask = np.zeros((cam["height"], cam["width"]), bool)
    for t in tiles:
        ty, tx = divmod(int(t), TX)
        mask[ty * TILE:(ty + 1) * TILE, tx * TILE:(tx + 1) * TILE] = True
    return mask
