"""gs_bin_pairs (emission, tile sort and ranges fused) on every route it
takes -- one ranking pass (at most 256 tiles), two passes of packed words, and
the emit-then-sort fallback (more than 65536 tiles) -- against the separate
gs_emit_pairs + gs_sort entry points (bit for bit) and against the oracle's
sorted keys and ranges; plus ragged images, empty and culled scenes and the
overflow contract."""
import numpy as np
import pytest

from paper_2604_18980_amd import scenes

from gpu_util import gpu_frame, oracle_mode

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "tiny128":            # 8 x 8 tiles: one pass
        sc, cam = scenes.tiny_scene(n=2000, seed=21)
        return sc, cam, {}
    if name == "tiny128_ada":
        sc, cam = scenes.tiny_scene(n=2000, seed=22)
        return sc, cam, dict(adagscale=True, K=0.1)
    if name == "ragged_257x129":     # 17 x 9 = 153 tiles: one pass, ragged edges
        sc, cam = scenes.tiny_scene(n=3000, seed=23)
        return sc, dict(cam, width=257, height=129, cx=128.0, cy=64.0), {}
    if name == "ragged_300x301":     # 19 x 19 = 361 tiles: two passes
        sc, cam = scenes.tiny_scene(n=3000, seed=24)
        return sc, dict(cam, width=300, height=301, cx=149.5, cy=150.0), {}
    if name == "mid_1920x1080":      # 8160 tiles: two passes, many owners per slice
        sc, cam = scenes.mid_scene(n=40_000, seed=3)
        return sc, cam, dict(adagscale=True, K=0.5)
    if name == "wide_4112x4112":     # 257 x 257 = 66049 tiles: fallback route
        sc, cam = scenes.mid_scene(n=20_000, seed=4, width=4112, height=4112)
        return sc, cam, {}
    if name == "giants_1024x2048":   # 64 x 128 tiles; 40 Gaussians up to the whole image
        # bands beyond 64 tile rows (one Gaussian's rows over several steps of
        # the span kernels' row walk) and spans beyond 16 tiles, among small ones
        sc, cam = scenes.tiny_scene(n=3000, seed=26)
        ls = sc.log_scales.copy()
        ls[:, :40] = np.log(np.linspace(0.3, 2.5, 40, dtype=np.float32))[None, :]
        sc = scenes.Scene(sc.means, ls, sc.quats, sc.opacity_logits, sc.sh, sc.sh_degree)
        return sc, scenes.make_camera(np.eye(3), np.zeros(3), 1024, 2048), {}
    raise KeyError(name)


CASES = ["tiny128", "tiny128_ada", "ragged_257x129", "ragged_300x301", "mid_1920x1080",
         "wide_4112x4112", "giants_1024x2048"]


@pytest.mark.parametrize("rule", [0, 1, 2], ids=["rect", "ellipse", "obb"])
@pytest.mark.parametrize("name", CASES)
def test_bin_equals_staged_and_oracle(O, name, rule):
    """Under the ellipse rule every case takes the emit-then-sort route, with
    the pairs emitted into the sort scratch (one pass), the outputs (two
    passes) or the route's own arrays (beyond the packed limits)."""
    sc, cam, mode = _case(name)
    mode = dict(mode, extent_rule=rule)
    print(f"bin case {name} rule {rule}: n={sc.n} {cam['width']}x{cam['height']}", flush=True)
    st = gpu_frame(sc, cam, mode, staged=True)
    bn = gpu_frame(sc, cam, mode, staged=False)
    P = st["num_pairs"]
    assert bn["num_pairs"] == P
    np.testing.assert_array_equal(bn["ranges"], st["ranges"])
    np.testing.assert_array_equal(bn["sorted_gids"][:P], st["sorted_gids"][:P])
    np.testing.assert_array_equal(bn["sorted_tiles"][:P], st["sorted_tiles"][:P])
    for k in ("image", "final_T", "n_contrib"):
        np.testing.assert_array_equal(bn[k], st[k])
    # against the oracle's sort (O13) and ranges (O14)
    fr = O.render(sc, cam, oracle_mode(O, mode), tiles=np.zeros(0, np.int32))
    assert fr.sorted_keys.size == P
    np.testing.assert_array_equal(bn["sorted_tiles"][:P], (fr.sorted_keys >> np.uint64(32)).astype(np.int64))
    np.testing.assert_array_equal(bn["sorted_gids"][:P], fr.sorted_vals.astype(np.int64))
    np.testing.assert_array_equal(bn["ranges"], fr.ranges)
    print(f"  pairs {P}", flush=True)


def test_bin_empty_and_culled(O):
    sc, cam = scenes.tiny_scene(n=500, seed=25)
    behind = dict(cam)
    vm = np.asarray(cam["viewmat"], np.float32).reshape(3, 4).copy()
    vm[2, 3] = -100.0  # every Gaussian behind the near plane
    behind["viewmat"] = vm.reshape(-1)
    g = gpu_frame(sc, behind, staged=False)
    assert g["num_pairs"] == 0 and not g["ranges"].any()
    empty = sc.subset(np.zeros(0, np.int64))
    g = gpu_frame(empty, cam, staged=False)
    assert g["num_pairs"] == 0 and not g["ranges"].any()
    assert np.all(g["final_T"] == 1.0) and not g["image"].any()


@pytest.mark.parametrize("rule", [0, 1], ids=["rect", "ellipse"])
@pytest.mark.parametrize("name", ["tiny128", "ragged_300x301", "wide_4112x4112", "giants_1024x2048"])
def test_bin_overflow_bins_nothing(O, name, rule):
    """Capacity below the pair count: the required count is reported, no list
    is produced (every range empty, image = background), and a regrown buffer
    gives the full result."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    sc, cam, mode = _case(name)
    mode = dict(mode, extent_rule=rule)
    full = gpu_frame(sc, cam, mode, staged=True)
    ds = R.DeviceScene.from_host(sc)
    cam_s, mode_s = gsr.camera_struct(cam), gsr.mode_struct(**mode)
    fb = R.FrameBuffers(ds.n, cam["width"], cam["height"], full["num_pairs"] // 3)
    R.enqueue_frame(ds, cam_s, mode_s, fb, bg=(0.25, 0.5, 0.75))
    torch.cuda.synchronize()
    assert int(fb.num_pairs.item()) == full["num_pairs"]
    assert not fb.ranges.cpu().numpy().any()
    img = fb.image.cpu().numpy()
    for c, v in enumerate((0.25, 0.5, 0.75)):
        assert np.all(img[c] == np.float32(v))
    fb.set_capacity(full["num_pairs"])
    R.enqueue_frame(ds, cam_s, mode_s, fb)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(fb.image.cpu().numpy(), full["image"])
    np.testing.assert_array_equal(fb.ranges.cpu().numpy().astype(np.uint32).astype(np.int64),
                                  full["ranges"])


def test_bin_reused_workspace_matches_fresh(O):
    """One set of buffers (and so one workspace, whose counters and digit
    group sums each call clears before use) serves frames with many, few and
    no visible Gaussians in turn; each frame equals a render into fresh
    buffers."""
    import torch
    from paper_2604_18980_amd import render as R
    sc, cam = scenes.mid_scene(n=40_000, seed=7, width=640, height=360)
    far = dict(cam)
    vm = np.asarray(cam["viewmat"], np.float32).reshape(3, 4).copy()
    vm[2, 3] += 60.0  # step back: fewer Gaussians get tiles
    far["viewmat"] = vm.reshape(-1)
    behind = dict(cam)
    vb = vm.copy()
    vb[2, 3] = -100.0  # nothing in front
    behind["viewmat"] = vb.reshape(-1)
    ds = R.DeviceScene.from_host(sc)
    fresh = {}
    for name, c in (("near", cam), ("far", far), ("behind", behind)):
        fb = R.render(ds, c, adagscale=True, K=0.3, slack=1.2)
        torch.cuda.synchronize()
        fresh[name] = (fb.image.clone(), fb.ranges.clone(), int(fb.num_pairs.item()))
    shared = R.FrameBuffers(ds.n, cam["width"], cam["height"], max(v[2] for v in fresh.values()) + 64)
    for name, c in (("near", cam), ("far", far), ("behind", behind), ("near", cam), ("far", far)):
        R.render(ds, c, adagscale=True, K=0.3, fb=shared)
        torch.cuda.synchronize()
        img, rg, P = fresh[name]
        print(f"  {name}: pairs {P}", flush=True)
        assert int(shared.num_pairs.item()) == P
        assert torch.equal(shared.ranges, rg)
        assert torch.equal(shared.image, img)


CANARY = -0x5A5A5A5B  # 0xA5A5A5A5 as int32


def _cut_capacities(pair_gids, P):
    """Capacities that stop the emission inside one Gaussian's run of pairs:
    a third of the pairs, mid-way through a run longer than 16 tiles (a long
    row span or several rows), and one pair into a short run."""
    g = pair_gids[:P]
    starts = np.flatnonzero(np.r_[True, g[1:] != g[:-1]])
    lens = np.diff(np.r_[starts, P])
    caps = [P // 3]
    long_runs = np.flatnonzero(lens > 16)
    if long_runs.size:
        i = long_runs[long_runs.size // 2]
        caps.append(int(starts[i] + lens[i] // 2))
    short = np.flatnonzero((lens >= 2) & (lens <= 16))
    if short.size:
        i = short[short.size // 2]
        caps.append(int(starts[i] + 1))
    return sorted(set(c for c in caps if 0 < c < P))


@pytest.mark.parametrize("staged", [True, False], ids=["staged", "bin"])
@pytest.mark.parametrize("rule", [1, 2], ids=["ellipse", "obb"])
def test_overflow_writes_nothing_past_capacity(O, rule, staged):
    """Capacity below the pair count, cutting into long and short spans of the
    giants frame: the pair and sorted arrays are views of larger buffers whose
    tail past the capacity holds a canary, and no store may reach it.  Staged
    emission writes exactly the first `capacity` pairs of the full emission,
    which gs_sort then sorts; gs_bin_pairs bins nothing."""
    import torch
    from paper_2604_18980_amd import gsr, render as R
    sc, cam, mode = _case("giants_1024x2048")
    mode = dict(mode, extent_rule=rule)
    full = gpu_frame(sc, cam, mode, staged=True)
    P = full["num_pairs"]
    caps = _cut_capacities(full["pair_gids"], P)
    assert len(caps) >= 3, caps
    ds = R.DeviceScene.from_host(sc)
    cam_s, mode_s = gsr.camera_struct(cam), gsr.mode_struct(**mode)
    tail = 1 << 20  # more than 64 Gaussians covering the whole 64 x 128-tile image
    for cap in caps:
        print(f"giants rule {rule} {'staged' if staged else 'bin'}: capacity {cap} of {P}", flush=True)
        fb = R.FrameBuffers(ds.n, cam["width"], cam["height"], cap)
        big = {}
        for name in ("pair_tiles", "pair_gids", "sorted_tiles", "sorted_gids"):
            big[name] = torch.full((cap + tail,), CANARY, dtype=torch.int32, device="cuda")
            setattr(fb, name, big[name][:cap])
        R.run_preprocess(ds, cam_s, mode_s, fb)
        if staged:
            R.run_emit(fb, cam_s)
            R.run_sort(fb, cam_s)
        else:
            R.run_bin(fb, cam_s, with_tiles=True)
        torch.cuda.synchronize()
        assert int(fb.num_pairs.item()) == P
        if not staged:  # gs_bin_pairs bins nothing when over capacity
            assert not fb.ranges.cpu().numpy().any()
        for name, b in big.items():
            t = b[cap:].cpu().numpy()
            assert np.all(t == CANARY), f"{name}: {int((t != CANARY).sum())} stores past capacity {cap}"
        if staged:
            # the emitted prefix, and gs_sort's stable sort of it (it reads
            # min(num_pairs, capacity) pairs)
            pt = fb.pair_tiles.cpu().numpy().astype(np.uint32).astype(np.int64)
            pg = fb.pair_gids.cpu().numpy().astype(np.uint32).astype(np.int64)
            np.testing.assert_array_equal(pt, full["pair_tiles"][:cap])
            np.testing.assert_array_equal(pg, full["pair_gids"][:cap])
            order = np.argsort(pt, kind="stable")
            np.testing.assert_array_equal(fb.sorted_tiles.cpu().numpy().astype(np.uint32), pt[order])
            np.testing.assert_array_equal(fb.sorted_gids.cpu().numpy().astype(np.uint32), pg[order])
