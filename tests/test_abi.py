"""The C-ABI library loads, exports every entry point declared in
include/gsr.h, and rejects invalid arguments on the host before any HIP call
(so these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def G():
    from paper_2604_18980_amd import gsr
    if not os.path.exists(gsr.LIB_PATH):
        from paper_2604_18980_amd import build
        build.build(verbose=False)
    gsr.load()
    return gsr


def test_exports_every_declared_symbol(G):
    names = declared()
    assert len(names) >= 10
    L = G.load()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(G.EXPORTS)


def exported_symbols():
    """Names in libgsr.so's dynamic symbol table that it defines."""
    import subprocess
    from paper_2604_18980_amd import gsr
    out = subprocess.run(["nm", "-D", "--defined-only", gsr.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    return {line.split()[-1] for line in out.splitlines() if line.strip()}


def test_exported_c_symbols_equal_header(G):
    """The C-linkage symbols libgsr.so exports are exactly the entry points
    gsr.h declares (hidden visibility by default).  Everything else it exports
    is a kernel handle (C++-mangled, the HIP runtime looks kernels up by name)
    or a compiler-generated compilation-unit id."""
    syms = exported_symbols()
    c_syms = {s for s in syms if not s.startswith("_Z") and not s.startswith("__hip_cuid_")}
    assert c_syms == set(declared()), sorted(c_syms ^ set(declared()))
    mangled = {s for s in syms if s.startswith("_Z")}
    # every mangled export is a __global__ function of the gsr kernels (k_...)
    assert all("k_" in s for s in mangled), sorted(s for s in mangled if "k_" not in s)


def test_plane_offsets_are_64_bit(tmp_path):
    """The structure-of-arrays plane offset k n + g the preprocess kernels and
    their adjoint index with, evaluated on the host (hipcc, no GPU) at the
    largest n the interface accepts: exact, where 32-bit arithmetic wraps for
    n above about 7.2e8."""
    import subprocess
    src = tmp_path / "plane.cpp"
    src.write_text(
        '#include "gsr_internal.hpp"\n#include <stdio.h>\n'
        "int main() {\n"
        "  const int n = 2147483647, g = n - 1;\n"
        "  for (int k = 0; k < 4; ++k) {\n"
        "    unsigned long long want = (unsigned long long)k * 2147483647ull + 2147483646ull;\n"
        "    if (gsr::plane_at(k, n, g) != want) { printf(\"bad %d\\n\", k); return 1; }\n"
        "  }\n"
        "  printf(\"ok\\n\");\n  return 0;\n}\n")
    exe = tmp_path / "plane"
    cmd = ["/opt/rocm/bin/hipcc", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2604_18980_amd", "csrc"), str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout


def test_scene_size_limit(G):
    """n is accepted below 2^31 (ids are 32-bit) and rejected from 2^31 on,
    before anything is enqueued."""
    L = G.load()
    P = C.c_void_p
    cam = _cam(G)
    mode = G.mode_struct()
    sc = G.GsScene()
    for p in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        setattr(sc, p, 4096)
    sc.n = 1 << 31
    assert L.gs_preprocess(C.byref(sc), C.byref(cam), C.byref(mode), P(1), P(1), P(1), None) == 1
    assert b"2^31" in L.gs_last_error()
    grads = G.GsSceneGrads(4096, 4096, 4096, 4096, 4096)
    assert L.gs_preprocess_backward(C.byref(sc), C.byref(cam), P(1), P(1), C.byref(grads),
                                    None) == 1


def test_version_and_status_strings(G):
    assert "gfx950" in G.gs_version()
    L = G.load()
    assert L.gs_status_string(0) == b"ok"
    assert L.gs_status_string(2) == b"capacity exceeded"


def test_workspace_size_grows(G):
    a = G.gs_workspace_size(1000, 10_000, 128, 128)
    b = G.gs_workspace_size(1000, 20_000, 128, 128)
    c = G.gs_workspace_size(2000, 20_000, 128, 128)
    assert 0 < a < b < c
    assert G.gs_workspace_size(0, 0, 1, 1) > 0
    assert G.gs_workspace_size(-1, 0, 1, 1) == 0


def _cam(G, w=64, h=64):
    from paper_2604_18980_amd import scenes
    import numpy as np
    return G.camera_struct(scenes.make_camera(np.eye(3), np.zeros(3), w, h))


def test_invalid_arguments_rejected_on_host(G):
    L = G.load()
    P = C.c_void_p
    cam = _cam(G)
    mode = G.mode_struct()
    sc = G.GsScene()
    sc.n = 10
    sc.sh_degree = 0
    # NULL scene arrays
    assert L.gs_preprocess(C.byref(sc), C.byref(cam), C.byref(mode), P(1), P(1), P(1), None) == 1
    assert b"NULL" in L.gs_last_error()
    sc.sh_degree = 4
    assert L.gs_preprocess(C.byref(sc), C.byref(cam), C.byref(mode), P(1), P(1), P(1), None) == 1
    assert b"sh_degree" in L.gs_last_error()
    sc.sh_degree = 0
    sc.n = -1
    assert L.gs_preprocess(C.byref(sc), C.byref(cam), C.byref(mode), P(1), P(1), P(1), None) == 1
    # bad camera
    bad = _cam(G, 0, 10)
    assert L.gs_rasterize(P(1), 1, P(1), P(1), C.byref(bad), (C.c_float * 3)(), None, P(1), P(1),
                          P(1), None, None) == 1
    bad = _cam(G)
    bad.fx = float("nan")
    assert L.gs_rasterize(P(1), 1, P(1), P(1), C.byref(bad), (C.c_float * 3)(), None, P(1), P(1),
                          P(1), None, None) == 1
    # bad mode
    sc.n = 10
    for p in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        setattr(sc, p, 4096)
    m = G.mode_struct(adagscale=True, K=-1.0)
    assert L.gs_preprocess(C.byref(sc), C.byref(cam), C.byref(m), P(1), P(1), P(1), None) == 1
    assert b"K" in L.gs_last_error()
    m = G.mode_struct(adagscale=True, K=0.1, t_upper=[2.0] * 20)
    assert L.gs_preprocess(C.byref(sc), C.byref(cam), C.byref(m), P(1), P(1), P(1), None) == 1
    m = G.mode_struct(extent_rule=3)
    assert L.gs_preprocess(C.byref(sc), C.byref(cam), C.byref(m), P(1), P(1), P(1), None) == 1
    assert b"extent_rule" in L.gs_last_error()
    # unknown extent rule at emission and binning
    assert L.gs_emit_pairs(P(1), P(1), P(1), 10, C.byref(cam), 3, P(1), P(1), 100, P(1), P(1),
                           1 << 40, None) == 1
    assert b"extent_rule" in L.gs_last_error()
    assert L.gs_bin_pairs(P(1), P(1), P(1), 10, C.byref(cam), -1, P(1), None, P(1), 100, P(1),
                          P(1), 1 << 40, None) == 1
    assert b"extent_rule" in L.gs_last_error()
    # workspace too small
    assert L.gs_emit_pairs(P(1), P(1), P(1), 10, C.byref(cam), 0, P(1), P(1), 100, P(1), P(1), 8,
                           None) == 2
    assert b"workspace" in L.gs_last_error()
    # capacity beyond 32-bit indices
    assert L.gs_sort(P(1), P(1), P(1), 1 << 33, C.byref(cam), P(2), P(2), P(1), P(1), 1 << 40,
                     None) == 1
    # sorted output aliasing the input
    assert L.gs_sort(P(1), P(1), P(1), 100, C.byref(cam), P(1), P(2), P(3), P(4), 1 << 40,
                     None) == 1
    # unsupported raster geometry
    cfg = G.GsRasterCfg(100, 1, 256)
    assert L.gs_rasterize(P(1), 1, P(1), P(1), C.byref(cam), (C.c_float * 3)(), C.byref(cfg), P(1),
                          P(1), P(1), None, None) == 4


def test_binding_raises_with_message(G):
    cam = _cam(G)
    with pytest.raises(G.GsrError, match="NULL"):
        sc = G.GsScene()
        sc.n = 5
        G.gs_preprocess(sc, cam, G.mode_struct(), None, None, None, stream=0)


def test_render_views_rejects_bad_arguments(G):
    L = G.load()
    P = C.c_void_p
    sc = G.GsScene()
    sc.n = 10
    sc.sh_degree = 0
    for p in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        setattr(sc, p, 4096)
    mode = G.mode_struct()
    frames = (G.GsViewFrame * 2)()
    for f in frames:
        f.cam = _cam(G)
        f.splats = f.rects = f.tiles_touched = f.sorted_gids = f.ranges = 4096
        f.num_pairs = f.image = f.final_T = f.n_contrib = f.ws = 4096
        f.pair_capacity = 100
        f.ws_bytes = 1 << 40
    bg = (C.c_float * 3)()
    args = lambda n, lanes, ws_bytes: (C.byref(sc), C.byref(mode), C.cast(frames, P), n, bg, None,
                                       lanes, None, P(4096), ws_bytes, None)
    assert L.gs_render_views(*args(0, 1, 1 << 40)) == 1
    assert L.gs_render_views(*args(65, 1, 1 << 40)) == 1
    assert L.gs_render_views(*args(2, 0, 1 << 40)) == 1
    assert L.gs_render_views(*args(2, 9, 1 << 40)) == 1
    assert b"lanes" in L.gs_last_error()
    assert L.gs_render_views(*args(2, 1, 16)) == 2          # views workspace too small
    frames[1].ws_bytes = 16
    assert L.gs_render_views(*args(2, 1, 1 << 40)) == 2     # view 1's binning workspace
    assert b"view 1" in L.gs_last_error()
    frames[1].ws_bytes = 1 << 40
    frames[0].pair_capacity = 1 << 33
    assert L.gs_render_views(*args(2, 1, 1 << 40)) == 1
    frames[0].pair_capacity = 100
    frames[1].cam.width = 0
    assert L.gs_render_views(*args(2, 1, 1 << 40)) == 1
    assert G.gs_render_views_workspace_size(64, 1_400_960) > G.gs_views_workspace_size(64, 1_400_960)


def test_sort_noalloc_limit(G):
    """gs_sort_noalloc rejects a pair capacity above its fixed scratch's limit
    on the host, before anything is enqueued, and the whole limit fits that
    scratch."""
    from paper_2604_18980_amd import scenes
    import numpy as np
    L = G.load()
    cam = G.camera_struct(scenes.make_camera(np.eye(3), np.zeros(3), 64, 64))
    P = C.c_void_p
    cap = G.SORT_NOALLOC_MAX_PAIRS + 1
    assert L.gs_sort_noalloc(P(16), P(32), P(48), cap, C.byref(cam), P(64), P(80), P(96),
                             None) == G.GS_ERR_INVALID_ARGUMENT
    assert b"limit" in L.gs_last_error()
    assert L.gs_workspace_size(0, G.SORT_NOALLOC_MAX_PAIRS, 0, 0) <= G.SORT_NOALLOC_SCRATCH_BYTES
