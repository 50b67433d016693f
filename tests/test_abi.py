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
