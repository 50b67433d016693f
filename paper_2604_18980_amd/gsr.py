"""Thin Python binding of libgsr's C-ABI (``include/gsr.h``).

Functions carry the C names and only marshal arguments: torch tensors supply
device memory (their data pointers) and the current HIP stream; every step of
the render runs in the library's HIP kernels.  There is no fallback: if
``libgsr.so`` is missing or fails to load, the import raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgsr.so")

GS_OK, GS_ERR_INVALID_ARGUMENT, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_UNSUPPORTED = range(5)
LUT_BINS = 20
TILE = 16
SORT_NOALLOC_MAX_PAIRS = 7_000_000          # GS_SORT_NOALLOC_MAX_PAIRS
SORT_NOALLOC_SCRATCH_BYTES = 64 << 20       # GS_SORT_NOALLOC_SCRATCH_BYTES

EXPORTS = ("gs_workspace_size", "gs_preprocess", "gs_emit_pairs", "gs_sort", "gs_sort_noalloc",
           "gs_bin_pairs",
           "gs_rasterize", "gs_raster_work", "gs_calibrate_t_upper", "gs_rasterize_skip",
           "gs_contribution_profile",
           "gs_rasterize_backward", "gs_preprocess_backward", "gs_views_workspace_size",
           "gs_rasterize_views", "gs_render_views_workspace_size", "gs_render_views",
           "gs_wall_clock_khz", "gs_status_string", "gs_last_error", "gs_version")


class GsrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


class GsScene(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("n", C.c_int64),
                ("sh_degree", C.c_int)]


class GsCamera(C.Structure):
    _fields_ = [("viewmat", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int), ("height", C.c_int)]


class GsMode(C.Structure):
    _fields_ = [("adagscale", C.c_int), ("K", C.c_float), ("t_upper", C.c_float * LUT_BINS),
                ("lut_depth_max", C.c_float), ("force_unit_scale", C.c_int),
                ("extent_rule", C.c_int)]


class GsRasterCfg(C.Structure):
    _fields_ = [("threads_per_tile", C.c_int), ("pixels_per_thread", C.c_int),
                ("lds_batch", C.c_int)]


class GsSceneGrads(C.Structure):
    _fields_ = [("d_means", C.c_void_p), ("d_log_scales", C.c_void_p), ("d_quats", C.c_void_p),
                ("d_opacity_logits", C.c_void_p), ("d_sh", C.c_void_p)]


_lib = None


def load():
    """Load libgsr.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2604_18980_amd.build`")
    L = C.CDLL(LIB_PATH)
    P, I64, I = C.c_void_p, C.c_int64, C.c_int
    L.gs_workspace_size.argtypes = [I64, I64, I, I]
    L.gs_workspace_size.restype = C.c_size_t
    L.gs_preprocess.argtypes = [P, P, P, P, P, P, P]
    L.gs_emit_pairs.argtypes = [P, P, P, I64, P, I, P, P, I64, P, P, C.c_size_t, P]
    L.gs_sort.argtypes = [P, P, P, I64, P, P, P, P, P, C.c_size_t, P]
    L.gs_sort_noalloc.argtypes = [P, P, P, I64, P, P, P, P, P]
    L.gs_bin_pairs.argtypes = [P, P, P, I64, P, I, P, P, P, I64, P, P, C.c_size_t, P]
    L.gs_rasterize.argtypes = [P, I64, P, P, P, P, P, P, P, P, P, P]
    L.gs_raster_work.argtypes = [P, I64, P, P, P, P, P]
    L.gs_calibrate_t_upper.argtypes = [P, I64, P, P, P, C.c_float, P, P, P]
    L.gs_rasterize_skip.argtypes = [P, I64, P, P, P, P, I, C.c_float, P, P, C.c_float, P, P, P, P,
                                    P]
    L.gs_contribution_profile.argtypes = [P, I64, P, P, P, I, C.c_float, P, P, P]
    L.gs_rasterize_backward.argtypes = [P, I64, P, P, P, P, P, P, P, P, P]
    L.gs_preprocess_backward.argtypes = [P, P, P, P, P, P]
    L.gs_render_views.argtypes = [P, P, P, I, P, P, I, P, P, C.c_size_t, P]
    L.gs_render_views.restype = C.c_int
    for f in ("gs_preprocess", "gs_emit_pairs", "gs_sort", "gs_sort_noalloc", "gs_bin_pairs",
              "gs_rasterize",
              "gs_raster_work", "gs_calibrate_t_upper", "gs_rasterize_skip", "gs_contribution_profile",
              "gs_rasterize_backward", "gs_preprocess_backward"):
        getattr(L, f).restype = C.c_int
    L.gs_status_string.argtypes = [I]
    L.gs_status_string.restype = C.c_char_p
    L.gs_last_error.restype = C.c_char_p
    L.gs_version.restype = C.c_char_p
    _lib = L
    return L


def _check(status):
    if status != GS_OK:
        msg = load().gs_last_error().decode()
        raise GsrError(status, msg)


def _ptr(t):
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def camera_struct(cam) -> GsCamera:
    c = GsCamera()
    vm = np.asarray(cam["viewmat"], np.float32).reshape(12)
    for i in range(12):
        c.viewmat[i] = float(vm[i])
    c.fx, c.fy, c.cx, c.cy = (float(np.float32(cam[k])) for k in ("fx", "fy", "cx", "cy"))
    c.width, c.height = int(cam["width"]), int(cam["height"])
    return c


def mode_struct(adagscale=False, K=0.0, t_upper=None, lut_depth_max=100.0,
                force_unit_scale=False, extent_rule=0) -> GsMode:
    m = GsMode()
    m.adagscale = 1 if adagscale else 0
    m.K = float(K)
    lut = np.ones(LUT_BINS, np.float32) if t_upper is None else np.asarray(t_upper, np.float32)
    for i in range(LUT_BINS):
        m.t_upper[i] = float(lut[i])
    m.lut_depth_max = float(lut_depth_max)
    m.force_unit_scale = 1 if force_unit_scale else 0
    m.extent_rule = int(extent_rule)
    return m


def scene_struct(means, log_scales, quats, opacity_logits, sh, sh_degree) -> GsScene:
    s = GsScene()
    s.means, s.log_scales, s.quats = _ptr(means), _ptr(log_scales), _ptr(quats)
    s.opacity_logits, s.sh = _ptr(opacity_logits), _ptr(sh)
    s.n = int(means.shape[-1])
    s.sh_degree = int(sh_degree)
    return s


# --------------------------------------------------------------------------- C-ABI mirrors
def gs_version() -> str:
    return load().gs_version().decode()


def gs_workspace_size(n, pair_capacity, width, height) -> int:
    return int(load().gs_workspace_size(int(n), int(pair_capacity), int(width), int(height)))


def gs_preprocess(scene: GsScene, cam: GsCamera, mode: GsMode, splats, rects, tiles_touched,
                  stream=None):
    _check(load().gs_preprocess(C.byref(scene), C.byref(cam), C.byref(mode), _ptr(splats),
                                _ptr(rects), _ptr(tiles_touched), _stream(stream)))


def gs_emit_pairs(splats, rects, tiles_touched, n, cam: GsCamera, extent_rule, pair_tiles,
                  pair_gids, pair_capacity, num_pairs, ws, stream=None):
    _check(load().gs_emit_pairs(_ptr(splats), _ptr(rects), _ptr(tiles_touched), int(n),
                                C.byref(cam), int(extent_rule), _ptr(pair_tiles), _ptr(pair_gids),
                                int(pair_capacity), _ptr(num_pairs), _ptr(ws),
                                int(ws.numel() * ws.element_size()) if ws is not None else 0,
                                _stream(stream)))


def gs_sort(pair_tiles, pair_gids, num_pairs, pair_capacity, cam: GsCamera, sorted_tiles,
            sorted_gids, ranges, ws, stream=None):
    _check(load().gs_sort(_ptr(pair_tiles), _ptr(pair_gids), _ptr(num_pairs), int(pair_capacity),
                          C.byref(cam), _ptr(sorted_tiles), _ptr(sorted_gids), _ptr(ranges),
                          _ptr(ws), int(ws.numel() * ws.element_size()) if ws is not None else 0,
                          _stream(stream)))


def gs_sort_noalloc(pair_tiles, pair_gids, num_pairs, pair_capacity, cam: GsCamera, sorted_tiles,
                    sorted_gids, ranges, stream=None):
    _check(load().gs_sort_noalloc(_ptr(pair_tiles), _ptr(pair_gids), _ptr(num_pairs),
                                  int(pair_capacity), C.byref(cam), _ptr(sorted_tiles),
                                  _ptr(sorted_gids), _ptr(ranges), _stream(stream)))


def gs_bin_pairs(splats, rects, tiles_touched, n, cam: GsCamera, extent_rule, sorted_gids,
                 sorted_tiles, ranges, pair_capacity, num_pairs, ws, stream=None):
    """sorted_tiles may be None (not written)."""
    _check(load().gs_bin_pairs(_ptr(splats), _ptr(rects), _ptr(tiles_touched), int(n),
                               C.byref(cam), int(extent_rule), _ptr(sorted_gids),
                               _ptr(sorted_tiles), _ptr(ranges),
                               int(pair_capacity), _ptr(num_pairs), _ptr(ws),
                               int(ws.numel() * ws.element_size()) if ws is not None else 0,
                               _stream(stream)))


def gs_rasterize(splats, n, sorted_gids, ranges, cam: GsCamera, bg, cfg, image, final_T,
                 n_contrib, n_evaluated=None, stream=None):
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check(load().gs_rasterize(_ptr(splats), int(n), _ptr(sorted_gids), _ptr(ranges),
                               C.byref(cam), bgv, C.byref(cfg) if cfg is not None else None,
                               _ptr(image), _ptr(final_T), _ptr(n_contrib), _ptr(n_evaluated),
                               _stream(stream)))


def gs_raster_work(splats, n, sorted_gids, ranges, cam: GsCamera, work, stream=None):
    _check(load().gs_raster_work(_ptr(splats), int(n), _ptr(sorted_gids), _ptr(ranges),
                                 C.byref(cam), _ptr(work), _stream(stream)))


def gs_calibrate_t_upper(splats, n, sorted_gids, ranges, cam: GsCamera, lut_depth_max, t_upper_bits,
                         max_t_bits=None, stream=None):
    _check(load().gs_calibrate_t_upper(_ptr(splats), int(n), _ptr(sorted_gids), _ptr(ranges),
                                       C.byref(cam), float(lut_depth_max), _ptr(t_upper_bits),
                                       _ptr(max_t_bits), _stream(stream)))


def gs_rasterize_skip(splats, n, sorted_gids, ranges, cam: GsCamera, bg, kind, theta, weight,
                      t_upper, lut_depth_max, image, final_T, n_contrib, counts=None, stream=None):
    """t_upper: host sequence of GS_LUT_BINS floats (kind 2) or None."""
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    lut = None if t_upper is None else (C.c_float * LUT_BINS)(*[float(x) for x in t_upper])
    _check(load().gs_rasterize_skip(_ptr(splats), int(n), _ptr(sorted_gids), _ptr(ranges),
                                    C.byref(cam), bgv, int(kind), float(theta), _ptr(weight), lut,
                                    float(lut_depth_max), _ptr(image), _ptr(final_T),
                                    _ptr(n_contrib), _ptr(counts), _stream(stream)))


def gs_contribution_profile(splats, n, sorted_gids, ranges, cam: GsCamera, nbins, bin_width, sums,
                            counts, stream=None):
    _check(load().gs_contribution_profile(_ptr(splats), int(n), _ptr(sorted_gids), _ptr(ranges),
                                          C.byref(cam), int(nbins), float(bin_width), _ptr(sums),
                                          _ptr(counts), _stream(stream)))


def gs_rasterize_backward(splats, n, sorted_gids, ranges, cam: GsCamera, bg, final_T, n_contrib,
                          dL_dimage, grad_splats, stream=None):
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check(load().gs_rasterize_backward(_ptr(splats), int(n), _ptr(sorted_gids), _ptr(ranges),
                                        C.byref(cam), bgv, _ptr(final_T), _ptr(n_contrib),
                                        _ptr(dL_dimage), _ptr(grad_splats), _stream(stream)))


def gs_preprocess_backward(scene: GsScene, cam: GsCamera, tiles_touched, grad_splats,
                           grads: GsSceneGrads, stream=None):
    _check(load().gs_preprocess_backward(C.byref(scene), C.byref(cam), _ptr(tiles_touched),
                                         _ptr(grad_splats), C.byref(grads), _stream(stream)))


class GsViewTarget(C.Structure):
    _fields_ = [("splats", C.c_void_p), ("sorted_gids", C.c_void_p), ("ranges", C.c_void_p),
                ("image", C.c_void_p), ("final_T", C.c_void_p), ("n_contrib", C.c_void_p),
                ("width", C.c_int), ("height", C.c_int)]


def gs_views_workspace_size(n_views, total_tiles) -> int:
    L = load()
    L.gs_views_workspace_size.argtypes = [C.c_int, C.c_int64]
    L.gs_views_workspace_size.restype = C.c_size_t
    return int(L.gs_views_workspace_size(int(n_views), int(total_tiles)))


def gs_rasterize_views(views_host, d_views, n_views, bg, cfg, clock, ws, stream=None):
    """views_host: ctypes array of GsViewTarget; d_views: a device tensor holding
    the same bytes."""
    L = load()
    L.gs_rasterize_views.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L.gs_rasterize_views.restype = C.c_int
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check(L.gs_rasterize_views(C.cast(views_host, C.c_void_p), _ptr(d_views), int(n_views), bgv,
                                C.byref(cfg) if cfg is not None else None, _ptr(clock), _ptr(ws),
                                int(ws.numel() * ws.element_size()), _stream(stream)))


class GsViewFrame(C.Structure):
    _fields_ = [("cam", GsCamera), ("splats", C.c_void_p), ("rects", C.c_void_p),
                ("tiles_touched", C.c_void_p), ("sorted_gids", C.c_void_p),
                ("ranges", C.c_void_p), ("pair_capacity", C.c_int64), ("num_pairs", C.c_void_p),
                ("ws", C.c_void_p), ("ws_bytes", C.c_size_t), ("image", C.c_void_p),
                ("final_T", C.c_void_p), ("n_contrib", C.c_void_p)]


def gs_render_views_workspace_size(n_views, total_tiles) -> int:
    L = load()
    L.gs_render_views_workspace_size.argtypes = [C.c_int, C.c_int64]
    L.gs_render_views_workspace_size.restype = C.c_size_t
    return int(L.gs_render_views_workspace_size(int(n_views), int(total_tiles)))


def gs_render_views(scene: GsScene, mode: GsMode, frames, n_views, bg, cfg, lanes, clock, ws,
                    stream=None):
    """frames: ctypes array of GsViewFrame (host)."""
    L = load()
    L.gs_render_views.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                  C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_size_t,
                                  C.c_void_p]
    L.gs_render_views.restype = C.c_int
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check(L.gs_render_views(C.byref(scene), C.byref(mode), C.cast(frames, C.c_void_p),
                             int(n_views), bgv, C.byref(cfg) if cfg is not None else None,
                             int(lanes), _ptr(clock), _ptr(ws),
                             int(ws.numel() * ws.element_size()), _stream(stream)))


def gs_wall_clock_khz(device=0) -> int:
    L = load()
    L.gs_wall_clock_khz.argtypes = [C.c_int]
    L.gs_wall_clock_khz.restype = C.c_int
    return int(L.gs_wall_clock_khz(int(device)))
