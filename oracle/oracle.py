"""Python face of the FP64 CPU oracle (``gs_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the HIP path.  The C library is
built with ``gcc -O2 -ffp-contract=off`` (``build()``); this module only
marshals numpy arrays and strings the stages together:

    preprocess -> emit -> sort -> ranges -> blend        (Sec. 2.1, eq. 1-2)
    AdaGScale: eq. (10) threshold, Th >= opacity cull,
               reduced tile extent (Sec. 3.1-3.3)
    backward:  analytic adjoint with frozen decisions

It also carries the image metrics (PSNR, SSIM) and the peripheral-score
helpers (eq. 4, eq. 8-9) used to pin eq. (10).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gs_oracle.c")
LIB = os.path.join(HERE, "libgs_oracle.so")
# The same source built with OpenMP: the per-Gaussian preprocess loop and the
# per-tile blend loop run on all the host's threads.  Used only to time the
# oracle as a CPU baseline; parity runs use the single-threaded build.
LIB_OMP = os.path.join(HERE, "libgs_oracle_omp.so")

TAU = 1.0 / 255.0
T_STOP = 1e-4
TILE = 16
LUT_BINS = 20


def _compile(out, openmp):
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", SRC, "-o", out, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.check_call(cmd)


def build(force: bool = True) -> str:
    for out, omp in ((LIB, False), (LIB_OMP, True)):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            _compile(out, omp)
    return LIB


_lib = None
_openmp = False


def use_openmp(on: bool = True):
    """Switch the wrappers to the OpenMP build (timing) or back to the
    single-threaded one (parity, the default)."""
    global _lib, _openmp
    if bool(on) != _openmp:
        _openmp = bool(on)
        _lib = None


def threads() -> int:
    return int(lib().orc_threads())


def lib():
    global _lib
    if _lib is None:
        path = LIB_OMP if _openmp else LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            _compile(path, _openmp)
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_sh_basis.argtypes = [C.c_int, P, P, P]
        L.orc_plain_extent.argtypes = [C.c_double] * 3
        L.orc_plain_extent.restype = C.c_double
        L.orc_adagscale.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, P, C.c_double,
                                    C.c_int, P, P]
        L.orc_adagscale.restype = C.c_int
        L.orc_preprocess.argtypes = ([C.c_int64, P, P, P, P, P, C.c_int, P, C.c_int, C.c_int,
                                      C.c_int, C.c_double, P, C.c_double, C.c_int, C.c_int]
                                     + [P] * 14)
        L.orc_emit.argtypes = [C.c_int64, P, P, P, C.c_int, C.c_int, P, P, P, P, P, P, P]
        L.orc_obb_spans.argtypes = [C.c_double] * 6 + [C.c_int] * 4 + [P, P]
        L.orc_obb_spans.restype = C.c_int
        L.orc_ellipse_spans.argtypes = [C.c_double] * 7 + [C.c_int] * 4 + [P]
        L.orc_ellipse_spans.restype = C.c_int
        L.orc_emit.restype = C.c_int64
        L.orc_sort.argtypes = [C.c_int64, P, P]
        L.orc_ranges.argtypes = [C.c_int64, P, C.c_int, P]
        L.orc_blend.argtypes = [C.c_int, C.c_int, P, P, P, P, P, C.c_int64, P, P, P, P, P, P, P, P,
                                P]
        L.orc_t_upper_accumulate.argtypes = [C.c_int64, P, P, C.c_double, P]
        L.orc_contrib_profile.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int, C.c_double, P, P]
        L.orc_blend_skip.argtypes = ([C.c_int, C.c_int, P, P, P, P, P, C.c_int64, C.c_int,
                                      C.c_double, P, P, P, C.c_double] + [P] * 6)
        L.orc_blend_bruteforce.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_int, P, P, P, P, P, P,
                                           P, P]
        L.orc_blend_backward.argtypes = [C.c_int, C.c_int, P, P, P, P, P, P, P, C.c_int64]
        L.orc_constants.argtypes = [P]
        L.orc_threads.restype = C.c_int
        L.orc_preprocess_backward.argtypes = [C.c_int64, P, P, P, P, P, C.c_int, P, C.c_int,
                                              C.c_int, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def cam_array(cam) -> np.ndarray:
    return np.concatenate([np.asarray(cam["viewmat"], np.float32).reshape(12),
                           np.array([cam["fx"], cam["fy"], cam["cx"], cam["cy"]], np.float32)])


def default_lut():
    return np.ones(LUT_BINS, dtype=np.float32)


@dataclass
class Mode:
    """Per-call method switch: plain 3D-GS (``adagscale=False``) or AdaGScale
    with peripheral-loss budget ``K`` and depth LUT ``t_upper`` over
    [0, ``lut_depth_max``] (Sec. 3.4).  K and lut_depth_max are single
    precision at the library interface, so the oracle rounds them the same way."""
    adagscale: bool = False
    K: float = 0.0
    t_upper: np.ndarray = None
    lut_depth_max: float = 100.0
    force_unit_scale: bool = False
    extent_rule: int = 0   # 0: tile rectangle; 1: alpha >= Th ellipse; 2: oriented 3-sigma box

    def lut(self):
        return _f32(self.t_upper if self.t_upper is not None else default_lut())


@dataclass
class Preproc:
    mean2d: np.ndarray
    conic: np.ndarray
    quad: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray
    depth: np.ndarray
    cov2d: np.ndarray
    extent: np.ndarray
    th: np.ndarray
    scale: np.ndarray
    rect: np.ndarray
    tiles_touched: np.ndarray
    radius: np.ndarray
    flags: np.ndarray
    extent_rule: int = 0

    def record(self, kind: str = "stored") -> np.ndarray:
        """Per-Gaussian record the blend reads, [n][9]: mean x, mean y, the
        conic of eq. (1) (Cxx, Cxy, Cyy: d^T Sigma2^-1 d = Cxx dx^2 + 2 Cxy dx dy
        + Cyy dy^2), opacity, r, g, b, in double.

        kind "stored": the values of the renderer's float32 splat record.  The
          mean, opacity and colour are rounded to float32, and so are the
          record's sum-of-squares fields A = Cxx, beta = Cxy / Cxx,
          gamma = Cyy - Cxy^2 / Cxx; the conic is then formed from those
          float32 values in double (Cxx = A, Cxy = A beta, Cyy = A beta^2 +
          gamma).
        kind "exact": nothing rounded but the mean, which the interface keeps
          as float32 pixel coordinates; the conic and every other value are
          the double-precision preprocess outputs (the inverse of the
          projected covariance, eq. 1).
        kind "double": nothing rounded (gradient checks)."""
        if kind == "stored":
            q = self.quad.astype(np.float32).astype(np.float64)
            A, beta, gamma = q[:, 0], q[:, 1], q[:, 2]
            conic = np.stack([A, A * beta, (A * beta) * beta + gamma], axis=1)
            mean = self.mean2d.astype(np.float32).astype(np.float64)
            att = np.concatenate([self.opacity[:, None], self.rgb], axis=1)
            att = att.astype(np.float32).astype(np.float64)
        elif kind in ("exact", "double"):
            conic = self.conic
            mean = self.mean2d
            if kind == "exact":
                mean = mean.astype(np.float32).astype(np.float64)
            att = np.concatenate([self.opacity[:, None], self.rgb], axis=1)
        else:
            raise ValueError(f"record kind {kind!r}")
        rec = np.concatenate([mean, conic, att], axis=1)
        return np.ascontiguousarray(rec, np.float64)

    @property
    def depth_f32(self):
        return self.depth.astype(np.float32)


def preprocess(scene, cam, mode: Mode = Mode()) -> Preproc:
    L = lib()
    n = scene.n
    out = Preproc(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), quad=np.zeros((n, 3)),
                  opacity=np.zeros(n),
                  rgb=np.zeros((n, 3)), depth=np.zeros(n), cov2d=np.zeros((n, 3)),
                  extent=np.zeros(n), th=np.zeros(n), scale=np.zeros(n),
                  rect=np.zeros((n, 4), np.int32), tiles_touched=np.zeros(n, np.int64),
                  radius=np.zeros(n, np.int32), flags=np.zeros(n, np.int32),
                  extent_rule=int(mode.extent_rule))
    arrs = [_f32(scene.means), _f32(scene.log_scales), _f32(scene.quats),
            _f32(scene.opacity_logits), _f32(scene.sh)]
    ca = cam_array(cam)
    lut = mode.lut()
    L.orc_preprocess(n, *[_p(a) for a in arrs], scene.sh_degree, _p(ca), cam["width"],
                     cam["height"], int(mode.adagscale), float(np.float32(mode.K)), _p(lut),
                     float(np.float32(mode.lut_depth_max)), int(mode.force_unit_scale),
                     int(mode.extent_rule), _p(out.mean2d), _p(out.conic), _p(out.quad), _p(out.opacity), _p(out.rgb),
                     _p(out.depth),
                     _p(out.cov2d), _p(out.extent), _p(out.th), _p(out.scale), _p(out.rect),
                     _p(out.tiles_touched), _p(out.radius), _p(out.flags))
    return out


def num_tiles(cam):
    return ((cam["width"] + TILE - 1) // TILE) * ((cam["height"] + TILE - 1) // TILE)


def emit(pre: Preproc, cam):
    L = lib()
    n = pre.rect.shape[0]
    d32 = _f32(pre.depth_f32)
    geo_arrays = [np.ascontiguousarray(a, np.float64)
                  for a in (pre.mean2d, pre.quad, pre.opacity, pre.th, pre.scale)]
    geo = [_p(a) for a in geo_arrays]
    args = (n, _p(pre.rect), _p(pre.tiles_touched), _p(d32), cam["width"], pre.extent_rule, *geo)
    np_ = L.orc_emit(*args, None, None)
    keys = np.zeros(max(np_, 1), np.uint64)
    vals = np.zeros(max(np_, 1), np.uint32)
    L.orc_emit(*args, _p(keys), _p(vals))
    return keys[:np_], vals[:np_]


def obb_spans(u, v, A, beta, gamma, s, ty0, ty1, cx0, cx1):
    """Rule-2 row test on explicit values: (ok, spans[rows][2], vertices[4][2])
    of the oriented 3-sigma box (scaled by s) of the covariance recovered from
    (A, beta, gamma)."""
    spans = np.zeros((max(ty1 - ty0, 0), 2), np.int32)
    verts = np.zeros((4, 2))
    ok = lib().orc_obb_spans(float(u), float(v), float(A), float(beta), float(gamma), float(s),
                             int(ty0), int(ty1), int(cx0), int(cx1), _p(spans), _p(verts))
    return bool(ok), spans, verts


def ellipse_spans(u, v, A, beta, gamma, sigma, t, ty0, ty1, cx0, cx1):
    """Rule-1 row test on explicit values: for tile rows ty0 .. ty1-1, the
    inclusive tile-column span [a, b] (empty when b < a) that meets the ellipse
    A (X + beta Y)^2 + gamma Y^2 <= 2 ln(sigma / t), clipped to [cx0, cx1].
    Returns (ok, spans[rows][2]); the values are used as given (no float32
    rounding)."""
    spans = np.zeros((max(ty1 - ty0, 0), 2), np.int32)
    ok = lib().orc_ellipse_spans(float(u), float(v), float(A), float(beta), float(gamma),
                                 float(sigma), float(t), int(ty0), int(ty1), int(cx0), int(cx1),
                                 _p(spans))
    return bool(ok), spans


def sort(keys, vals):
    k = np.ascontiguousarray(keys, np.uint64).copy()
    v = np.ascontiguousarray(vals, np.uint32).copy()
    lib().orc_sort(k.size, _p(k), _p(v))
    return k, v


def ranges(sorted_keys, ntiles):
    r = np.zeros((ntiles, 2), np.int64)
    k = np.ascontiguousarray(sorted_keys, np.uint64)
    lib().orc_ranges(k.size, _p(k), ntiles, _p(r))
    return r


@dataclass
class Frame:
    pre: Preproc
    keys: np.ndarray         # emitted, Gaussian-major
    vals: np.ndarray
    sorted_keys: np.ndarray
    sorted_vals: np.ndarray
    ranges: np.ndarray
    image: np.ndarray = None
    final_T: np.ndarray = None
    n_contrib: np.ndarray = None
    margin: np.ndarray = None
    evals: np.ndarray = None
    sig: np.ndarray = None


def blend(frame_or_parts, cam, bg=(0.0, 0.0, 0.0), tiles=None, rec=None, bound=False):
    """Blend every tile (or the tile ids in ``tiles``).  Returns image [3][H][W],
    final_T [H][W], n_contrib [H][W], per-pixel decision margin (distance to
    the nearest threshold in units of a float32 renderer's first-order error
    bound; below 1 the float32 decision may differ), evaluation counts and
    blend signatures; pixels outside the selected tiles are 0.  With
    ``bound``, also the per-pixel first-order float32 error bound of the
    image, [3][H][W], appended to the tuple."""
    f = frame_or_parts
    W, H = cam["width"], cam["height"]
    if rec is None:
        rec = f.pre.record()
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int64)
    mg = np.full((H, W), np.inf)
    ev = np.zeros((H, W), np.int64)
    sg = np.zeros((H, W), np.uint64)
    bgv = np.asarray(bg, np.float64)
    rg = np.ascontiguousarray(f.ranges, np.int64)
    sv = np.ascontiguousarray(f.sorted_vals, np.uint32)
    if tiles is None:
        sel, nsel = None, -1
    else:
        sel = np.ascontiguousarray(tiles, np.int32)
        nsel = sel.size
    bd = np.zeros((3, H, W)) if bound else None
    lib().orc_blend(W, H, _p(rg), _p(sv), _p(rec), _p(bgv), _p(sel), nsel, _p(img), _p(T),
                    _p(nc), _p(mg), _p(ev), _p(sg), None, None, _p(bd))
    if bound:
        return img, T, nc, mg, ev, sg, bd
    return img, T, nc, mg, ev, sg


def blend_counts(frame: "Frame", cam, tiles=None, rec=None):
    """Per-pixel work of the blend: (list entries evaluated, Gaussians
    blended, decision margin), each [H][W]; pixels outside ``tiles`` are 0."""
    W, H = cam["width"], cam["height"]
    if rec is None:
        rec = frame.pre.record()
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int64)
    mg = np.full((H, W), np.inf)
    ev = np.zeros((H, W), np.int64)
    bl = np.zeros((H, W), np.int64)
    bgv = np.zeros(3)
    rg = np.ascontiguousarray(frame.ranges, np.int64)
    sv = np.ascontiguousarray(frame.sorted_vals, np.uint32)
    sel = None if tiles is None else np.ascontiguousarray(tiles, np.int32)
    nsel = -1 if sel is None else sel.size
    lib().orc_blend(W, H, _p(rg), _p(sv), _p(rec), _p(bgv), _p(sel), nsel, _p(img), _p(T),
                    _p(nc), _p(mg), _p(ev), None, _p(bl), None, None)
    return ev, bl, mg


def blend_skip(frame: "Frame", cam, kind, theta, weight=None, lut=None, lut_depth_max=100.0,
               bg=(0.0, 0.0, 0.0), tiles=None, rec=None):
    """Blend with the contribution-skip rule (Sec. 2.4, 3.2): a blend whose
    contribution is below theta is skipped (no colour, no T update).  kind 0:
    alpha T (eq. 3); 1: alpha weight[i] (max(T^i)); 2: alpha T_up(depth_i) from
    the 20-bin `lut` over [0, lut_depth_max].  Returns (image, final_T,
    n_contrib, margin, blended per pixel, skipped blends in total)."""
    W, H = cam["width"], cam["height"]
    rec = np.ascontiguousarray(frame.pre.record() if rec is None else rec, np.float64)
    n = rec.shape[0]
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int64)
    mg = np.full((H, W), np.inf)
    bl = np.zeros((H, W), np.int64)
    sk = np.zeros(1, np.int64)
    bgv = np.asarray(bg, np.float64)
    w = np.ascontiguousarray(weight if weight is not None else np.zeros(max(n, 1)), np.float64)
    d32 = _f32(frame.pre.depth_f32) if frame.pre is not None else np.zeros(max(n, 1), np.float32)
    lt = np.ascontiguousarray(lut if lut is not None else np.ones(LUT_BINS), np.float64)
    rg = np.ascontiguousarray(frame.ranges, np.int64)
    sv = np.ascontiguousarray(frame.sorted_vals, np.uint32)
    sel = None if tiles is None else np.ascontiguousarray(tiles, np.int32)
    nsel = -1 if sel is None else sel.size
    lib().orc_blend_skip(W, H, _p(rg), _p(sv), _p(rec), _p(bgv), _p(sel), nsel, int(kind),
                         float(theta), _p(w), _p(d32), _p(lt), float(lut_depth_max), _p(img),
                         _p(T), _p(nc), _p(mg), _p(bl), _p(sk))
    return img, T, nc, mg, bl, int(sk[0])


def contrib_profile(frame: "Frame", cam, nbins=34, bin_width=0.1, rec=None):
    """Fig. 4(b): per bin of the Mahalanobis distance between pixel and mean,
    the sum and count of the contributions alpha T of the frame's blends."""
    rec = np.ascontiguousarray(frame.pre.record() if rec is None else rec, np.float64)
    sums = np.zeros(nbins)
    counts = np.zeros(nbins, np.int64)
    lib().orc_contrib_profile(cam["width"], cam["height"], _p(np.ascontiguousarray(frame.ranges, np.int64)),
                              _p(np.ascontiguousarray(frame.sorted_vals, np.uint32)), _p(rec),
                              int(nbins), float(bin_width), _p(sums), _p(counts))
    return sums, counts


def max_transmittance(frame: "Frame", cam, rec=None):
    """Per Gaussian, the largest transmittance in front of it over the pixels
    where it is blended (max(T^i), Sec. 3.2); 0 where it is never blended.
    Also returns the per-pixel decision margin."""
    W, H = cam["width"], cam["height"]
    if rec is None:
        rec = frame.pre.record()
    n = rec.shape[0]
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int64)
    mg = np.full((H, W), np.inf)
    mt = np.zeros(max(n, 1))
    rg = np.ascontiguousarray(frame.ranges, np.int64)
    sv = np.ascontiguousarray(frame.sorted_vals, np.uint32)
    lib().orc_blend(W, H, _p(rg), _p(sv), _p(np.ascontiguousarray(rec, np.float64)), _p(np.zeros(3)),
                    None, -1, _p(img), _p(T), _p(nc), _p(mg), None, None, None, _p(mt), None)
    return mt[:n], mg


def t_upper_accumulate(depth_f32, max_t, lut_depth_max, lut=None):
    """Raise the 20-bin T_upper table (Sec. 3.4) with one view's per-Gaussian
    max transmittance, binned by the float32 depth; returns the table."""
    lut = np.zeros(20) if lut is None else np.ascontiguousarray(lut, np.float64)
    d = np.ascontiguousarray(depth_f32, np.float32)
    m = np.ascontiguousarray(max_t, np.float64)
    lib().orc_t_upper_accumulate(d.size, _p(d), _p(m), float(lut_depth_max), _p(lut))
    return lut


def t_upper_finish(lut):
    """Bins no calibration Gaussian fell in get 1 (the trivial bound)."""
    lut = np.asarray(lut, np.float64).copy()
    lut[~(lut > 0)] = 1.0
    return lut


def render(scene, cam, mode: Mode = Mode(), bg=(0.0, 0.0, 0.0), tiles=None) -> Frame:
    pre = preprocess(scene, cam, mode)
    keys, vals = emit(pre, cam)
    sk, sv = sort(keys, vals)
    rg = ranges(sk, num_tiles(cam))
    fr = Frame(pre, keys, vals, sk, sv, rg)
    fr.image, fr.final_T, fr.n_contrib, fr.margin, fr.evals, fr.sig = blend(fr, cam, bg, tiles)
    return fr


def blend_bruteforce(pre: Preproc, cam, mode_id=1, bg=(0.0, 0.0, 0.0)):
    W, H = cam["width"], cam["height"]
    n = pre.rect.shape[0]
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int64)
    rec = pre.record()
    d32 = _f32(pre.depth_f32)
    bgv = np.asarray(bg, np.float64)
    lib().orc_blend_bruteforce(mode_id, n, W, H, _p(pre.rect), _p(pre.flags), _p(d32), _p(rec),
                               _p(bgv), _p(img), _p(T), _p(nc))
    return img, T, nc


def blend_backward(frame: Frame, cam, dL_dimage, bg=(0.0, 0.0, 0.0), rec=None, tiles=None):
    """Per-Gaussian gradients of the blend: [N][9] = d(mean x, mean y, Cxx,
    Cxy, Cyy, opacity, r, g, b), the record's entries (see Preproc.record).
    With ``tiles``, only those tiles' pixels are differentiated (dL/dimage is
    taken as zero elsewhere)."""
    n = frame.pre.rect.shape[0]
    if rec is None:
        rec = frame.pre.record()
    g2d = np.zeros((n, 9))
    bgv = np.asarray(bg, np.float64)
    dL = np.ascontiguousarray(dL_dimage, np.float64)
    sel = None if tiles is None else np.ascontiguousarray(tiles, np.int32)
    lib().orc_blend_backward(cam["width"], cam["height"], _p(np.ascontiguousarray(frame.ranges)),
                             _p(np.ascontiguousarray(frame.sorted_vals, np.uint32)), _p(rec),
                             _p(bgv), _p(dL), _p(g2d), _p(sel), -1 if sel is None else sel.size)
    return g2d


def preprocess_backward(scene, cam, pre: Preproc, g2d):
    n, K = scene.n, (scene.sh_degree + 1) ** 2
    out = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opacity_logits=np.zeros(n), sh=np.zeros((K, 3, n)))
    arrs = [_f32(scene.means), _f32(scene.log_scales), _f32(scene.quats),
            _f32(scene.opacity_logits), _f32(scene.sh)]
    ca = cam_array(cam)
    lib().orc_preprocess_backward(n, *[_p(a) for a in arrs], scene.sh_degree, _p(ca), cam["width"],
                                  cam["height"], _p(pre.flags), _p(np.ascontiguousarray(g2d)),
                                  _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]),
                                  _p(out["opacity_logits"]), _p(out["sh"]))
    return out


def constants():
    out = np.zeros(10)
    lib().orc_constants(_p(out))
    keys = ["tau", "t_stop", "lut_bins", "two_pi", "alpha_max", "near_z", "dilation",
            "frustum_slack", "lambda_floor", "tile"]
    return dict(zip(keys, out.tolist()))


def sh_basis(degree, d, with_grad=False):
    d = np.ascontiguousarray(d, np.float64)
    k = (degree + 1) ** 2
    Y = np.zeros(k)
    dY = np.zeros((k, 3)) if with_grad else None
    lib().orc_sh_basis(degree, _p(d), _p(Y), _p(dY))
    return (Y, dY) if with_grad else Y


def plain_extent(a, b, c):
    return lib().orc_plain_extent(a, b, c)


def adagscale(det, sigma, depth, K, t_upper=None, lut_depth_max=100.0, force_unit_scale=False):
    lut = _f32(t_upper if t_upper is not None else default_lut())
    th = np.zeros(1)
    s = np.zeros(1)
    keep = lib().orc_adagscale(det, sigma, depth, K, _p(lut), lut_depth_max,
                               int(force_unit_scale), _p(th), _p(s))
    return bool(keep), float(th[0]), float(s[0])


# ---------------------------------------------------------------------------
# Image metrics (AdaGScale is compared with the plain render; Sec. 4.1 uses PSNR)
# ---------------------------------------------------------------------------
def psnr(a, b):
    a = np.clip(np.asarray(a, np.float64), 0, 1)
    b = np.clip(np.asarray(b, np.float64), 0, 1)
    mse = np.mean((a - b) ** 2)
    return float("inf") if mse == 0 else float(10 * np.log10(1.0 / mse))


def _gauss_window(size=11, sigma=1.5):
    x = np.arange(size) - (size - 1) / 2
    g = np.exp(-x ** 2 / (2 * sigma ** 2))
    g /= g.sum()
    return np.outer(g, g)


def ssim(a, b, k1=0.01, k2=0.03):
    """SSIM of Wang et al. (2004): 11x11 Gaussian window (sigma 1.5), valid
    region, C1 = (k1)^2, C2 = (k2)^2 for unit dynamic range, mean over channels."""
    from scipy.signal import correlate2d
    a = np.clip(np.asarray(a, np.float64), 0, 1)
    b = np.clip(np.asarray(b, np.float64), 0, 1)
    w = _gauss_window()
    c1, c2 = k1 ** 2, k2 ** 2
    vals = []
    for ch in range(a.shape[0]):
        x, y = a[ch], b[ch]
        f = lambda z: correlate2d(z, w, mode="valid")
        mx, my = f(x), f(y)
        sxx = f(x * x) - mx * mx
        syy = f(y * y) - my * my
        sxy = f(x * y) - mx * my
        m = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
        vals.append(m.mean())
    return float(np.mean(vals))
