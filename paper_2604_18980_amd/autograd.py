"""torch.autograd.Function over the C-ABI: the forward runs the four stages,
the backward runs gs_rasterize_backward (recomputing transmittance from the
stored final T and n_contrib) and gs_preprocess_backward.  The pair set is a
discrete choice of the forward (AdaGScale's scaled extent included) and is
held fixed for the backward."""
from __future__ import annotations

import torch

from . import gsr
from . import render as R


class RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, sh_degree, cam, mode, bg):
        scene = R.DeviceScene(means.detach().contiguous(), log_scales.detach().contiguous(),
                              quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                              sh.detach().contiguous(), int(sh_degree))
        fb = R.render(scene, cam, bg=bg, **(mode or {}))
        ctx.scene, ctx.fb, ctx.cam, ctx.bg = scene, fb, cam, tuple(bg)
        return fb.image.clone()

    @staticmethod
    def backward(ctx, grad_image):
        scene, fb = ctx.scene, ctx.fb
        cam_s = gsr.camera_struct(ctx.cam)
        grad_splats = torch.empty_like(fb.splats)
        gsr.gs_rasterize_backward(fb.splats, fb.n, fb.sorted_gids, fb.ranges, cam_s, ctx.bg,
                                  fb.final_T, fb.n_contrib, grad_image.contiguous(), grad_splats)
        out = [torch.empty_like(t) for t in (scene.means, scene.log_scales, scene.quats,
                                             scene.opacity_logits, scene.sh)]
        grads = gsr.GsSceneGrads(*[t.data_ptr() for t in out])
        gsr.gs_preprocess_backward(scene.struct(), cam_s, fb.tiles_touched, grad_splats, grads)
        ctx.grad_splats = grad_splats
        return (*out, None, None, None, None)


def rasterize(means, log_scales, quats, opacity_logits, sh, sh_degree, cam, bg=(0.0, 0.0, 0.0),
              **mode):
    """Differentiable render of one view: image [3][H][W].  Parameters in the
    library's layouts: means/log_scales [3][n], quats [4][n], opacity_logits
    [n], sh [n][(d+1)^2][3] (render.sh_to_device_layout converts a host
    [(d+1)^2][3][n] array); gradients come back in the same layouts."""
    return RasterizeFn.apply(means, log_scales, quats, opacity_logits, sh, sh_degree, cam, mode, bg)
