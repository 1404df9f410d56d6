"""torch.autograd.Function over the hand-written HIP adjoint.

forward(means, scales, quats, opacity, sh) -> (C, F, T) renders every view of
the rasterizer; backward(dC, dF, dT) calls fh_render_bwd (Appendix A.2 of the
paper: the adjoint through w_i = alpha_i T_i, transmittance recovered back to
front from the stored final T and last-contributor index) and returns the
gradients of the five differentiable inputs.  Backward reads the binning and
traversal state its forward left in the rasterizer's workspace, so it raises if
the rasterizer ran another forward (or re-planned) in between.  The feature
tensor is frozen
(Section 3.2: f_i is non-differentiable) and gets no gradient.
"""
from __future__ import annotations

import torch

from ._lib import FhError
from .raster import Gaussians, Rasterizer


class RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, feat, rasterizer: Rasterizer, sh_degree: int):
        g = Gaussians(means.contiguous(), scales.contiguous(), quats.contiguous(), opacity.contiguous(),
                      sh.contiguous(), None if feat is None else feat.contiguous(), sh_degree)
        img = rasterizer.forward(g)
        ctx.rasterizer = rasterizer
        ctx.generation = rasterizer.generation
        ctx.g = g
        ctx.img = img
        ctx.mark_non_differentiable(img.n_iter)
        F = img.F if img.F is not None else torch.zeros(img.C.shape[0], 0, device=img.C.device)
        return img.C, F, img.T, img.n_iter

    @staticmethod
    def backward(ctx, dC, dF, dT, _dn):
        r: Rasterizer = ctx.rasterizer
        if r.generation != ctx.generation:
            # the workspace no longer holds this forward's binning and traversal
            raise FhError("the rasterizer ran another forward (or re-planned) after this one: "
                          "backward needs the state of its own forward; use one Rasterizer per forward in flight")
        dC = torch.zeros_like(ctx.img.C) if dC is None else dC.contiguous().float()
        dF = None if (dF is None or ctx.img.F is None) else dF.contiguous().float()
        dT = None if dT is None else dT.contiguous().float()
        grads = r.render_bwd(ctx.g, ctx.img, dC, dF, dT)
        return grads["means"], grads["scales"], grads["quats"], grads["opacity"], grads["sh"], None, None, None


def rasterize(rasterizer: Rasterizer, means, scales, quats, opacity, sh, feat, sh_degree: int):
    """(C [P,3], F [P,D], T [P], n_iter [P]) for all views of `rasterizer`."""
    return RasterizeFn.apply(means, scales, quats, opacity, sh, feat, rasterizer, sh_degree)
