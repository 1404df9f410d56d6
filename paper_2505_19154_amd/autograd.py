"""torch.autograd.Function over the hand-written HIP adjoint.

forward(means, scales, quats, opacity, sh) -> (C, F, T) renders every view of
the rasterizer; backward(dC, dF, dT) calls fh_render_bwd (Appendix A.2 of the
paper: the adjoint through w_i = alpha_i T_i, transmittance recovered back to
front from the stored final T and last-contributor index) and returns the
gradients of the five differentiable inputs.  Backward reads the binning and
traversal state its forward left in the rasterizer's workspace, so it raises if
the rasterizer ran another forward (or re-planned) in between.  The paper
freezes the features (Section 3.2: f_i is non-differentiable); when a caller
asks for their gradient anyway (feat.requires_grad), dL/df_i = sum_p w_i(p)
dF(p) is the unnormalised fusion of the map dF, computed by fh_fuse_features
(in the BF16 form, which fuses BF16 targets, as the fusion of dF's BF16 hi
part plus that of its lo part into the same compensated accumulators).
"""
from __future__ import annotations

import torch

from ._lib import FH_FORM_BF16, FhError
from .raster import FusionAcc, Gaussians, Rasterizer


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
        dfeat = None
        if ctx.needs_input_grad[5] and ctx.g.feat is not None:
            dfeat = _feature_grad(r, ctx.g, ctx.img, dF)
        return grads["means"], grads["scales"], grads["quats"], grads["opacity"], grads["sh"], dfeat, None, None


def _feature_grad(r: Rasterizer, g: Gaussians, img, dF) -> torch.Tensor:
    """dL/df = sum_p w(p) dF(p) per Gaussian (zero without dF)."""
    feat = g.feat
    if dF is None:
        return torch.zeros_like(feat)
    acc = FusionAcc.zeros(feat.shape[0], feat.shape[1], feat.device)
    if r.plan.form == FH_FORM_BF16:
        hi = dF.to(torch.bfloat16)
        lo = (dF - hi.float()).to(torch.bfloat16)
        r.fuse_features(g, img, hi.contiguous(), acc)
        r.fuse_features(g, img, lo.contiguous(), acc)
    else:
        r.fuse_features(g, img, dF.contiguous(), acc)
    return (acc.sum + acc.comp).to(feat.dtype)


def rasterize(rasterizer: Rasterizer, means, scales, quats, opacity, sh, feat, sh_degree: int):
    """(C [P,3], F [P,D], T [P], n_iter [P]) for all views of `rasterizer`."""
    return RasterizeFn.apply(means, scales, quats, opacity, sh, feat, rasterizer, sh_degree)
