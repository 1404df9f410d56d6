"""The training step around the rasterizer (Algorithm 1 of the paper), on the
GPU through the C ABI: render, photometric loss, adjoint, Adam update of the
raw parameters, densification statistics, and periodic adaptive density
control (clone / split / prune).  Argument marshalling only: every step runs in
libfhgs.so.

Raw parameters: means, log_scales (scale = exp), quats (raw), logit_opacity
(opacity = sigmoid), sh.  The activated scales and opacities that rendering
reads are kept beside them and rewritten by every update.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib as L
from .raster import Gaussians, Rasterizer, _same_device, _stream, check_tensor

GROUPS = ("means", "log_scales", "quats", "logit_opacity", "sh")
_F32 = (torch.float32,)


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Params:
    """Raw parameters (FP32, contiguous, on one device) and their activations."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    logit_opacity: torch.Tensor
    sh: torch.Tensor
    scales: torch.Tensor = field(default=None)
    opacity: torch.Tensor = field(default=None)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def sh_degree(self) -> int:
        return int(round(self.sh.shape[1] ** 0.5)) - 1

    def check(self, name: str = "params") -> None:
        n, nb, dev = self.n, self.sh.shape[1], self.means.device
        for k, shp in (("means", (n, 3)), ("log_scales", (n, 3)), ("quats", (n, 4)), ("logit_opacity", (n,)),
                       ("sh", (n, nb, 3))):
            check_tensor(getattr(self, k), f"{name}.{k}", shp, _F32, dev)
        if nb not in (1, 4, 9, 16):
            raise L.FhError(f"{name}.sh must hold (L+1)^2 <= 16 coefficient rows, not {nb}")

    def struct(self) -> L.FhParams:
        return L.FhParams(*[_vp(getattr(self, k)) for k in GROUPS])

    @staticmethod
    def zeros_like(p: "Params") -> "Params":
        return Params(*[torch.zeros_like(getattr(p, k)) for k in GROUPS])

    def gaussians(self, feat: torch.Tensor | None) -> Gaussians:
        return Gaussians(self.means, self.scales, self.quats, self.opacity, self.sh, feat, self.sh_degree)


def activate(p: Params) -> Params:
    """Fill p.scales and p.opacity from the raw values (fh_activate; afterwards
    the Adam and densification kernels keep them current)."""
    p.check()
    n, dev = p.n, p.means.device
    p.scales = torch.empty(n, 3, dtype=torch.float32, device=dev)
    p.opacity = torch.empty(n, dtype=torch.float32, device=dev)
    L.check(L.load().fh_activate(n, _vp(p.log_scales), _vp(p.logit_opacity), _vp(p.scales), _vp(p.opacity),
                                 _stream()), "fh_activate")
    return p


def adam_step(p: Params, m: Params, v: Params, grads: dict, step: int, lr: dict, betas=(0.9, 0.999),
              eps: float = 1e-15) -> None:
    """One Adam step of every group in place (fh_adam_step); grads are the
    rasterizer's gradients of the activated parameters."""
    lib = L.load()
    for q, nm in ((p, "params"), (m, "m"), (v, "v")):
        q.check(nm)
    n, nb, dev = p.n, p.sh.shape[1], p.means.device
    check_tensor(p.scales, "params.scales", (n, 3), _F32, dev)
    check_tensor(p.opacity, "params.opacity", (n,), _F32, dev)
    for k, shp in (("means", (n, 3)), ("scales", (n, 3)), ("quats", (n, 4)), ("opacity", (n,)), ("sh", (n, nb, 3))):
        check_tensor(grads[k], f"grads[{k!r}]", shp, _F32, dev)
    cfg = L.FhAdam((ctypes.c_float * 5)(*[float(lr[k]) for k in GROUPS]), float(betas[0]), float(betas[1]),
                   float(eps), int(step))
    gr = L.FhGrads(*[_vp(grads[k]) for k in ("means", "scales", "quats", "opacity", "sh")])
    ps, ms, vs = p.struct(), m.struct(), v.struct()
    L.check(lib.fh_adam_step(n, p.sh_degree, ctypes.byref(ps), ctypes.byref(ms), ctypes.byref(vs), ctypes.byref(gr),
                             ctypes.byref(cfg), _vp(p.scales), _vp(p.opacity), _stream()), "fh_adam_step")


def densify_stats(r: Rasterizer, grad_sum: torch.Tensor, count: torch.Tensor) -> None:
    """Add the last fh_render_bwd's |dL/d(u, v)| of every view that binned each
    Gaussian into grad_sum [n] and count the views in count [n] (int32)."""
    check_tensor(grad_sum, "grad_sum", (r.n,), _F32, r.device)
    check_tensor(count, "count", (r.n,), (torch.int32,), r.device)
    L.check(r.lib.fh_densify_stats(ctypes.byref(r.plan), _vp(r.ws), _vp(grad_sum), _vp(count), _stream()),
            "fh_densify_stats")


def densify(p: Params, m: Params, v: Params, grad_sum: torch.Tensor, count: torch.Tensor, z: torch.Tensor,
            grad_threshold: float, log_scale_threshold: float, prune_logit: float,
            extra_rows: tuple = ()) -> tuple:
    """Adaptive density control (fh_densify_plan + fh_densify_apply): returns
    the new (params, m, v) and the densified copies of `extra_rows` (per-Gaussian
    tensors such as the frozen features).  z [n, 2, 3]: standard normal draws
    for the split children.  Reads the new size back from the device (one
    synchronisation)."""
    lib = L.load()
    n, dev = p.n, p.means.device
    for q, nm in ((p, "params"), (m, "m"), (v, "v")):
        q.check(nm)
    check_tensor(grad_sum, "grad_sum", (n,), _F32, dev)
    check_tensor(count, "count", (n,), (torch.int32,), dev)
    check_tensor(z, "z", (n, 2, 3), _F32, dev)
    dws = torch.empty(max(int(lib.fh_densify_workspace_size(n)), 256), dtype=torch.uint8, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    cfg = L.FhDensifyConfig(float(grad_threshold), float(log_scale_threshold), float(prune_logit))
    L.check(lib.fh_densify_plan(n, _vp(grad_sum), _vp(count), _vp(p.log_scales), _vp(p.logit_opacity),
                                ctypes.byref(cfg), _vp(dws), _vp(counts), _stream()), "fh_densify_plan")
    n_out, n_keep = (int(x) for x in counts.cpu().tolist())
    nb = p.sh.shape[1]
    e = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)
    mk = lambda: Params(e(n_out, 3), e(n_out, 3), e(n_out, 4), e(n_out), e(n_out, nb, 3))
    out, mo, vo = mk(), mk(), mk()
    out.scales, out.opacity = e(n_out, 3), e(n_out)
    ps, ms, vs, os_, mos, vos = (q.struct() for q in (p, m, v, out, mo, vo))
    L.check(lib.fh_densify_apply(n, p.sh_degree, _vp(dws), ctypes.byref(ps), ctypes.byref(ms), ctypes.byref(vs),
                                 _vp(z), n_out, n_keep, ctypes.byref(os_), ctypes.byref(mos), ctypes.byref(vos),
                                 _vp(out.scales), _vp(out.opacity), _stream()), "fh_densify_apply")
    rows = []
    for t in extra_rows:
        if t is None:
            rows.append(None)
            continue
        if not _same_device(t.device, dev) or not t.is_contiguous() or t.shape[0] != n:
            raise L.FhError("extra rows must be contiguous, on the parameters' device, one row per Gaussian")
        o = torch.empty((n_out,) + tuple(t.shape[1:]), dtype=t.dtype, device=dev)
        row_bytes = t[0].numel() * t.element_size() if n else 0
        L.check(lib.fh_densify_copy_rows(n, _vp(dws), _vp(t), _vp(o), row_bytes, n_out, n_keep, _stream()),
                "fh_densify_copy_rows")
        rows.append(o)
    return out, mo, vo, rows


class PhotometricLoss:
    """Mean squared error of a rendered image against its target and its
    adjoint dC (fh_photometric_loss), with the workspace kept across calls."""

    def __init__(self, n_pixels: int, device="cuda"):
        self.lib = L.load()
        self.P = int(n_pixels)
        self.device = torch.device(device)
        self.lws = torch.empty(max(int(self.lib.fh_loss_workspace_size(self.P)), 256), dtype=torch.uint8,
                               device=self.device)
        self.loss = torch.empty(1, dtype=torch.float32, device=self.device)

    def __call__(self, C: torch.Tensor, C_target: torch.Tensor, dC: torch.Tensor | None = None):
        for t, nm in ((C, "C"), (C_target, "C_target")):
            check_tensor(t, nm, (self.P, 3), _F32, self.device)
        dC = torch.empty_like(C) if dC is None else dC
        check_tensor(dC, "dC", (self.P, 3), _F32, self.device)
        L.check(self.lib.fh_photometric_loss(self.P, _vp(C), _vp(C_target), _vp(dC), _vp(self.loss), _vp(self.lws),
                                             _stream()), "fh_photometric_loss")
        return self.loss, dC


class Trainer:
    """Algorithm 1 on synthetic views: for step i, view i mod V is rendered,
    compared with its target image, differentiated, and the Gaussians updated
    by Adam; densification statistics accumulate after every backward, and
    every `densify_every` steps the density control runs (new Gaussians get
    their split draws from `z_source(n)`)."""

    def __init__(self, params: Params, feat: torch.Tensor | None, cams, targets, lr: dict, form: str = "f32",
                 densify_every: int = 0, grad_threshold: float = 2e-4, log_scale_threshold: float = -3.0,
                 prune_logit: float = -5.3, z_source=None, device="cuda"):
        self.p = params if params.scales is not None else activate(params)
        self.feat = feat
        self.cams = list(cams)
        self.targets = list(targets)
        self.lr = dict(lr)
        self.form = form
        self.densify_every = int(densify_every)
        self.thr = (float(grad_threshold), float(log_scale_threshold), float(prune_logit))
        self.z_source = z_source
        self.device = torch.device(device)
        self.m = Params.zeros_like(self.p)
        self.v = Params.zeros_like(self.p)
        self.t = 0
        self.losses = [PhotometricLoss(c.width * c.height, device) for c in self.cams]
        self._reset_stats()
        self._rasterizers()

    def _reset_stats(self):
        self.grad_sum = torch.zeros(self.p.n, dtype=torch.float32, device=self.device)
        self.count = torch.zeros(self.p.n, dtype=torch.int32, device=self.device)

    def _rasterizers(self):
        d = 0 if self.feat is None else int(self.feat.shape[1])
        fdt = "bf16" if (self.feat is not None and self.feat.dtype == torch.bfloat16) else "f32"
        self.r = [Rasterizer([c], self.p.n, self.p.sh_degree, d, feat_dtype=fdt, form=self.form, device=self.device)
                  for c in self.cams]

    def step(self) -> torch.Tensor:
        """One iteration; returns the loss of the rendered view (device scalar)."""
        vi = self.t % len(self.cams)
        r = self.r[vi]
        g = self.p.gaussians(self.feat)
        img = r.forward(g)
        loss, dC = self.losses[vi](img.C, self.targets[vi])
        grads = r.render_bwd(g, img, dC)
        densify_stats(r, self.grad_sum, self.count)
        self.t += 1
        adam_step(self.p, self.m, self.v, grads, self.t, self.lr)
        if self.densify_every and self.t % self.densify_every == 0:
            self.densify()
        return loss

    def densify(self) -> None:
        z = self.z_source(self.p.n)
        self.p, self.m, self.v, rows = densify(self.p, self.m, self.v, self.grad_sum, self.count, z, *self.thr,
                                               extra_rows=(self.feat,))
        self.feat = rows[0]
        self._reset_stats()
        self._rasterizers()
