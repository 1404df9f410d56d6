"""Per-pixel brute force without tiles, in torch float64 on the CPU.

The plain definition of what the tiled method computes: for every pixel, take
every visible Gaussian (camera depth beyond the near plane, float32 depth as
the binning decides it), order them by (depth, index), and composite front to
back (Section 3.1: c = sum_i c_i w_i, w_i = alpha_i T_i, T_i = prod_{j<i}
(1 - alpha_j)) with the skip and stop rules of the rasterizer.  No tiles, no
keys, no ranges.  Written with torch float64 operations so that autograd gives
gradients that do not depend on the hand-written adjoint; intended for scenes
of at most a few hundred Gaussians and a few thousand pixels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binspec, consts, sh


def _sh_torch(degree: int, d: torch.Tensor) -> torch.Tensor:
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    cols = []
    for b in range(sh.num_bases(degree)):
        acc = torch.zeros_like(x)
        for (i, j, k), c in sh._POLYS[b].items():
            acc = acc + c * x ** i * y ** j * z ** k
        cols.append(acc)
    return torch.stack(cols, 1)


def _rot(qn: torch.Tensor) -> torch.Tensor:
    w, x, y, z = qn.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def render(params: dict, g_meta: dict, cam, feat: np.ndarray | None, keep_w: list | None = None):
    """params: float64 torch leaves means [N,3], scales [N,3], quats [N,4],
    opacity [N], sh [N,B,3].  Returns C [P,3], F [P,D] or None, T [P], niter [P]
    and the depth order.  keep_w, if a list, receives the weight map w [P] of
    every position of the order (zero where the Gaussian did not blend)."""
    bq = binspec.bin_quantities(g_meta, cam)
    vis = np.nonzero(bq["visible"])[0]
    order = vis[np.lexsort((vis, bq["depth"][vis]))]

    mu, s, q, op, shc = (params[k] for k in ("means", "scales", "quats", "opacity", "sh"))
    Rc = torch.tensor(np.asarray(cam.R, np.float64))
    tc = torch.tensor(np.asarray(cam.t, np.float64))
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    p = mu @ Rc.T + tc
    u = fx * p[:, 0] / p[:, 2] + cx
    v = fy * p[:, 1] / p[:, 2] + cy
    qn = q / q.norm(dim=1, keepdim=True)
    M = _rot(qn) * s[:, None, :]
    S3 = M @ M.transpose(1, 2)
    zero = torch.zeros_like(p[:, 2])
    J = torch.stack([torch.stack([fx / p[:, 2], zero, -fx * p[:, 0] / p[:, 2] ** 2], 1),
                     torch.stack([zero, fy / p[:, 2], -fy * p[:, 1] / p[:, 2] ** 2], 1)], 1)
    Tm = J @ Rc
    S2 = Tm @ S3 @ Tm.transpose(1, 2)
    a = S2[:, 0, 0] + consts.LOWPASS
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + consts.LOWPASS
    det = a * c - b * b
    A, B, C = c / det, -b / det, a / det
    campos = -Rc.T @ tc
    dv = mu - campos
    dirn = dv / dv.norm(dim=1, keepdim=True)
    Y = _sh_torch(int(g_meta["sh_degree"]), dirn)
    rgb = torch.clamp(torch.einsum("nb,nbc->nc", Y, shc) + 0.5, min=0.0)

    W, H = int(cam.width), int(cam.height)
    yy, xx = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(W, dtype=torch.float64),
                            indexing="ij")
    x = xx.reshape(-1) + 0.5
    y = yy.reshape(-1) + 0.5
    P = W * H
    T = torch.ones(P, dtype=torch.float64)
    col = torch.zeros(P, 3, dtype=torch.float64)
    featt = None if feat is None else torch.tensor(np.asarray(feat, np.float64))
    F = None if featt is None else torch.zeros(P, featt.shape[1], dtype=torch.float64)
    done = torch.zeros(P, dtype=torch.bool)
    niter = torch.zeros(P, dtype=torch.int64)
    for pos, gi in enumerate(order.tolist()):
        dx = x - u[gi]
        dy = y - v[gi]
        power = -0.5 * (A[gi] * dx * dx + 2.0 * B[gi] * dx * dy + C[gi] * dy * dy)
        alpha = torch.clamp(op[gi] * torch.exp(power), max=consts.ALPHA_MAX)
        ok = (alpha.detach() >= consts.ALPHA_MIN) & ~done
        Tn = T * (1.0 - alpha)
        stop = ok & (Tn.detach() < consts.T_MIN)
        done = done | stop
        contrib = ok & ~stop
        w = torch.where(contrib, alpha * T, torch.zeros_like(T))
        if keep_w is not None:
            keep_w.append(w)
        col = col + w[:, None] * rgb[gi][None, :]
        if F is not None:
            F = F + w[:, None] * featt[gi][None, :]
        T = torch.where(contrib, Tn, T)
        niter = torch.where(contrib, torch.full_like(niter, pos + 1), niter)
    return col, F, T, niter, order


def render_surfel(params: dict, g_meta: dict, cam, feat: np.ndarray | None, keep_w: list | None = None):
    """The surfel primitive (Section 3.1) by its definition, without tiles:
    every pixel's ray c_w + t d_w (camera centre, direction through the pixel
    centre) meets the plane p + u T_u + v T_v (T_u = s_u t_u, T_v = s_v t_v,
    world tangents from the quaternion) where, by Cramer's rule on
    [T_u, T_v, -d_w] (u, v, t) = c_w - p,
      u = r . (T_v x -d) / det,  v = T_u . (r x -d) / det,  det = T_u . (T_v x -d),
    r = c_w - p; G = exp(-(u^2 + v^2) / 2) (0 for a parallel ray, det = 0),
    alpha = min(0.99, o G).  Every surfel that binning keeps visible (float32
    depth beyond the near plane, opacity above 1/255, its disc in front of the
    camera) is composited in (depth, index) order with the rasterizer's skip
    and stop rules.  Torch float64, so autograd gives gradients independent of
    the hand-written adjoint.  Returns C [P,3], F [P,D] or None, T [P], niter [P]
    and the depth order; keep_w as for render."""
    bq = binspec.bin_quantities(g_meta, cam, "surfel")
    vis = np.nonzero(bq["visible"])[0]
    order = vis[np.lexsort((vis, bq["depth"][vis]))]
    mu, s, q, op, shc = (params[k] for k in ("means", "scales", "quats", "opacity", "sh"))
    Rc = torch.tensor(np.asarray(cam.R, np.float64))
    tc = torch.tensor(np.asarray(cam.t, np.float64))
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    qn = q / q.norm(dim=1, keepdim=True)
    Rq = _rot(qn)
    Tu = Rq[:, :, 0] * s[:, 0:1]
    Tv = Rq[:, :, 1] * s[:, 1:2]
    campos = -Rc.T @ tc
    dv = mu - campos
    dirn = dv / dv.norm(dim=1, keepdim=True)
    Y = _sh_torch(int(g_meta["sh_degree"]), dirn)
    rgb = torch.clamp(torch.einsum("nb,nbc->nc", Y, shc) + 0.5, min=0.0)

    W, H = int(cam.width), int(cam.height)
    yy, xx = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(W, dtype=torch.float64),
                            indexing="ij")
    x = xx.reshape(-1) + 0.5
    y = yy.reshape(-1) + 0.5
    P = W * H
    dcam = torch.stack([(x - cx) / fx, (y - cy) / fy, torch.ones_like(x)], 1)     # [P, 3]
    dw = dcam @ Rc                                                              # R_c^T d
    T = torch.ones(P, dtype=torch.float64)
    col = torch.zeros(P, 3, dtype=torch.float64)
    featt = None if feat is None else torch.tensor(np.asarray(feat, np.float64))
    F = None if featt is None else torch.zeros(P, featt.shape[1], dtype=torch.float64)
    done = torch.zeros(P, dtype=torch.bool)
    niter = torch.zeros(P, dtype=torch.int64)
    for pos, gi in enumerate(order.tolist()):
        r = (campos - mu[gi])[None, :].expand(P, 3)
        nd = -dw
        tvxd = torch.cross(Tv[gi][None, :].expand(P, 3), nd, dim=1)
        det = (Tu[gi][None, :] * tvxd).sum(1)
        uu = (r * tvxd).sum(1)
        vv = (Tu[gi][None, :] * torch.cross(r, nd, dim=1)).sum(1)
        live = det != 0
        dsafe = torch.where(live, det, torch.ones_like(det))
        u = uu / dsafe
        v = vv / dsafe
        G = torch.where(live, torch.exp(-0.5 * (u * u + v * v)), torch.zeros_like(u))
        alpha = torch.clamp(op[gi] * G, max=consts.ALPHA_MAX)
        ok = (alpha.detach() >= consts.ALPHA_MIN) & ~done
        Tn = T * (1.0 - alpha)
        stop = ok & (Tn.detach() < consts.T_MIN)
        done = done | stop
        contrib = ok & ~stop
        w = torch.where(contrib, alpha * T, torch.zeros_like(T))
        if keep_w is not None:
            keep_w.append(w)
        col = col + w[:, None] * rgb[gi][None, :]
        if F is not None:
            F = F + w[:, None] * featt[gi][None, :]
        T = torch.where(contrib, Tn, T)
        niter = torch.where(contrib, torch.full_like(niter, pos + 1), niter)
    return col, F, T, niter, order


def leaves(g: dict) -> dict:
    return {k: torch.tensor(np.asarray(g[k], np.float64), requires_grad=True)
            for k in ("means", "scales", "quats", "opacity", "sh")}


def unit_rows(x: np.ndarray) -> np.ndarray:
    """Rows scaled to unit length (a zero row stays zero)."""
    x = np.asarray(x, np.float64)
    n = np.sqrt((x * x).sum(1, keepdims=True))
    return np.where(n > 0, x / np.where(n > 0, n, 1.0), 0.0)


def ndfd_losses(params: dict, g_meta: dict, cam, feat: np.ndarray, gt: np.ndarray, lam: float, k: float,
                surfels: bool = False):
    """The NDFD losses of every pixel by their definitions (Section 3.3,
    Appendix A.1), without the O(N) rearrangement: with unit features and
    sigma_i = 1 / (1 + exp(k (cos(f_i, F_gt) - lambda))),
        L_gt = sum_i w_i sigma_i,
        L_cf = sum_i sum_{j<i} sigma_i w_i w_j (1 - cos(f_i, f_j))   (the double sum).
    Returns (L_gt [P], L_cf [P]) as differentiable float64 tensors.  surfels:
    the blend weights of the surfel primitive (render_surfel)."""
    ws = []
    _, _, _, _, order = (render_surfel if surfels else render)(params, g_meta, cam, None, keep_w=ws)
    if not ws:
        P = int(cam.width) * int(cam.height)
        z = torch.zeros(P, dtype=torch.float64)
        return z, z
    Wm = torch.stack(ws, 0)                                   # [positions, P]
    fh = torch.tensor(unit_rows(np.asarray(feat, np.float64)[order]))
    gh = torch.tensor(unit_rows(gt))
    sig = 1.0 / (1.0 + torch.exp(k * (fh @ gh.T - lam)))     # [positions, P], constant
    Lgt = (Wm * sig).sum(0)
    pair = 1.0 - fh @ fh.T                                    # [positions, positions]
    lower = torch.tril(pair, diagonal=-1)                     # j < i
    Lcf = (sig * Wm * (lower @ Wm)).sum(0)
    return Lgt, Lcf
