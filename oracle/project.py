"""Per-Gaussian projection to the screen and its adjoint chain, in FP64 (numpy).

Forward (one camera, all Gaussians; Algorithm 2's screen-space Gaussians step):
  p      = R_c mu + t_c                       camera-space centre
  (u, v) = (fx p_x / p_z + cx, fy p_y / p_z + cy)
  R_q    = rotation of q / |q| (Hamilton, (w, x, y, z))
  Sigma3 = R_q diag(s)^2 R_q^T
  J      = [[fx/p_z, 0, -fx p_x/p_z^2], [0, fy/p_z, -fy p_y/p_z^2]]   (first-order EWA)
  Sigma2 = (J R_c) Sigma3 (J R_c)^T + LOWPASS * I  = [[a, b], [b, c]]
  conic  = Sigma2^-1 = (A, B, C) = (c, -b, a) / (a c - b^2)
  rgb    = max(0, sum_b sh_b Y_b(dir) + 1/2),  dir = (mu - cam_centre) / |mu - cam_centre|

The screen-space density is exp(power) with
  power(x, y) = -1/2 (A dx^2 + 2 B dx dy + C dy^2),  (dx, dy) = (x - u, y - v),
and alpha = opacity * exp(power) (Section 3.1).

Backward: given per-Gaussian adjoints of (u, v, A, B, C, opacity, rgb), the
chain rule back to (means, scales, quats, opacity, sh).  `magnitude=True`
evaluates the same chain with every local factor replaced by its absolute value
and every upstream adjoint by its magnitude companion; the result bounds the
size of the terms that cancel and sets the elementwise tolerance scale.
"""
from __future__ import annotations

import numpy as np

from . import consts, sh


def quat_to_rot(qn: np.ndarray) -> np.ndarray:
    """Rotation matrix of unit quaternions qn [N,4] = (w, x, y, z) -> [N,3,3]."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    R = np.empty((qn.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _drot_dq(qn: np.ndarray) -> np.ndarray:
    """dR_kl / dq_i for the rotation above: [N, 4, 3, 3]."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    zero = np.zeros_like(w)
    dw = np.stack([np.stack([zero, -2 * z, 2 * y], -1),
                   np.stack([2 * z, zero, -2 * x], -1),
                   np.stack([-2 * y, 2 * x, zero], -1)], -2)
    dx = np.stack([np.stack([zero, 2 * y, 2 * z], -1),
                   np.stack([2 * y, -4 * x, -2 * w], -1),
                   np.stack([2 * z, 2 * w, -4 * x], -1)], -2)
    dy = np.stack([np.stack([-4 * y, 2 * x, 2 * w], -1),
                   np.stack([2 * x, zero, 2 * z], -1),
                   np.stack([-2 * w, 2 * z, -4 * y], -1)], -2)
    dz = np.stack([np.stack([-4 * z, -2 * w, 2 * x], -1),
                   np.stack([2 * w, -4 * z, 2 * y], -1),
                   np.stack([2 * x, 2 * y, zero], -1)], -2)
    return np.stack([dw, dx, dy, dz], 1)


def project(g: dict, cam) -> dict:
    """FP64 projection of every Gaussian for one camera (no culling here)."""
    mu = np.asarray(g["means"], np.float64)
    s = np.asarray(g["scales"], np.float64)
    q = np.asarray(g["quats"], np.float64)
    op = np.asarray(g["opacity"], np.float64)
    shc = np.asarray(g["sh"], np.float64)
    degree = int(g["sh_degree"])
    Rc = np.asarray(cam.R, np.float64)
    tc = np.asarray(cam.t, np.float64)
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)

    p = mu @ Rc.T + tc
    px, py, pz = p[:, 0], p[:, 1], p[:, 2]
    u = fx * px / pz + cx
    v = fy * py / pz + cy

    qnorm = np.linalg.norm(q, axis=1)
    qn = q / qnorm[:, None]
    Rq = quat_to_rot(qn)
    M = Rq * s[:, None, :]
    Sigma3 = M @ np.transpose(M, (0, 2, 1))

    n = mu.shape[0]
    J = np.zeros((n, 2, 3))
    J[:, 0, 0] = fx / pz
    J[:, 0, 2] = -fx * px / pz ** 2
    J[:, 1, 1] = fy / pz
    J[:, 1, 2] = -fy * py / pz ** 2
    T = J @ Rc
    Sigma2 = T @ Sigma3 @ np.transpose(T, (0, 2, 1))
    a = Sigma2[:, 0, 0] + consts.LOWPASS
    b = Sigma2[:, 0, 1]
    c = Sigma2[:, 1, 1] + consts.LOWPASS
    det = a * c - b * b
    A, B, C = c / det, -b / det, a / det

    cam_centre = -Rc.T @ tc
    dv = mu - cam_centre
    dlen = np.linalg.norm(dv, axis=1)
    dirn = dv / dlen[:, None]
    Y = sh.eval_sh(degree, dirn)
    raw = np.einsum("nb,nbc->nc", Y, shc) + 0.5
    rgb = np.maximum(raw, 0.0)
    # magnitude companion of the colour sum, and the Gaussians whose clamp
    # decision (raw > 0) sits within rounding reach of its threshold
    # (Y_b is itself a sum of monomials: its companion sums their magnitudes)
    Ymag = sh.eval_sh(degree, dirn, magnitude=True)
    rgb_mag = np.einsum("nb,nbc->nc", Ymag, np.abs(shc)) + 0.5
    clamp_amb = (np.abs(raw) <= consts.AMBIG_REL * rgb_mag).any(axis=1)

    return dict(p=p, u=u, v=v, depth=pz, qn=qn, qnorm=qnorm, Rq=Rq, M=M, Sigma3=Sigma3,
                J=J, T=T, a=a, b=b, c=c, det=det, A=A, B=B, C=C, opacity=op,
                dirn=dirn, dlen=dlen, Y=Y, Ymag=Ymag, raw=raw, rgb=rgb, rgb_mag=rgb_mag, clamp_amb=clamp_amb,
                scales=s, Rc=Rc,
                fx=fx, fy=fy, sh=shc, degree=degree)


def project_bwd(pr: dict, up: dict, magnitude: bool = False) -> dict:
    """Adjoint of `project` for one camera.

    up: dict of per-Gaussian adjoints u, v, A, B, C, opacity [N] and rgb [N,3]
    (or their magnitude companions when magnitude=True).  Returns adjoints of
    means [N,3], scales [N,3], quats [N,4], opacity [N], sh [N,B,3].
    """
    F = np.abs if magnitude else (lambda t: t)
    det = pr["det"]
    a, b, c = pr["a"], pr["b"], pr["c"]
    d2 = det * det
    upA, upB, upC = up["A"], up["B"], up["C"]

    # conic (A, B, C) = (c, -b, a)/det  ->  (a, b, c)
    up_a = F(-c * c / d2) * upA + F(b * c / d2) * upB + F(-b * b / d2) * upC
    up_b = F(2 * b * c / d2) * upA + F(-(a * c + b * b) / d2) * upB + F(2 * a * b / d2) * upC
    up_c = F(-b * b / d2) * upA + F(a * b / d2) * upB + F(-a * a / d2) * upC

    T, S3 = pr["T"], pr["Sigma3"]
    t0, t1 = T[:, 0, :], T[:, 1, :]
    # a = t0 S3 t0 + lp, b = t0 S3 t1, c = t1 S3 t1 + lp, expanded term by term
    S3t0 = np.einsum("nkj,nj->nk", F(S3), F(t0)) if magnitude else np.einsum("nkj,nj->nk", S3, t0)
    S3t1 = np.einsum("nkj,nj->nk", F(S3), F(t1)) if magnitude else np.einsum("nkj,nj->nk", S3, t1)
    up_t0 = 2 * up_a[:, None] * S3t0 + up_b[:, None] * S3t1
    up_t1 = up_b[:, None] * S3t0 + 2 * up_c[:, None] * S3t1
    G3 = (up_a[:, None, None] * F(t0[:, :, None] * t0[:, None, :])
          + up_b[:, None, None] * F(t0[:, :, None] * t1[:, None, :])
          + up_c[:, None, None] * F(t1[:, :, None] * t1[:, None, :]))

    # T = J R_c
    Rc = pr["Rc"]
    up_J00 = np.einsum("nk,k->n", up_t0, F(Rc[0]))
    up_J02 = np.einsum("nk,k->n", up_t0, F(Rc[2]))
    up_J11 = np.einsum("nk,k->n", up_t1, F(Rc[1]))
    up_J12 = np.einsum("nk,k->n", up_t1, F(Rc[2]))

    # J and (u, v) -> camera-space centre p
    fx, fy = pr["fx"], pr["fy"]
    px, py, pz = pr["p"][:, 0], pr["p"][:, 1], pr["p"][:, 2]
    upu, upv = up["u"], up["v"]
    up_px = F(fx / pz) * upu + F(-fx / pz ** 2) * up_J02
    up_py = F(fy / pz) * upv + F(-fy / pz ** 2) * up_J12
    up_pz = (F(-fx * px / pz ** 2) * upu + F(-fy * py / pz ** 2) * upv
             + F(-fx / pz ** 2) * up_J00 + F(2 * fx * px / pz ** 3) * up_J02
             + F(-fy / pz ** 2) * up_J11 + F(2 * fy * py / pz ** 3) * up_J12)
    up_p = np.stack([up_px, up_py, up_pz], 1)
    up_mu = up_p @ F(Rc)            # p = R_c mu + t: d/dmu = R_c^T up_p

    # Sigma3 = M M^T, M = R_q diag(s)
    M, Rq, s = pr["M"], pr["Rq"], pr["scales"]
    up_M = np.einsum("nij,njl->nil", G3 + np.transpose(G3, (0, 2, 1)), F(M))
    up_R = up_M * F(s)[:, None, :]
    up_s = np.einsum("nkl,nkl->nl", up_M, F(Rq))

    # R_q(qn), qn = q / |q|
    dR = _drot_dq(pr["qn"])
    up_qn = np.einsum("nikl,nkl->ni", F(dR), up_R)
    qn, qnorm = pr["qn"], pr["qnorm"]
    proj = (np.eye(4)[None] - qn[:, :, None] * qn[:, None, :]) / qnorm[:, None, None]
    up_q = np.einsum("nij,nj->ni", F(proj), up_qn)

    # colour: rgb = max(0, sum_b sh_b Y_b(dir) + 1/2)
    mask = (pr["raw"] > 0.0).astype(np.float64)
    up_raw = up["rgb"] * mask
    Y = pr["Y"]
    up_sh = (pr["Ymag"] if magnitude else Y)[:, :, None] * up_raw[:, None, :]
    dY = sh.eval_sh_grad(pr["degree"], pr["dirn"])         # [N,B,3]
    up_dir = np.einsum("nbk,nbc,nc->nk", F(dY), F(pr["sh"]), up_raw)
    dirn, dlen = pr["dirn"], pr["dlen"]
    projd = (np.eye(3)[None] - dirn[:, :, None] * dirn[:, None, :]) / dlen[:, None, None]
    up_mu = up_mu + np.einsum("nij,nj->ni", F(projd), up_dir)

    return dict(means=up_mu, scales=up_s, quats=up_q, opacity=up["opacity"].copy(), sh=up_sh)
