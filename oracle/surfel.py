"""Surfel primitive (Section 3.1): projection to a per-view record and its
adjoint chain, in FP64 (numpy).  TEST INFRASTRUCTURE ONLY.

A surfel has centre p (means), orthogonal tangents t_u, t_v (the first two
columns of the rotation of the quaternion), planar scales (s_u, s_v)
(scales[:, 0:2]; scales[:, 2] plays no part), opacity, SH colour and a
feature.  A point of its tangent plane is P(u, v) = p + s_u t_u u + s_v t_v v
and its density there G(u, v) = exp(-(u^2 + v^2) / 2).  A pixel (x, y) takes
the density at the point of the plane its ray meets, i.e. the (u, v) with
(x z, y z, z) = K (R_c P(u, v) + t_c) (the paper's x = W H (u, v, 1, 1)^T).

In camera space, with p_c = R_c p + t_c and T_u = s_u R_c t_u, T_v = s_v R_c
t_v, the map (u, v, 1) -> (x z, y z, z) has columns K T_u, K T_v, K p_c.
Divided by z_c = p_c.z and taken relative to the projected centre
(x_c, y_c) = (fx p_c.x / z_c + cx, fy p_c.y / z_c + cy), pixel offsets
(dx, dy) = (x - x_c, y - y_c) satisfy
  (dx w, dy w, w) = [[a0, a1, 0], [b0, b1, 0], [c0, c1, 1]] (u, v, 1),
  a_i = fx (T_i.x z_c - p_c.x T_i.z) / z_c^2,  b_i = fy (T_i.y z_c - p_c.y T_i.z) / z_c^2,
  c_i = T_i.z / z_c                            (T_0 = T_u, T_1 = T_v).
The ray of (dx, dy) meets the plane where (u, v, 1) is parallel to the cross
product of the two plane rows h_x = (a0 - dx c0, a1 - dx c1, -dx) and
h_y = (b0 - dy c0, b1 - dy c1, -dy):
  k0 = dx b1 - dy a1,   k1 = dy a0 - dx b0,   k2 = D - dy e1 - dx e2,
  D = a0 b1 - a1 b0,  e1 = a0 c1 - a1 c0,  e2 = c0 b1 - c1 b0,
  (u, v) = (k0, k1) / k2;  G = 0 where k2 = 0 (a ray parallel to the plane).
The per-view record is (x_c, y_c, a0, a1, b0, b1, D, e1, e2), opacity and
colour; alpha = min(0.99, o G) and the walk are those of the Gaussian case.
Depth order: z_c.  Binning: oracle.binspec's surfel rule (the image of the
disc u^2 + v^2 <= kappa_i).

Backward: given per-view adjoints of the nine record entries, the opacity and
the colour, the chain back to means, scales (s_u, s_v; zero for the third),
quats, opacity and SH, optionally with every local factor replaced by its
magnitude (see oracle.project).
"""
from __future__ import annotations

import numpy as np

from . import consts, project as eproj, sh

SRF = ("xc", "yc", "a0", "a1", "b0", "b1", "D", "e1", "e2")


def project_surfel(g: dict, cam) -> dict:
    """FP64 surfel records of every primitive for one camera (no culling here)."""
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
    qnorm = np.linalg.norm(q, axis=1)
    qn = q / qnorm[:, None]
    Rq = eproj.quat_to_rot(qn)
    du = Rq[:, :, 0] @ Rc.T                 # R_c t_u
    dv = Rq[:, :, 1] @ Rc.T                 # R_c t_v
    Tu = s[:, 0:1] * du
    Tv = s[:, 1:2] * dv
    z = p[:, 2]
    z2 = z * z
    xc = fx * p[:, 0] / z + cx
    yc = fy * p[:, 1] / z + cy
    a0 = fx * (Tu[:, 0] * z - p[:, 0] * Tu[:, 2]) / z2
    a1 = fx * (Tv[:, 0] * z - p[:, 0] * Tv[:, 2]) / z2
    b0 = fy * (Tu[:, 1] * z - p[:, 1] * Tu[:, 2]) / z2
    b1 = fy * (Tv[:, 1] * z - p[:, 1] * Tv[:, 2]) / z2
    c0 = Tu[:, 2] / z
    c1 = Tv[:, 2] / z
    D = a0 * b1 - a1 * b0
    e1 = a0 * c1 - a1 * c0
    e2 = c0 * b1 - c1 * b0
    srf = np.stack([xc, yc, a0, a1, b0, b1, D, e1, e2], 1)

    cam_centre = -Rc.T @ tc
    dvec = mu - cam_centre
    dlen = np.linalg.norm(dvec, axis=1)
    dirn = dvec / dlen[:, None]
    Y = sh.eval_sh(degree, dirn)
    raw = np.einsum("nb,nbc->nc", Y, shc) + 0.5
    rgb = np.maximum(raw, 0.0)
    Ymag = sh.eval_sh(degree, dirn, magnitude=True)
    rgb_mag = np.einsum("nb,nbc->nc", Ymag, np.abs(shc)) + 0.5
    clamp_amb = (np.abs(raw) <= consts.AMBIG_REL * rgb_mag).any(axis=1)
    return dict(srf=srf, p=p, z=z, depth=z, du=du, dv=dv, Tu=Tu, Tv=Tv, c0=c0, c1=c1,
                a0=a0, a1=a1, b0=b0, b1=b1, qn=qn, qnorm=qnorm, Rq=Rq, scales=s, Rc=Rc,
                fx=fx, fy=fy, opacity=op, dirn=dirn, dlen=dlen, Y=Y, Ymag=Ymag, raw=raw, rgb=rgb,
                rgb_mag=rgb_mag, clamp_amb=clamp_amb, sh=shc, degree=degree)


def plane_coords(srf: np.ndarray, x: np.ndarray, y: np.ndarray):
    """(u, v, k2) of the ray of pixel centre (x, y) for records srf [..., 9]
    (the formula of the module docstring; k2 = 0 marks a parallel ray)."""
    xc, yc, a0, a1, b0, b1, D, e1, e2 = (srf[..., i] for i in range(9))
    dx, dy = x - xc, y - yc
    k0 = dx * b1 - dy * a1
    k1 = dy * a0 - dx * b0
    k2 = D - dy * e1 - dx * e2
    with np.errstate(all="ignore"):
        u = np.where(k2 != 0, k0 / np.where(k2 != 0, k2, 1.0), np.inf)
        v = np.where(k2 != 0, k1 / np.where(k2 != 0, k2, 1.0), np.inf)
    return u, v, k2


def project_surfel_bwd(pr: dict, up: dict, magnitude: bool = False) -> dict:
    """Adjoint of `project_surfel` for one camera.

    up: "srf" [N, 9] adjoints of (x_c, y_c, a0, a1, b0, b1, D, e1, e2),
    "opacity" [N], "rgb" [N, 3] (magnitude companions when magnitude=True).
    Returns adjoints of means [N,3], scales [N,3], quats [N,4], opacity [N],
    sh [N,B,3]."""
    F = np.abs if magnitude else (lambda t: t)
    g = up["srf"]
    gxc, gyc, ga0, ga1, gb0, gb1, gD, ge1, ge2 = (g[:, i].copy() for i in range(9))
    a0, a1, b0, b1, c0, c1 = pr["a0"], pr["a1"], pr["b0"], pr["b1"], pr["c0"], pr["c1"]
    # D = a0 b1 - a1 b0, e1 = a0 c1 - a1 c0, e2 = c0 b1 - c1 b0
    ga0 = ga0 + F(b1) * gD + F(c1) * ge1
    gb1 = gb1 + F(a0) * gD + F(c0) * ge2
    ga1 = ga1 + F(-b0) * gD + F(-c0) * ge1
    gb0 = gb0 + F(-a1) * gD + F(-c1) * ge2
    gc0 = F(-a1) * ge1 + F(b1) * ge2
    gc1 = F(a0) * ge1 + F(-b0) * ge2

    fx, fy = pr["fx"], pr["fy"]
    p, z, Tu, Tv = pr["p"], pr["z"], pr["Tu"], pr["Tv"]
    px, py = p[:, 0], p[:, 1]
    z2, z3 = z * z, z * z * z
    gTu = np.zeros_like(Tu)
    gTv = np.zeros_like(Tv)
    gp = np.zeros_like(p)
    # x_c = fx p_x / z + cx, y_c = fy p_y / z + cy
    gp[:, 0] += F(fx / z) * gxc
    gp[:, 1] += F(fy / z) * gyc
    gp[:, 2] += F(-fx * px / z2) * gxc + F(-fy * py / z2) * gyc
    # a_i = fx (T.x / z - p_x T.z / z^2), b_i = fy (T.y / z - p_y T.z / z^2), c_i = T.z / z
    for T, gT, gai, gbi, gci in ((Tu, gTu, ga0, gb0, gc0), (Tv, gTv, ga1, gb1, gc1)):
        gT[:, 0] += F(fx / z) * gai
        gT[:, 1] += F(fy / z) * gbi
        gT[:, 2] += F(-fx * px / z2) * gai + F(-fy * py / z2) * gbi + F(1.0 / z) * gci
        gp[:, 0] += F(-fx * T[:, 2] / z2) * gai
        gp[:, 1] += F(-fy * T[:, 2] / z2) * gbi
        gp[:, 2] += ((F(-fx * T[:, 0] / z2) + F(2.0 * fx * px * T[:, 2] / z3)) * gai
                     + (F(-fy * T[:, 1] / z2) + F(2.0 * fy * py * T[:, 2] / z3)) * gbi
                     + F(-T[:, 2] / z2) * gci)
    Rc = pr["Rc"]
    up_mu = gp @ F(Rc)                                  # p_c = R_c mu + t_c
    # T_u = s_u R_c t_u, T_v = s_v R_c t_v  (t_u, t_v: columns 0 and 1 of R_q)
    s = pr["scales"]
    up_s = np.zeros_like(s)
    up_s[:, 0] = np.einsum("nk,nk->n", gTu, F(pr["du"]))
    up_s[:, 1] = np.einsum("nk,nk->n", gTv, F(pr["dv"]))
    up_R = np.zeros((s.shape[0], 3, 3))
    up_R[:, :, 0] = (gTu @ F(Rc)) * F(s[:, 0:1])
    up_R[:, :, 1] = (gTv @ F(Rc)) * F(s[:, 1:2])
    dR = eproj._drot_dq(pr["qn"])
    up_qn = np.einsum("nikl,nkl->ni", F(dR), up_R)
    qn, qnorm = pr["qn"], pr["qnorm"]
    projq = (np.eye(4)[None] - qn[:, :, None] * qn[:, None, :]) / qnorm[:, None, None]
    up_q = np.einsum("nij,nj->ni", F(projq), up_qn)

    # colour, as for the Gaussian primitive
    mask = (pr["raw"] > 0.0).astype(np.float64)
    up_raw = up["rgb"] * mask
    Y = pr["Y"]
    up_sh = (pr["Ymag"] if magnitude else Y)[:, :, None] * up_raw[:, None, :]
    dY = sh.eval_sh_grad(pr["degree"], pr["dirn"])
    up_dir = np.einsum("nbk,nbc,nc->nk", F(dY), F(pr["sh"]), up_raw)
    dirn, dlen = pr["dirn"], pr["dlen"]
    projd = (np.eye(3)[None] - dirn[:, :, None] * dirn[:, None, :]) / dlen[:, None, None]
    up_mu = up_mu + np.einsum("nij,nj->ni", F(projd), up_dir)
    return dict(means=up_mu, scales=up_s, quats=up_q, opacity=up["opacity"].copy(), sh=up_sh)
