"""Pins of the oracle's FP64 projection and its adjoint chain (oracle/project.py)."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

import scenegen
from oracle import consts, project


def _scene(n=40, deg=2, seed=0):
    return scenegen.make_gaussians(n, 1.0, deg, 4, seed=seed)


def test_rotation_orthonormal_and_scipy():
    q = np.random.default_rng(0).normal(size=(30, 4))
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    R = project.quat_to_rot(qn)
    assert np.allclose(R @ np.transpose(R, (0, 2, 1)), np.eye(3), atol=1e-15)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-14)
    ref = Rotation.from_quat(np.concatenate([qn[:, 1:], qn[:, :1]], 1)).as_matrix()  # scalar-last
    assert np.allclose(R, ref, atol=1e-14)


def test_sigma3_eigenvalues_are_squared_scales():
    g = _scene()
    cam = scenegen.make_cameras("front64x64")[0]
    pr = project.project(g, cam)
    ev = np.sort(np.linalg.eigvalsh(pr["Sigma3"]), 1)
    ref = np.sort(np.asarray(g["scales"], np.float64) ** 2, 1)
    assert np.allclose(ev, ref, rtol=1e-12, atol=1e-18)


def test_isotropic_on_axis_closed_form():
    # isotropic Gaussian of std sigma on the optical axis at depth z:
    # Sigma2 = (f sigma / z)^2 I + lowpass I, (u, v) = (cx, cy), for any rotation
    cam = scenegen.make_cameras("front64x48")[0]
    sigma = 0.05
    n = 8
    q = np.random.default_rng(1).normal(size=(n, 4)).astype(np.float32)
    g = dict(means=np.zeros((n, 3), np.float32), scales=np.full((n, 3), sigma, np.float32),
             quats=q, opacity=np.full(n, 0.5, np.float32),
             sh=np.zeros((n, 1, 3), np.float32), sh_degree=0, d=0, feat=None)
    pr = project.project(g, cam)
    z = 4.0
    s2 = (cam.fx * float(np.float32(sigma)) / z) ** 2 + consts.LOWPASS
    assert np.allclose(pr["u"], cam.cx, atol=1e-9) and np.allclose(pr["v"], cam.cy, atol=1e-9)
    assert np.allclose(pr["a"], s2, rtol=1e-6) and np.allclose(pr["c"], s2, rtol=1e-6)
    assert np.allclose(pr["b"], 0.0, atol=1e-9 * s2)
    assert np.allclose(pr["A"], 1 / s2, rtol=1e-6) and np.allclose(pr["B"], 0, atol=1e-9)
    assert np.allclose(pr["depth"], z, rtol=1e-7)


def test_rigid_motion_invariance():
    # moving the scene and the camera by one rigid motion leaves the screen-space
    # Gaussian (uv, conic, depth) unchanged
    g = _scene(30, 0)
    cam = scenegen.make_cameras("front64x64")[0]
    Rm = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    tm = np.array([0.4, -1.0, 0.7])
    g2 = dict(g)
    g2["means"] = (np.asarray(g["means"], np.float64) @ Rm.T + tm)
    qm = Rotation.from_matrix(Rm)
    qg = Rotation.from_quat(np.concatenate([g["quats"][:, 1:], g["quats"][:, :1]], 1))
    qq = (qm * qg).as_quat()
    g2["quats"] = np.concatenate([qq[:, 3:], qq[:, :3]], 1)
    cam2 = scenegen.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                           np.asarray(cam.R, np.float64) @ Rm.T,
                           np.asarray(cam.t, np.float64) - np.asarray(cam.R, np.float64) @ Rm.T @ tm)
    p1, p2 = project.project(g, cam), project.project(g2, cam2)
    for k in ("u", "v", "A", "B", "C", "depth"):
        assert np.allclose(p1[k], p2[k], rtol=1e-10, atol=1e-10), k


def test_adjoint_chain_matches_central_differences():
    g = _scene(12, 3, seed=4)
    g = {k: (np.asarray(v, np.float64) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    cam = scenegen.make_cameras("front64x64")[0]
    rng = np.random.default_rng(5)
    n = g["means"].shape[0]
    up = dict(u=rng.normal(size=n), v=rng.normal(size=n), A=rng.normal(size=n) * 10,
              B=rng.normal(size=n) * 10, C=rng.normal(size=n) * 10, opacity=rng.normal(size=n),
              rgb=rng.normal(size=(n, 3)))

    def loss(gg):
        pr = project.project(gg, cam)
        return (up["u"] * pr["u"] + up["v"] * pr["v"] + up["A"] * pr["A"] + up["B"] * pr["B"]
                + up["C"] * pr["C"] + up["opacity"] * pr["opacity"] + (up["rgb"] * pr["rgb"]).sum(1)).sum()

    grads = project.project_bwd(project.project(g, cam), up)
    for key in ("means", "scales", "quats", "opacity", "sh"):
        x = g[key]
        flat = x.reshape(-1)
        fd = np.zeros_like(flat)
        for i in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[i]))
            xp = flat.copy(); xp[i] += h
            xm = flat.copy(); xm[i] -= h
            gp = dict(g); gp[key] = xp.reshape(x.shape)
            gm = dict(g); gm[key] = xm.reshape(x.shape)
            fd[i] = (loss(gp) - loss(gm)) / (2 * h)
        an = grads[key].reshape(-1)
        scale = np.abs(an).max() + 1e-12
        assert np.abs(an - fd).max() <= 1e-5 * scale, key


def test_magnitude_bounds_value():
    g = _scene(20, 3, seed=6)
    cam = scenegen.make_cameras("front64x64")[0]
    rng = np.random.default_rng(7)
    n = 20
    up = dict(u=rng.normal(size=n), v=rng.normal(size=n), A=rng.normal(size=n),
              B=rng.normal(size=n), C=rng.normal(size=n), opacity=rng.normal(size=n),
              rgb=rng.normal(size=(n, 3)))
    upm = {k: np.abs(v) for k, v in up.items()}
    pr = project.project(g, cam)
    gv = project.project_bwd(pr, up)
    gm = project.project_bwd(pr, upm, magnitude=True)
    for k in gv:
        assert np.all(np.abs(gv[k]) <= gm[k] * (1 + 1e-12) + 1e-300), k
