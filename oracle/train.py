"""The training step around the rasterizer (Algorithm 1: render, loss, Adam
update, and periodic densification), in FP64 numpy, written from its
definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Parameters are held raw and activated for rendering: means; log-scales
(scale = exp); the raw quaternion (normalised inside the projection); the
opacity logit (opacity = sigmoid); SH coefficients.  Features are frozen.

Adam (Kingma and Ba, 2015), per parameter element with gradient g at step t:
    m = b1 m + (1 - b1) g,   v = b2 v + (1 - b2) g^2,
    x = x - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Gradients of the raw parameters from those of the activated ones:
    dL/d log s = s dL/ds,   dL/d logit = o (1 - o) dL/do.

Photometric loss (Algorithm 1, Photometric Loss; the paper leaves the function
open): the mean squared error over pixels and channels,
    L = sum (C - C_target)^2 / (3 P),   dL/dC = 2 (C - C_target) / (3 P).

Densification (the adaptive density control the paper inherits; Algorithm 1,
Densification): per Gaussian, over the views of the iterations since the
last refinement, the norm of its screen-space mean gradient |dL/d(u, v)| is
summed over the views that binned it (at least one tile instance, the
visibility rule of 3DGS), and those views counted.  At a
refinement, with avg = sum / count:
    avg >= grad_thr and max log-scale <= log_scale_thr  ->  clone (a copy is
        appended);
    avg >= grad_thr and max log-scale  > log_scale_thr  ->  split: the
        Gaussian is replaced by two, means mu + R diag(s) z_j (z_j given, two
        per split Gaussian), log-scales log s - ln 1.6, other parameters copied;
    then every Gaussian (old or new) with opacity logit < prune_logit
    (opacity below sigmoid(prune_logit)) is removed.
These decisions are integers decided by floating point, so they are taken in
float32 on float32 values, as the kernels take them: avg = sum / count, and
the comparisons of the float32 parameters with float32 thresholds.
New Gaussians start with zero Adam moments; survivors keep theirs.  Order of
the result: the kept originals in index order (a split Gaussian keeps its
first child in its place), then the clones and the second children, in the
index order of their parents.
"""
from __future__ import annotations

import numpy as np

GROUPS = ("means", "log_scales", "quats", "logit_opacity", "sh")


def activate(raw: dict) -> dict:
    """Rendering parameters from raw ones."""
    return dict(means=raw["means"], scales=np.exp(raw["log_scales"]), quats=raw["quats"],
                opacity=1.0 / (1.0 + np.exp(-raw["logit_opacity"])), sh=raw["sh"])


def raw_grads(raw: dict, grads: dict) -> dict:
    """Gradients of the raw parameters from gradients of the activated ones."""
    act = activate(raw)
    o = act["opacity"]
    return dict(means=grads["means"], log_scales=grads["scales"] * act["scales"], quats=grads["quats"],
                logit_opacity=grads["opacity"] * o * (1.0 - o), sh=grads["sh"])


def photometric_loss(C: np.ndarray, C_target: np.ndarray):
    """(L, dL/dC) of the mean squared error, in FP64."""
    e = np.asarray(C, np.float64) - np.asarray(C_target, np.float64)
    return float((e * e).sum() / e.size), 2.0 * e / e.size


def densify_stats(g2d_views: list, binned_views: list):
    """(grad_sum, count) over views: g2d_views[v] [N, >= 2] holds each
    Gaussian's dL/du, dL/dv in view v, binned_views[v] [N] whether view v binned
    it; the norms are summed in FP64."""
    gs = np.zeros(np.asarray(g2d_views[0]).shape[0])
    cnt = np.zeros(gs.shape[0], np.int64)
    for g2d, b in zip(g2d_views, binned_views):
        g2d = np.asarray(g2d, np.float64)
        b = np.asarray(b, bool)
        gs += np.where(b, np.hypot(g2d[:, 0], g2d[:, 1]), 0.0)
        cnt += b
    return gs, cnt


def adam_step(raw: dict, g: dict, m: dict, v: dict, t: int, lr: dict, b1=0.9, b2=0.999, eps=1e-15):
    """One Adam update of every parameter group (new raw, m, v)."""
    out_raw, out_m, out_v = {}, {}, {}
    for k in GROUPS:
        mk = b1 * m[k] + (1.0 - b1) * g[k]
        vk = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mh = mk / (1.0 - b1 ** t)
        vh = vk / (1.0 - b2 ** t)
        out_raw[k] = raw[k] - lr[k] * mh / (np.sqrt(vh) + eps)
        out_m[k], out_v[k] = mk, vk
    return out_raw, out_m, out_v


def quat_rotation(q: np.ndarray) -> np.ndarray:
    """Rotation matrices of (w, x, y, z) quaternions (normalised first)."""
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def densify_actions(grad_sum: np.ndarray, count: np.ndarray, log_scales: np.ndarray, grad_thr: float,
                    log_scale_thr: float) -> np.ndarray:
    """0 keep, 1 clone, 2 split (decided in float32 from float32 statistics)."""
    gs = np.asarray(grad_sum, np.float32)
    cnt = np.asarray(count, np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        avg = np.where(cnt > 0, gs / np.where(cnt > 0, cnt, np.float32(1)), np.float32(0)).astype(np.float32)
    lmax = np.asarray(log_scales, np.float32).max(1)
    hot = avg >= np.float32(grad_thr)
    act = np.zeros(gs.shape[0], np.int32)
    act[hot & (lmax <= np.float32(log_scale_thr))] = 1
    act[hot & (lmax > np.float32(log_scale_thr))] = 2
    return act


def densify(raw: dict, m: dict, v: dict, act: np.ndarray, z: np.ndarray, prune_logit: float):
    """Apply clone / split actions, then prune; z [n_split, 2, 3] are the
    standard normal draws of the split Gaussians (in index order)."""
    n = act.shape[0]
    split = np.nonzero(act == 2)[0]
    clone = np.nonzero(act == 1)[0]
    R = quat_rotation(np.asarray(raw["quats"], np.float64)[split])
    s = np.exp(np.asarray(raw["log_scales"], np.float64)[split])
    mu = np.asarray(raw["means"], np.float64)[split]
    child = [mu + np.einsum("nij,nj->ni", R, s * z[:, j, :]) for j in range(2)]
    new_raw = {k: np.asarray(raw[k], np.float64).copy() for k in GROUPS}
    new_raw["means"][split] = child[0]
    new_raw["log_scales"][split] = new_raw["log_scales"][split] - np.log(1.6)
    # appended: clones and second children, in parent index order
    extra = np.sort(np.concatenate([clone, split]))
    out_raw = {}
    for k in GROUPS:
        add = new_raw[k][extra].copy()
        if k == "means":
            sec = {int(i): c for i, c in zip(split, child[1])}
            for r, i in enumerate(extra):
                if int(i) in sec:
                    add[r] = sec[int(i)]
        out_raw[k] = np.concatenate([new_raw[k], add])
    out_m = {k: np.concatenate([np.asarray(m[k], np.float64), np.zeros_like(np.asarray(m[k])[extra])])
             for k in GROUPS}
    out_v = {k: np.concatenate([np.asarray(v[k], np.float64), np.zeros_like(np.asarray(v[k])[extra])])
             for k in GROUPS}
    # split parents' moments restart as well (their parameters changed)
    for k in GROUPS:
        out_m[k][split] = 0.0
        out_v[k][split] = 0.0
    keep = np.asarray(out_raw["logit_opacity"], np.float32) >= np.float32(prune_logit)
    return ({k: out_raw[k][keep] for k in GROUPS}, {k: out_m[k][keep] for k in GROUPS},
            {k: out_v[k][keep] for k in GROUPS}, keep, n)
