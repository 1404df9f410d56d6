"""Pins of the FP64 compositing oracle (oracle/raster.c) and of brute force vs tiles."""
import json
import os

import numpy as np
import torch

import scenegen
from oracle import brute, consts, pipeline, raster

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


class _Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


def _one_tile(us, vs, A, B, C, op, rgb, feat=None, w=16, h=16, **kw):
    """Composite Gaussians listed nearest-first in a single 16x16 tile."""
    n = len(us)
    proj = dict(u=np.asarray(us, float), v=np.asarray(vs, float), A=np.asarray(A, float),
                B=np.asarray(B, float), C=np.asarray(C, float), opacity=np.asarray(op, float),
                rgb=np.asarray(rgb, float).reshape(n, 3))
    ranges = np.array([[0, n]])
    return raster.render_view(_Cam(w, h), ranges, np.arange(n), proj, feat=feat, **kw)


def test_single_gaussian_closed_form():
    gold = GOLD["single_isotropic"]
    o = gold["opacity"]
    u0, v0 = 7.5, 7.5   # centre on pixel (7, 7)
    out = _one_tile([u0], [v0], [1.0], [0.0], [1.0], [o], [[0.2, 0.5, 1.0]],
                    feat=np.array([[2.0, -1.0]]))
    for case in gold["cases"]:
        px, py = int(7 + case["dx"]), int(7 + case["dy"])
        p = py * 16 + px
        a = case["alpha"]
        assert np.allclose(out["C"][p], np.array([0.2, 0.5, 1.0]) * a, rtol=1e-14, atol=1e-300)
        assert np.allclose(out["F"][p], np.array([2.0, -1.0]) * a, rtol=1e-14, atol=1e-300)
        assert np.isclose(out["T"][p], 1 - a, rtol=1e-14)
        assert out["niter"][p] == (1 if a > 0 else 0)


def test_stack_termination():
    gold = GOLD["stack_095"]
    n = gold["n_gaussians"]
    out = _one_tile([7.5] * n, [7.5] * n, [1.0] * n, [0.0] * n, [1.0] * n, [gold["alpha"]] * n,
                    [[1.0, 1.0, 1.0]] * n, feat=np.ones((n, 1)))
    p = 7 * 16 + 7
    assert np.isclose(out["T"][p], gold["T_final"], rtol=1e-12)
    assert out["niter"][p] == gold["n_iter"]
    assert np.isclose(out["C"][p, 0], gold["sum_w"], rtol=1e-12)
    assert np.isclose(out["F"][p, 0], gold["sum_w"], rtol=1e-12)


def test_two_concentric_order():
    gold = GOLD["two_concentric"]
    out = _one_tile([7.5, 7.5], [7.5, 7.5], [1, 1], [0, 0], [1, 1],
                    [gold["alpha_near"], gold["alpha_far"]], [gold["rgb_near"], gold["rgb_far"]])
    p = 7 * 16 + 7
    assert np.allclose(out["C"][p], gold["C"], rtol=1e-14)
    assert np.isclose(out["T"][p], gold["T_final"], rtol=1e-14)


def test_clamp():
    gold = GOLD["clamp"]
    out = _one_tile([7.5], [7.5], [1], [0], [1], [1.0], [[1, 1, 1]])
    p = 7 * 16 + 7
    assert np.isclose(out["T"][p], gold["T_final"], rtol=1e-14)
    assert np.isclose(out["C"][p, 0], gold["alpha"], rtol=1e-14)


def _random_scene_oracle(seed, n=120, d=5, recipe="front48x40", deg=1):
    g = scenegen.make_gaussians(n, 1.0, deg, d, seed=seed)
    cams = scenegen.make_cameras(recipe)
    o = pipeline.run(g, cams)
    return g, cams, o


def test_weight_sum_invariant_and_ones_features():
    g, cams, _ = _random_scene_oracle(3)
    g["feat"] = np.ones((g["means"].shape[0], 1), np.float32)
    o = pipeline.run(g, cams)
    v = o["views"][0]
    # all-ones features: F = sum w = 1 - T_final
    assert np.allclose(v["F"][:, 0], 1 - v["T"], atol=1e-14)


def test_linear_in_features_and_colour():
    g, cams, o1 = _random_scene_oracle(4)
    g2 = dict(g)
    g2["feat"] = 2.0 * g["feat"]          # exact in float32
    o2 = pipeline.run(g2, cams)
    assert np.allclose(o2["views"][0]["F"], 2.0 * o1["views"][0]["F"], rtol=1e-14, atol=1e-300)
    # colour: scale the per-Gaussian rgb at the compositing level
    rng = np.random.default_rng(9)
    n = 5
    args = ([7.5 + rng.normal() for _ in range(n)], [7.5 + rng.normal() for _ in range(n)],
            [0.3] * n, [0.05] * n, [0.2] * n, list(rng.uniform(0.2, 0.9, n)))
    rgb = rng.uniform(0, 1, (n, 3))
    c1 = _one_tile(*args, rgb)["C"]
    c2 = _one_tile(*args, 0.5 * rgb)["C"]
    assert np.allclose(c2, 0.5 * c1, rtol=1e-14, atol=1e-300)


def test_permutation_invariance():
    g, cams, o1 = _random_scene_oracle(5)
    perm = np.random.default_rng(0).permutation(g["means"].shape[0])
    g2 = {k: (v[perm] if isinstance(v, np.ndarray) and v.shape[:1] == (g["means"].shape[0],) else v)
          for k, v in g.items()}
    o2 = pipeline.run(g2, cams)
    v1, v2 = o1["views"][0], o2["views"][0]
    assert np.allclose(v1["C"], v2["C"], atol=1e-13)
    assert np.allclose(v1["F"], v2["F"], atol=1e-13)
    assert np.allclose(v1["T"], v2["T"], atol=1e-13)


def test_brute_force_equals_tiled():
    for seed, recipe in ((6, "front48x40"), (7, "front33x21"), (8, "front70x50")):
        g, cams, o = _random_scene_oracle(seed, n=150, recipe=recipe, deg=2)
        L = brute.leaves(g)
        with torch.no_grad():
            C, F, T, niter, order = brute.render(L, g, cams[0], g["feat"])
        v = o["views"][0]
        assert np.allclose(C.numpy(), v["C"], atol=1e-13)
        assert np.allclose(F.numpy(), v["F"], atol=1e-13)
        assert np.allclose(T.numpy(), v["T"], atol=1e-13)
        # the last contributor is the same Gaussian
        ranges = pipeline.view_slice(o["bins"], 0, cams[0])
        W = cams[0].width
        tx = (np.arange(T.numel()) % W) // 16
        ty = (np.arange(T.numel()) // W) // 16
        tile = ty * ((W + 15) // 16) + tx
        tiled_last = np.where(v["niter"] > 0, o["bins"]["gids"][np.maximum(ranges[tile, 0] + v["niter"] - 1, 0)], -1)
        brute_last = np.where(niter.numpy() > 0, order[np.maximum(niter.numpy() - 1, 0)], -1)
        assert np.array_equal(tiled_last, brute_last)


def test_colour_magnitude_companion():
    # rgb_mag bounds |rgb| (so Cmag bounds |C|) and equals rgb when every SH
    # term is non-negative; the clamp is flagged ambiguous exactly near raw = 0
    from oracle import project
    g = scenegen.make_gaussians(400, 1.2, 2, 0, seed=8)
    cam = scenegen.make_cameras("front64x48")[0]
    ora = pipeline.run(g, [cam])
    v = ora["views"][0]
    assert np.all(v["Cmag"] >= np.abs(v["C"]) * (1 - 1e-15))
    pr = v["proj"]
    assert np.all(pr["rgb_mag"] >= np.abs(pr["rgb"]))
    g0 = scenegen.make_gaussians(300, 1.2, 0, 0, seed=9)
    g0["sh"] = np.abs(g0["sh"])
    ora0 = pipeline.run(g0, [cam])
    assert np.array_equal(ora0["views"][0]["Cmag"], ora0["views"][0]["C"])
    # a DC coefficient that puts raw exactly at 0 (and one clearly away from it)
    g1 = scenegen.make_gaussians(2, 1.0, 0, 0, seed=10)
    y00 = 0.5 / np.sqrt(np.pi)
    g1["sh"][0, 0, :] = np.float32(-0.5 / y00)
    g1["sh"][1, 0, :] = np.float32(0.3 / y00)
    pr1 = project.project(g1, cam)
    assert pr1["clamp_amb"][0] and not pr1["clamp_amb"][1]


def test_ambiguity_companions():
    # two concentric Gaussians, the front one's alpha at the centre pixel within
    # rounding of 1/255: that pixel is flagged, the front Gaussian (the decider)
    # is flagged, the back one keeps its terms and gets a non-zero g2d_amb;
    # an alpha just above the 0.99 clamp contributes unclamped magnitudes
    u = v = 7.5
    a_front = (1.0 / 255.0) * (1.0 + 1e-7)
    out = _one_tile([u, u], [v, v], [0.02, 0.02], [0.0, 0.0], [0.02, 0.02], [a_front, 0.6],
                    [[0.2, 0.5, 1.0], [1.0, 0.3, 0.1]], dC=np.ones((256, 3)), dT=np.zeros(256))
    p = 7 * 16 + 7
    assert out["flags"][p] & 1
    assert out["gflags"][0] & 1 and not out["gflags"][1] & 1
    assert np.all(out["g2d_amb"] >= 0) and np.any(out["g2d_amb"][1] > 0)
    assert out["g2d_amb"][0, 5] > 0          # the decider's would-be opacity term
    assert np.all(out["g2d_amb"][1] <= out["g2d_mag"][1] * (1 + 1e-12))
    # no near-threshold decision: nothing to bound
    out = _one_tile([u], [v], [0.02], [0.0], [0.02], [0.5], [[0.2, 0.5, 1.0]], dC=np.ones((256, 3)),
                    dT=np.zeros(256))
    assert not np.any(out["flags"] & 1) and np.all(out["g2d_amb"] == 0)
    # alpha clamped at the centre by a hair: its power/opacity terms there are
    # zero in the FP64 adjoint but bounded by their unclamped magnitude
    out = _one_tile([u], [v], [0.02], [0.0], [0.02], [0.99 * (1 + 1e-7)], [[0.2, 0.5, 1.0]],
                    dC=np.ones((256, 3)), dT=np.zeros(256))
    assert out["flags"][p] & 2
    assert out["g2d_amb"][0, 5] > 0 and out["g2d_amb"][0, 0:5].sum() >= 0
