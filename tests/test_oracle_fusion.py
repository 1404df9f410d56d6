"""Pins of the oracle's w-weighted feature fusion."""
import numpy as np

import scenegen
from oracle import pipeline, raster


def _run(seed, target_fn, n=120, d=4, views="front48x40"):
    g = scenegen.make_gaussians(n, 1.0, 1, d, seed=seed)
    if views == "three":
        cams = [scenegen.look_at_camera(p, 40, 32) for p in ((0, -4, 0), (3, -2, 1), (-2, 1, 3.5))]
    else:
        cams = scenegen.make_cameras(views)
    vt = [scenegen.make_view_tensors(i, c.npix, d) for i, c in enumerate(cams)]
    for i, c in enumerate(cams):
        vt[i]["target"] = target_fn(c.npix, d, i)
    return g, pipeline.run(g, cams, vt, fusion=True)


def test_constant_target_gives_the_constant():
    const = np.array([0.25, -1.5, 3.0, 7.0])
    g, o = _run(1, lambda p, d, i: np.tile(const, (p, 1)))
    fhat = pipeline.finalize_fusion(o["fsum"], o["wsum"], g["feat"])
    hit = o["wsum"] > 0
    assert hit.sum() > 10
    assert np.allclose(fhat[hit], const, rtol=1e-14)
    # never-blended Gaussians keep their feature
    assert np.array_equal(fhat[~hit], np.asarray(g["feat"], np.float64)[~hit])


def test_single_gaussian_weighted_average():
    class Cam:
        width, height = 16, 16
    proj = dict(u=np.array([6.3]), v=np.array([9.1]), A=np.array([0.2]), B=np.array([0.05]),
                C=np.array([0.3]), opacity=np.array([0.7]), rgb=np.ones((1, 3)))
    rng = np.random.default_rng(2)
    tgt = rng.normal(size=(256, 3))
    out = raster.render_view(Cam, np.array([[0, 1]]), np.array([0]), proj, feat=np.zeros((1, 3)),
                             dC=np.zeros((256, 3)), dF=np.zeros((256, 3)), dT=np.zeros(256), target=tgt)
    ys, xs = np.mgrid[0:16, 0:16]
    dx, dy = xs.reshape(-1) + 0.5 - 6.3, ys.reshape(-1) + 0.5 - 9.1
    alpha = 0.7 * np.exp(-0.5 * (0.2 * dx * dx + 2 * 0.05 * dx * dy + 0.3 * dy * dy))
    alpha = np.where(alpha >= 1 / 255, np.minimum(alpha, 0.99), 0.0)
    assert np.isclose(out["wsum"][0], alpha.sum(), rtol=1e-13)
    assert np.allclose(out["fsum"][0], alpha @ tgt, rtol=1e-12)


def test_linear_in_target_and_multi_view_sum():
    rng_t = lambda p, d, i: np.random.default_rng(50 + i).normal(size=(p, d))
    g, o1 = _run(3, rng_t, views="three")
    g, o2 = _run(3, lambda p, d, i: 2.0 * rng_t(p, d, i), views="three")
    # parallel FP64 accumulation order varies: compare against the magnitude companion
    assert np.all(np.abs(o2["fsum"] - 2.0 * o1["fsum"]) <= 1e-14 * o2["fsum_mag"] + 1e-300)
    assert np.allclose(o2["wsum"], o1["wsum"], rtol=1e-14, atol=0)
    # the multi-view sums are the sums of the single-view runs
    g = scenegen.make_gaussians(120, 1.0, 1, 4, seed=3)
    cams = [scenegen.look_at_camera(p, 40, 32) for p in ((0, -4, 0), (3, -2, 1), (-2, 1, 3.5))]
    tot = np.zeros_like(o1["fsum"])
    for i, c in enumerate(cams):
        vt = scenegen.make_view_tensors(i, c.npix, 4)
        vt["target"] = rng_t(c.npix, 4, i)
        tot += pipeline.run(g, [c], [vt], fusion=True)["fsum"]
    assert np.all(np.abs(tot - o1["fsum"]) <= 1e-14 * o1["fsum_mag"] + 1e-300)
