"""Pins of the opacity-aware binning rule (oracle/binspec.py, rule="opacity"):
each Gaussian's box factor kappa_i = min(KAPPA, 2 ln(255 o_i) + 1/256), with
the logarithm evaluated by a fixed float32 sequence of basic operations."""
import numpy as np

import scenegen
from oracle import binspec, consts, pipeline, project


def test_float32_log_tracks_the_fp64_log():
    # every float32 from just above 1 to 255 in a dense sweep, plus powers of two
    # and the range-reduction boundary sqrt 2
    x = np.concatenate([np.linspace(1.0, 255.0, 200001), 2.0 ** np.arange(0, 8),
                        [np.sqrt(2.0) * (1 - 1e-7), np.sqrt(2.0), np.sqrt(2.0) * (1 + 1e-7)]]).astype(np.float32)
    got = binspec.ln_f32(x).astype(np.float64)
    ref = np.log(x.astype(np.float64))
    err = np.abs(got - ref)
    # a few float32 ulps of ln x (at most 5.55 here: ulp 4.8e-7)
    assert err.max() <= 2e-6, err.max()
    assert np.all(np.diff(got[:200001]) >= 0)        # monotone along the sweep


def test_kappa_bounds_the_exact_threshold_from_above():
    o = np.concatenate([np.linspace(1.0 / 255.0, 1.0, 100001), [0.5 / 255.0, 1.0 / 255.0, 0.99, 1.0]])
    o = o.astype(np.float32)
    kap, live = binspec.opacity_kappa(o)
    x = 255.0 * o.astype(np.float64)
    exact = 2.0 * np.log(np.maximum(x, 1e-300))
    assert np.array_equal(live, np.float32(255.0) * o > np.float32(1.0))
    k = kap[live].astype(np.float64)
    # at least the exact factor (no pixel where alpha can reach 1/255 lost) ...
    assert np.all(k >= np.minimum(exact[live], consts.KAPPA))
    # ... and never more than the box rule or the margin above the exact one
    assert np.all(k <= consts.KAPPA_F32)
    assert np.all(k <= exact[live] + 1.0 / 256.0 + 1e-5)
    # a fully opaque Gaussian stays just under the box rule's factor
    assert abs(float(kap[-1]) - (2.0 * np.log(255.0) + 1.0 / 256.0)) < 1e-5 and kap[-1] < consts.KAPPA_F32
    assert not live[o <= np.float32(1.0 / 255.0)].any()


def test_opacity_box_holds_every_pixel_alpha_can_reach():
    # alpha = o exp(power) >= 1/255 at a pixel centre => that pixel's tile is in the rect
    g = scenegen.make_gaussians(400, 1.2, 0, 0, seed=4)
    cam = scenegen.make_cameras("front128x96")[0]
    bq = binspec.bin_quantities(g, cam, "opacity")
    pr = project.project(g, cam)
    ys, xs = np.mgrid[0:96, 0:128]
    x = xs.reshape(-1) + 0.5
    y = ys.reshape(-1) + 0.5
    checked = 0
    for i in range(400):
        if not (pr["depth"][i] > consts.Z_NEAR):
            continue
        dx, dy = x - pr["u"][i], y - pr["v"][i]
        power = -0.5 * (pr["A"][i] * dx * dx + 2 * pr["B"][i] * dx * dy + pr["C"][i] * dy * dy)
        hit = min(1.0, pr["opacity"][i]) * np.exp(power) >= consts.ALPHA_MIN
        if not hit.any():
            continue
        checked += 1
        assert bq["binned"][i]
        tx, ty = (x[hit] // 16).astype(int), (y[hit] // 16).astype(int)
        assert np.all((tx >= bq["x0"][i]) & (tx <= bq["x1"][i]) & (ty >= bq["y0"][i]) & (ty <= bq["y1"][i]))
    assert checked > 100


def test_opacity_rule_keeps_a_subset_of_the_box_rule_instances():
    g = scenegen.make_gaussians(3000, 1.5, 0, 0, seed=6)
    cam = scenegen.make_cameras("front200x150")[0]
    box = binspec.bin_quantities(g, cam, "box")
    opa = binspec.bin_quantities(g, cam, "opacity")
    b = opa["binned"]
    assert np.all(box["binned"][b])
    for k in ("x0", "y0"):
        assert np.all(opa[k][b] >= box[k][b])
    for k in ("x1", "y1"):
        assert np.all(opa[k][b] <= box[k][b])
    assert opa["ntiles"].sum() < box["ntiles"].sum()
    # the depth keys do not depend on the rule
    assert np.array_equal(opa["depth"].view(np.uint32), box["depth"].view(np.uint32))


def test_opacity_rule_changes_no_composited_value():
    """Every instance the opacity rule drops has alpha < 1/255 in every pixel
    of its tile, so the walk only loses skipped entries: colour, features,
    transmittance, gradients and fusion sums are those of the box rule (up to
    the order of the per-Gaussian FP64 sums); only n_iter, a list position,
    shrinks."""
    g = scenegen.make_gaussians(1500, 1.2, 1, 8, seed=8)
    cams = [scenegen.look_at_camera(p, w, h) for p, w, h in (((0, -4, 0), 96, 80), ((3, -2.5, 1.2), 80, 64))]
    vts = [scenegen.make_view_tensors(i, c.npix, 8, with_dT=True) for i, c in enumerate(cams)]
    box = pipeline.run(g, cams, vts, fusion=True)
    opa = pipeline.run(g, cams, vts, fusion=True, bin_rule="opacity")
    assert opa["bins"]["keys"].size < box["bins"]["keys"].size
    for vb, vo in zip(box["views"], opa["views"]):
        for k in ("C", "F", "T"):
            assert np.allclose(vo[k], vb[k], rtol=1e-13, atol=1e-15), k
        assert np.all(vo["niter"] <= vb["niter"])
        assert np.array_equal(vo["niter"] > 0, vb["niter"] > 0)
    for k in box["grads"]:
        assert np.allclose(opa["grads"][k], box["grads"][k], rtol=1e-11, atol=1e-13), k
    assert np.allclose(opa["fsum"], box["fsum"], rtol=1e-11, atol=1e-13)
    assert np.allclose(opa["wsum"], box["wsum"], rtol=1e-11, atol=1e-13)
    assert opa["counts"][1] == box["counts"][1]            # the same contributing blends
    assert opa["counts"][2] < box["counts"][2]             # fewer alpha evaluations
