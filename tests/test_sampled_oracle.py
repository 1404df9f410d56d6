"""The sampled form of the oracle (tests/sampled.py), used at the batched
workloads' full sizes, equals the full oracle pipeline on a small two-view
scene: forward outputs of the walked tiles, and the sampled Gaussians'
gradient, magnitude and fusion sums over both views."""
import numpy as np
import pytest

import scenegen
from oracle import binspec, pipeline
from tests import sampled as S


@pytest.mark.parametrize("prim", ["gaussian", "surfel"])
def test_sampled_oracle_equals_full_pipeline(prim):
    surf = prim == "surfel"
    g = scenegen.make_gaussians(900, 1.5, 2, 8, seed=21, feat_dtype="bf16")
    if surf:
        g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    cams = [scenegen.look_at_camera(p, w, h) for p, w, h in (((0, -4, 0), 96, 80), ((3, -2.5, 1.2), 112, 64))]
    vts = [dict(scenegen.make_view_tensors(i, c.npix, 8, with_dT=True)) for i, c in enumerate(cams)]
    full = pipeline.run(g, cams, vts, fusion=True, want_Fmag=True, bin_rule="surfel" if surf else "box")
    bqs = full["bins"]["per_view"]
    counts = [binspec.tile_counts(bq) for bq in bqs]
    cand = S.pick_gaussians(bqs, 10, seed=3)
    assert cand.size == 10
    views = S.plan(bqs, counts, cams, cand, extra_tiles=2, seed=4)
    ora = S.run(g, cams, bqs, cand, views, lambda vi, key, pix: vts[vi][key][pix], 8, surfels=surf)
    for vi, vw in enumerate(views):
        f, ref = vw["fwd"], full["views"][vi]
        p = f["pix"]
        assert np.array_equal(f["niter"], ref["niter"][p])
        for k in ("C", "Cmag", "T", "F", "Fmag", "Cden", "Tden", "Fden"):
            assert np.allclose(f[k], ref[k][p], rtol=1e-12, atol=1e-300), k
    for k in S.GRAD_KEYS:
        scale = np.maximum(full["grads_mag"][k][cand], 1e-300)
        assert np.all(np.abs(ora["sums"][k] - full["grads"][k][cand]) <= 1e-10 * scale), k
        assert np.allclose(ora["mags"][k], full["grads_mag"][k][cand], rtol=1e-10, atol=1e-300), k
        assert np.allclose(ora["ambs"][k], full["grads_amb"][k][cand], rtol=1e-10, atol=1e-300), k
    assert np.allclose(ora["fsum"], full["fsum"][cand], rtol=1e-10, atol=1e-12)
    assert np.allclose(ora["wsum"], full["wsum"][cand], rtol=1e-12, atol=1e-300)
    assert np.array_equal(ora["gflag"] != 0, full["gflags"][cand] != 0)


def test_footprint_central_differences_match_the_oracle_adjoint():
    # FP64 central differences of the forward over a Gaussian's footprint tiles
    # equal the hand-written adjoint (for perturbations that keep the depth order)
    g = scenegen.make_gaussians(700, 1.5, 1, 8, seed=22)
    cam = scenegen.look_at_camera((0, -4, 0), 96, 80)
    vt = scenegen.make_view_tensors(0, cam.npix, 8)
    full = pipeline.run(g, [cam], [vt], fusion=False)
    bq = full["bins"]["per_view"][0]
    rows = lambda vi, key, pix: None if key in ("target", "dT") else vt[key][pix]
    forward_axis = np.abs(np.asarray(cam.R)[2])
    assert forward_axis[0] < 1e-6 and forward_axis[2] < 1e-6   # means x and z keep the depth
    cand = [i for i in S.pick_gaussians([bq], 40, seed=5) if full["gflags"][i] == 0][:4]
    assert len(cand) == 4
    for gi in cand:
        for key, comp in (("means", 0), ("means", 2), ("scales", 1), ("quats", 3), ("opacity", 0), ("sh", 4)):
            x = float(np.asarray(g[key]).reshape(700, -1)[gi, comp])
            fd = S.central_difference(g, cam, bq, rows, 8, gi, key, comp, 1e-6 * max(abs(x), 0.05))
            an = float(full["grads"][key].reshape(700, -1)[gi, comp])
            mag = float(full["grads_mag"][key].reshape(700, -1)[gi, comp])
            assert abs(fd - an) <= 1e-6 * mag + 1e-9, (gi, key, comp, fd, an)
