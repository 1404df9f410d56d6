"""The sampled form of the oracle (tests/sampled.py), used at the batched
workloads' full sizes, equals the full oracle pipeline on a small two-view
scene: forward outputs of the walked tiles, and the sampled Gaussians'
gradient, magnitude and fusion sums over both views."""
import numpy as np

import scenegen
from oracle import binspec, pipeline
from tests import sampled as S


def test_sampled_oracle_equals_full_pipeline():
    g = scenegen.make_gaussians(900, 1.5, 2, 8, seed=21, feat_dtype="bf16")
    cams = [scenegen.look_at_camera(p, w, h) for p, w, h in (((0, -4, 0), 96, 80), ((3, -2.5, 1.2), 112, 64))]
    vts = [dict(scenegen.make_view_tensors(i, c.npix, 8, with_dT=True)) for i, c in enumerate(cams)]
    full = pipeline.run(g, cams, vts, fusion=True, want_Fmag=True)
    bqs = full["bins"]["per_view"]
    counts = [binspec.tile_counts(bq) for bq in bqs]
    cand = S.pick_gaussians(bqs, 10, seed=3)
    assert cand.size == 10
    views = S.plan(bqs, counts, cams, cand, extra_tiles=2, seed=4)
    ora = S.run(g, cams, bqs, cand, views, lambda vi, key, pix: vts[vi][key][pix], 8)
    for vi, vw in enumerate(views):
        f, ref = vw["fwd"], full["views"][vi]
        p = f["pix"]
        assert np.array_equal(f["niter"], ref["niter"][p])
        for k in ("C", "Cmag", "T", "F", "Fmag"):
            assert np.allclose(f[k], ref[k][p], rtol=1e-12, atol=1e-300), k
    for k in S.GRAD_KEYS:
        scale = np.maximum(full["grads_mag"][k][cand], 1e-300)
        assert np.all(np.abs(ora["sums"][k] - full["grads"][k][cand]) <= 1e-10 * scale), k
        assert np.allclose(ora["mags"][k], full["grads_mag"][k][cand], rtol=1e-10, atol=1e-300), k
    assert np.allclose(ora["fsum"], full["fsum"][cand], rtol=1e-10, atol=1e-12)
    assert np.allclose(ora["wsum"], full["wsum"][cand], rtol=1e-12, atol=1e-300)
    assert np.array_equal(ora["gflag"] != 0, full["gflags"][cand] != 0)
