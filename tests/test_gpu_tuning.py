"""Launch-shape tuning: every candidate of fh_tuning_candidates gives the same
results bit for bit (no arithmetic depends on the launch shape), and the
autotuner picks one of them, reusing a cached pick for the same workload key."""
import json

import numpy as np
import pytest
import torch

import scenegen
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form,d", [("f32", 64), ("bf16", 64), ("bf16", 256)])
def test_every_launch_shape_gives_identical_results(form, d, tmp_path):
    from paper_2505_19154_amd import _lib as L
    from paper_2505_19154_amd.raster import FusionAcc, Rasterizer
    # (d = 256 brings the BF16 forward's 4-row and 256-channel shapes)
    g = scenegen.make_gaussians(3000, 1.5, 3, d, seed=31, feat_dtype="bf16")
    cams = [scenegen.look_at_camera(p, w, h) for p, w, h in (((0, -4, 0), 120, 88), ((3, -2.5, 1.2), 100, 72))]
    vts = U.view_maps(cams, d, target_dtype="bf16")
    dg = U.device_gaussians(g)
    dC, dF, dT = U.concat(vts, "dC"), U.concat(vts, "dF"), U.concat(vts, "dT")
    target = U.concat(vts, "target_bits")
    r = Rasterizer(cams, dg.n, dg.sh_degree, dg.d, feat_dtype="bf16", form=form)
    img = r.forward(dg)
    ref_img = {k: getattr(img, k).clone() for k in ("C", "F", "T", "n_iter")}
    acc0 = FusionAcc.zeros(dg.n, d, "cuda")
    ref_grads = {k: v.clone() for k, v in r.render_bwd(dg, img, dC, dF, dT, target=target, acc=acc0).items()}
    torch.cuda.synchronize()
    default = (int(r.plan.tuning.fwd_slice), int(r.plan.tuning.bwd_chunk), int(r.plan.tuning.fwd_rows),
               int(r.plan.tuning.schedule))
    fwd_c = r.tuning_candidates(L.FH_K_RENDER_FWD)
    bwd_c = r.tuning_candidates(L.FH_K_RENDER_BWD)
    print(f"[tuning {form} d{d}] default {default}, forward {fwd_c}, backward {bwd_c}", flush=True)
    assert default in fwd_c and default in bwd_c
    for sl, ch, rows, sc in fwd_c + bwd_c:
        r.set_tuning(sl, ch, rows, sc)
        out = r.render_fwd(dg)
        for k, v in ref_img.items():
            assert torch.equal(getattr(out, k), v), (sl, ch, rows, sc, k)
        acc = FusionAcc.zeros(dg.n, d, "cuda")
        grads = r.render_bwd(dg, out, dC, dF, dT, target=target, acc=acc)
        torch.cuda.synchronize()
        for k, v in ref_grads.items():
            assert torch.equal(grads[k], v), (sl, ch, rows, sc, k)
        assert torch.equal(acc.sum, acc0.sum) and torch.equal(acc.wsum, acc0.wsum), (sl, ch, rows, sc)
    # the autotuner picks a candidate and caches it under the workload key
    cache = str(tmp_path / "tune.json")
    r.set_tuning(*default)
    img = r.render_fwd(dg)
    pick = r.autotune(dg, img, dC, dF, dT, target=target, reps=2, cache=cache)
    print(f"[tuning {form} d{d}] picked {pick}", flush=True)
    assert (pick["fwd_slice"], pick["fwd_rows"]) in [(c[0], c[2]) for c in fwd_c]
    assert pick["bwd_chunk"] in [c[1] for c in bwd_c] and pick["schedule"] in (0, 1)
    table = json.load(open(cache))
    assert table[r.tuning_key()] == pick
    # a new plan for the same workload takes the cached pick without timing
    r2 = Rasterizer(cams, dg.n, dg.sh_degree, dg.d, feat_dtype="bf16", form=form)
    img2 = r2.forward(dg)
    assert r2.autotune(dg, img2, cache=cache) == pick
    img2 = r2.forward(dg)
    assert torch.equal(img2.F, ref_img["F"]) and torch.equal(img2.C, ref_img["C"])
    # a shape outside the candidates is refused before any launch
    r2.set_tuning(48, 32)
    with pytest.raises(L.FhError):
        r2.render_fwd(dg)
