"""GPU vs oracle at the benchmark's full sizes, in the launch configuration
bench.py times, on outputs the oracle can compute in seconds:

* binning: every key and every tile range, bit for bit (the oracle's float32
  binning runs on all Gaussians);
* forward: every pixel of a block of tiles;
* gradients and fusion: Gaussians of the front layer (the only ones the walk
  reaches at this density: the nearest with a rect of at most 12x12 tiles at
  800x800, or of at most 20x20 tiles within a 1500-tile budget at 1080p), with
  the oracle walking every tile of their rects, so their sums are complete
  (tests/sampled.py); up to 64 that contribute are compared.
The c3 parameters are also checked as surfels (Section 3.1) in the BF16 form,
the surfel step bench.py times beside the headline.
"""
import numpy as np
import pytest
import torch

import scenegen
from oracle import binspec, pipeline, project, raster, surfel
from tests import gpu_util as U
from tests import sampled as S

pytestmark = pytest.mark.gpu

# workload, form, tile block (x0, y0, size) for the forward check, primitive
CASES = [
    ("c2", "f32", (22, 20, 6), "gaussian"),
    ("c3", "f32", (56, 30, 5), "gaussian"),
    ("c3", "bf16", (56, 30, 5), "gaussian"),
    ("c3", "bf16", (56, 30, 5), "surfel"),
]
# front-layer sample per workload: (max rect side in tiles, nearest count, tile budget)
FRONT = {"c2": (12, 5000, None), "c3": (20, 100000, 1500)}
# elementwise bounds (units of the magnitude companion), per arithmetic form
RT = {f: dict(F=r, grad=r, fuse=r) for f, r in U.RTOL_FORM.items()}


@pytest.fixture(scope="module", params=CASES, ids=[f"{w}-{f}" + ("" if p == "gaussian" else f"-{p}")
                                                    for w, f, _, p in CASES])
def run(request):
    wname, form, (bx, by, bs), prim = request.param
    surf = prim == "surfel"
    rule = "surfel" if surf else "box"
    wl = scenegen.WORKLOADS[wname]
    print(f"\n[full {wname} {form} {prim}] generating", flush=True)
    g = scenegen.make_gaussians(wl.n, wl.half_extent, wl.sh_degree, wl.d, seed=0, feat_dtype=wl.feat_dtype)
    cams = scenegen.make_cameras(wl.views)
    vts = [scenegen.make_view_tensors(0, cams[0].npix, wl.d, with_dT=True,
                                      target_dtype="bf16" if wl.feat_dtype == "bf16" else "f32")]
    gpu = U.run_gpu(g, cams, vts, fusion=wl.fusion, form=form, margin=1.02, bin_rule=rule)
    print(f"[full {wname} {form} {prim}] gpu done: {gpu['counters'].n_instances} instances", flush=True)
    bins = binspec.bin_views(g, cams, rule)
    cam = cams[0]
    tiles_x = bins["per_view"][0]["tiles_x"]
    sel = np.array([(by + j) * tiles_x + (bx + i) for j in range(bs) for i in range(bs)], np.int64)
    pr = (surfel.project_surfel if surf else project.project)(g, cam)
    vt = vts[0]
    out = raster.render_view(cam, pipeline.view_slice(bins, 0, cam), bins["gids"], pr,
                             feat=np.asarray(g["feat"], np.float64), dC=vt["dC"], dF=vt["dF"], dT=vt["dT"],
                             target=vt["target"] if wl.fusion else None, tile_sel=sel, want_F=True,
                             want_Fmag=True, want_fusion=wl.fusion)
    print(f"[full {wname} {form} {prim}] oracle done", flush=True)
    return dict(wl=wl, form=form, g=g, cams=cams, gpu=gpu, bins=bins, out=out, pr=pr, vt=vt,
                block=(bx, by, bs), sel=sel, surf=surf)


def test_binning_bit_exact_full(run):
    gpu, bins = run["gpu"], run["bins"]
    c = gpu["counters"]
    assert c.n_instances == bins["keys"].size
    keys, gids = gpu["r"].bin_keys(int(c.n_instances))
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), bins["keys"])
    assert np.array_equal(gids.cpu().numpy().astype(np.int64), bins["gids"])
    ranges = gpu["r"].ws_view("ranges", torch.int32, gpu["r"].n_tiles * 2).cpu().numpy().reshape(-1, 2)
    assert np.array_equal(ranges.astype(np.int64), bins["ranges"])


def _block_pixels(run):
    cam = run["cams"][0]
    bx, by, bs = run["block"]
    ys, xs = np.mgrid[by * 16:(by + bs) * 16, bx * 16:(bx + bs) * 16]
    ok = (xs < cam.width) & (ys < cam.height)
    return (ys[ok] * cam.width + xs[ok]).astype(np.int64)


def test_forward_block(run):
    gpu, out = run["gpu"], run["out"]
    pix = _block_pixels(run)
    img = gpu["img"]
    flags = out["flags"][pix]
    ok = (flags & 1) == 0
    print(f"[full] ambiguous pixels in block {1 - ok.mean():.2e}", flush=True)
    C, T = img.C.cpu().numpy()[pix], img.T.cpu().numpy()[pix]
    nit = img.n_iter.cpu().numpy()[pix].astype(np.int64)
    assert np.array_equal(nit[ok], out["niter"][pix][ok])
    assert U.elementwise(C, out["C"][pix], out["Cmag"][pix], mask=ok[:, None].repeat(3, 1),
                         amb=out["Cden"][pix])[0] <= 1.0
    assert U.elementwise(T, out["T"][pix], out["T"][pix], mask=ok, amb=out["Tden"][pix])[0] <= 1.0
    F = img.F.cpu().numpy()[pix]
    rt = RT[run["form"]]["F"]
    mF, aF = U.elementwise(F, out["F"][pix], out["Fmag"][pix], rtol=rt, mask=ok[:, None].repeat(F.shape[1], 1),
                           amb=out["Fden"][pix])
    err = np.abs(F - out["F"][pix])[ok] / np.maximum(out["Fmag"][pix][ok], 1e-30)
    print(f"[full] F ratio max/mean {mF:.3f}/{aF:.3f}; |dF|/M max {err.max():.2e} mean {err.mean():.2e}", flush=True)
    assert mF <= 1.0


@pytest.fixture(scope="module")
def front(run):
    """The sampled oracle over the front layer's tiles (see the module docstring)."""
    g, cam = run["g"], run["cams"][0]
    bq = run["bins"]["per_view"][0]
    wl = run["wl"]
    vt = run["vt"]
    cand = S.pick_front(bq, *FRONT[wl.name])
    views = [dict(tiles=np.array(sorted(set().union(*[S._rect_tiles(bq, int(i)) for i in cand]))), tile_off=0,
                  pix_off=0)]
    rows = lambda vi, key, pix: vt[key][pix] if (key != "target" or wl.fusion) else None
    ora = S.run(g, [cam], [bq], cand, views, rows, wl.d, surfels=run["surf"])
    keep = np.nonzero(U.checkable(ora["gflag"]) & (np.abs(ora["sums"]["opacity"]) > 0))[0][:64]
    print(f"[full] front layer: {cand.size} Gaussians over {views[0]['tiles'].size} tiles, {keep.size} compared",
          flush=True)
    return dict(cand=cand, keep=keep, **ora)


def test_gradients_of_front_gaussians(run, front):
    gpu = run["gpu"]
    keep = front["keep"]
    assert keep.size >= 8
    gid = front["cand"][keep]
    rt = RT[run["form"]]["grad"]
    for k in S.GRAD_KEYS:
        got = gpu["grads"][k].cpu().numpy()[gid]
        mx, mean = U.elementwise(got, front["sums"][k][keep], front["mags"][k][keep], rtol=rt,
                                 amb=front["ambs"][k][keep])
        print(f"[full] grad {k}: ratio max/mean {mx:.3f}/{mean:.3f} (rtol {rt:g})", flush=True)
        assert mx <= 1.0, k


def test_fusion_of_front_gaussians(run, front):
    if not run["wl"].fusion:
        pytest.skip("workload without fusion")
    acc = run["gpu"]["acc"]
    keep = front["keep"]
    gid = front["cand"][keep]
    s = (acc.sum + acc.comp).cpu().numpy()[gid]
    w = (acc.wsum + acc.wcomp).cpu().numpy()[gid]
    rt = RT[run["form"]]["fuse"]
    mx, mean = U.elementwise(s, front["fsum"][keep], front["fsum_mag"][keep], rtol=rt, amb=front["fsum_amb"][keep])
    mw, _ = U.elementwise(w, front["wsum"][keep], front["wsum"][keep], rtol=rt, amb=front["wsum_amb"][keep])
    print(f"[full] fusion ratio max/mean {mx:.3f}/{mean:.3f}, wsum {mw:.3f} (rtol {rt:g})", flush=True)
    assert mx <= 1.0 and mw <= 1.0
