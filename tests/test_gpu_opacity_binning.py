"""GPU vs oracle under the opacity-aware binning rule (fh_plan.bin_rule =
FH_BIN_OPACITY): keys, rects and ranges bit for bit (the float32 ln sequence
and per-Gaussian box factors of oracle/binspec.py), outputs under the
tolerance rule of tests/gpu_util.py, and the same composited values as the
box rule with fewer instances."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import binspec
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

SCENES = {
    # name: (n, half_extent, sh_degree, d, feat_dtype, cameras, form)
    "sh3_ragged": (3000, 1.5, 3, 32, "f32", [((0, -4, 0), 200, 150)], "f32"),
    "mfma_d64_multiview": (2000, 1.2, 2, 64, "bf16", [((0, -4, 0), 96, 80), ((3, -2.5, 1.2), 130, 70)], "bf16"),
    # every third Gaussian's opacity straddles the rule's cut-off 255 o = 1
    # (no instances at or below it; tiny boxes just above): uniform in
    # [0.5/255, 2/255], plus float32(1/255) and its two neighbours
    "low_opacity": (2400, 1.2, 1, 32, "bf16", [((0, -4, 0), 112, 88)], "bf16", "low_opacity"),
}


def _low_opacity(g):
    op = np.asarray(g["opacity"], np.float32).copy()
    idx = np.arange(0, op.size, 3)
    op[idx] = np.random.default_rng(11).uniform(0.5 / 255, 2.0 / 255, idx.size).astype(np.float32)
    c = np.float32(1.0 / 255.0)
    op[idx[:3]] = [np.nextafter(c, np.float32(0)), c, np.nextafter(c, np.float32(1))]
    g["opacity"] = op


@pytest.fixture(scope="module", params=list(SCENES))
def case(request):
    n, h, deg, d, fdt, cams_spec, form = SCENES[request.param][:7]
    g = scenegen.make_gaussians(n, h, deg, d, seed=0, feat_dtype=fdt)
    if SCENES[request.param][7:] == ("low_opacity",):
        _low_opacity(g)
    cams = [scenegen.look_at_camera(p, w, hh) for p, w, hh in cams_spec]
    vts = U.view_maps(cams, d, with_dT=True, target_dtype="bf16" if form == "bf16" else "f32")
    print(f"\n[opacity-binning {request.param}]", flush=True)
    gpu = U.run_gpu(g, cams, vts, fusion=True, form=form, bin_rule="opacity")
    box = U.run_gpu(g, cams, vts, fusion=True, form=form)
    ora = U.run_oracle(g, cams, vts, fusion=True, bin_rule="opacity")
    return dict(name=request.param, g=g, cams=cams, gpu=gpu, box=box, ora=ora, form=form)


def test_binning_bit_exact(case):
    gpu, ora = case["gpu"], case["ora"]
    c = gpu["counters"]
    assert not c.inst_overflow
    assert c.n_instances == ora["bins"]["keys"].size
    assert c.n_instances < case["box"]["counters"].n_instances
    keys, gids = gpu["r"].bin_keys(int(c.n_instances))
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ora["bins"]["keys"])
    assert np.array_equal(gids.cpu().numpy().astype(np.int64), ora["bins"]["gids"])
    ranges = gpu["r"].ws_view("ranges", torch.int32, gpu["r"].n_tiles * 2).cpu().numpy().reshape(-1, 2)
    assert np.array_equal(ranges.astype(np.int64), ora["bins"]["ranges"])
    if case["name"] == "low_opacity":
        # the cut-off itself: no instance at or below 255 o = 1, boxes just above
        op = np.asarray(case["g"]["opacity"])
        has = np.zeros(op.size, bool)
        has[np.unique(gids.cpu().numpy().astype(np.int64))] = True
        below, above = op < 0.99 / 255, (op > 1.01 / 255) & (op < 2.0 / 255)
        assert below.sum() > 100 and not has[below].any()
        assert above.sum() > 100 and has[above].all()
        assert has[[0, 3, 6]].tolist() == [False, False, True]   # 1/255's neighbour below, 1/255, neighbour above
    n = case["g"]["means"].shape[0]
    rect = gpu["r"].ws_view("rect", torch.int32, 4 * n * len(case["cams"])).cpu().numpy().reshape(-1, 4)
    for vi, bq in enumerate(ora["bins"]["per_view"]):
        b = bq["binned"]
        rv = rect[vi * n:(vi + 1) * n]
        assert np.array_equal(rv[b, 0], bq["x0"][b]) and np.array_equal(rv[b, 2], bq["x1"][b])
        assert np.array_equal(rv[b, 1], bq["y0"][b]) and np.array_equal(rv[b, 3], bq["y1"][b])


def test_outputs_match_the_oracle_and_the_box_rule(case):
    gpu, box, ora = case["gpu"], case["box"], case["ora"]
    rt = U.RTOL_FORM[case["form"]]
    ok = np.concatenate([(v["flags"] & 1) == 0 for v in ora["views"]])
    img, bimg = gpu["img"], box["img"]
    Cr = np.concatenate([v["C"] for v in ora["views"]])
    Cm = np.concatenate([v["Cmag"] for v in ora["views"]])
    Fr = np.concatenate([v["F"] for v in ora["views"]])
    Fm = np.concatenate([v["Fmag"] for v in ora["views"]])
    nr = np.concatenate([v["niter"] for v in ora["views"]])
    assert np.array_equal(img.n_iter.cpu().numpy().astype(np.int64)[ok], nr[ok])
    for got in (img, bimg):     # both rules against the oracle's values
        assert U.elementwise(got.C.cpu().numpy(), Cr, Cm, mask=ok[:, None].repeat(3, 1))[0] <= 1.0
        d = Fr.shape[1]
        assert U.elementwise(got.F.cpu().numpy(), Fr, Fm, rtol=rt, mask=ok[:, None].repeat(d, 1))[0] <= 1.0
    # fewer list positions walked, the same pixels reached
    assert torch.all(img.n_iter <= bimg.n_iter)
    keep = U.checkable(ora["gflags"])
    for k in ("means", "scales", "quats", "opacity", "sh"):
        ref = ora["grads"][k]
        m = keep.reshape((-1,) + (1,) * (ref.ndim - 1)) & np.ones(ref.shape, bool)
        mx, _ = U.elementwise(gpu["grads"][k].cpu().numpy(), ref, ora["grads_mag"][k], rtol=rt, mask=m,
                              amb=ora["grads_amb"][k])
        assert mx <= 1.0, k
    s = (gpu["acc"].sum + gpu["acc"].comp).cpu().numpy()
    mx, _ = U.elementwise(s, ora["fsum"], ora["fsum_mag"], rtol=rt, mask=keep[:, None] & np.ones(s.shape, bool),
                          amb=ora["fsum_amb"])
    assert mx <= 1.0


def test_full_size_binning_bit_exact_1080p():
    """500k Gaussians, 1920x1080: every key and range of the opacity rule."""
    wl = scenegen.WORKLOADS["c3"]
    g = scenegen.make_gaussians(wl.n, wl.half_extent, wl.sh_degree, wl.d, seed=0, feat_dtype=wl.feat_dtype)
    cams = scenegen.make_cameras(wl.views)
    from paper_2505_19154_amd.raster import Rasterizer
    dg = U.device_gaussians(g)
    r = Rasterizer(cams, dg.n, dg.sh_degree, dg.d, feat_dtype="bf16", form="bf16", bin_rule="opacity")
    c = r.prepare(dg, margin=1.02)
    bins = binspec.bin_views(g, cams, "opacity")
    box_n = int(binspec.bin_views(g, cams)["keys"].size)
    print(f"[opacity-binning 1080p] {c.n_instances} instances (box rule: {box_n})", flush=True)
    assert c.n_instances == bins["keys"].size < box_n
    keys, gids = r.bin_keys(int(c.n_instances))
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), bins["keys"])
    assert np.array_equal(gids.cpu().numpy().astype(np.int64), bins["gids"])
    ranges = r.ws_view("ranges", torch.int32, r.n_tiles * 2).cpu().numpy().reshape(-1, 2)
    assert np.array_equal(ranges.astype(np.int64), bins["ranges"])
