"""GPU (HIP, through the C ABI) vs the FP64 oracle on seeded synthetic scenes.

Sizes are small enough for the oracle to finish in seconds while spanning
several tiles, ragged edge tiles and (for the batched scene) several views of
different resolution.  Binning is compared bit for bit; floating-point outputs
under the tolerance rule of tests/gpu_util.py.
"""
import numpy as np
import pytest
import torch

import scenegen
from oracle import consts
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

SCENES = {
    # name: (n, half_extent, sh_degree, d, feat_dtype, cameras, form)
    "c1": (1000, 1.0, 0, 16, "f32", "front128", "f32"),
    "sh3_ragged": (3000, 1.5, 3, 32, "f32", "front200x150", "f32"),
    "bf16_feat": (2000, 1.5, 2, 24, "bf16", "front100x70", "f32"),
    "multiview": (1500, 1.2, 1, 8, "f32", "three", "f32"),
    "mfma_d32": (2500, 1.5, 3, 32, "bf16", "front120x90", "bf16"),
    "mfma_d128_multiview": (1500, 1.2, 1, 128, "bf16", "three", "bf16"),
    # the other BF16-form widths: 64 and 96 (16-row forward, one slice), 256
    # (8-row forward, one 256-channel slice; the adjoint's widest dF tile)
    "mfma_d64": (2000, 1.5, 3, 64, "bf16", "front100x70", "bf16"),
    "mfma_d96": (2000, 1.5, 2, 96, "bf16", "front90x60", "bf16"),
    "mfma_d256": (1200, 1.5, 3, 256, "bf16", "front96x80", "bf16"),
    # wider than 256: the adjoint and fusion in channel slices (d = 512: two of
    # 256 channels; d = 384: three of 128, so f . dF is carried over two slices)
    "mfma_d512": (900, 1.5, 1, 512, "bf16", "front64x48", "bf16"),
    "mfma_d384": (900, 1.5, 2, 384, "bf16", "front64x48", "bf16"),
    # FP32 form with FP32 features at d = 128 and 256: the MFMA forward with
    # three-term splits in its 8-row shapes (128- and 256-channel slices)
    "fsplit_d128": (1500, 1.5, 1, 128, "f32", "front100x70", "f32"),
    "fsplit_d256": (1200, 1.5, 1, 256, "f32", "front96x80", "f32"),
    # images smaller than one tile (the only tile ragged in both directions):
    # 7 x 5 pixels in the BF16-MFMA form, a single pixel in the FP32 form, and
    # 13 x 3 pixels of surfels at d = 64 (none of their pixels decides a
    # near-threshold skip or stop)
    "subtile_7x5_mfma": (400, 1.0, 2, 32, "bf16", "front7x5", "bf16"),
    "one_pixel": (300, 1.0, 1, 8, "f32", "front1x1", "f32"),
    "subtile_surfel_13x3": (400, 1.0, 1, 64, "bf16", "front13x3", "bf16", "surfel"),
    # the largest sizes the plan accepts: d = 1024 (BF16 form: the adjoint and
    # fusion in four 256-channel slices) and 32 views (a ring of small cameras
    # of 20 different sizes, one plan, one sort)
    "max_d1024": (600, 1.5, 1, 1024, "bf16", "front48x40", "bf16"),
    "max_views32": (800, 1.2, 1, 8, "f32", "ring32", "f32"),
    # splats of 1-2 tiles: some 2048-instance duplication ranges span more
    # than 1024 ranks (up to 1260) and take the per-instance rank search
    "tiny_splats": (4000, 1.5, 0, 8, "f32", "front40x40", "f32"),
    # surfels (Section 3.1's planar primitive): ray-plane intersection,
    # disc-image binning; scales x3 so that most span pixels.  FP32 form (VALU
    # kernels), then the BF16-MFMA form: 16-row forward at d = 64, the 8-row
    # 256-channel forward and the widest resident dF tile at d = 256 over three
    # views, two 256-channel slices at d = 512
    "surfel_sh2": (2000, 1.5, 2, 16, "f32", "front120x90", "f32", "surfel"),
    "surfel_multiview_bf16feat": (1500, 1.2, 1, 32, "bf16", "three", "f32", "surfel"),
    "surfel_mfma_d64": (2000, 1.5, 2, 64, "bf16", "front120x90", "bf16", "surfel"),
    "surfel_mfma_d256_multiview": (1200, 1.2, 1, 256, "bf16", "three", "bf16", "surfel"),
    "surfel_mfma_d512": (900, 1.5, 1, 512, "bf16", "front64x48", "bf16", "surfel"),
    # every tenth surfel edge-on (the plane z = 0 holds the view direction):
    # the middle pixel row (odd height) casts rays inside those planes, where
    # the intersection does not exist and the density is zero, and their
    # disc images bin as one row of tiles
    "surfel_edge_on": (1500, 1.5, 1, 32, "bf16", "front96x81", "bf16", "surfel", "edge_on"),
}
# BF16-MFMA form: F, the feature part of the adjoint and the fusion sums are
# contractions over two-term BF16 splits (tests/gpu_util.py: RTOL_FORM).
F_RTOL = U.RTOL_FORM


def _rule(name):
    return SCENES[name][7] if len(SCENES[name]) > 7 else "box"


def _scene(name, seed=0):
    n, h, deg, d, fdt, camr, _ = SCENES[name][:7]
    g = scenegen.make_gaussians(n, h, deg, d, seed=seed, feat_dtype=fdt)
    if _rule(name) == "surfel":
        g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    if SCENES[name][8:] == ("edge_on",):
        idx = np.arange(0, n, 10)
        q, m = np.asarray(g["quats"]).copy(), np.asarray(g["means"]).copy()
        q[idx] = [1.0, 0.0, 0.0, 0.0]   # tangents x and y: the plane z = const
        m[idx, 2] = 0.0                 # through the camera centre's height
        g["quats"], g["means"] = q.astype(np.float32), m.astype(np.float32)
    if camr == "three":
        cams = [scenegen.look_at_camera(p, w, hh) for p, w, hh in
                (((0, -4, 0), 96, 80), ((3, -2.5, 1.2), 130, 70), ((-2, 1.5, 3.2), 64, 64))]
    elif camr == "ring32":
        cams = [scenegen.look_at_camera((4.0 * np.cos(a), 4.0 * np.sin(a), 0.8 * np.sin(3 * a)),
                                        20 + (i % 5) * 3, 16 + (i % 4) * 5)
                for i, a in enumerate(np.linspace(0.0, 2.0 * np.pi, 32, endpoint=False))]
    else:
        cams = scenegen.make_cameras(camr)
    return g, cams


@pytest.fixture(scope="module", params=list(SCENES))
def case(request):
    g, cams = _scene(request.param)
    form = SCENES[request.param][6]
    # the BF16 form takes a BF16 fusion target (an MFMA operand as stored)
    vts = U.view_maps(cams, g["d"], with_dT=True, target_dtype="bf16" if form == "bf16" else "f32")
    print(f"\n[case {request.param}] n={g['means'].shape[0]} views={len(cams)}", flush=True)
    rule = _rule(request.param)
    gpu = U.run_gpu(g, cams, vts, fusion=g["d"] > 0, form=form, bin_rule=rule)
    ora = U.run_oracle(g, cams, vts, fusion=g["d"] > 0, bin_rule=rule)
    return dict(name=request.param, g=g, cams=cams, vts=vts, gpu=gpu, ora=ora, form=form)


def test_binning_bit_exact(case):
    gpu, ora = case["gpu"], case["ora"]
    c = gpu["counters"]
    assert not c.inst_overflow
    keys_ref = ora["bins"]["keys"]
    assert c.n_instances == keys_ref.size
    keys, gids = gpu["r"].bin_keys(int(c.n_instances))
    keys = keys.cpu().numpy().view(np.uint64)
    gids = gids.cpu().numpy().astype(np.int64)
    assert np.array_equal(keys, keys_ref)
    assert np.array_equal(gids, ora["bins"]["gids"])
    ranges = gpu["r"].ws_view("ranges", torch.int32, gpu["r"].n_tiles * 2).cpu().numpy().reshape(-1, 2)
    assert np.array_equal(ranges.astype(np.int64), ora["bins"]["ranges"])
    # per-(view, Gaussian) depth keys and rects
    n = case["g"]["means"].shape[0]
    dk = gpu["r"].ws_view("depth_key", torch.int32, n * len(case["cams"])).cpu().numpy().view(np.uint32)
    rect = gpu["r"].ws_view("rect", torch.int32, 4 * n * len(case["cams"])).cpu().numpy().reshape(-1, 4)
    for vi, bq in enumerate(ora["bins"]["per_view"]):
        b = bq["binned"]
        assert np.array_equal(dk[vi * n:(vi + 1) * n][b], bq["depth"].view(np.uint32)[b])
        assert np.all(dk[vi * n:(vi + 1) * n][~b] == 0xFFFFFFFF)
        rv = rect[vi * n:(vi + 1) * n]
        assert np.array_equal(rv[b, 0], bq["x0"][b]) and np.array_equal(rv[b, 2], bq["x1"][b])
        assert np.array_equal(rv[b, 1], bq["y0"][b]) and np.array_equal(rv[b, 3], bq["y1"][b])


def _pixel_masks(case):
    flags = np.concatenate([v["flags"] for v in case["ora"]["views"]])
    # bit 0: a skip/stop decision near its threshold (value ambiguous); bit 1
    # (alpha near the clamp) leaves the pixel's value continuous
    return (flags & 1) == 0, flags


def test_forward_parity(case):
    gpu, ora = case["gpu"], case["ora"]
    img = gpu["img"]
    C = img.C.cpu().numpy()
    T = img.T.cpu().numpy()
    nit = img.n_iter.cpu().numpy().astype(np.int64)
    Cr = np.concatenate([v["C"] for v in ora["views"]])
    Cm = np.concatenate([v["Cmag"] for v in ora["views"]])
    Tr = np.concatenate([v["T"] for v in ora["views"]])
    Cd = np.concatenate([v["Cden"] for v in ora["views"]])
    Td = np.concatenate([v["Tden"] for v in ora["views"]])
    nr = np.concatenate([v["niter"] for v in ora["views"]])
    ok, flags = _pixel_masks(case)
    amb = 1.0 - ok.mean()
    print(f"[{case['name']}] ambiguous pixels {amb:.2e}", flush=True)
    assert amb < 1e-2
    assert np.array_equal(nit[ok], nr[ok])
    mC, aC = U.elementwise(C, Cr, Cm, mask=ok[:, None].repeat(3, 1), amb=Cd)
    mT, aT = U.elementwise(T, Tr, Tr, mask=ok, amb=Td)
    print(f"[{case['name']}] C max/mean ratio {mC:.3f}/{aC:.3f}  T {mT:.3f}/{aT:.3f}  "
          f"norm C {U.normwise(C, Cr):.2e} T {U.normwise(T, Tr):.2e}", flush=True)
    assert mC <= 1.0 and mT <= 1.0
    assert U.normwise(C, Cr) <= U.RTOL and U.normwise(T, Tr) <= U.RTOL
    if img.F is not None:
        F = img.F.cpu().numpy()
        Fr = np.concatenate([v["F"] for v in ora["views"]])
        Fm = np.concatenate([v["Fmag"] for v in ora["views"]])
        Fd = np.concatenate([v["Fden"] for v in ora["views"]])
        rt = F_RTOL[case["form"]]
        mF, aF = U.elementwise(F, Fr, Fm, rtol=rt, mask=ok[:, None].repeat(F.shape[1], 1), amb=Fd)
        err = np.abs(F - Fr)[ok] / np.maximum(Fm[ok], 1e-30)
        print(f"[{case['name']}] F max/mean ratio {mF:.3f}/{aF:.3f} (rtol {rt:g}) norm {U.normwise(F, Fr):.2e} "
              f"max/mean |dF|/M {err.max():.2e}/{err.mean():.2e}", flush=True)
        assert mF <= 1.0 and U.normwise(F, Fr) <= rt


def test_backward_parity(case):
    gpu, ora = case["gpu"], case["ora"]
    keep = U.checkable(ora["gflags"])
    print(f"[{case['name']}] Gaussians excluded (ambiguous colour clamp) {1 - keep.mean():.2e}", flush=True)
    for k in ("means", "scales", "quats", "opacity", "sh"):
        got = gpu["grads"][k].cpu().numpy()
        ref = ora["grads"][k]
        mag = ora["grads_mag"][k]
        m = keep.reshape((-1,) + (1,) * (ref.ndim - 1)) & np.ones(ref.shape, bool)
        rt = U.RTOL_FORM[case["form"]]
        mx, mean = U.elementwise(got, ref, mag, rtol=rt, mask=m, amb=ora["grads_amb"][k])
        nw = U.normwise(got, ref)
        print(f"[{case['name']}] grad {k}: max/mean ratio {mx:.3f}/{mean:.3f} (rtol {rt:g}) norm {nw:.2e}",
              flush=True)
        assert mx <= 1.0, k
        assert nw <= rt, k


def test_fusion_parity(case):
    gpu, ora = case["gpu"], case["ora"]
    if case["g"]["d"] == 0:
        pytest.skip("no features")
    acc = gpu["acc"]
    s = (acc.sum + acc.comp).cpu().numpy()
    w = (acc.wsum + acc.wcomp).cpu().numpy()
    keep = U.checkable(ora["gflags"])
    rt = U.RTOL_FORM[case["form"]]
    mx, mean = U.elementwise(s, ora["fsum"], ora["fsum_mag"], rtol=rt, mask=keep[:, None] & np.ones(s.shape, bool),
                             amb=ora["fsum_amb"])
    mw, _ = U.elementwise(w, ora["wsum"], ora["wsum"], rtol=rt, mask=keep, amb=ora["wsum_amb"])
    print(f"[{case['name']}] fusion sum max/mean ratio {mx:.3f}/{mean:.3f} wsum {mw:.3f} "
          f"norm {U.normwise(s, ora['fsum']):.2e}", flush=True)
    assert mx <= 1.0 and mw <= 1.0
    assert U.normwise(s, ora["fsum"]) <= rt and U.normwise(w, ora["wsum"]) <= rt


def test_deterministic_rerun(case):
    g, cams, vts = case["g"], case["cams"], case["vts"]
    again = U.run_gpu(g, cams, vts, fusion=g["d"] > 0, form=case["form"], bin_rule=_rule(case["name"]))
    a, b = case["gpu"], again
    assert torch.equal(a["img"].C, b["img"].C) and torch.equal(a["img"].T, b["img"].T)
    for k in a["grads"]:
        assert torch.equal(a["grads"][k], b["grads"][k]), k
    if a["acc"] is not None:
        assert torch.equal(a["acc"].sum, b["acc"].sum)


def test_c1_takes_every_decision_as_the_oracle_does(monkeypatch):
    """The 1k-Gaussian 128x128 workload has no decision within 2e-5 relative of
    its threshold (well beyond FP32's decision error of ~1e-5 at the longest
    walks here), so the GPU must agree with the oracle on every pixel and every
    Gaussian with no pixel masked and no ambiguity allowance: n_iter exactly,
    C, T, F, gradients and fusion sums under the FP32 rule."""
    from oracle import consts as oconsts
    monkeypatch.setattr(oconsts, "AMBIG_REL", 2e-5)
    g, cams = _scene("c1")
    vts = U.view_maps(cams, g["d"], with_dT=True)
    ora = U.run_oracle(g, cams, vts, fusion=True)
    v = ora["views"][0]
    assert np.all(v["flags"] == 0) and np.all(ora["gflags"] == 0)
    gpu = U.run_gpu(g, cams, vts, fusion=True)
    img = gpu["img"]
    assert np.array_equal(img.n_iter.cpu().numpy().astype(np.int64), v["niter"])
    assert U.elementwise(img.C.cpu().numpy(), v["C"], v["Cmag"])[0] <= 1.0
    assert U.elementwise(img.T.cpu().numpy(), v["T"], v["T"])[0] <= 1.0
    assert U.elementwise(img.F.cpu().numpy(), v["F"], v["Fmag"])[0] <= 1.0
    for k in ("means", "scales", "quats", "opacity", "sh"):
        assert U.elementwise(gpu["grads"][k].cpu().numpy(), ora["grads"][k], ora["grads_mag"][k])[0] <= 1.0, k
    s = (gpu["acc"].sum + gpu["acc"].comp).cpu().numpy()
    w = (gpu["acc"].wsum + gpu["acc"].wcomp).cpu().numpy()
    assert U.elementwise(s, ora["fsum"], ora["fsum_mag"])[0] <= 1.0
    assert U.elementwise(w, ora["wsum"], ora["wsum"])[0] <= 1.0
