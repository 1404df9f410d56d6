"""GPU edge cases, error paths, accumulation across calls, finalisation and the
autograd.Function (checked against central differences of the GPU forward)."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import pipeline
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _raster(g, cams, form="f32", **kw):
    from paper_2505_19154_amd.raster import Rasterizer
    dg = U.device_gaussians(g)
    return dg, Rasterizer(cams, dg.n, dg.sh_degree, dg.d, feat_dtype=g.get("feat_dtype", "f32"), form=form, **kw)


def test_all_culled_scene():
    g = scenegen.make_gaussians(200, 0.5, 1, 8, seed=1)
    g["means"] = g["means"] + np.float32([0.0, -5.0, 0.0])   # behind the camera at y = -4
    cams = scenegen.make_cameras("front64x48")
    dg, r = _raster(g, cams)
    img = r.forward(dg)
    torch.cuda.synchronize()
    assert r.counters().n_instances == 0
    assert torch.all(img.C == 0) and torch.all(img.T == 1) and torch.all(img.n_iter == 0)
    assert torch.all(img.F == 0)
    vts = U.view_maps(cams, 8)
    grads = r.render_bwd(dg, img, U.concat(vts, "dC"), U.concat(vts, "dF"), U.concat(vts, "dT"))
    torch.cuda.synchronize()
    for k, v in grads.items():
        assert torch.all(v == 0), k


@pytest.mark.parametrize("form,prim", [("f32", "gaussian"), ("bf16", "gaussian"), ("bf16", "surfel")])
def test_empty_scene(form, prim):
    """No Gaussians at all (n = 0, the arrays empty): every pixel of both views
    keeps C = 0, T = 1, n_iter = 0, F = 0; the adjoint with fusion and the NDFD
    gradient, the NDFD losses and the finalisation run and return empty
    per-Gaussian results and zero losses."""
    from paper_2505_19154_amd.raster import FusionAcc, Rasterizer, fuse_finalize
    d = 32
    g = scenegen.make_gaussians(0, 1.0, 1, d, seed=0, feat_dtype="bf16")
    cams = [scenegen.look_at_camera((0, -4, 0), 40, 24), scenegen.look_at_camera((3, -2.5, 1.2), 23, 17)]
    dg = U.device_gaussians(g)
    print(f"\n[empty scene {form} {prim}]", flush=True)
    r = Rasterizer(cams, 0, 1, d, feat_dtype="bf16", form=form, primitive=prim, ndfd=True)
    img = r.forward(dg)
    torch.cuda.synchronize()
    c = r.counters()
    assert c.n_instances == 0 and c.n_visited == 0
    assert torch.all(img.C == 0) and torch.all(img.T == 1) and torch.all(img.n_iter == 0) and torch.all(img.F == 0)
    vts = U.view_maps(cams, d, with_dT=True, target_dtype="bf16")
    tg = U.concat(vts, "target_bits")
    P = r.n_pixels
    ab = torch.ones(P, device="cuda")
    Lgt = torch.full((P,), float("nan"), device="cuda")
    Lcf = torch.full((P,), float("nan"), device="cuda")
    acc = FusionAcc.zeros(0, d, "cuda")
    grads = r.render_bwd(dg, img, U.concat(vts, "dC"), U.concat(vts, "dF"), U.concat(vts, "dT"), target=tg, acc=acc,
                         ndfd=dict(gt=tg, a=ab, b=ab, lam=0.5, k=20.0, Lgt=Lgt, Lcf=Lcf))
    l_gt, l_cf = r.ndfd_losses(dg, img, tg)
    out = fuse_finalize(acc, None)
    torch.cuda.synchronize()
    for k, v in grads.items():
        assert v.shape[0] == 0, k
    assert torch.all(Lgt == 0) and torch.all(Lcf == 0) and torch.all(l_gt == 0) and torch.all(l_cf == 0)
    assert tuple(out.shape) == (0, d)


def test_single_gaussian_matches_oracle():
    g = scenegen.make_gaussians(1, 0.1, 2, 16, seed=3)
    g["opacity"][:] = 0.8
    g["scales"][:] = 0.08
    cams = scenegen.make_cameras("front40x40")
    vts = U.view_maps(cams, 16)
    gpu = U.run_gpu(g, cams, vts, fusion=True)
    ora = U.run_oracle(g, cams, vts, fusion=True)
    v = ora["views"][0]
    ok = (v["flags"] & 1) == 0
    assert U.elementwise(gpu["img"].C.cpu().numpy(), v["C"], v["Cmag"], mask=ok[:, None].repeat(3, 1))[0] <= 1.0
    for k in ("means", "scales", "quats", "opacity"):
        assert U.elementwise(gpu["grads"][k].cpu().numpy(), ora["grads"][k], ora["grads_mag"][k],
                             amb=ora["grads_amb"][k])[0] <= 1.0, k


def test_nonfinite_gaussians_are_culled_and_counted():
    g = scenegen.make_gaussians(300, 1.0, 0, 8, seed=4)
    g["means"][5] = [np.nan, 0, 0]
    g["scales"][7] = [np.inf, 0.1, 0.1]
    g["quats"][9] = [np.nan, 0, 0, 1]
    cams = scenegen.make_cameras("front64x48")
    dg, r = _raster(g, cams)
    img = r.forward(dg)
    torch.cuda.synchronize()
    assert r.counters().n_culled_nonfinite == 3
    assert torch.isfinite(img.C).all() and torch.isfinite(img.F).all()
    ora = U.run_oracle(g, cams)
    assert r.counters().n_instances == ora["bins"]["keys"].size


def test_capacity_overflow_is_reported_not_faulted():
    g = scenegen.make_gaussians(500, 1.0, 0, 8, seed=5)
    cams = scenegen.make_cameras("front64x48")
    dg, r = _raster(g, cams, inst_capacity=64, visit_capacity=64)
    r.project(dg)
    r.bin_sort()
    c = r.counters()
    assert c.inst_overflow == 1 and c.n_instances > 64
    img = r.render_fwd(dg)   # skipped on the device: nothing is read out of bounds
    torch.cuda.synchronize()
    # grows and recovers
    img = r.forward(dg)
    c = r.counters()
    assert not c.inst_overflow and not c.visit_overflow
    ora = U.run_oracle(g, cams)
    ok = (ora["views"][0]["flags"] & 1) == 0
    assert U.elementwise(img.C.cpu().numpy(), ora["views"][0]["C"], ora["views"][0]["Cmag"],
                         mask=ok[:, None].repeat(3, 1))[0] <= 1.0


@pytest.mark.parametrize("form,d,prim", [("f32", 32, "gaussian"), ("bf16", 32, "gaussian"), ("bf16", 512, "gaussian"),
                                         ("f32", 32, "surfel"), ("bf16", 64, "surfel")])
def test_fusion_accumulates_across_calls_and_finalises(form, d, prim):
    # (d = 512 in the BF16 form: the fusion kernel in two 256-channel slices;
    # surfels: the fusion kernel's own walk with surfel records)
    from paper_2505_19154_amd.raster import FusionAcc, fuse_finalize
    g = scenegen.make_gaussians(800, 1.0, 1, d, seed=6, feat_dtype="bf16")
    if prim == "surfel":
        g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    cams = [scenegen.look_at_camera(p, 48, 40) for p in ((0, -4, 0), (3, -2.5, 1.2))]
    # exactly representable in BF16 (the BF16 form feeds the target to the MFMA in BF16)
    const = ((np.arange(d) % 32) * 0.125 - 2.0).astype(np.float32)
    acc = FusionAcc.zeros(800, d, "cuda")
    dg = U.device_gaussians(g)
    for cam in cams:     # one call per view into the same accumulators
        from paper_2505_19154_amd.raster import Rasterizer
        r = Rasterizer([cam], dg.n, dg.sh_degree, dg.d, feat_dtype="bf16", form=form, primitive=prim)
        img = r.forward(dg)
        tgt = torch.from_numpy(np.tile(const, (cam.npix, 1))).cuda()
        if form == "bf16":
            tgt = tgt.to(torch.bfloat16)      # exact: const is representable
        r.fuse_features(dg, img, tgt, acc)
    fin = fuse_finalize(acc, torch.from_numpy(g["feat"]).cuda())
    torch.cuda.synchronize()
    w = (acc.wsum + acc.wcomp).cpu().numpy()
    hit = w > 0
    assert hit.sum() > 50
    # a constant target map fuses to that constant; unseen Gaussians keep their feature
    f = fin.cpu().numpy()
    rt = 1e-6 if form == "f32" else U.RTOL_FORM["bf16"]
    assert np.allclose(f[hit], const[None, :], rtol=rt, atol=rt)
    assert np.array_equal(f[~hit], g["feat"][~hit])
    # the two calls equal one two-view call (oracle sums)
    vts = [dict(scenegen.make_view_tensors(i, c.npix, d), target=np.tile(const, (c.npix, 1))) for i, c in enumerate(cams)]
    ora = pipeline.run(g, cams, vts, fusion=True, bin_rule="surfel" if prim == "surfel" else "box")
    keep = U.checkable(ora["gflags"])
    assert U.elementwise(w, ora["wsum"], ora["wsum"], rtol=U.RTOL_FORM[form], mask=keep, amb=ora["wsum_amb"])[0] <= 1.0


def test_autograd_function_against_central_differences():
    """RasterizeFn on the 800x800 scene (200k Gaussians, SH3, D=64, FP32):
    autograd gradients of L = sum dC . C + sum dF . F for a 64-Gaussian subset
    against central differences of the FP64 forward, taken over each
    Gaussian's footprint tiles (all other pixels are unchanged by the step).
    The subset: among the 5000 nearest Gaussians with a footprint of at most
    12x12 tiles, the first 64 (by index) with no near-threshold decision in any
    pixel they touch (oracle flags and ambiguity bound) and a non-zero opacity
    gradient (at this density only the front
    layer is ever reached).  Steps keep the depth order (mean components across the view
    axis, scales, rotation, opacity, SH); a step along the view axis reorders
    Gaussians at this density and has no central difference."""
    from paper_2505_19154_amd.autograd import rasterize
    from paper_2505_19154_amd.raster import Rasterizer
    from oracle import binspec
    from tests import sampled as S
    wl = scenegen.WORKLOADS["c2"]
    g = scenegen.make_gaussians(wl.n, wl.half_extent, wl.sh_degree, wl.d, seed=0)
    cams = scenegen.make_cameras(wl.views)
    cam = cams[0]
    vt = scenegen.make_view_tensors(0, cam.npix, wl.d)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    params = [t(g[k]).requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    r = Rasterizer(cams, wl.n, wl.sh_degree, wl.d)
    C, F, T, _ = rasterize(r, *params, t(g["feat"]), wl.sh_degree)
    loss = (C.double() * t(vt["dC"]).double()).sum() + (F.double() * t(vt["dF"]).double()).sum()
    loss.backward()
    grads = {k: p.grad.cpu().numpy().reshape(wl.n, -1) for k, p in zip(S.GRAD_KEYS, params)}

    bq = binspec.bin_quantities(g, cam)
    rows = lambda vi, key, pix: None if key in ("target", "dT") else vt[key][pix]
    # the nearest such Gaussians (most of the far ones are never reached before pixels saturate)
    first = S.pick_front(bq, 12, 5000)
    views = [dict(tiles=np.array(sorted(set().union(*[S._rect_tiles(bq, i) for i in first]))), tile_off=0,
                  pix_off=0)]
    ora = S.run(g, [cam], [bq], first, views, rows, wl.d)
    # no near-threshold decision in any pixel they touch (a step could cross it:
    # no flag and a zero ambiguity bound) and a contribution
    amb_any = sum(np.abs(ora["ambs"][k]).reshape(first.size, -1).sum(1) for k in S.GRAD_KEYS)
    ok = (ora["gflag"] == 0) & (amb_any == 0) & (np.abs(ora["sums"]["opacity"]) > 0)
    subset = first[ok][:64]
    assert subset.size == 64
    depth_axis = np.abs(np.asarray(cam.R, np.float64)[2])
    across = [c for c in range(3) if depth_axis[c] < 1e-6]
    assert across, "no mean component keeps the depth for this camera"
    rng = np.random.default_rng(0)
    worst = 0.0
    tight = total = 0
    lists = {}      # unperturbed tile lists, shared by all differences
    for n_i, gi in enumerate(subset):
        k = int(np.nonzero(first == gi)[0][0])
        for key, comp in (("means", across[n_i % len(across)]), ("scales", int(rng.integers(3))),
                          ("quats", int(rng.integers(4))), ("opacity", 0), ("sh", int(rng.integers(grads["sh"].shape[1])))):
            if (n_i % 4 and key in ("quats", "sh")) or (n_i % 2 and key == "scales"):
                continue       # every Gaussian: means, opacity; every 2nd scales; every 4th quats and SH
            x = float(np.asarray(g[key], np.float64).reshape(wl.n, -1)[gi, comp])
            # small steps where the footprint moves (fewer skip/stop flips), larger where L is linear
            h = (1e-3 if key == "sh" else 1e-5) * max(abs(x), 0.05)
            fd, fd_small, fd_big = (S.central_difference(g, cam, bq, rows, wl.d, int(gi), key, comp, s * h, lists)
                                    for s in (1.0, 0.1, 10.0))
            # the quotient's own error (rounding, curvature, a skip/stop decision crossed by the step)
            spread = max(abs(fd - fd_small), abs(fd - fd_big))
            an = float(grads[key][gi, comp])
            mag = float(ora["mags"][key].reshape(first.size, -1)[k, comp])
            amb = float(ora["ambs"][key].reshape(first.size, -1)[k, comp])
            # the FP32 gradient's bound (1e-5 M, doubled; ambiguous decisions as in the
            # parity tests) plus the quotient's error
            ratio = abs(an - fd) / (2e-5 * mag + U.AMB_FACTOR * amb + 2 * spread + 1e-30)
            worst = max(worst, ratio)
            total += 1
            tight += 2 * spread <= 2e-5 * mag
            if ratio > 1.0:
                print(f"FD mismatch g={gi} {key}[{comp}]: fd={fd:.7g} (h/10: {fd_small:.7g}, 10h: {fd_big:.7g}) "
                      f"autograd={an:.7g} "
                      f"magnitude={mag:.3g}", flush=True)
    print(f"[fd] {total} differences, {tight} decisive; worst ratio {worst:.3f}", flush=True)
    assert worst <= 1.0 and tight >= 0.75 * total


@pytest.mark.parametrize("form,prim", [("f32", "gaussian"), ("bf16", "gaussian"), ("f32", "surfel"), ("bf16", "surfel")])
def test_graph_replay_matches_eager(form, prim):
    """A captured step replayed several times, with eager work and host
    synchronisation between replays, reproduces the eager results bit for bit."""
    from paper_2505_19154_amd.raster import FusionAcc, Rasterizer
    g = scenegen.make_gaussians(3000, 1.5, 3, 32, seed=7, feat_dtype="bf16")
    if prim == "surfel":
        g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    cams = [scenegen.look_at_camera(p, w, h) for p, w, h in (((0, -4, 0), 96, 80), ((3, -2.5, 1.2), 130, 70))]
    vts = U.view_maps(cams, 32, target_dtype="bf16")
    dg = U.device_gaussians(g)
    dC, dF, dT = U.concat(vts, "dC"), U.concat(vts, "dF"), U.concat(vts, "dT")
    target = U.concat(vts, "target_bits")
    r = Rasterizer(cams, dg.n, dg.sh_degree, dg.d, feat_dtype="bf16", form=form, primitive=prim)
    img = r.forward(dg)
    acc_e = FusionAcc.zeros(dg.n, 32, "cuda")
    grads_e = r.render_bwd(dg, img, dC, dF, dT, target=target, acc=acc_e)
    C_e, F_e, T_e = img.C.clone(), img.F.clone(), img.T.clone()
    torch.cuda.synchronize()
    acc = FusionAcc.zeros(dg.n, 32, "cuda")
    graph, grads = r.capture_step(dg, img, dC, dF, dT, target=target, acc=acc)
    for rep in range(3):
        for t_ in (img.C, img.F, img.T, acc.sum, acc.comp, acc.wsum, acc.wcomp):
            t_.zero_()
        for t_ in grads.values():
            t_.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        c = r.counters()
        assert not c.inst_overflow and not c.visit_overflow
        assert torch.equal(img.C, C_e) and torch.equal(img.F, F_e) and torch.equal(img.T, T_e), rep
        for k in grads:
            assert torch.equal(grads[k], grads_e[k]), (rep, k)
        assert torch.equal(acc.sum, acc_e.sum) and torch.equal(acc.wsum, acc_e.wsum), rep
        _ = (dC * 2).sum().item()   # unrelated eager work between replays


def _column_wall_scene(d):
    """32x16 view (two tiles).  In front, four layers of near-opaque Gaussians,
    narrow in x, cover pixel column 0 of every row, which stops within the
    first chunk of 32; behind, 96 faint wide Gaussians keep every other pixel
    walking for several chunks.  A workgroup must not stop while any of its
    pixels walks."""
    rng = np.random.default_rng(11)
    cam = scenegen.Camera(width=32, height=16, fx=50.0, fy=50.0, cx=16.0, cy=8.0,
                          R=np.eye(3, dtype=np.float32), t=np.float32([0.0, 0.0, 4.0]))
    means, scales, opac = [], [], []
    for layer in range(4):
        zc = 2.0 + 0.01 * layer
        for i in range(8):
            u, v = 0.5, 1.0 + 2.0 * i
            means.append([(u - 16.0) * zc / 50.0, (v - 8.0) * zc / 50.0, zc - 4.0])
            scales.append([0.2 * zc / 50.0, 2.0 * zc / 50.0, 0.2 * zc / 50.0])
            opac.append(0.99)
    for i in range(96):
        zc = 4.0 + 0.005 * i
        u, v = rng.uniform(0, 32), rng.uniform(0, 16)
        means.append([(u - 16.0) * zc / 50.0, (v - 8.0) * zc / 50.0, zc - 4.0])
        s = 12.0 * zc / 50.0
        scales.append([s, s, s])
        opac.append(0.06)
    n = len(means)
    g = scenegen.make_gaussians(n, 1.0, 0, d, seed=12, feat_dtype="bf16")
    g["means"] = np.float32(means)
    g["scales"] = np.float32(scales)
    g["quats"] = np.tile(np.float32([1.0, 0.0, 0.0, 0.0]), (n, 1))
    g["opacity"] = np.float32(opac)
    return g, [cam]


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_forward_runs_until_every_pixel_stops(form):
    g, cams = _column_wall_scene(32)
    gpu = U.run_gpu(g, cams, None, form=form)
    ora = U.run_oracle(g, cams)
    v = ora["views"][0]
    niter = v["niter"].reshape(16, 32)
    # the premise: column 0 stops within the first chunk, the other columns walk past several
    assert niter[:, 0].max() <= 32 and niter[:, 2:].min() > 64
    ok = (v["flags"] & 1) == 0
    img = gpu["img"]
    assert np.array_equal(img.n_iter.cpu().numpy().astype(np.int64)[ok], v["niter"][ok])
    assert U.elementwise(img.C.cpu().numpy(), v["C"], v["Cmag"], mask=ok[:, None].repeat(3, 1))[0] <= 1.0
    assert U.elementwise(img.T.cpu().numpy(), v["T"], v["T"], mask=ok)[0] <= 1.0
    assert U.elementwise(img.F.cpu().numpy(), v["F"], v["Fmag"], rtol=U.RTOL_FORM[form],
                         mask=ok[:, None].repeat(32, 1))[0] <= 1.0


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_overflow_leaves_zero_gradients_not_stale_ones(form):
    """A backward whose visits overflow the capacity writes zero gradients and
    leaves the fusion accumulators alone, although the workspace still holds
    the per-(view, Gaussian) adjoints of an earlier, complete backward."""
    from paper_2505_19154_amd.raster import FusionAcc
    g = scenegen.make_gaussians(600, 1.0, 1, 32, seed=21, feat_dtype="bf16")
    cams = scenegen.make_cameras("front64x48")
    few = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    few["means"] = g["means"].copy()
    few["means"][40:] += np.float32([0.0, -9.0, 0.0])     # all but 40 behind the camera
    vts = U.view_maps(cams, 32, target_dtype="bf16")
    dC, dF, dT = U.concat(vts, "dC"), U.concat(vts, "dF"), U.concat(vts, "dT")
    target = U.concat(vts, "target_bits")
    dfew, r = _raster(few, cams, form=form)
    r.forward(dfew)
    c = r.counters()
    r.reserve(int(c.n_instances), int(c.n_visited))      # capacities exactly those of the 40
    img = r.forward(dfew)
    grads = r.render_bwd(dfew, img, dC, dF, dT)
    torch.cuda.synchronize()
    assert any(bool(torch.any(v != 0)) for v in grads.values())
    dg = U.device_gaussians(g)
    r.project(dg)
    r.bin_sort()
    r.render_fwd(dg, img)
    acc = FusionAcc.zeros(dg.n, 32, "cuda")
    grads = {k: torch.full_like(v, float("nan")) for k, v in grads.items()}
    r.render_bwd(dg, img, dC, dF, dT, target=target, acc=acc, grads=grads)
    torch.cuda.synchronize()
    c = r.counters()
    assert c.inst_overflow or c.visit_overflow
    for k, v in grads.items():
        assert torch.all(v == 0), k
    for t_ in (acc.sum, acc.comp, acc.wsum, acc.wcomp):
        assert torch.all(t_ == 0)


def test_backward_after_another_forward_raises():
    """RasterizeFn.backward needs its own forward's binning in the workspace:
    a second forward on the same rasterizer in between is refused."""
    from paper_2505_19154_amd._lib import FhError
    from paper_2505_19154_amd.autograd import rasterize
    g = scenegen.make_gaussians(300, 1.0, 0, 8, seed=22)
    cams = scenegen.make_cameras("front64x48")
    dg, r = _raster(g, cams)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    p1 = [t(g[k]).requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    p2 = [t(g[k]).requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    C1, _, _, _ = rasterize(r, *p1, t(g["feat"]), 0)
    C2, _, _, _ = rasterize(r, *p2, t(g["feat"]), 0)
    with pytest.raises(FhError):
        C1.sum().backward()
    C2.sum().backward()          # the latest forward still backpropagates
    assert p2[3].grad is not None and torch.isfinite(p2[3].grad).all()


def test_binding_rejects_misshapen_tensors_before_launch():
    from paper_2505_19154_amd._lib import FhError
    g = scenegen.make_gaussians(300, 1.0, 0, 8, seed=23)
    cams = scenegen.make_cameras("front64x48")
    dg, r = _raster(g, cams)
    img = r.forward(dg)
    P = r.n_pixels
    dC = torch.zeros(P, 3, device="cuda")
    with pytest.raises(FhError):
        r.render_bwd(dg, img, torch.zeros(P - 1, 3, device="cuda"))
    with pytest.raises(FhError):
        r.render_bwd(dg, img, dC, dF=torch.zeros(8, P, device="cuda").t())      # not contiguous
    from paper_2505_19154_amd.raster import FusionAcc
    acc = FusionAcc.zeros(dg.n, 8, "cuda")
    with pytest.raises(FhError):
        r.render_bwd(dg, img, dC, target=torch.zeros(P, 8, dtype=torch.float16, device="cuda"), acc=acc)
    with pytest.raises(FhError):
        r.render_bwd(dg, img, dC, target=torch.zeros(P, 8, device="cuda"), acc=FusionAcc.zeros(dg.n - 1, 8, "cuda"))
    with pytest.raises(FhError):
        r.fuse_features(dg, img, torch.zeros(P, 8, dtype=torch.float64, device="cuda"), acc)


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_autograd_function_with_surfels(form):
    """RasterizeFn with a surfel rasterizer: autograd gradients of
    L = sum dC . C + dF . F + dT . T equal the oracle's surfel adjoint (Section
    3.1) under the parity rule, and C, T the oracle's images."""
    from paper_2505_19154_amd.autograd import rasterize
    from paper_2505_19154_amd.raster import Rasterizer
    d = 64 if form == "bf16" else 16
    g = scenegen.make_gaussians(700, 1.0, 1, d, seed=23, feat_dtype="bf16")
    g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    cams = scenegen.make_cameras("front64x48")
    vts = U.view_maps(cams, d, with_dT=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    params = [t(g[k]).requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    feat = U.device_gaussians(g).feat
    r = Rasterizer(cams, len(g["opacity"]), 1, d, feat_dtype="bf16", form=form, primitive="surfel")
    C, F, T, _ = rasterize(r, *params, feat, 1)
    loss = ((C.double() * t(vts[0]["dC"]).double()).sum() + (F.double() * t(vts[0]["dF"]).double()).sum()
            + (T.double() * t(vts[0]["dT"]).double()).sum())
    loss.backward()
    ora = U.run_oracle(g, cams, vts, bin_rule="surfel")
    v = ora["views"][0]
    ok = (v["flags"] & 1) == 0
    assert U.elementwise(C.detach().cpu().numpy(), v["C"], v["Cmag"], mask=ok[:, None].repeat(3, 1),
                         amb=v["Cden"])[0] <= 1.0
    assert U.elementwise(T.detach().cpu().numpy(), v["T"], v["T"], mask=ok, amb=v["Tden"])[0] <= 1.0
    keep = U.checkable(ora["gflags"])
    rt = U.RTOL_FORM[form]
    for k, p in zip(("means", "scales", "quats", "opacity", "sh"), params):
        got = p.grad.cpu().numpy()
        m = keep.reshape((-1,) + (1,) * (got.ndim - 1)) & np.ones(got.shape, bool)
        assert U.elementwise(got, ora["grads"][k], ora["grads_mag"][k], rtol=rt, mask=m,
                             amb=ora["grads_amb"][k])[0] <= 1.0, k
    # the third scale takes no part in a surfel
    assert torch.all(params[1].grad[:, 2] == 0)


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_autograd_feature_gradient_is_the_fusion_of_dF(form):
    """With feat.requires_grad, RasterizeFn returns dL/df_i = sum_p w_i(p) dF(p)
    (the unnormalised fusion of dF; the paper's features are frozen, so this is
    asked for explicitly), against the oracle's fusion sums of the map dF."""
    from paper_2505_19154_amd.autograd import rasterize
    from paper_2505_19154_amd.raster import Rasterizer
    d = 32
    fdt = "bf16" if form == "bf16" else "f32"
    g = scenegen.make_gaussians(900, 1.2, 1, d, seed=24, feat_dtype=fdt)
    cams = scenegen.make_cameras("front64x48")
    vt = scenegen.make_view_tensors(0, cams[0].npix, d, with_dT=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    params = [t(g[k]).requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    feat = U.device_gaussians(g).feat.clone().requires_grad_(True)
    r = Rasterizer(cams, len(g["opacity"]), 1, d, feat_dtype=fdt, form=form)
    C, F, T, _ = rasterize(r, *params, feat, 1)
    loss = (F.double() * t(vt["dF"]).double()).sum() + (C.double() * t(vt["dC"]).double()).sum()
    loss.backward()
    got = feat.grad.float().cpu().numpy()
    # the oracle: fusion of the target map dF, unnormalised
    ora = pipeline.run(g, cams, [dict(vt, target=vt["dF"])], fusion=True)
    keep = U.checkable(ora["gflags"])
    m = keep[:, None] & np.ones(got.shape, bool)
    if form == "f32":
        assert U.elementwise(got, ora["fsum"], ora["fsum_mag"], rtol=U.RTOL_FORM[form], mask=m,
                             amb=ora["fsum_amb"])[0] <= 1.0
    else:
        # returned in the features' BF16: within half a BF16 unit of the magnitude, plus the form's rule
        assert U.elementwise(got, ora["fsum"], ora["fsum_mag"], rtol=2.0 ** -8 + U.RTOL_FORM[form], mask=m,
                             amb=ora["fsum_amb"])[0] <= 1.0
    assert np.abs(got).max() > 0


def test_get_status_matches_read_counters_without_a_sync():
    """fh_get_status copies the counters on the stream (device destination,
    no host synchronisation) and agrees with fh_read_counters."""
    g = scenegen.make_gaussians(500, 1.0, 0, 8, seed=25)
    cams = scenegen.make_cameras("front64x48")
    dg, r = _raster(g, cams)
    img = r.forward(dg)
    out = torch.full((4,), -1, dtype=torch.int64, device="cuda")
    r.status_async(out)
    c = r.counters()      # (synchronises)
    got = out.cpu().numpy()
    flags = got[3:4].view(np.int32)
    assert got[0] == c.n_instances and got[1] == c.n_visited and got[2] == c.n_culled_nonfinite
    assert flags[0] == c.inst_overflow and flags[1] == c.visit_overflow
    assert c.n_instances > 0 and c.n_visited > 0
