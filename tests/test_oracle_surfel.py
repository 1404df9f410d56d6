"""Pins of the oracle's surfel primitive (Section 3.1; oracle/surfel.py, the
surfel rule of oracle/binspec.py and the surfel branch of oracle/raster.c)
against what the geometry fixes: the ray-plane intersection solved in world
space, a fronto-parallel surfel's closed form, the untiled per-pixel
definition (torch float64) for the images, its autograd for the adjoint,
central differences, and brute-force coverage of the tile rects."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import binspec, brute, consts, pipeline, surfel


def _scene(seed, n=80, d=5, recipe="front48x40", deg=1, half=1.0):
    g = scenegen.make_gaussians(n, half, deg, d, seed=seed)
    # surfels a little larger than the default splats, so that most cover several pixels
    g["scales"] = (np.asarray(g["scales"]) * 2.0).astype(np.float32)
    cams = scenegen.make_cameras(recipe)
    return g, cams


def _world_uv(g, cam, i, x, y):
    """(u, v) of pixel centres (x, y) on surfel i by a 3x3 solve in world space."""
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    c = -R.T @ t
    q = np.asarray(g["quats"][i], np.float64)
    from oracle.project import quat_to_rot
    Rq = quat_to_rot((q / np.linalg.norm(q))[None])[0]
    s = np.asarray(g["scales"][i], np.float64)
    p = np.asarray(g["means"][i], np.float64)
    out = []
    for xx, yy in zip(x, y):
        d = R.T @ np.array([(xx - cam.cx) / cam.fx, (yy - cam.cy) / cam.fy, 1.0])
        A = np.stack([s[0] * Rq[:, 0], s[1] * Rq[:, 1], -d], 1)
        uvt = np.linalg.solve(A, c - p)
        out.append(uvt[:2])
    return np.array(out)


def test_plane_coords_match_a_world_space_solve():
    g, cams = _scene(3, n=30)
    cam = cams[0]
    pr = surfel.project_surfel(g, cam)
    rng = np.random.default_rng(0)
    for i in range(30):
        x = rng.uniform(0, cam.width, 7)
        y = rng.uniform(0, cam.height, 7)
        u, v, k2 = surfel.plane_coords(pr["srf"][i][None].repeat(7, 0), x, y)
        ref = _world_uv(g, cam, i, x, y)
        assert np.all(k2 != 0)
        scale = np.maximum(1.0, np.abs(ref))
        assert np.all(np.abs(u - ref[:, 0]) <= 1e-9 * scale[:, 0]), i
        assert np.all(np.abs(v - ref[:, 1]) <= 1e-9 * scale[:, 1]), i


def test_fronto_parallel_surfel_closed_form():
    # camera at the origin looking down +z, surfel in the plane z = 4 with its
    # tangents along x and y: u = (x - x_c) z / (fx s_u), v = (y - y_c) z / (fy s_v)
    cam = scenegen.Camera(64, 48, 60.0, 55.0, 32.0, 24.0, np.eye(3, dtype=np.float32),
                          np.zeros(3, np.float32))
    g = dict(means=np.array([[0.3, -0.2, 4.0]], np.float32), scales=np.array([[0.15, 0.25, 0.01]], np.float32),
             quats=np.array([[1.0, 0.0, 0.0, 0.0]], np.float32), opacity=np.array([0.8], np.float32),
             sh=np.zeros((1, 1, 3), np.float32), sh_degree=0, feat=None, d=0)
    pr = surfel.project_surfel(g, cam)
    m = g["means"][0].astype(np.float64)        # (the float32 values)
    xc, yc = 60.0 * m[0] / m[2] + 32.0, 55.0 * m[1] / m[2] + 24.0
    assert np.allclose(pr["srf"][0, :2], [xc, yc], rtol=1e-12, atol=1e-12)
    ys, xs = np.mgrid[0:48, 0:64] + 0.5
    u, v, _ = surfel.plane_coords(pr["srf"][0], xs, ys)
    su, sv = float(np.float32(0.15)), float(np.float32(0.25))
    assert np.allclose(u, (xs - xc) * m[2] / (60.0 * su), rtol=1e-12, atol=1e-12)
    assert np.allclose(v, (ys - yc) * m[2] / (55.0 * sv), rtol=1e-12, atol=1e-12)
    # the tiled oracle composites alpha = min(0.99, o exp(-(u^2 + v^2)/2)) of that one surfel
    o = pipeline.run(g, [cam], bin_rule="surfel")
    a = np.minimum(consts.ALPHA_MAX, float(np.float32(0.8)) * np.exp(-0.5 * (u * u + v * v))).reshape(-1)
    a = np.where(a >= consts.ALPHA_MIN, a, 0.0)
    assert np.allclose(o["views"][0]["T"], 1.0 - a, rtol=0, atol=1e-14)


def test_rect_holds_every_pixel_where_alpha_reaches_the_threshold():
    g, cams = _scene(5, n=120, half=1.5)
    cam = cams[0]
    bq = binspec.bin_quantities(g, cam, "surfel")
    pr = surfel.project_surfel(g, cam)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width] + 0.5
    checked = 0
    for i in np.nonzero(bq["visible"])[0]:
        u, v, k2 = surfel.plane_coords(pr["srf"][i], xs, ys)
        with np.errstate(all="ignore"):
            a = float(g["opacity"][i]) * np.exp(-0.5 * (u * u + v * v))
        hit = (k2 != 0) & (a >= consts.ALPHA_MIN)
        if not hit.any():
            continue
        ty, tx = np.nonzero(hit)
        tx, ty = tx // consts.TILE, ty // consts.TILE
        assert bq["binned"][i]
        assert tx.min() >= bq["x0"][i] and tx.max() <= bq["x1"][i], i
        assert ty.min() >= bq["y0"][i] and ty.max() <= bq["y1"][i], i
        checked += 1
    assert checked > 40
    # culled: opacity at most 1/255, or behind the near plane
    assert not np.any(bq["binned"] & (np.asarray(g["opacity"]) * 255.0 <= 1.0))


@pytest.mark.parametrize("seed", [1, 2])
def test_tiled_surfel_oracle_equals_the_untiled_definition(seed):
    g, cams = _scene(seed)
    o = pipeline.run(g, cams, bin_rule="surfel")
    L = brute.leaves(g)
    C, F, T, _, _ = brute.render_surfel(L, g, cams[0], g["feat"])
    v = o["views"][0]
    assert np.abs(v["T"] - T.detach().numpy()).max() < 1e-12
    assert np.abs(v["C"] - C.detach().numpy()).max() < 1e-12
    assert np.abs(v["F"] - F.detach().numpy()).max() < 1e-12
    assert (v["T"] < 0.999).sum() > 200


def test_surfel_adjoint_matches_torch_autograd():
    for seed in (1, 2, 3):
        g, cams = _scene(seed)
        vt = [scenegen.make_view_tensors(0, cams[0].npix, g["d"], with_dT=True)]
        o = pipeline.run(g, cams, vt, bin_rule="surfel")
        L = brute.leaves(g)
        C, F, T, _, _ = brute.render_surfel(L, g, cams[0], g["feat"])
        loss = ((torch.tensor(vt[0]["dC"], dtype=torch.float64) * C).sum()
                + (torch.tensor(vt[0]["dF"], dtype=torch.float64) * F).sum()
                + (torch.tensor(vt[0]["dT"], dtype=torch.float64) * T).sum())
        loss.backward()
        for k in ("means", "scales", "quats", "opacity", "sh"):
            ref = L[k].grad.numpy()
            got = o["grads"][k]
            mag = o["grads_mag"][k]
            assert np.all(np.abs(got - ref) <= 1e-10 * mag + 1e-12), k
            assert np.all(mag >= np.abs(got) * (1 - 1e-12))
        # the third scale takes no part in a surfel
        assert np.all(o["grads"]["scales"][:, 2] == 0)
        assert np.abs(o["grads"]["means"]).max() > 0


def test_surfel_adjoint_matches_central_differences():
    g, cams = _scene(11, n=50)
    vt = [scenegen.make_view_tensors(0, cams[0].npix, g["d"], with_dT=True)]
    o = pipeline.run(g, cams, vt, bin_rule="surfel")

    def loss(gg):
        v = pipeline.run(gg, cams, bin_rule="surfel")["views"][0]
        return float((vt[0]["dC"] * v["C"]).sum() + (vt[0]["dF"] * v["F"]).sum() + (vt[0]["dT"] * v["T"]).sum())

    ok = np.nonzero((o["gflags"] == 0) & (np.abs(o["grads"]["opacity"]) > 1e-6))[0][:5]
    assert ok.size >= 3
    g64 = {k: (np.asarray(v, np.float64) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    for key, comps in (("means", 3), ("scales", 2), ("quats", 4), ("opacity", 1)):
        for i in ok:
            for c in range(comps):
                h = 1e-7 * max(1.0, abs(float(np.asarray(g64[key])[i].reshape(-1)[c])))
                gp = dict(g64); gp[key] = g64[key].copy()
                gm = dict(g64); gm[key] = g64[key].copy()
                if comps == 1:
                    gp[key][i] += h; gm[key][i] -= h
                else:
                    gp[key][i, c] += h; gm[key][i, c] -= h
                fd = (loss(gp) - loss(gm)) / (2 * h)
                an = o["grads"][key][i] if comps == 1 else o["grads"][key][i, c]
                mag = o["grads_mag"][key][i] if comps == 1 else o["grads_mag"][key][i, c]
                assert abs(fd - an) <= 1e-5 * mag + 1e-7, (key, i, c, fd, an)


def test_surfel_fusion_of_a_constant_map_returns_the_constant():
    g, cams = _scene(7)
    d = g["d"]
    const = np.linspace(-1.0, 2.0, d)
    vt = [dict(scenegen.make_view_tensors(0, cams[0].npix, d), target=np.tile(const, (cams[0].npix, 1)))]
    o = pipeline.run(g, cams, vt, fusion=True, bin_rule="surfel")
    hit = o["wsum"] > 1e-6
    assert hit.sum() > 20
    fin = pipeline.finalize_fusion(o["fsum"], o["wsum"], g["feat"])
    assert np.allclose(fin[hit], const[None, :], rtol=1e-12, atol=1e-12)


# --- the ambiguity bound with surfel records (the flips of tests/test_oracle_ambiguity.py) ---

def _surfel_proj(seed, n=14, w=32, h=16):
    """Surfel records with footprints of 2-7 px, random orientation and a
    mild perspective (|c| <= 0.02), plus opacity and colour."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0, np.pi, n)
    s1, s2 = rng.uniform(2, 7, n), rng.uniform(2, 7, n)
    ct, st = np.cos(th), np.sin(th)
    a0, a1, b0, b1 = ct * s1, -st * s2, st * s1, ct * s2
    c0, c1 = rng.uniform(-0.02, 0.02, n), rng.uniform(-0.02, 0.02, n)
    srf = np.stack([rng.uniform(0, w, n), rng.uniform(0, h, n), a0, a1, b0, b1,
                    a0 * b1 - a1 * b0, a0 * c1 - a1 * c0, c0 * b1 - c1 * b0], 1)
    return dict(srf=srf, opacity=rng.uniform(0.15, 0.6, n), rgb=rng.uniform(0, 1, (n, 3)))


@pytest.mark.parametrize("kind,m,seed", [(k, m, s) for k in ("skip", "stop", "clamp") for m in (0, 5, 11)
                                         for s in range(3) if not (k == "stop" and m == 0)])
def test_surfel_flipped_decision_stays_within_the_bound(kind, m, seed):
    from tests import gpu_util as U
    from tests.test_oracle_ambiguity import DELTA, KEYS, _max_ratio, _render, _scene as _escene
    proj = _surfel_proj(seed)
    _, feat, maps = _escene(seed)
    rng = np.random.default_rng(2000 + seed)
    px, py = int(rng.integers(2, 30)), int(rng.integers(2, 14))
    x, y = px + 0.5, py + 0.5
    if kind == "stop":
        # equal front layers centred on the pixel leave T = 0.004 there
        proj["srf"][:m, 0], proj["srf"][:m, 1] = x, y
        proj["opacity"][:m] = 1.0 - 0.004 ** (1.0 / m)

    def alpha_at(p, j):
        u, v, k2 = surfel.plane_coords(p["srf"][j], np.array(x), np.array(y))
        return min(consts.ALPHA_MAX, p["opacity"][j] * float(np.exp(-0.5 * (u * u + v * v)))) if k2 != 0 else 0.0

    def decider(sign):
        p = {k: v.copy() for k, v in proj.items()}
        p["srf"][m, 0], p["srf"][m, 1] = x, y        # alpha there is the opacity exactly
        f = 1.0 + sign * DELTA
        if kind == "skip":
            p["opacity"][m] = consts.ALPHA_MIN * f
        elif kind == "clamp":
            p["opacity"][m] = consts.ALPHA_MAX * f
        else:
            T = 1.0
            for j in range(m):
                a = alpha_at(p, j)
                if a >= consts.ALPHA_MIN:
                    T *= 1 - a
            p["opacity"][m] = 1.0 - consts.T_MIN * f / T
        return p

    hi = _render(decider(+1), feat, maps)
    lo = _render(decider(-1), feat, maps)
    pix = py * 32 + px
    assert (hi["flags"][pix] != 0) and (lo["flags"][pix] != 0)
    assert max(float(np.abs(hi[k] - lo[k]).max()) for k in KEYS) > 1e-9
    r = _max_ratio(hi, lo, U.AMB_FACTOR)
    for key in KEYS:
        assert r[key] <= 1.0, (key, r)


# --- the density-rounding allowance (the surfel branch of oracle/raster.c) ---

def _composite_f32_density(g, cam, vt, ndfd=None):
    """The untiled composite with every surfel density evaluated from the
    record rounded to float32 and the intersection in float32 (the rest in
    torch float64, opacity a leaf): C, T and dL/dopacity for the loss
    dC . C + dF . F + dT . T, or with ndfd = (lam, k) the NDFD losses by
    their double-sum definition and dL/dopacity of sum a L_gt + b L_cf."""
    pr = surfel.project_surfel(g, cam)
    bq = binspec.bin_quantities(g, cam, "surfel")
    vis = np.nonzero(bq["visible"])[0]
    order = vis[np.lexsort((vis, bq["depth"][vis]))]
    W, H = int(cam.width), int(cam.height)
    ys, xs = np.mgrid[0:H, 0:W]
    x = xs.reshape(-1) + 0.5
    y = ys.reshape(-1) + 0.5
    op = torch.tensor(np.asarray(g["opacity"], np.float64), requires_grad=True)
    rgb = torch.tensor(pr["rgb"])
    feat = torch.tensor(np.asarray(g["feat"], np.float64))
    P = W * H
    T = torch.ones(P, dtype=torch.float64)
    C = torch.zeros(P, 3, dtype=torch.float64)
    F = torch.zeros(P, feat.shape[1], dtype=torch.float64)
    done = torch.zeros(P, dtype=torch.bool)
    ws = []
    for gi in order.tolist():
        r = pr["srf"][gi].astype(np.float32)
        dx = (x - pr["srf"][gi][0]).astype(np.float32)
        dy = (y - pr["srf"][gi][1]).astype(np.float32)
        k0 = dx * r[5] - dy * r[3]
        k1 = dy * r[2] - dx * r[4]
        k2 = r[6] - dy * r[7] - dx * r[8]
        with np.errstate(all="ignore"):
            u = np.where(k2 != 0, k0 / k2, np.float32(0))
            v = np.where(k2 != 0, k1 / k2, np.float32(0))
            G32 = np.where(k2 != 0, np.exp(np.float32(-0.5) * (u * u + v * v)), np.float32(0))
        G = torch.tensor(G32.astype(np.float64))
        alpha = torch.clamp(op[gi] * G, max=consts.ALPHA_MAX)
        ok = (alpha.detach() >= consts.ALPHA_MIN) & ~done
        Tn = T * (1.0 - alpha)
        stop = ok & (Tn.detach() < consts.T_MIN)
        done = done | stop
        c = ok & ~stop
        w = torch.where(c, alpha * T, torch.zeros_like(T))
        ws.append(w)
        C = C + w[:, None] * rgb[gi][None]
        F = F + w[:, None] * feat[gi][None]
        T = torch.where(c, Tn, T)
    if ndfd is None:
        loss = ((torch.tensor(vt["dC"]) * C).sum() + (torch.tensor(vt["dF"]) * F).sum()
                + (torch.tensor(vt["dT"]) * T).sum())
        loss.backward()
        return C.detach().numpy(), T.detach().numpy(), op.grad.numpy()
    lam, k = ndfd
    Wm = torch.stack(ws, 0)
    fh = torch.tensor(brute.unit_rows(np.asarray(g["feat"], np.float64)[order]))
    gh = torch.tensor(brute.unit_rows(vt["gt"]))
    sig = 1.0 / (1.0 + torch.exp(k * (fh @ gh.T - lam)))
    Lgt = (Wm * sig).sum(0)
    Lcf = (sig * Wm * (torch.tril(1.0 - fh @ fh.T, diagonal=-1) @ Wm)).sum(0)
    loss = (torch.tensor(vt["ndfd_a"]) * Lgt).sum() + (torch.tensor(vt["ndfd_b"]) * Lcf).sum()
    loss.backward()
    return Lgt.detach().numpy(), Lcf.detach().numpy(), op.grad.numpy()


@pytest.mark.parametrize("n,deg,d,seed", [(1500, 1, 5, 2), (2000, 2, 16, 0)])
def test_density_allowance_covers_a_float32_density(n, deg, d, seed):
    """Rounding the surfel records to float32 and intersecting in float32
    changes T, C and the opacity gradient by no more than the oracle's
    density-rounding allowance (Cden, Tden, grads_amb) on every pixel and
    surfel that no near-threshold decision touches; the scene holds surfels
    seen close to edge-on, where that change exceeds the plain relative
    tolerance of 1e-5 by far."""
    g = scenegen.make_gaussians(n, 1.5, deg, d, seed=seed)
    g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    cams = scenegen.make_cameras("front120x90")
    cam = cams[0]
    vt = scenegen.make_view_tensors(0, cam.npix, g["d"], with_dT=True)
    o = pipeline.run(g, cams, [vt], bin_rule="surfel")
    v = o["views"][0]
    C32, T32, gop32 = _composite_f32_density(g, cam, vt)
    px = (v["flags"] & 1) == 0
    assert px.mean() > 0.99
    assert np.all(np.abs(T32 - v["T"])[px] <= 1.05 * v["Tden"][px] + 1e-13)
    assert np.all((np.abs(C32 - v["C"]) <= 1.05 * v["Cden"] + 1e-13)[px])
    keep = o["gflags"] == 0
    d = np.abs(gop32 - o["grads"]["opacity"])
    assert np.all((d <= 1.05 * o["grads_amb"]["opacity"] + 1e-10 * o["grads_mag"]["opacity"])[keep])
    # the allowance is needed: the plain tolerance fails somewhere, and it is
    # not vacuous: the typical opacity gradient keeps a tight bound
    assert np.any((d > 1e-5 * o["grads_mag"]["opacity"])[keep])
    ref = np.abs(o["grads"]["opacity"])
    hit = keep & (ref > 0)
    assert np.median((o["grads_amb"]["opacity"] + 1e-5 * o["grads_mag"]["opacity"])[hit] / ref[hit]) < 1e-2


# --- the NDFD branch with surfels (Section 3.3 along the surfel walk) ---

def test_surfel_ndfd_losses_and_gradient_equal_the_definition():
    """L_gt and L_cf of the surfel walk (the oracle's forward-indexed O(N)
    form) equal the double-sum definition over the untiled surfel composite,
    and their gradient through w equals torch autograd of that definition."""
    lam, k = 0.5, 20.0
    for seed in (4, 6):
        g, cams = _scene(seed, n=90, d=8)
        cam = cams[0]
        P = cam.npix
        rng = np.random.default_rng(700 + seed)
        F = pipeline.run(g, cams, bin_rule="surfel")["views"][0]["F"]
        gt = F + 0.3 * rng.normal(size=F.shape) * np.abs(F).mean()
        vt = dict(dC=np.zeros((P, 3)), dF=np.zeros((P, g["d"])), dT=np.zeros(P), gt=gt,
                  ndfd_a=rng.normal(size=P), ndfd_b=rng.normal(size=P))
        o = pipeline.run(g, cams, [vt], ndfd=dict(lam=lam, k=k), bin_rule="surfel")
        v = o["views"][0]
        L = brute.leaves(g)
        Lgt, Lcf = brute.ndfd_losses(L, g, cam, g["feat"], gt, lam, k, surfels=True)
        assert np.allclose(v["Lgt"], Lgt.detach().numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(v["Lcf"], Lcf.detach().numpy(), rtol=1e-11, atol=1e-13)
        assert v["Lgt"].max() > 0 and np.abs(v["Lcf"]).max() > 0
        loss = (torch.tensor(vt["ndfd_a"]) * Lgt).sum() + (torch.tensor(vt["ndfd_b"]) * Lcf).sum()
        loss.backward()
        for key in ("means", "scales", "quats", "opacity"):
            ref = L[key].grad.numpy()
            got, mag = o["grads"][key], o["grads_mag"][key]
            assert np.all(np.abs(got - ref) <= 1e-10 * mag + 1e-13), key
        assert np.abs(o["grads"]["means"]).max() > 0
        assert np.all(o["grads"]["sh"] == 0)      # colour does not enter NDFD


def test_density_allowance_covers_the_ndfd_losses_and_gradient():
    """With the density evaluated in float32, the NDFD losses and the opacity
    gradient of sum a L_gt + b L_cf stay within the oracle's density
    allowance (Lgt_den, Lcf_den, grads_amb) wherever no near-threshold
    decision is involved."""
    lam, k = 0.5, 20.0
    g = scenegen.make_gaussians(1500, 1.5, 1, 5, seed=2)
    g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    cams = scenegen.make_cameras("front120x90")
    cam = cams[0]
    P = cam.npix
    rng = np.random.default_rng(31)
    F = pipeline.run(g, cams, bin_rule="surfel")["views"][0]["F"]
    gt = F + 0.3 * rng.normal(size=F.shape) * np.abs(F).mean()
    vt = dict(dC=np.zeros((P, 3)), dF=np.zeros((P, g["d"])), dT=np.zeros(P), gt=gt,
              ndfd_a=rng.normal(size=P), ndfd_b=rng.normal(size=P))
    o = pipeline.run(g, cams, [vt], ndfd=dict(lam=lam, k=k), bin_rule="surfel")
    v = o["views"][0]
    Lgt32, Lcf32, gop32 = _composite_f32_density(g, cam, vt, ndfd=(lam, k))
    px = (v["flags"] & 1) == 0
    assert np.all((np.abs(Lgt32 - v["Lgt"]) <= 1.05 * v["Lgt_den"] + 1e-13)[px])
    assert np.all((np.abs(Lcf32 - v["Lcf"]) <= 1.05 * v["Lcf_den"] + 1e-13)[px])
    keep = o["gflags"] == 0
    dd = np.abs(gop32 - o["grads"]["opacity"])
    assert np.all((dd <= 1.05 * o["grads_amb"]["opacity"] + 1e-10 * o["grads_mag"]["opacity"])[keep])
    # the allowance is needed: the plain relative tolerance fails for the gradient somewhere
    assert np.any((dd > 1e-5 * o["grads_mag"]["opacity"])[keep])
