"""GPU parity of the NDFD feature branch (Section 3.3, Appendix A.1-A.2)
against the oracle: the per-pixel losses L_gt and L_cf (fh_ndfd_losses and the
same sweep inside fh_render_bwd), and the gradient of sum_p (a L_gt + b L_cf)
through the blend weights, alone and joined with the colour and feature
adjoint.  Scenes: BF16 features at every supported width, the ground-truth
map the oracle's rendered features plus noise (so that sigma spreads over
(0, 1)), rounded to BF16 and fed to both sides; seeds whose walks hold no
near-threshold decision (the oracle's ambiguity bound does not cover the NDFD
terms), which the test asserts.  The surfel scenes (Section 3.1's primitive,
the configuration the paper trains) add the oracle's density-rounding
allowance of the losses and the gradient."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import pipeline
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

LAM, K = 0.5, 20.0
# the NDFD walk contracts on MFMA with two-term BF16 splits of its FP32
# operands (weights, the running vectors): the BF16 form's bound
RT = U.RTOL_FORM["bf16"]

SCENES = {
    # name: (n, half extent, d, seed, [(camera position, width, height)][, primitive])
    "d32": (900, 1.5, 32, 13, [((0, -4, 0), 72, 56)]),
    "d64_two_views": (1200, 1.2, 64, 17, [((0, -4, 0), 64, 48), ((3, -2.5, 1.2), 50, 40)]),
    "d96": (1000, 1.5, 96, 5, [((0, -4, 0), 56, 40)]),
    "d128": (900, 1.5, 128, 12, [((0, -4, 0), 60, 44)]),
    "d256": (800, 1.5, 256, 7, [((0, -4, 0), 48, 40)]),
    # surfels (scales x3 so that most span pixels)
    "surfel_d64": (700, 1.5, 64, 2, [((0, -4, 0), 56, 44)], "surfel"),
    "surfel_d256": (600, 1.5, 256, 1, [((0, -4, 0), 48, 40)], "surfel"),
    "surfel_d32_two_views": (700, 1.5, 32, 7, [((0, -4, 0), 64, 48), ((3, -2.5, 1.2), 50, 40)], "surfel"),
    # zero vectors, whose unit vector is taken as zero: the features of every
    # seventh Gaussian and F_gt of every fifth pixel
    "d64_zero_vectors": (1200, 1.2, 64, 17, [((0, -4, 0), 64, 48)], "gaussian", "zeros"),
}


def _prim(name):
    return SCENES[name][5] if len(SCENES[name]) > 5 else "gaussian"


def _scene(name, with_colour=False):
    n, h, d, seed, camspec = SCENES[name][:5]
    g = scenegen.make_gaussians(n, h, 1, d, seed=seed, feat_dtype="bf16")
    if _prim(name) == "surfel":
        g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    g["primitive"] = _prim(name)
    zeros = SCENES[name][6:] == ("zeros",)
    if zeros:
        g["feat_bits"] = np.asarray(g["feat_bits"]).copy()
        g["feat_bits"][::7] = 0
        g["feat"] = scenegen.bf16_bits_to_f32(g["feat_bits"]).astype(np.asarray(g["feat"]).dtype)
    cams = [scenegen.look_at_camera(p, w, hh) for p, w, hh in camspec]
    F = pipeline.run(g, cams, bin_rule=_rule(g))["views"]
    rng = np.random.default_rng(700 + seed)
    vts = []
    for vi, c in enumerate(cams):
        Fv = F[vi]["F"]
        gt = Fv + 0.5 * rng.normal(size=Fv.shape) * (np.abs(Fv).mean() + 1e-3)
        gtb = scenegen.to_bf16_bits(gt.astype(np.float32))
        if zeros:
            gtb[::5] = 0
        P = c.npix
        vt = dict(dC=np.zeros((P, 3)), dF=np.zeros((P, d)), dT=np.zeros(P),
                  gt=scenegen.bf16_bits_to_f32(gtb).astype(np.float64), gt_bits=gtb,
                  ndfd_a=rng.normal(size=P), ndfd_b=rng.normal(size=P))
        if with_colour:
            vt["dC"] = rng.normal(size=(P, 3))
            vt["dF"] = rng.normal(size=(P, d)).astype(np.float32).astype(np.float64)
        vts.append(vt)
    return g, cams, vts


def _rule(g):
    return "surfel" if g.get("primitive") == "surfel" else "box"


def _gpu(g, cams, vts, form):
    from paper_2505_19154_amd.raster import Rasterizer
    dg = U.device_gaussians(g)
    r = Rasterizer(cams, dg.n, 1, g["d"], feat_dtype="bf16", form=form, ndfd=True,
                   primitive=g.get("primitive", "gaussian"))
    img = r.forward(dg)
    cat = lambda k: torch.from_numpy(np.ascontiguousarray(np.concatenate([v[k] for v in vts]), np.float32)).cuda()
    gt = torch.from_numpy(np.concatenate([v["gt_bits"] for v in vts]).view(np.int16)).cuda().view(torch.bfloat16)
    Lgt0, Lcf0 = r.ndfd_losses(dg, img, gt, LAM, K)
    P = r.n_pixels
    Lgt = torch.empty(P, dtype=torch.float32, device="cuda")
    Lcf = torch.empty(P, dtype=torch.float32, device="cuda")
    grads = r.render_bwd(dg, img, cat("dC"), cat("dF"), cat("dT"),
                         ndfd=dict(gt=gt, a=cat("ndfd_a"), b=cat("ndfd_b"), lam=LAM, k=K, Lgt=Lgt, Lcf=Lcf))
    torch.cuda.synchronize()
    return dict(Lgt0=Lgt0.cpu().numpy(), Lcf0=Lcf0.cpu().numpy(), Lgt=Lgt.cpu().numpy(), Lcf=Lcf.cpu().numpy(),
                grads={k: v.cpu().numpy() for k, v in grads.items()})


def _check(name, g, cams, vts, gpu):
    ora = pipeline.run(g, cams, vts, ndfd=dict(lam=LAM, k=K), bin_rule=_rule(g))
    # precondition: no near-threshold decision anywhere (see the module docstring)
    assert all(int((v["flags"] != 0).sum()) == 0 for v in ora["views"]) and int((ora["gflags"] != 0).sum()) == 0
    ref = lambda k: np.concatenate([v[k] for v in ora["views"]])
    # the losses: elementwise against their companions, normwise
    for nm in ("Lgt", "Lcf"):
        r_, m_, den = ref(nm), ref(nm + "_mag"), ref(nm + "_den")
        for got in (gpu[nm + "0"], gpu[nm]):
            ratio = U.elementwise(got, r_, m_, rtol=RT, amb=den)[0]
            nw = U.normwise(got, r_)
            print(f"[ndfd {name}] {nm} ratio {ratio:.3f} norm {nw:.2e}", flush=True)
            assert ratio <= 1.0 and nw <= RT, nm
    # the standalone losses and the backward's sweep are the same walk
    assert np.array_equal(gpu["Lgt0"], gpu["Lgt"]) and np.array_equal(gpu["Lcf0"], gpu["Lcf"])
    assert ref("Lgt").max() > 0 and np.std(ref("Lgt") / np.maximum(ref("WN"), 1e-12)) > 0.05
    for k in ("means", "scales", "quats", "opacity", "sh"):
        got, r_, m_ = gpu["grads"][k], ora["grads"][k], ora["grads_mag"][k]
        # (no near-threshold decision: the bound holds only the surfel density allowance)
        ratio = U.elementwise(got, r_, m_, rtol=RT, amb=ora["grads_amb"][k])[0]
        nw = U.normwise(got, r_)
        print(f"[ndfd {name}] grad {k} ratio {ratio:.3f} norm {nw:.2e}", flush=True)
        assert ratio <= 1.0 and nw <= RT, k


@pytest.mark.parametrize("name", list(SCENES))
def test_ndfd_losses_and_gradient_match_oracle(name):
    g, cams, vts = _scene(name)
    gpu = _gpu(g, cams, vts, "bf16")
    # the NDFD gradient alone: nothing else reaches the colour
    assert np.all(gpu["grads"]["sh"] == 0)
    _check(name, g, cams, vts, gpu)


@pytest.mark.parametrize("name,form", [("d64_two_views", "bf16"), ("d128", "f32"), ("surfel_d64", "bf16"),
                                       ("surfel_d32_two_views", "f32")])
def test_ndfd_joins_the_colour_and_feature_adjoint(name, form):
    # g_k = rgb_k . dC + f_k . dF + h_k: the NDFD partials are added to the
    # gradient kernel's (either form) before the per-Gaussian reduction
    g, cams, vts = _scene(name, with_colour=True)
    gpu = _gpu(g, cams, vts, form)
    _check(name, g, cams, vts, gpu)


def test_ndfd_rejects_fp32_features_and_bad_maps():
    from paper_2505_19154_amd._lib import FhError
    from paper_2505_19154_amd.raster import Rasterizer
    g = scenegen.make_gaussians(200, 1.0, 0, 32, seed=3)
    cams = [scenegen.look_at_camera((0, -4, 0), 32, 32)]
    dg = U.device_gaussians(g)
    r = Rasterizer(cams, dg.n, 0, 32)
    img = r.forward(dg)
    gt = torch.zeros(r.n_pixels, 32, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(FhError):
        r.ndfd_losses(dg, img, gt)                       # FP32 features
    gb = scenegen.make_gaussians(200, 1.0, 0, 32, seed=3, feat_dtype="bf16")
    dgb = U.device_gaussians(gb)
    rb = Rasterizer(cams, dgb.n, 0, 32, feat_dtype="bf16", form="bf16")
    imgb = rb.forward(dgb)
    with pytest.raises(FhError):
        rb.ndfd_losses(dgb, imgb, gt[:-1])               # wrong shape
    with pytest.raises(FhError):
        rb.ndfd_losses(dgb, imgb, gt.float())            # not BF16
    # the gradient needs a plan with the NDFD storage; the losses alone do not
    Lgt, Lcf = rb.ndfd_losses(dgb, imgb, gt)
    dC = torch.zeros(rb.n_pixels, 3, device="cuda")
    with pytest.raises(FhError):
        rb.render_bwd(dgb, imgb, dC, ndfd=dict(gt=gt))
    from paper_2505_19154_amd import _lib as L
    import ctypes
    from paper_2505_19154_amd.raster import _ptr, _stream
    gs, im = dgb.struct(), imgb.struct()
    up = L.FhUpstream(_ptr(dC), None, None)
    up.ndfd_gt = _ptr(gt)
    gr = rb.new_grads()
    grs = L.FhGrads(*[_ptr(gr[k]) for k in ("means", "scales", "quats", "opacity", "sh")])
    st = rb.lib.fh_render_bwd(ctypes.byref(rb.plan), ctypes.byref(gs), _ptr(rb.ws), ctypes.byref(im), ctypes.byref(up),
                              None, 0, None, ctypes.byref(grs), _stream())
    assert st == L.FH_E_INVALID
