"""GPU parity of the training step (Algorithm 1) against the oracle
(oracle/train.py): Adam over raw parameters with the activation chain, the
activations, the densification statistics, the clone / split / prune
densification, the photometric loss, and an end-to-end convergence check on
a synthetic scene whose target images the oracle renders."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import pipeline, train as otrain
from paper_2505_19154_amd import train as T
from paper_2505_19154_amd.raster import Rasterizer
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

LR = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, logit_opacity=5e-2, sh=2.5e-3)


def _raw(n, nb, seed):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4))
    return dict(means=rng.uniform(-1, 1, size=(n, 3)), log_scales=rng.normal(-3, 0.5, size=(n, 3)),
                quats=q, logit_opacity=rng.normal(size=n), sh=rng.normal(0, 0.3, size=(n, nb, 3)))


def _f32(d):
    return {k: np.asarray(v, np.float32) for k, v in d.items()}


def _dev(d):
    return {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda() for k, v in d.items()}


def _params(raw32) -> T.Params:
    t = _dev(raw32)
    return T.activate(T.Params(t["means"], t["log_scales"], t["quats"], t["logit_opacity"], t["sh"]))


def _np(p: T.Params):
    return {k: getattr(p, k).cpu().numpy().astype(np.float64) for k in T.GROUPS}


@pytest.mark.parametrize("n", [1, 257, 3001])
def test_activate_matches_fp64(n):
    raw = _f32(_raw(n, 4, 1))
    p = _params(raw)
    torch.cuda.synchronize()
    s_ref = np.exp(raw["log_scales"].astype(np.float64))
    o_ref = 1.0 / (1.0 + np.exp(-raw["logit_opacity"].astype(np.float64)))
    assert np.all(np.abs(p.scales.cpu().numpy() - s_ref) <= 4e-7 * s_ref)
    assert np.all(np.abs(p.opacity.cpu().numpy() - o_ref) <= 4e-7 * o_ref)


@pytest.mark.parametrize("n,sh_degree", [(1, 0), (1003, 3), (4096, 1)])
def test_adam_steps_match_oracle(n, sh_degree):
    nb = (sh_degree + 1) ** 2
    raw = _f32(_raw(n, nb, 2))
    p = _params(raw)
    m, v = T.Params.zeros_like(p), T.Params.zeros_like(p)
    ora_raw = {k: x.astype(np.float64) for k, x in raw.items()}
    ora_m = {k: np.zeros_like(x) for k, x in ora_raw.items()}
    ora_v = {k: np.zeros_like(x) for k, x in ora_raw.items()}
    rng = np.random.default_rng(3)
    gabs = {k: np.zeros_like(x) for k, x in ora_raw.items()}
    g2abs = {k: np.zeros_like(x) for k, x in ora_raw.items()}
    for t in range(1, 4):
        ga = _f32(dict(means=rng.normal(size=(n, 3)), scales=rng.normal(size=(n, 3)), quats=rng.normal(size=(n, 4)),
                       opacity=rng.normal(size=n), sh=rng.normal(size=(n, nb, 3))))
        # the oracle's raw gradients at the activated values the kernel reads
        gr = otrain.raw_grads(ora_raw, {k: x.astype(np.float64) for k, x in ga.items()})
        ora_raw, ora_m, ora_v = otrain.adam_step(ora_raw, gr, ora_m, ora_v, t, LR)
        for k in gabs:
            gabs[k] = 0.9 * gabs[k] + np.abs(gr[k])
            g2abs[k] = 0.999 * g2abs[k] + gr[k] ** 2
        T.adam_step(p, m, v, _dev(ga), t, LR)
    torch.cuda.synchronize()
    gx, gm, gv = _np(p), _np(m), _np(v)
    for k in T.GROUPS:
        # three steps of FP32 arithmetic: a few ulp of x plus 1e-6 of each step
        bx = 4e-7 * np.abs(ora_raw[k]) + 3e-6 * LR[k] * 3
        assert np.all(np.abs(gx[k] - ora_raw[k]) <= bx), k
        assert np.all(np.abs(gm[k] - ora_m[k]) <= 1e-6 * gabs[k] + 1e-30), k
        assert np.all(np.abs(gv[k] - ora_v[k]) <= 1e-6 * g2abs[k] + 1e-30), k
    # the activations now follow the updated raw values
    s_ref = np.exp(gx["log_scales"])
    o_ref = 1.0 / (1.0 + np.exp(-gx["logit_opacity"]))
    assert np.all(np.abs(p.scales.cpu().numpy() - s_ref) <= 4e-7 * s_ref)
    assert np.all(np.abs(p.opacity.cpu().numpy() - o_ref) <= 4e-7 * o_ref)


def test_adam_rejects_bad_arguments():
    from paper_2505_19154_amd._lib import FhError
    p = _params(_f32(_raw(10, 1, 4)))
    m, v = T.Params.zeros_like(p), T.Params.zeros_like(p)
    g = _dev(dict(means=np.zeros((10, 3)), scales=np.zeros((10, 3)), quats=np.zeros((10, 4)), opacity=np.zeros(10),
                  sh=np.zeros((10, 1, 3))))
    with pytest.raises(FhError):
        T.adam_step(p, m, v, g, 0, LR)            # step must be >= 1
    with pytest.raises(FhError):
        T.adam_step(p, m, v, dict(g, means=g["means"][:5]), 1, LR)


@pytest.mark.parametrize("n,seed", [(1, 5), (2500, 6), (70001, 7)])
def test_densify_matches_oracle(n, seed):
    nb = 9
    rng = np.random.default_rng(seed)
    raw = _f32(_raw(n, nb, seed))
    raw["logit_opacity"] = rng.normal(0, 3, size=n).astype(np.float32)
    grad_sum = np.abs(rng.normal(0, 3e-4, size=n)).astype(np.float32)
    count = rng.integers(0, 4, size=n).astype(np.int32)
    z = rng.normal(size=(n, 2, 3)).astype(np.float32)
    feat = rng.normal(size=(n, 24)).astype(np.float32)
    thr, lthr, prune = 2e-4, -3.0, -2.0
    m = {k: rng.normal(size=x.shape).astype(np.float32) for k, x in raw.items()}
    v = {k: np.abs(rng.normal(size=x.shape)).astype(np.float32) for k, x in raw.items()}
    # oracle
    act = otrain.densify_actions(grad_sum, count, raw["log_scales"], thr, lthr)
    split = np.nonzero(act == 2)[0]
    o_raw, o_m, o_v, keep, _ = otrain.densify({k: x.astype(np.float64) for k, x in raw.items()},
                                              {k: x.astype(np.float64) for k, x in m.items()},
                                              {k: x.astype(np.float64) for k, x in v.items()}, act,
                                              z[split].astype(np.float64), prune)
    # GPU
    p = _params(raw)
    pm = T.Params(*[_dev(m)[k] for k in T.GROUPS])
    pv = T.Params(*[_dev(v)[k] for k in T.GROUPS])
    out, om, ov, rows = T.densify(p, pm, pv, torch.from_numpy(grad_sum).cuda(), torch.from_numpy(count).cuda(),
                                  torch.from_numpy(z).cuda(), thr, lthr, prune,
                                  extra_rows=(torch.from_numpy(feat).cuda(),))
    torch.cuda.synchronize()
    assert out.n == o_raw["means"].shape[0]
    g = _np(out)
    for k in ("quats", "logit_opacity", "sh"):
        assert np.array_equal(g[k], o_raw[k]), k          # copies: bit for bit
    # means of split children: FP32 mu + R diag(s) z against FP64
    mag = np.abs(o_raw["means"]) + 3 * np.exp(o_raw["log_scales"]).max(1, keepdims=True) * 4.0
    assert np.all(np.abs(g["means"] - o_raw["means"]) <= 2e-7 * mag)
    assert np.all(np.abs(g["log_scales"] - o_raw["log_scales"]) <= 2e-7 * (np.abs(o_raw["log_scales"]) + 0.5))
    for k in T.GROUPS:
        assert np.array_equal(_np(om)[k], o_m[k]) and np.array_equal(_np(ov)[k], o_v[k]), k
    # activations of the new set, and the frozen features carried to every copy
    s_ref = np.exp(g["log_scales"])
    assert np.all(np.abs(out.scales.cpu().numpy() - s_ref) <= 4e-7 * s_ref)
    parent = np.concatenate([np.arange(n), np.sort(np.nonzero(act != 0)[0])])[keep]
    assert np.array_equal(rows[0].cpu().numpy(), feat[parent])


def test_densify_stats_match_oracle():
    g = scenegen.make_gaussians(600, 1.0, 1, 0, seed=11)
    cams = [scenegen.look_at_camera((0.0, -4.0, 0.3), 96, 80), scenegen.look_at_camera((3.0, -2.5, 0.5), 64, 64),
            scenegen.look_at_camera((-2.0, -3.0, -1.0), 80, 48)]
    vts = U.view_maps(cams, 0)
    ora = pipeline.run(g, cams, vts)
    gpu = U.run_gpu(g, cams, vts)
    r = gpu["r"]
    gs = torch.zeros(r.n, dtype=torch.float32, device="cuda")
    cnt = torch.zeros(r.n, dtype=torch.int32, device="cuda")
    T.densify_stats(r, gs, cnt)
    T.densify_stats(r, gs, cnt)        # accumulates
    torch.cuda.synchronize()
    binned = [ora["bins"]["per_view"][v]["binned"] for v in range(len(cams))]
    ref, rcnt = otrain.densify_stats([ora["views"][v]["g2d"] for v in range(len(cams))], binned)
    assert np.array_equal(cnt.cpu().numpy(), 2 * rcnt)
    bound = np.zeros(r.n)
    for v in range(len(cams)):
        mag = ora["views"][v]["g2d_mag"][:, :2].sum(1)
        amb = ora["views"][v]["g2d_amb"][:, :2].sum(1)
        bound += np.where(binned[v], U.RTOL * mag + U.AMB_FACTOR * amb, 0.0)
    err = np.abs(gs.cpu().numpy() - 2 * ref)
    assert np.all(err <= 2 * bound + 1e-30), float((err / np.maximum(2 * bound, 1e-300)).max())
    assert (rcnt > 0).sum() > 100 and (ref > 0).sum() > 50


@pytest.mark.parametrize("shape", [(1, 1), (37, 29), (640, 480)])
def test_photometric_loss_matches_oracle(shape):
    P = shape[0] * shape[1]
    rng = np.random.default_rng(P)
    C = rng.uniform(size=(P, 3)).astype(np.float32)
    Ct = rng.uniform(size=(P, 3)).astype(np.float32)
    pl = T.PhotometricLoss(P)
    loss, dC = pl(torch.from_numpy(C).cuda(), torch.from_numpy(Ct).cuda())
    torch.cuda.synchronize()
    L_ref, dC_ref = otrain.photometric_loss(C, Ct)
    assert abs(float(loss.item()) - L_ref) <= 1e-5 * L_ref
    e = np.abs(C.astype(np.float64) - Ct)
    assert np.all(np.abs(dC.cpu().numpy() - dC_ref) <= 4e-7 * 2 * e / (3 * P) + 1e-30)


@pytest.mark.timeout(300)
def test_training_converges_on_a_synthetic_scene():
    # ground truth: 400 Gaussians; targets rendered by the oracle from three views
    nb = 4
    gt = scenegen.make_gaussians(400, 1.0, 1, 0, seed=21)
    cams = [scenegen.look_at_camera((0.0, -4.0, 0.0), 96, 72), scenegen.look_at_camera((3.0, -2.5, 0.5), 96, 72),
            scenegen.look_at_camera((-2.5, -3.0, -1.0), 96, 72)]
    ora = pipeline.run(gt, cams)
    targets = [torch.from_numpy(np.ascontiguousarray(ora["views"][v]["C"], np.float32)).cuda()
               for v in range(len(cams))]
    # start: the same Gaussians with perturbed means, scales, opacities and colours
    rng = np.random.default_rng(22)
    raw = dict(means=gt["means"] + rng.normal(0, 0.03, size=gt["means"].shape),
               log_scales=np.log(gt["scales"]) + rng.normal(0, 0.3, size=gt["scales"].shape),
               quats=gt["quats"], logit_opacity=np.zeros(400),
               sh=gt["sh"] + rng.normal(0, 0.3, size=gt["sh"].shape))
    p = _params(_f32(raw))
    zrng = torch.Generator(device="cuda").manual_seed(23)
    # every Gaussian counts as hot at the one refinement (step 240): the small
    # ones are cloned, the large ones split
    tr = T.Trainer(p, None, cams, targets, LR, densify_every=240, grad_threshold=1e-12, log_scale_threshold=-2.5,
                   prune_logit=-4.6, z_source=lambda n: torch.randn(n, 2, 3, generator=zrng, device="cuda"))
    first = [float(tr.step().item()) for _ in range(3)]
    n0 = tr.p.n
    for _ in range(237):
        tr.step()
    assert tr.p.n > n0            # densified at step 240
    n1 = tr.p.n
    for _ in range(357):
        tr.step()
    last = []
    for _ in range(3):
        last.append(float(tr.step().item()))
    print(f"[train] loss {np.mean(first):.3e} -> {np.mean(last):.3e}, Gaussians {n0} -> {n1}", flush=True)
    assert np.mean(last) < 0.5 * np.mean(first)
