"""Pins of the oracle's NDFD feature branch (Section 3.3, Appendix A.1-A.2):
the losses L_gt and L_cf along each ray, and their gradient through the blend
weights w."""
import numpy as np
import torch

import scenegen
from oracle import brute, pipeline

LAM, K = 0.5, 20.0


def _case(seed, n=90, d=8, recipe="front48x40", correlated=True):
    g = scenegen.make_gaussians(n, 1.0, 1, d, seed=seed)
    cams = scenegen.make_cameras(recipe)
    P = cams[0].npix
    rng = np.random.default_rng(500 + seed)
    if correlated:
        # a ground-truth map near the rendered feature, so that cosines spread
        # over [-1, 1] and sigma over (0, 1)
        F = pipeline.run(g, cams)["views"][0]["F"]
        gt = F + 0.3 * rng.normal(size=F.shape) * np.abs(F).mean()
    else:
        gt = rng.normal(size=(P, d))
    vt = dict(dC=np.zeros((P, 3)), dF=np.zeros((P, d)), dT=np.zeros(P), gt=gt,
              ndfd_a=rng.normal(size=P), ndfd_b=rng.normal(size=P))
    return g, cams, vt


def test_losses_equal_the_double_sum_definition():
    for seed in (1, 2):
        g, cams, vt = _case(seed)
        o = pipeline.run(g, cams, [vt], ndfd=dict(lam=LAM, k=K))
        v = o["views"][0]
        Lgt, Lcf = brute.ndfd_losses(brute.leaves(g), g, cams[0], g["feat"], vt["gt"], LAM, K)
        assert np.allclose(v["Lgt"], Lgt.detach().numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(v["Lcf"], Lcf.detach().numpy(), rtol=1e-11, atol=1e-13)
        assert np.all(np.abs(v["Lcf"]) <= v["Lcf_mag"] + 1e-15)
        # sigma spreads (the test is not all sigma = 1)
        assert v["Lgt"].max() > 0 and np.std(v["Lgt"] / np.maximum(v["WN"], 1e-12)) > 0.05
        # the recorded W_N is 1 - T_final
        assert np.allclose(v["WN"], 1.0 - v["T"], rtol=1e-12, atol=1e-14)


def test_gradient_equals_autograd_of_the_definition():
    for seed in (3, 4):
        g, cams, vt = _case(seed)
        o = pipeline.run(g, cams, [vt], ndfd=dict(lam=LAM, k=K))
        L = brute.leaves(g)
        Lgt, Lcf = brute.ndfd_losses(L, g, cams[0], g["feat"], vt["gt"], LAM, K)
        loss = (torch.tensor(vt["ndfd_a"]) * Lgt).sum() + (torch.tensor(vt["ndfd_b"]) * Lcf).sum()
        loss.backward()
        for k in ("means", "scales", "quats", "opacity"):
            ref = L[k].grad.numpy()
            got, mag = o["grads"][k], o["grads_mag"][k]
            assert np.all(np.abs(got - ref) <= 1e-10 * mag + 1e-13), k
        assert np.all(o["grads"]["sh"] == 0)      # colour does not enter NDFD


def _ray(seed, n=12, d=5):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(n, d))
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    w = rng.uniform(0.01, 0.2, n)
    sig = rng.uniform(0, 1, n)
    return f, w, sig


def test_forward_indexed_and_reversed_gradients_agree():
    """dL_cf/dw_k in the forward-indexed form, in the reversed (back-to-front)
    form with the recorded totals W_N and F_N, by torch autograd of the double
    sum, and by central differences, on random rays (sigma held constant)."""
    for seed in range(5):
        f, w, sig = _ray(seed)
        n = w.size
        G = f @ f.T
        # forward-indexed: sigma_k (W_{k-1} - F_{k-1}.f_k) + sum_{i>k} sigma_i w_i (1 - f_i.f_k)
        fwd = np.array([sig[k] * (w[:k].sum() - (w[:k, None] * f[:k]).sum(0) @ f[k])
                        + sum(sig[i] * w[i] * (1 - G[i, k]) for i in range(k + 1, n)) for k in range(n)])
        # reversed: q counts from the far end; W_q, F_q include q; the second sum runs over the farther ones
        WN, FN = w.sum(), (w[:, None] * f).sum(0)
        rev = np.empty(n)
        Wq, Fq = 0.0, np.zeros(f.shape[1])
        far = []
        for k in range(n - 1, -1, -1):
            Wq += w[k]
            Fq = Fq + w[k] * f[k]
            rev[k] = sig[k] * ((WN - Wq) - (FN - Fq) @ f[k]) + sum(sig[i] * w[i] * (1 - G[i, k]) for i in far)
            far.append(k)
        wt = torch.tensor(w, requires_grad=True)
        lower = torch.tril(torch.tensor(1 - G), diagonal=-1)
        Lcf = (torch.tensor(sig) * wt * (lower @ wt)).sum()
        Lcf.backward()
        auto = wt.grad.numpy()

        def lcf(ww):
            return float((sig * ww * (np.tril(1 - G, -1) @ ww)).sum())

        fd = np.array([(lcf(w + 1e-6 * np.eye(n)[k]) - lcf(w - 1e-6 * np.eye(n)[k])) / 2e-6 for k in range(n)])
        assert np.allclose(fwd, auto, rtol=1e-12, atol=1e-14)
        assert np.allclose(rev, auto, rtol=1e-12, atol=1e-14)
        assert np.allclose(fd, auto, rtol=1e-7, atol=1e-9)
        # the O(N) form of L_cf equals the double sum
        Wp = np.concatenate([[0.0], np.cumsum(w)[:-1]])
        Fp = np.vstack([np.zeros(f.shape[1]), np.cumsum(w[:, None] * f, 0)[:-1]])
        on = (sig * w * (Wp - (Fp * f).sum(1))).sum()
        assert np.isclose(on, lcf(w), rtol=1e-13)


def test_identical_features_closed_form():
    """All features equal: every cosine is 1, so L_cf = 0 and its gradient
    vanishes; with F_gt along the same direction sigma = 1/(1 + e^{k(1 - lambda)})
    everywhere and L_gt = sigma (1 - T_final)."""
    g, cams, vt = _case(7, correlated=False)
    d = g["feat"].shape[1]
    g["feat"] = np.tile(np.float32(np.arange(1, d + 1)), (g["feat"].shape[0], 1))
    vt["gt"] = np.tile(np.arange(1, d + 1, dtype=np.float64) * 3.0, (vt["gt"].shape[0], 1))
    vt["ndfd_a"] = np.zeros_like(vt["ndfd_a"])
    o = pipeline.run(g, cams, [vt], ndfd=dict(lam=LAM, k=K))
    v = o["views"][0]
    sig = 1.0 / (1.0 + np.exp(K * (1.0 - LAM)))
    assert np.allclose(v["Lcf"], 0.0, atol=1e-14)
    assert np.allclose(v["Lgt"], sig * (1.0 - v["T"]), rtol=1e-12, atol=1e-16)
    for k in ("means", "scales", "quats", "opacity"):
        assert np.allclose(o["grads"][k], 0.0, atol=1e-12 * (1 + np.abs(o["grads_mag"][k]).max())), k


def test_sigma_companion_bounds_the_cosine_rounding():
    """sigma's companion carries the cosine's rounding through the sigmoid's
    slope: scaling the ground-truth map's components by (1 + eps s), s = +-1,
    changes every cosine by at most 2 eps sum_c |fh_c gh_c| (the components and
    the norm), so L_gt and L_cf change by at most 2 eps (M - their slope-free
    part) to first order; the slope-free companion alone is exceeded."""
    g, cams, vt = _case(8)
    eps = 1e-7
    rng = np.random.default_rng(9)
    o0 = pipeline.run(g, cams, [vt], ndfd=dict(lam=LAM, k=K))["views"][0]
    vt2 = dict(vt, gt=vt["gt"] * (1.0 + eps * rng.choice([-1.0, 1.0], size=vt["gt"].shape)))
    o1 = pipeline.run(g, cams, [vt2], ndfd=dict(lam=LAM, k=K))["views"][0]
    dgt = np.abs(o1["Lgt"] - o0["Lgt"])
    slope_gt = o0["Lgt_mag"] - o0["Lgt"]              # sum w k sigma (1 - sigma) phi_mag
    assert np.all(dgt <= 2.05 * eps * slope_gt + 1e-18)
    assert np.all(o0["Lgt_mag"] >= o0["Lgt"]) and np.all(o0["Lcf_mag"] >= np.abs(o0["Lcf"]))
    # the change is real and larger than the slope-free companion allows
    hit = o0["Lgt"] > 0
    assert (dgt[hit] / (eps * o0["Lgt"][hit])).max() > 2.05
    dcf = np.abs(o1["Lcf"] - o0["Lcf"])
    assert np.all(dcf <= 2.05 * eps * o0["Lcf_mag"] + 1e-18)


def test_gradient_companion_bounds_the_gradient():
    g, cams, vt = _case(5)
    o = pipeline.run(g, cams, [vt], ndfd=dict(lam=LAM, k=K))
    for k in ("means", "scales", "quats", "opacity"):
        assert np.all(np.abs(o["grads"][k]) <= o["grads_mag"][k] * (1 + 1e-12) + 1e-300), k
