"""Pins of the oracle's training step (oracle/train.py): Adam and the
densification rules."""
import numpy as np
import torch

from oracle import train


def _raw(n=40, nb=4, seed=0):
    rng = np.random.default_rng(seed)
    return dict(means=rng.normal(size=(n, 3)), log_scales=rng.normal(-3, 0.5, size=(n, 3)),
                quats=rng.normal(size=(n, 4)), logit_opacity=rng.normal(size=n), sh=rng.normal(size=(n, nb, 3)))


def _zeros(raw):
    return {k: np.zeros_like(v) for k, v in raw.items()}


LR = dict(means=1e-3, log_scales=5e-3, quats=1e-3, logit_opacity=5e-2, sh=2.5e-3)


def test_first_adam_step_moves_every_element_by_lr_against_the_gradient_sign():
    # at t = 1, m_hat = g and v_hat = g^2, so the step is lr g / (|g| + eps)
    raw = _raw()
    rng = np.random.default_rng(1)
    g = {k: rng.normal(size=v.shape) for k, v in raw.items()}
    new, m, v = train.adam_step(raw, g, _zeros(raw), _zeros(raw), 1, LR)
    for k in raw:
        assert np.allclose(raw[k] - new[k], LR[k] * np.sign(g[k]), rtol=1e-12, atol=1e-14), k
        assert np.allclose(m[k], 0.1 * g[k]) and np.allclose(v[k], 0.001 * g[k] ** 2)


def test_adam_matches_torch_adam_over_several_steps():
    raw = _raw(seed=2)
    rng = np.random.default_rng(3)
    params = {k: torch.tensor(v, requires_grad=True) for k, v in raw.items()}
    opt = torch.optim.Adam([dict(params=[params[k]], lr=LR[k]) for k in train.GROUPS], betas=(0.9, 0.999), eps=1e-15)
    m, v = _zeros(raw), _zeros(raw)
    for t in range(1, 6):
        g = {k: rng.normal(size=x.shape) for k, x in raw.items()}
        raw, m, v = train.adam_step(raw, g, m, v, t, LR)
        opt.zero_grad()
        for k in train.GROUPS:
            params[k].grad = torch.tensor(g[k])
        opt.step()
        for k in train.GROUPS:
            assert np.allclose(raw[k], params[k].detach().numpy(), rtol=1e-12, atol=1e-14), (t, k)


def test_raw_gradients_match_autograd_of_the_activations():
    raw = _raw(seed=4)
    rng = np.random.default_rng(5)
    ga = dict(means=rng.normal(size=(40, 3)), scales=rng.normal(size=(40, 3)), quats=rng.normal(size=(40, 4)),
              opacity=rng.normal(size=40), sh=rng.normal(size=(40, 4, 3)))
    got = train.raw_grads(raw, ga)
    ls = torch.tensor(raw["log_scales"], requires_grad=True)
    lo = torch.tensor(raw["logit_opacity"], requires_grad=True)
    ((torch.exp(ls) * torch.tensor(ga["scales"])).sum() + (torch.sigmoid(lo) * torch.tensor(ga["opacity"])).sum()
     ).backward()
    assert np.allclose(got["log_scales"], ls.grad.numpy(), rtol=1e-13)
    assert np.allclose(got["logit_opacity"], lo.grad.numpy(), rtol=1e-13)


def test_densify_actions_and_results():
    raw = _raw(n=10, seed=6)
    raw["log_scales"][:] = -4.0
    raw["log_scales"][[2, 5]] = -1.0                      # large: split when hot
    raw["logit_opacity"][:] = 2.0
    raw["logit_opacity"][7] = -8.0                        # transparent: pruned
    gsum = np.zeros(10, np.float32)
    cnt = np.full(10, 4, np.int32)
    gsum[[1, 2, 3]] = 0.01                                # avg 2.5e-3 >= 2e-4
    act = train.densify_actions(gsum, cnt, raw["log_scales"], 2e-4, np.log(0.05))
    assert act.tolist() == [0, 1, 2, 1, 0, 0, 0, 0, 0, 0]
    z = np.random.default_rng(7).normal(size=(1, 2, 3))
    m, v = _zeros(raw), _zeros(raw)
    m["means"][:] = 1.0
    out, om, ov, keep, n0 = train.densify(raw, m, v, act, z, prune_logit=np.log(0.005 / 0.995))
    # 10 + 2 clones + 1 second child - 1 pruned
    assert out["means"].shape[0] == 12 and n0 == 10
    # originals in order without the pruned one, then the appended ones (parents 1, 2, 3)
    assert np.allclose(out["means"][:2], raw["means"][:2])
    R = train.quat_rotation(raw["quats"][[2]])[0]
    s = np.exp(raw["log_scales"][2])
    assert np.allclose(out["means"][2], raw["means"][2] + R @ (s * z[0, 0]))
    assert np.allclose(out["means"][10], raw["means"][2] + R @ (s * z[0, 1]))
    assert np.allclose(out["log_scales"][[2, 10]], -1.0 - np.log(1.6))
    assert np.allclose(out["means"][9], raw["means"][1]) and np.allclose(out["means"][11], raw["means"][3])
    # the split children's mean is the parent's in expectation: average over many draws
    zz = np.random.default_rng(8).normal(size=(20000, 2, 3))
    act1 = np.array([2])
    one = {k: v[[2]] for k, v in raw.items()}
    kids = []
    for zi in zz[:2000]:
        o1, _, _, _, _ = train.densify(one, _zeros(one), _zeros(one), act1, zi[None], -1e9)
        kids.append(o1["means"])
    kids = np.concatenate(kids)
    cov = np.cov((kids - raw["means"][2]).T)
    assert np.allclose(kids.mean(0), raw["means"][2], atol=4 * s.max() / np.sqrt(4000) + 1e-12)
    # the children scatter with the parent's covariance R diag(s^2) R^T
    assert np.allclose(cov, R @ np.diag(s ** 2) @ R.T, atol=0.1 * s.max() ** 2)
    # moments: kept originals keep theirs, split parents and new ones restart
    assert np.all(om["means"][[0, 1, 3]] == 1.0) and np.all(om["means"][[2, 9, 10, 11]] == 0.0)
    assert keep.sum() == 12 and not keep[7]


def test_photometric_loss_and_its_gradient_by_central_differences():
    rng = np.random.default_rng(9)
    C, Ct = rng.uniform(size=(7, 3)), rng.uniform(size=(7, 3))
    L, dC = train.photometric_loss(C, Ct)
    # hand value for a one-pixel image: ((0.5)^2 + 0 + (-1)^2) / 3
    assert train.photometric_loss(np.array([[1.0, 2.0, 3.0]]), np.array([[0.5, 2.0, 4.0]]))[0] == 1.25 / 3
    h = 1e-6
    for i, c in ((0, 0), (3, 2), (6, 1)):
        Cp, Cm = C.copy(), C.copy()
        Cp[i, c] += h
        Cm[i, c] -= h
        fd = (train.photometric_loss(Cp, Ct)[0] - train.photometric_loss(Cm, Ct)[0]) / (2 * h)
        assert abs(fd - dC[i, c]) <= 1e-9


def test_densify_stats_hand_case():
    # three Gaussians, two views: (3, 4) -> 5 in view 0 only where binned
    g0 = np.array([[3.0, 4.0], [1.0, 0.0], [0.0, 0.0]])
    g1 = np.array([[0.0, -2.0], [6.0, 8.0], [5.0, 12.0]])
    b0 = np.array([True, False, True])
    b1 = np.array([True, True, False])
    gs, cnt = train.densify_stats([g0, g1], [b0, b1])
    assert gs.tolist() == [7.0, 10.0, 0.0] and cnt.tolist() == [2, 1, 1]
