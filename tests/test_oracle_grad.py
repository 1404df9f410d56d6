"""Pins of the oracle's hand-written adjoint (raster.c backward + project_bwd)."""
import numpy as np
import torch

import scenegen
from oracle import brute, pipeline


def _case(seed, n=100, d=6, recipe="front48x40", deg=2, dT=True):
    g = scenegen.make_gaussians(n, 1.0, deg, d, seed=seed)
    cams = scenegen.make_cameras(recipe)
    vt = [scenegen.make_view_tensors(0, cams[0].npix, d, with_dT=dT)]
    return g, cams, vt


def test_adjoint_matches_torch_autograd_of_brute_force():
    for seed in (1, 2, 3):
        g, cams, vt = _case(seed)
        o = pipeline.run(g, cams, vt)
        L = brute.leaves(g)
        C, F, T, _, _ = brute.render(L, g, cams[0], g["feat"])
        loss = ((torch.tensor(vt[0]["dC"], dtype=torch.float64) * C).sum()
                + (torch.tensor(vt[0]["dF"], dtype=torch.float64) * F).sum()
                + (torch.tensor(vt[0]["dT"], dtype=torch.float64) * T).sum())
        loss.backward()
        for k in ("means", "scales", "quats", "opacity", "sh"):
            ref = L[k].grad.numpy()
            got = o["grads"][k]
            mag = o["grads_mag"][k]
            assert np.all(np.abs(got - ref) <= 1e-10 * mag + 1e-12), k


def test_adjoint_matches_central_differences():
    g, cams, vt = _case(11, n=60, deg=1)
    o = pipeline.run(g, cams, vt)

    def loss(gg):
        oo = pipeline.run(gg, cams)
        v = oo["views"][0]
        return float((vt[0]["dC"] * v["C"]).sum() + (vt[0]["dF"] * v["F"]).sum() + (vt[0]["dT"] * v["T"]).sum())

    # Gaussians with no ambiguous decision and a few contributing pixels
    ok = np.nonzero((o["gflags"] == 0) & (np.abs(o["grads"]["opacity"]) > 1e-6))[0][:6]
    assert ok.size >= 3
    g64 = {k: (np.asarray(v, np.float64) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    for key, comps in (("means", 3), ("scales", 3), ("quats", 4), ("opacity", 1)):
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


def test_feature_gradient_equals_fusion_with_target_dF():
    # dL/df_g = sum_p w_g(p) dF(p) is the unnormalised fusion of the map dF
    g, cams, vt = _case(12)
    vt2 = [dict(vt[0], target=vt[0]["dF"])]
    o = pipeline.run(g, cams, vt2, fusion=True, want_dfeat=True)
    assert np.allclose(o["dfeat"], o["fsum"], rtol=1e-13, atol=1e-15)
