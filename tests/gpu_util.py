"""Helpers shared by the GPU parity tests: move a scenegen scene to the device,
run the HIP path through the C ABI, run the oracle on the same inputs, and
compare under the tolerance rule.

Tolerance rule (FP32 path vs FP64 oracle), per output x with reference r:
  * elementwise  |x - r| <= rtol * M + atol, where M is the oracle's magnitude
    companion (the same sums with every term replaced by its absolute value),
    checked on pixels whose float decisions are not ambiguous (no alpha within
    1e-4 relative of 1/255 or of the 0.99 clamp, no T' within 1e-4 relative of
    1e-4 along the pixel's walk); for per-Gaussian sums, on Gaussians that
    decide no ambiguous decision, with AMB_FACTOR times the oracle's bound of
    what the ambiguous decisions could change added to the bound;
  * normwise     ||x - r||_2 <= rtol * ||r||_2 over everything on the small
    scenes; over the elements free of near-threshold decisions at full frame,
    where flipped stop decisions (T changes by up to its whole value) are
    bound to occur, with the all-element value reported beside it.
"""
from __future__ import annotations

import numpy as np
import torch

import scenegen
from oracle import pipeline

RTOL = 1e-5
# The BF16-MFMA form feeds the feature contractions two-term BF16 splits
# (x = hi + lo, hi = bf16(x), lo = bf16(x - hi)) of the FP32 operands w and dF,
# which carry each operand to within 2^-18 relative; on top of the FP32 budget
# that gives 1e-5 + 2^-18 (3.8e-6), rounded up.
RTOL_FORM = {"f32": RTOL, "bf16": 2e-5}


def device_gaussians(g: dict, device="cuda"):
    from paper_2505_19154_amd.raster import Gaussians
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    feat = None
    if g["d"] > 0:
        if g.get("feat_dtype") == "bf16":
            feat = torch.from_numpy(g["feat_bits"].view(np.int16)).to(device).view(torch.bfloat16)
        else:
            feat = t(g["feat"])
    return Gaussians(t(g["means"]), t(g["scales"]), t(g["quats"]), t(g["opacity"]), t(g["sh"]), feat,
                     int(g["sh_degree"]))


def view_maps(cams, d, with_dT=True, target_dtype="f32"):
    return [scenegen.make_view_tensors(i, c.npix, d, with_dT=with_dT, target_dtype=target_dtype)
            for i, c in enumerate(cams)]


def concat(vts, key, device="cuda"):
    if key == "target_bits":
        a = np.concatenate([v[key] for v in vts]).view(np.int16)
        return torch.from_numpy(a).to(device).view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(np.concatenate([v[key] for v in vts]), np.float32)).to(device)


def run_gpu(g: dict, cams, vts=None, fusion=False, form="f32", margin=1.05, bin_rule="box"):
    """bin_rule "surfel" renders the primitives as surfels (with their own binning rule)."""
    from paper_2505_19154_amd.raster import FusionAcc, Rasterizer
    dg = device_gaussians(g)
    surf = bin_rule == "surfel"
    r = Rasterizer(cams, dg.n, dg.sh_degree, dg.d, feat_dtype=g.get("feat_dtype", "f32"), form=form,
                   bin_rule="box" if surf else bin_rule, primitive="surfel" if surf else "gaussian")
    img = r.forward(dg, margin)
    out = dict(r=r, g=dg, img=img)
    if vts is not None:
        dC = concat(vts, "dC")
        dF = concat(vts, "dF") if dg.d else None
        dT = concat(vts, "dT")
        acc = None
        target = None
        if fusion:
            acc = FusionAcc.zeros(dg.n, dg.d, "cuda")
            target = concat(vts, "target_bits") if "target_bits" in vts[0] else concat(vts, "target")
        grads = r.render_bwd(dg, img, dC, dF, dT, target=target, acc=acc)
        out.update(grads=grads, acc=acc)
    torch.cuda.synchronize()
    out["counters"] = r.counters()
    return out


def run_oracle(g: dict, cams, vts=None, fusion=False, bin_rule="box"):
    return pipeline.run(g, cams, vts, fusion=fusion, want_Fmag=True, bin_rule=bin_rule)


def split_views(arr, cams):
    offs = np.cumsum([0] + [c.npix for c in cams])
    return [arr[offs[i]:offs[i + 1]] for i in range(len(cams))]


# A near-threshold decision of one Gaussian may go the other way in FP32 and
# change its own and the other contributors' terms in that pixel; the oracle
# bounds that change to first order (grads_amb, fsum_amb, wsum_amb).  Taking a
# single decision both ways in FP64 changes the sums by at most the bound itself
# (tests/test_oracle_ambiguity.py; the decider's own would-be blend meets it
# exactly).  The factor covers what first order leaves out: FP32 flips happen
# within ~1e-6 relative of a threshold (second-order terms of that size), the
# rounding of the terms a flip adds or removes (within 2e-5 of them), and k skip
# decisions of one pixel flipping together, where a later decider's would-be
# blend also carries the earlier ones' transmittance factors, up to
# (1 - 1/255)^-(k-1): 1.05 covers k <= 13.
AMB_FACTOR = 1.05


def checkable(gflags):
    """Gaussians whose per-Gaussian sums are compared elementwise: all but those
    with a near-threshold colour clamp (oracle gflags bit 2), whose SH gradient
    and colour terms switch as a whole; near-threshold skip/stop/alpha-clamp
    decisions are covered by the amb bound instead."""
    return (np.asarray(gflags) & 4) == 0


def elementwise(got, ref, mag, rtol=RTOL, mask=None, atol=1e-30, amb=None):
    """max and mean of |got - ref| / (rtol mag + AMB_FACTOR amb + atol)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    mag = np.asarray(mag, np.float64)
    err = np.abs(got - ref)
    bound = rtol * mag + atol
    if amb is not None:
        bound = bound + AMB_FACTOR * np.asarray(amb, np.float64)
    ratio = err / np.maximum(bound, 1e-300)
    if mask is not None:
        ratio = ratio[mask]
    return float(ratio.max()) if ratio.size else 0.0, float(ratio.mean()) if ratio.size else 0.0


def normwise(got, ref):
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / nr) if nr > 0 else float(np.linalg.norm(got - ref))
