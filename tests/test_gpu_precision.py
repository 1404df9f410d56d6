"""Full-frame parity and the precision statement at the 1080p benchmark
workload (500k Gaussians, SH3, D=256 BF16 features, fusion of a BF16 target).

Both arithmetic forms run the whole step on the GPU; the FP64 oracle walks
every tile of the frame twice:
  * fed the same BF16-rounded features and target the GPU reads: every pixel
    and every Gaussian must meet the tolerance rule (tests/gpu_util.py), and
    the per-output error is recorded (the arithmetic error of the form);
  * fed the unrounded FP32 draws of the same features and target: the
    difference is recorded as the error of storing them in BF16.
The statement (max and mean |x - r| / M per output, M the oracle's magnitude
companion, and the normwise error ||x - r|| / ||r|| over the same elements
and over all of them) is written as JSON to
profiles/precision_c3.json, or to $FH_PRECISION_OUT.
"""
import json
import os
import time

import numpy as np
import pytest

import scenegen
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GRADS = ("means", "scales", "quats", "opacity", "sh")


def _stats(got, ref, mag, ok=None, amb=None, rtol=None):
    """max and mean |got - ref| / mag over `ok` & (mag > 0), the tolerance-rule
    ratio over the same set (when rtol is given), and the normwise error."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    mag = np.asarray(mag, np.float64)
    err = np.abs(got - ref)
    sel = mag > 0
    if ok is not None:
        sel &= ok
    r = err[sel] / mag[sel]
    # normwise over the same elements (those no near-threshold decision can
    # reach), and over every element for the record: a flipped stop decision
    # changes a pixel's T by up to its whole value, a skip flip a Gaussian's
    # sums by up to its bound, in FP32 as in any precision short of FP64
    out = dict(max_rel=float(r.max()) if r.size else 0.0, mean_rel=float(r.mean()) if r.size else 0.0,
               normwise=U.normwise(got[sel], ref[sel]), normwise_all=U.normwise(got, ref),
               checked=int(sel.sum()), total=int(err.size))
    # where the oracle's magnitude is zero nothing contributed (away from
    # near-threshold decisions): the value must be exactly zero
    zero = ~(mag > 0) if ok is None else (~(mag > 0) & ok)
    out["zero_where_untouched"] = bool(np.all(got[zero] == 0))
    if rtol is not None:
        bound = rtol * mag + 1e-30
        if amb is not None:
            bound = bound + U.AMB_FACTOR * np.asarray(amb, np.float64)
        rr = err / bound
        out["rule_ratio_max"] = float(rr[ok].max()) if ok is not None else float(rr.max())
    return out


def _rows_mask(ok_px, d):
    return np.repeat(ok_px[:, None], d, axis=1)


@pytest.fixture(scope="module")
def c3():
    wl = scenegen.WORKLOADS["c3"]
    t0 = time.time()
    g = scenegen.make_gaussians(wl.n, wl.half_extent, wl.sh_degree, wl.d, seed=0, feat_dtype="bf16")
    cams = scenegen.make_cameras(wl.views)
    vt = scenegen.make_view_tensors(0, cams[0].npix, wl.d, with_dT=True, target_dtype="bf16")
    gpu = {}
    for form in ("bf16", "f32"):
        r = U.run_gpu(g, cams, [vt], fusion=True, form=form, margin=1.02)
        img = r["img"]
        gpu[form] = dict(C=img.C.cpu().numpy(), T=img.T.cpu().numpy(), F=img.F.cpu().numpy(),
                         niter=img.n_iter.cpu().numpy().astype(np.int64),
                         grads={k: v.cpu().numpy() for k, v in r["grads"].items()},
                         fsum=(r["acc"].sum + r["acc"].comp).cpu().numpy(),
                         wsum=(r["acc"].wsum + r["acc"].wcomp).cpu().numpy())
        del r
        print(f"[precision] gpu {form} done ({time.time() - t0:.0f} s)", flush=True)
    ora = U.run_oracle(g, cams, [vt], fusion=True)
    print(f"[precision] oracle (same BF16 values) done ({time.time() - t0:.0f} s)", flush=True)
    # the unrounded draws of the same features and target
    g32 = scenegen.make_gaussians(wl.n, wl.half_extent, wl.sh_degree, wl.d, seed=0, feat_dtype="f32")
    vt32 = scenegen.make_view_tensors(0, cams[0].npix, wl.d, with_dT=True, target_dtype="f32")
    from oracle import pipeline
    ora32 = pipeline.run(g32, cams, [vt32], fusion=True, want_Fmag=False, magnitudes=False)
    print(f"[precision] oracle (FP32 features and target) done ({time.time() - t0:.0f} s)", flush=True)
    return dict(wl=wl, gpu=gpu, ora=ora, ora32=ora32)


@pytest.mark.timeout(2400)
def test_full_frame_parity_and_precision_statement(c3):
    ora, ora32 = c3["ora"], c3["ora32"]
    v = ora["views"][0]
    v32 = ora32["views"][0]
    ok_px = (v["flags"] & 1) == 0
    keep = U.checkable(ora["gflags"])
    d = c3["wl"].d
    report = dict(workload=c3["wl"].description, pixels=int(ok_px.size),
                  ambiguous_pixels=int((~ok_px).sum()), gaussians=int(keep.size),
                  excluded_gaussians_colour_clamp=int((~keep).sum()),
                  tolerance=dict(rule="|x - r| <= rtol M + 1.05 amb elementwise; ||x - r|| <= rtol ||r|| over the "
                                      "elements free of near-threshold decisions (normwise_all: every element, "
                                      "reported)",
                                 rtol=dict(U.RTOL_FORM)),
                  forms={})
    failures = []
    for form, got in c3["gpu"].items():
        rt = U.RTOL_FORM[form]
        same, storage = {}, {}
        # per-pixel outputs over every unambiguous pixel of the frame
        same["n_iter_mismatches"] = int((got["niter"][ok_px] != v["niter"][ok_px]).sum())
        same["C"] = _stats(got["C"], v["C"], v["Cmag"], _rows_mask(ok_px, 3), rtol=U.RTOL)
        same["T"] = _stats(got["T"], v["T"], v["T"], ok_px, rtol=U.RTOL)
        same["F"] = _stats(got["F"], v["F"], v["Fmag"], _rows_mask(ok_px, d), rtol=rt)
        storage["F"] = _stats(got["F"], v32["F"], v["Fmag"], _rows_mask(ok_px, d))
        for k in GRADS:
            ref, mag, amb = ora["grads"][k], ora["grads_mag"][k], ora["grads_amb"][k]
            m = keep.reshape((-1,) + (1,) * (ref.ndim - 1)) & np.ones(ref.shape, bool)
            same["grad_" + k] = _stats(got["grads"][k], ref, mag, m & (amb == 0), amb=amb, rtol=rt)
            same["grad_" + k]["rule_ratio_max"] = _stats(got["grads"][k], ref, mag, m, amb=amb,
                                                         rtol=rt)["rule_ratio_max"]
            storage["grad_" + k] = _stats(got["grads"][k], ora32["grads"][k], mag, m & (amb == 0))
        mf = keep[:, None] & np.ones(got["fsum"].shape, bool)
        same["fusion_sum"] = _stats(got["fsum"], ora["fsum"], ora["fsum_mag"], mf & (ora["fsum_amb"] == 0),
                                    rtol=rt)
        same["fusion_sum"]["rule_ratio_max"] = _stats(got["fsum"], ora["fsum"], ora["fsum_mag"], mf,
                                                      amb=ora["fsum_amb"], rtol=rt)["rule_ratio_max"]
        same["fusion_weight"] = _stats(got["wsum"], ora["wsum"], ora["wsum"], keep & (ora["wsum_amb"] == 0),
                                       rtol=rt)
        same["fusion_weight"]["rule_ratio_max"] = _stats(got["wsum"], ora["wsum"], ora["wsum"], keep,
                                                         amb=ora["wsum_amb"], rtol=rt)["rule_ratio_max"]
        storage["fusion_sum"] = _stats(got["fsum"], ora32["fsum"], ora["fsum_mag"], mf & (ora["fsum_amb"] == 0))
        report["forms"][form] = dict(rtol=rt, vs_oracle_same_bf16_values=same,
                                     vs_oracle_fp32_features_and_target=storage)
        for name, st in same.items():
            if name == "n_iter_mismatches":
                if st:
                    failures.append((form, name, st))
                continue
            if st["rule_ratio_max"] > 1.0 or st["normwise"] > rt or not st["zero_where_untouched"]:
                failures.append((form, name, st))
        print(f"[precision] {form}: " + "; ".join(
            f"{k} {s['max_rel']:.2e}/{s['mean_rel']:.2e} (rule {s['rule_ratio_max']:.3f}, norm {s['normwise']:.2e}, "
            f"all {s['normwise_all']:.2e})"
            for k, s in same.items() if k != "n_iter_mismatches"), flush=True)
        print(f"[precision] {form} storage: " + "; ".join(
            f"{k} {s['max_rel']:.2e}/{s['mean_rel']:.2e} norm {s['normwise']:.2e}" for k, s in storage.items()),
            flush=True)
    path = os.environ.get("FH_PRECISION_OUT", os.path.join(ROOT, "profiles", "precision_c3.json"))
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(report, f, indent=1)
    assert not failures, failures
