#!/usr/bin/env python3
"""Benchmark: one step = project -> bin_sort -> render_fwd -> render_bwd (+ feature
fusion) over one batch of synthetic views, all through the C ABI on one GPU.

    python bench.py [--steps K] [--warmup W] [--workload c3] [--form f32|bf16] [--batched c4]

Prints ONE JSON line: Gaussian-pixel blends per second (sum over pixels of the
list positions each pixel walks, n_iter) with inputs resident in HBM, the
roofline position of the dominant kernel (timed live with HIP events on its
own stream), and the FP64 CPU oracle timed on a bounded sample of the same
workload.  The line also carries the batched workload ("batched": 16 views
of uneven size by default), both arithmetic forms, each step captured in one
HIP graph and timed as graph replays.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ms/view and Gaussian-pixel blends/s, 1080p D=256, BF16 vs FP32"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--form", default="auto", choices=["auto", "f32", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU-oracle sample time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare", type=int, default=1, help="also time the other arithmetic form")
    ap.add_argument("--kernel", default="render_bwd",
                    choices=["project", "bin", "render_fwd", "render_bwd", "reduce", "project_bwd"])
    ap.add_argument("--autotune", type=int, default=1, help="pick the launch shape by timing before the steps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB read + 1 GiB write kernel (for scaling HBM counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU: turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-calibration run into profiles/traffic_<kernel>_<workload>_<form>.json")
    ap.add_argument("--traffic-command", default="", help="the profiled command, recorded with --traffic-from")
    ap.add_argument("--extras", type=int, default=1,
                    help="also time the NDFD branch and the training-step kernels on the headline workload")
    ap.add_argument("--batched", default="c4",
                    help="batched workload timed after the headline as one graph-replayed step per form "
                         "('' to skip)")
    return ap.parse_args()


def alg_bytes(kernel: str, wl, P: int, n_vis: int, n_inst: int, feat_b: int, tgt_b: int) -> tuple[float, str]:
    """Algorithmic bytes one launch of `kernel` must move: each input it needs read
    once and each output written once, per pixel and per visible Gaussian."""
    D = wl.d
    nsh = 3 * (wl.sh_degree + 1) ** 2
    if kernel == "render_bwd":
        per_pix = 24 + 4 * D + (D * tgt_b if wl.fusion else 0)
        per_g = 48 + D * feat_b + 48 + (4 * D + 4 if wl.fusion else 0)
        return P * per_pix + n_vis * per_g, f"{per_pix} B/pixel + {per_g} B/visible Gaussian"
    if kernel == "render_fwd":
        per_pix = 20 + 4 * D
        per_g = 48 + D * feat_b
        return P * per_pix + n_vis * per_g + 8 * n_inst, f"{per_pix} B/pixel + {per_g} B/visible Gaussian + 8 B/instance"
    if kernel == "bin":
        return 44 * n_inst + 24 * wl.n, "44 B/instance + 24 B/Gaussian"
    if kernel in ("project", "project_bwd"):
        per_g = 44 + 4 * nsh + 64
        return per_g * wl.n, f"{per_g} B/Gaussian"
    if kernel == "reduce":
        per_g = 48 + (8 * D + 8 if wl.fusion else 0) * 2
        return per_g * n_vis, f"{per_g} B/visible Gaussian"
    raise ValueError(kernel)


# the source files that define each bracket's kernels (plus the shared headers)
BRACKET_SOURCES = {
    ("project", "f32"): ("project.hip",), ("project", "bf16"): ("project.hip",),
    ("render_fwd", "f32"): ("render_f32.hip",), ("render_fwd", "bf16"): ("render_bf16.hip",),
    ("render_bwd", "f32"): ("render_f32.hip", "reduce.hip"), ("render_bwd", "bf16"): ("render_bwd_bf16.hip", "reduce.hip"),
    ("project_bwd", "f32"): ("project.hip",), ("project_bwd", "bf16"): ("project.hip",),
}


def kernel_src_digest(kernel: str, form: str) -> str:
    """Digest of the sources of one bracket's kernels (all kernel sources when
    the bracket has no entry)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_19154_amd", "csrc")
    files = BRACKET_SOURCES.get((kernel, form))
    names = sorted(os.listdir(csrc)) if files is None else sorted(("common.hpp", "kernels.hpp") + files)
    for f in names:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


# the kernels each event bracket of the C ABI launches (base names), for the
# brackets whose kernels no other bracket launches
BRACKET_KERNELS = {
    ("project", "f32"): ("k_project",), ("project", "bf16"): ("k_project",),
    ("render_fwd", "f32"): ("k_render_fwd_f32",), ("render_fwd", "bf16"): ("k_render_fwd_bf16",),
    ("render_bwd", "f32"): ("k_visit_stage", "k_render_bwd_f32"),
    ("render_bwd", "bf16"): ("k_visit_stage", "k_render_bwd_bf16", "k_fuse_bf16", "k_fuse_rec_bf16", "k_gk_bf16"),
    ("project_bwd", "f32"): ("k_project_bwd",), ("project_bwd", "bf16"): ("k_project_bwd",),
}
COPY_BYTES = 1 << 30       # the calibration kernel reads and writes this many bytes


def _short_name(kname: str) -> str:
    n = kname.split("(")[0]
    n = n.replace("void ", "").strip()
    return n.split("::")[-1]


def _counter_rows(path: str):
    import csv
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            yield row


def traffic_from(fetch_csv: str, write_csv: str, kernel: str, workload: str, form: str, command: str):
    """HBM bytes per launch of the `kernel` bracket from two rocprofv3 --pmc runs,
    each counter scaled by what it reads for the 1 GiB calibration copy."""
    if (kernel, form) not in BRACKET_KERNELS:
        raise SystemExit(f"no counter attribution for the {kernel} bracket")
    pats = BRACKET_KERNELS[(kernel, form)]
    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per_kernel: dict[str, list[float]] = {}
        calib = []
        for row in _counter_rows(path):
            if row.get("Counter_Name") != counter:
                continue
            name = _short_name(row["Kernel_Name"])
            val = float(row["Counter_Value"])
            if "neg_kernel" in row["Kernel_Name"] or "neg" == name:
                calib.append(val)
            elif name.split("<")[0] in pats:
                per_kernel.setdefault(name, []).append(val)
        if not calib:
            raise SystemExit(f"{path}: no calibration copy kernel found")
        # the largest neg dispatch is the 1 GiB copy
        kib = max(calib)
        scale = COPY_BYTES / (kib * 1024.0)
        launch_kib = sum(sum(v) / len(v) for v in per_kernel.values())
        out[counter] = dict(calibration_kib=kib, scale=scale, kib_per_launch=launch_kib,
                            per_kernel={k: sum(v) / len(v) for k, v in per_kernel.items()},
                            dispatches={k: len(v) for k, v in per_kernel.items()})
    hbm = sum(out[c]["kib_per_launch"] * 1024.0 * out[c]["scale"] for c in out)
    res = dict(kernel=kernel, workload=workload, form=form, kernel_src_digest=kernel_src_digest(kernel, form),
               hbm_bytes_per_launch=hbm, counters=out, command=command,
               note="FETCH_SIZE and WRITE_SIZE from separate rocprofv3 --pmc runs, KiB per dispatch averaged over "
                    "dispatches and summed over the kernels of the bracket; each scaled by calibration bytes / "
                    "counter bytes of a plain copy (torch.neg) of 1 GiB in, 1 GiB out")
    path = os.path.join(PROFILES, f"traffic_{kernel}_{workload}_{form}.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(dict(path=path, hbm_bytes_per_launch=hbm)))


def measured_traffic(kernel: str, workload: str, form: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it is
    for the current kernel sources; else None."""
    path = os.path.join(PROFILES, f"traffic_{kernel}_{workload}_{form}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_src_digest") != kernel_src_digest(kernel, form):
        return None
    return float(t["hbm_bytes_per_launch"])


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _ranges(cpus) -> str:
    cpus = sorted(cpus)
    out, i = [], 0
    while i < len(cpus):
        j = i
        while j + 1 < len(cpus) and cpus[j + 1] == cpus[j] + 1:
            j += 1
        out.append(str(cpus[i]) if i == j else f"{cpus[i]}-{cpus[j]}")
        i = j + 1
    return ",".join(out)


def cpu_baseline(g, cams, vts, wl, target_seconds: float):
    """The FP64 oracle on a random sample of tiles (fwd + bwd + fusion), with the
    O(N) stages (binning, projection, projection adjoint) run in full; on all
    the threads OpenMP takes, then on one thread (a smaller sample)."""
    import numpy as np

    from oracle import binspec, pipeline, project, raster

    cam = cams[0]
    feat = np.asarray(g["feat"], np.float64)
    vt = vts[0]
    dC = np.asarray(vt["dC"], np.float64)
    dF = np.asarray(vt["dF"], np.float64)
    dT = np.asarray(vt["dT"], np.float64)
    tgt = np.asarray(vt["target"], np.float64) if wl.fusion else None
    t0 = time.perf_counter()
    bins = binspec.bin_views(g, [cam])
    t1 = time.perf_counter()
    pr = project.project(g, cam)
    t2 = time.perf_counter()
    ntiles = int(bins["num_tiles"])
    rng = np.random.default_rng(7)
    perm = rng.permutation(ntiles)
    ranges = pipeline.view_slice(bins, 0, cam)

    def walk(sel):
        return raster.render_view(cam, ranges, bins["gids"], pr, feat=feat, dC=dC, dF=dF, dT=dT, target=tgt,
                                  tile_sel=sel, want_F=True, want_fusion=wl.fusion)

    def sampled(seconds, first):
        # calibrate on a few tiles, then size the sample to the time target
        tp0 = time.perf_counter()
        walk(perm[first:first + 8])
        per_tile = max((time.perf_counter() - tp0) / 8, 1e-4)
        k = int(min(ntiles - first, max(16, seconds / per_tile)))
        sel = perm[first:first + k]
        ta = time.perf_counter()
        out = walk(sel)
        return out, k, time.perf_counter() - ta

    threads = raster.num_threads()
    out, k, t_walk = sampled(target_seconds, 0)
    t4 = time.perf_counter()
    project.project_bwd(pr, pipeline._unpack(out["g2d"]))
    t5 = time.perf_counter()
    frac = k / ntiles
    t_on = (t1 - t0) + (t2 - t1) + (t5 - t4)        # the O(N) stages (numpy, one thread)
    t_equiv = t_on + t_walk / frac
    blends = float(out["counts"][0]) / frac
    raster.set_num_threads(1)
    try:
        out1, k1, t_walk1 = sampled(max(2.0, target_seconds / 4), 0)
    finally:
        raster.set_num_threads(threads)
    t_equiv1 = t_on + t_walk1 / (k1 / ntiles)
    blends1 = float(out1["counts"][0]) / (k1 / ntiles)
    try:
        aff = _ranges(os.sched_getaffinity(0))
    except AttributeError:
        aff = "unknown"
    return dict(value=blends / t_equiv, unit="Gaussian-pixel blends/s", cores=threads, kind="oracle",
                sample=(f"{k} of {ntiles} tiles (random, seed 7) composited fwd+bwd{'+fusion' if wl.fusion else ''} "
                        f"in FP64 on {threads} threads ({t_walk:.1f} s), scaled by the tile fraction; binning "
                        f"{t1 - t0:.1f} s, projection {t2 - t1:.1f} s and its adjoint {t5 - t4:.1f} s run on all "
                        f"Gaussians"),
                ms_per_view=1000.0 * t_equiv, cpu_model=_cpu_model(), nproc=os.cpu_count(), affinity=aff,
                one_core=dict(value=blends1 / t_equiv1, ms_per_view=1000.0 * t_equiv1,
                              sample=f"{k1} of {ntiles} tiles on 1 thread ({t_walk1:.1f} s), same O(N) stages"))


DEVICE_MAPS_ABOVE = 4_000_000      # pixels: per-view maps drawn on the device beyond this


def load_workload(wl, dev):
    """Gaussians, cameras and per-view maps of a workload, resident on `dev`.
    Small workloads draw their maps on the host (the CPU baseline reads them);
    the batched ones draw them on the device (scenegen.make_view_tensors_device)."""
    import numpy as np
    import torch

    import scenegen
    from paper_2505_19154_amd.raster import Gaussians

    g = scenegen.make_gaussians(wl.n, wl.half_extent, wl.sh_degree, wl.d, seed=0, feat_dtype=wl.feat_dtype)
    cams = scenegen.make_cameras(wl.views)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    feat = (torch.from_numpy(g["feat_bits"].view(np.int16)).to(dev).view(torch.bfloat16) if wl.feat_dtype == "bf16"
            else t(g["feat"]))
    dg = Gaussians(t(g["means"]), t(g["scales"]), t(g["quats"]), t(g["opacity"]), t(g["sh"]), feat, wl.sh_degree)
    P = sum(c.npix for c in cams)
    tdt = wl.feat_dtype
    vts = None
    if P <= DEVICE_MAPS_ABOVE:
        vts = [scenegen.make_view_tensors(i, c.npix, wl.d, with_dT=False, target_dtype=tdt) for i, c in enumerate(cams)]
        cat = lambda k: np.concatenate([v[k] for v in vts])
        dC, dF, dT = t(cat("dC")), t(cat("dF")), t(cat("dT"))
        target = None
        if wl.fusion:
            target = (torch.from_numpy(cat("target_bits").view(np.int16)).to(dev).view(torch.bfloat16)
                      if tdt == "bf16" else t(cat("target")))
    else:
        dC = torch.empty(P, 3, device=dev)
        dF = torch.empty(P, wl.d, device=dev)
        dT = torch.empty(P, device=dev)
        target = torch.empty(P, wl.d, device=dev, dtype=torch.bfloat16 if tdt == "bf16" else torch.float32)
        off = 0
        for i, c in enumerate(cams):
            m = scenegen.make_view_tensors_device(i, c.npix, wl.d, dev, with_dT=False, target_dtype=tdt)
            for dst, k in ((dC, "dC"), (dF, "dF"), (dT, "dT"), (target, "target")):
                dst[off:off + c.npix] = m[k]
            del m
            off += c.npix
        if not wl.fusion:
            target = None
    return dict(wl=wl, g=g, cams=cams, dg=dg, vts=vts, dC=dC, dF=dF, dT=dT, target=target)


KERNEL_IDS = None


def run_form(W, form_name: str, kernel: str, args, dev, graph: bool = False, primitive: str = "gaussian"):
    """Warm up, then time K steps of one arithmetic form.  The chosen kernel is
    bracketed by HIP events on its own stream over K eager steps.  With graph,
    the step is captured in one HIP graph and the K timed steps are replays.
    primitive: "gaussian" or "surfel" (the workload's parameters taken as
    surfels: scales[:, 0:2] the planar scales)."""
    import torch

    from paper_2505_19154_amd import _lib as L
    from paper_2505_19154_amd.raster import FusionAcc, Rasterizer

    kid = {"project": L.FH_K_PROJECT, "bin": L.FH_K_BIN, "render_fwd": L.FH_K_RENDER_FWD,
           "render_bwd": L.FH_K_RENDER_BWD, "reduce": L.FH_K_REDUCE, "project_bwd": L.FH_K_PROJECT_BWD}
    wl, cams, dg = W["wl"], W["cams"], W["dg"]
    dC, dF, dT, target = W["dC"], W["dF"], W["dT"], W["target"]
    tag = f"[bench] {wl.name} {form_name}" + ("" if primitive == "gaussian" else f" {primitive}")
    r = Rasterizer(cams, wl.n, wl.sh_degree, wl.d, feat_dtype=wl.feat_dtype, form=form_name, device=dev,
                   primitive=primitive)
    img = r.forward(dg, margin=1.02)
    tuning = r.autotune(dg, img, dC, dF, dT, target=target, reps=2) if args.autotune else None
    acc = FusionAcc.zeros(wl.n, wl.d, dev) if wl.fusion else None
    grads = r.new_grads()

    def step():
        r.project(dg)
        r.bin_sort()
        r.render_fwd(dg, img)
        r.render_bwd(dg, img, dC, dF, dT, target=target, acc=acc, grads=grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    c = r.counters()
    if c.inst_overflow or c.visit_overflow:
        raise RuntimeError("capacity overflow during warm-up")
    print(f"{tag}: warm-up done, {c.n_instances} instances, {c.n_visited} visited", file=sys.stderr, flush=True)
    K = args.steps
    ks = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ke = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for e in ks + ke:
        e.record()
    torch.cuda.synchronize()
    arr_s = (ctypes.c_void_p * K)(*[e._as_parameter_ for e in ks])
    arr_e = (ctypes.c_void_p * K)(*[e._as_parameter_ for e in ke])
    L.check(r.lib.fh_set_kernel_events(kid[kernel], arr_s, arr_e, K), "fh_set_kernel_events")
    def timed(fn):
        """K calls of fn between K + 1 events: (mean, median) ms per call."""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(K):
            fn()
            ev[i + 1].record()
        torch.cuda.synchronize()
        per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(K))
        return ev[0].elapsed_time(ev[K]) / K, per[K // 2] if K % 2 else 0.5 * (per[K // 2 - 1] + per[K // 2])

    eager_ms, eager_med = timed(step)
    L.check(r.lib.fh_set_kernel_events(kid[kernel], None, None, 0), "fh_set_kernel_events")
    kms = sum(a.elapsed_time(b) for a, b in zip(ks, ke)) / K
    ms, med = eager_ms, eager_med
    if graph:
        g_obj, grads = r.capture_step(dg, img, dC, dF, dT, target=target, acc=acc, grads=grads)
        for _ in range(args.warmup):
            g_obj.replay()
        ms, med = timed(g_obj.replay)
    c = r.counters()
    if c.inst_overflow or c.visit_overflow:
        raise RuntimeError("capacity overflow during the timed steps")
    blends = int(img.n_iter.to(torch.int64).sum().item())
    print(f"{tag}: {ms:.3f} ms/step{' (graph replay; eager %.3f)' % eager_ms if graph else ''}, "
          f"{kernel} {kms:.3f} ms", file=sys.stderr, flush=True)
    return dict(r=r, img=img, c=c, ms=ms, median_ms=med, eager_ms=eager_ms, kms=kms, blends=blends,
                tuning=tuning or r.tuning_dict())


def visible_count(r, wl, n_views) -> int:
    import torch
    return int((r.ws_view("depth_key", torch.int32, wl.n * n_views) != -1).sum().item())


def batched_leg(args, dev):
    """Both arithmetic forms of a batched workload, each step one graph replay."""
    import torch

    import scenegen
    wl = scenegen.WORKLOADS[args.batched]
    print(f"[bench] batched workload {wl.name}: {wl.description}", file=sys.stderr, flush=True)
    W = load_workload(wl, dev)
    feat_b = 2 if wl.feat_dtype == "bf16" else 4
    out = dict(workload=f"{wl.name}: {wl.description}", views=len(W["cams"]),
               pixels=sum(c.npix for c in W["cams"]), graph_replay=True, forms={})
    for form_name in ("f32", "bf16"):
        res = run_form(W, form_name, args.kernel, args, dev, graph=True)
        n_vis = visible_count(res["r"], wl, len(W["cams"]))
        ab, per_unit = alg_bytes(args.kernel, wl, res["r"].n_pixels, n_vis, int(res["c"].n_instances), feat_b, feat_b)
        achieved = ab / (res["kms"] * 1e-3) / 1e9
        out["forms"][form_name] = dict(
            ms_per_step=res["ms"], ms_per_step_median=res["median_ms"], ms_per_view=res["ms"] / len(W["cams"]),
            eager_ms_per_step=res["eager_ms"],
            blends=res["blends"], blends_per_s=res["blends"] / (res["ms"] * 1e-3),
            instances=int(res["c"].n_instances), visited_instances=int(res["c"].n_visited), visible_gaussians=n_vis,
            tuning=res["tuning"],
            roofline=dict(kernel=args.kernel, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=achieved / HBM_PEAK_GBS, kernel_ms=res["kms"], algorithmic_bytes=ab,
                          per_unit=per_unit))
        del res
        torch.cuda.empty_cache()
    out["bf16_speedup_over_f32"] = out["forms"]["f32"]["ms_per_step"] / out["forms"]["bf16"]["ms_per_step"]
    del W
    torch.cuda.empty_cache()
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0


def _event_ms(fn, K):
    """Mean ms of K calls of fn between two events on the current stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(K):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / K


def extras_leg(W, args, dev):
    """The NDFD branch (Section 3.3) and the training-step kernels (Algorithm 1)
    on the headline workload, BF16 form.  NDFD: the losses alone
    (fh_ndfd_losses) and the backward with the NDFD gradient joined, the NDFD
    kernel bracketed by HIP events on its stream; roofline against the BF16
    MFMA peak with the algorithmic flops 10 D per walked (pixel, position) for
    the gradient launch (phi, x, the running F, y, the running sigma-weighted
    suffix) and 6 D for the losses; the gradient launch also records two floats
    per (position, pixel) in its forward sweep and reads them back.  Training: Adam over the raw parameters,
    the photometric loss, and one whole training step (render, loss, adjoint,
    densification statistics, Adam) with HBM rooflines for the elementwise
    kernels."""
    import torch

    from paper_2505_19154_amd import _lib as L
    from paper_2505_19154_amd import train as T
    from paper_2505_19154_amd.raster import Rasterizer

    wl, cams, dg = W["wl"], W["cams"], W["dg"]
    K = args.steps
    out = {}
    r = Rasterizer(cams, wl.n, wl.sh_degree, wl.d, feat_dtype=wl.feat_dtype, form="bf16", device=dev, ndfd=True)
    img = r.forward(dg, margin=1.02)
    blends = int(img.n_iter.to(torch.int64).sum().item())
    P = r.n_pixels
    gt = W["target"]                      # a BF16 [P, D] map stands in for F_gt
    a = torch.full((P,), 1.0 / P, device=dev)
    b = torch.full((P,), 0.1 / P, device=dev)
    nd = dict(gt=gt, a=a, b=b, lam=0.5, k=20.0)
    grads = r.new_grads()
    for _ in range(args.warmup):
        r.ndfd_losses(dg, img, gt)
        r.render_bwd(dg, img, W["dC"], W["dF"], None, grads=grads, ndfd=nd)
    ms_loss = _event_ms(lambda: r.ndfd_losses(dg, img, gt), K)
    ks = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ke = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for e in ks + ke:
        e.record()
    torch.cuda.synchronize()
    arr_s = (ctypes.c_void_p * K)(*[e._as_parameter_ for e in ks])
    arr_e = (ctypes.c_void_p * K)(*[e._as_parameter_ for e in ke])
    L.check(r.lib.fh_set_kernel_events(L.FH_K_NDFD, arr_s, arr_e, K), "fh_set_kernel_events")
    ms_bwd_ndfd = _event_ms(lambda: r.render_bwd(dg, img, W["dC"], W["dF"], None, grads=grads, ndfd=nd), K)
    L.check(r.lib.fh_set_kernel_events(L.FH_K_NDFD, None, None, 0), "fh_set_kernel_events")
    kms = sum(x.elapsed_time(y) for x, y in zip(ks, ke)) / K
    ms_bwd = _event_ms(lambda: r.render_bwd(dg, img, W["dC"], W["dF"], None, grads=grads), K)
    flops = 10.0 * wl.d * blends
    ach = flops / (kms * 1e-3) / 1e12
    out["ndfd"] = dict(
        losses_ms=ms_loss, render_bwd_with_ndfd_ms=ms_bwd_ndfd, render_bwd_ms=ms_bwd, ndfd_kernel_ms=kms,
        walked_positions=blends,
        roofline=dict(kernel="k_ndfd (gradient)", bound="mfma", achieved=ach, peak=MFMA_BF16_PEAK_TFLOPS,
                      unit="TFLOP/s", frac=ach / MFMA_BF16_PEAK_TFLOPS, algorithmic_flops=flops,
                      per_unit=f"10 D = {10 * wl.d} flops per walked (pixel, position)"))
    print(f"[bench] ndfd: losses {ms_loss:.3f} ms, kernel {kms:.3f} ms, backward {ms_bwd:.3f} -> {ms_bwd_ndfd:.3f} ms",
          file=sys.stderr, flush=True)
    # training step kernels, on this workload's Gaussians as raw parameters
    p = T.Params(dg.means.clone(), torch.log(dg.scales), dg.quats.clone(),
                 torch.log(dg.opacity) - torch.log1p(-dg.opacity), dg.sh.clone())
    p = T.activate(p)
    m, v = T.Params.zeros_like(p), T.Params.zeros_like(p)
    lr = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, logit_opacity=5e-2, sh=2.5e-3)
    step = [0]

    def adam():
        step[0] += 1
        T.adam_step(p, m, v, grads, step[0], lr)

    for _ in range(args.warmup):
        adam()
    ms_adam = _event_ms(adam, K)
    nb = (wl.sh_degree + 1) ** 2
    per_g = (3 + 3 + 4 + 1 + 3 * nb) * 28 + 4 * 8
    adam_bytes = per_g * wl.n
    pl = T.PhotometricLoss(P, dev)
    target_img = img.C.flip(0).contiguous()
    dC = torch.empty_like(img.C)
    for _ in range(args.warmup):
        pl(img.C, target_img, dC)
    ms_pl = _event_ms(lambda: pl(img.C, target_img, dC), K)
    gsum = torch.zeros(wl.n, dtype=torch.float32, device=dev)
    cnt = torch.zeros(wl.n, dtype=torch.int32, device=dev)
    tr_grads = r.new_grads()

    def train_step():
        g = p.gaussians(dg.feat)
        r.project(g)
        r.bin_sort()
        r.render_fwd(g, img)
        pl(img.C, target_img, dC)
        r.render_bwd(g, img, dC, None, None, grads=tr_grads)
        T.densify_stats(r, gsum, cnt)
        step[0] += 1
        T.adam_step(p, m, v, tr_grads, step[0], lr)

    r.reserve(int(r.plan.inst_capacity) * 2, int(r.plan.visit_capacity) * 2)
    for _ in range(args.warmup):
        train_step()
    ms_train = _event_ms(train_step, K)
    c = r.counters()
    out["train"] = dict(
        adam_ms=ms_adam, photometric_loss_ms=ms_pl, step_ms=ms_train,
        step=("project, bin_sort, render_fwd, photometric loss, render_bwd, densification statistics, Adam "
              "(BF16 form, no fusion; capacities reserved at twice the first step's counts)"),
        step_overflow=bool(c.inst_overflow or c.visit_overflow),
        adam_roofline=dict(kernel="k_adam", bound="hbm", achieved=adam_bytes / (ms_adam * 1e-3) / 1e9,
                           peak=HBM_PEAK_GBS, unit="GB/s", frac=adam_bytes / (ms_adam * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           algorithmic_bytes=adam_bytes,
                           per_unit=f"{per_g} B per Gaussian (x, g, m, v read; x, m, v written; 59 floats; "
                                    f"activated scales and opacity read and written)"),
        loss_roofline=dict(kernel="k_loss_partial + k_loss_final", bound="hbm",
                           achieved=36.0 * P / (ms_pl * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                           frac=36.0 * P / (ms_pl * 1e-3) / 1e9 / HBM_PEAK_GBS, per_unit="36 B per pixel"))
    print(f"[bench] train: adam {ms_adam:.3f} ms, loss {ms_pl:.3f} ms, step {ms_train:.3f} ms",
          file=sys.stderr, flush=True)
    del r, img
    torch.cuda.empty_cache()
    out["surfel"] = surfel_leg(W, args, dev)
    return out


def surfel_leg(W, args, dev):
    """The surfel primitive (Section 3.1) on the headline workload: the same
    parameters taken as surfels (scales[:, 0:2] the planar scales), the whole
    step (project, bin_sort, render_fwd, render_bwd with fusion), autotuned,
    in both arithmetic forms.  The gradient launch's roofline counts the
    surfel record (64 B) and partial row (64 B) per visited Gaussian in place
    of the Gaussian's 48 B each."""
    import torch

    wl = W["wl"]
    out = {}
    for form in ("bf16", "f32"):
        res = run_form(W, form, "render_bwd", args, dev, primitive="surfel")
        n_vis = visible_count(res["r"], wl, len(W["cams"]))
        feat_b = 2 if wl.feat_dtype == "bf16" else 4
        ab, per_unit = alg_bytes("render_bwd", wl, res["r"].n_pixels, n_vis, int(res["c"].n_instances), feat_b,
                                 feat_b)
        ab += 32 * n_vis
        achieved = ab / (res["kms"] * 1e-3) / 1e9
        out[form] = dict(
            ms_per_step=res["ms"], ms_per_step_median=res["median_ms"], blends=res["blends"],
            blends_per_s=res["blends"] / (res["ms"] * 1e-3), instances=int(res["c"].n_instances),
            visited_instances=int(res["c"].n_visited), visible_surfels=n_vis, tuning=res["tuning"],
            roofline=dict(kernel="render_bwd", bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=achieved / HBM_PEAK_GBS, kernel_ms=res["kms"], algorithmic_bytes=ab,
                          per_unit=per_unit + " (+32 B per visible surfel: larger record and partial row)"))
        del res
        torch.cuda.empty_cache()
    out["bf16_speedup_over_f32"] = out["f32"]["ms_per_step"] / out["bf16"]["ms_per_step"]
    out["bf16"]["ndfd"] = _surfel_ndfd(W, args, dev)
    return out


def _surfel_ndfd(W, args, dev):
    """The NDFD branch (Section 3.3) along the surfel walk, BF16 form: the
    losses alone and the backward with the NDFD gradient joined, against the
    backward without it (the configuration the paper trains)."""
    import torch

    from paper_2505_19154_amd.raster import Rasterizer

    wl, cams, dg = W["wl"], W["cams"], W["dg"]
    K = args.steps
    r = Rasterizer(cams, wl.n, wl.sh_degree, wl.d, feat_dtype=wl.feat_dtype, form="bf16", device=dev, ndfd=True,
                   primitive="surfel")
    img = r.forward(dg, margin=1.02)
    P = r.n_pixels
    gt = W["target"]
    nd = dict(gt=gt, a=torch.full((P,), 1.0 / P, device=dev), b=torch.full((P,), 0.1 / P, device=dev),
              lam=0.5, k=20.0)
    grads = r.new_grads()
    for _ in range(args.warmup):
        r.ndfd_losses(dg, img, gt)
        r.render_bwd(dg, img, W["dC"], W["dF"], None, grads=grads, ndfd=nd)
    res = dict(losses_ms=_event_ms(lambda: r.ndfd_losses(dg, img, gt), K),
               render_bwd_with_ndfd_ms=_event_ms(
                   lambda: r.render_bwd(dg, img, W["dC"], W["dF"], None, grads=grads, ndfd=nd), K),
               render_bwd_ms=_event_ms(lambda: r.render_bwd(dg, img, W["dC"], W["dF"], None, grads=grads), K))
    print(f"[bench] surfel ndfd: losses {res['losses_ms']:.3f} ms, backward {res['render_bwd_ms']:.3f} -> "
          f"{res['render_bwd_with_ndfd_ms']:.3f} ms", file=sys.stderr, flush=True)
    del r, img
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.traffic_from:
        import scenegen
        wl = scenegen.WORKLOADS[args.workload]
        form = args.form if args.form != "auto" else ("bf16" if wl.feat_dtype == "bf16" else "f32")
        traffic_from(*args.traffic_from, args.kernel, wl.name, form, args.traffic_command)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus}: runs over several GPUs are not implemented",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import scenegen

    wl = scenegen.WORKLOADS[args.workload]
    mfma_ok = wl.feat_dtype == "bf16" and (wl.d in (32, 64, 96) or (wl.d > 0 and wl.d % 128 == 0))
    form = args.form if args.form != "auto" else ("bf16" if mfma_ok else "f32")
    print(f"[bench] workload {wl.name}: {wl.description}; form {form}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W = load_workload(wl, dev)
    cams = W["cams"]
    print("[bench] inputs resident on the GPU", file=sys.stderr, flush=True)
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        print(f"[bench] calibration copy of {COPY_BYTES} bytes done", file=sys.stderr, flush=True)

    other = {"bf16": "f32", "f32": "bf16"}[form]
    res_other = None
    if args.compare and (other == "f32" or wl.feat_dtype == "bf16"):
        res_other = run_form(W, other, args.kernel, args, dev)
        del res_other["r"], res_other["img"]
        torch.cuda.empty_cache()
    main_run = run_form(W, form, args.kernel, args, dev)
    r, img, c, ms, kms, blends = (main_run[k] for k in ("r", "img", "c", "ms", "kms", "blends"))
    n_vis = visible_count(r, wl, len(cams))
    feat_b = 2 if wl.feat_dtype == "bf16" else 4
    ab, per_unit = alg_bytes(args.kernel, wl, r.n_pixels, n_vis, int(c.n_instances), feat_b, feat_b)
    achieved = ab / (kms * 1e-3) / 1e9
    traffic = measured_traffic(args.kernel, wl.name, form)
    res = {
        "metric": METRIC,
        "value": blends / (ms * 1e-3),
        "unit": "Gaussian-pixel blends/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if form == "bf16" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: {wl.description}",
            "gaussians": wl.n, "views": len(cams), "resolution": f"{cams[0].width}x{cams[0].height}",
            "d": wl.d, "feat_storage": wl.feat_dtype, "form": form, "fusion": wl.fusion,
            "instances": int(c.n_instances), "visited_instances": int(c.n_visited), "visible_gaussians": n_vis,
            "blends": blends, "ms_per_view": ms / len(cams), "ms_per_step_median": main_run["median_ms"],
            "tuning": main_run["tuning"],
            "other_form": None if res_other is None else {
                "form": other, "ms_per_step": res_other["ms"], "ms_per_view": res_other["ms"] / len(cams),
                "blends_per_s": res_other["blends"] / (res_other["ms"] * 1e-3),
                f"{args.kernel}_ms": res_other["kms"], "tuning": res_other["tuning"]},
        },
        "roofline": {
            "kernel": args.kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel_ms": kms,
            "algorithmic_bytes": ab, "per_unit": per_unit,
        },
    }
    del main_run, r, img
    torch.cuda.empty_cache()
    if args.extras and wl.feat_dtype == "bf16" and wl.fusion:
        res["extras"] = extras_leg(W, args, dev)
    if not args.no_cpu_baseline and W["vts"] is not None:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(W["g"], cams, W["vts"], wl, args.cpu_seconds)
    else:
        res["cpu_baseline"] = None
    del W
    if args.batched:
        res["batched"] = batched_leg(args, dev)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
