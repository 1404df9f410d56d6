"""Python front end of the HIP rasterizer: device memory and streams from PyTorch,
every computation in libfhgs.so.

`Rasterizer` owns one plan (sizes, capacities, workspace layout) and its
workspace tensor for a fixed set of cameras, and exposes the C-ABI calls with
the same names: project, bin_sort, render_fwd, render_bwd, fuse_features,
fuse_finalize.  Capacities for the data-dependent instance and visit counts
grow on demand (eager use reads the device counters once per call); callers
that must not synchronise (graph capture, the benchmark's timed loop) fix the
capacities up front with `reserve` and check the counters afterwards.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import torch

from . import _lib as L

# indices of workspace sub-buffers (order of the WsBuf enum in csrc/common.hpp)
_WS = {name: i for i, name in enumerate(
    ["counters", "rec", "depth_key", "rect", "order", "order_tmp", "dkey_tmp", "dkey_tmp2", "inst_off",
     "scan_tmp", "hist", "ranges", "tile_niter", "tile_voff", "grad2d", "rank_of", "keys_a",
     "keys_b", "vals_a", "vals_b", "vseg", "part_geom", "part_fuse", "vkey_a", "vkey_b", "vval_a", "vval_b",
     "long", "vrec", "vgid", "rrec", "unit_owner", "upart", "part_ndfd", "ndfd_sc", "torder_ka", "torder_kb",
     "torder_va", "torder_vb", "wrec", "grec"])}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _same_device(a, b) -> bool:
    a, b = torch.device(a), torch.device(b)
    if a.type != b.type:
        return False
    if a.type != "cuda":
        return True
    cur = lambda d: d.index if d.index is not None else torch.cuda.current_device()
    return cur(a) == cur(b)


def check_tensor(t, name: str, shape: tuple, dtypes: tuple, device) -> None:
    """Raise FhError unless `t` can be handed to a kernel as `name`: a tensor on
    `device`, contiguous, of one of `dtypes`, of exactly `shape`, and with its
    data 16-byte aligned (the kernels index rows by the stated shape and load
    four floats at a time)."""
    if not isinstance(t, torch.Tensor):
        raise L.FhError(f"{name} must be a tensor")
    if not _same_device(t.device, device):
        raise L.FhError(f"{name} must be on {device}, not {t.device}")
    if t.dtype not in dtypes:
        raise L.FhError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)}, not {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise L.FhError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")
    if not t.is_contiguous():
        raise L.FhError(f"{name} must be contiguous")
    if t.numel() and t.data_ptr() % 16:
        raise L.FhError(f"{name} must be 16-byte aligned")


_F32 = (torch.float32,)


@dataclass
class Gaussians:
    """Device tensors of the Gaussians (activated parameters, see include/fhgs.h)."""
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opacity: torch.Tensor
    sh: torch.Tensor
    feat: torch.Tensor | None
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def d(self) -> int:
        return 0 if self.feat is None else int(self.feat.shape[1])

    @property
    def feat_dtype(self) -> int:
        return L.FH_BF16 if (self.feat is not None and self.feat.dtype == torch.bfloat16) else L.FH_F32

    def struct(self) -> L.FhGaussians:
        for name in ("means", "scales", "quats", "opacity", "sh"):
            t = getattr(self, name)
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise L.FhError(f"{name} must be a contiguous float32 CUDA tensor")
        if self.feat is not None and (not self.feat.is_contiguous() or self.feat.dtype not in (torch.float32, torch.bfloat16)):
            raise L.FhError("feat must be contiguous float32 or bfloat16")
        return L.FhGaussians(_ptr(self.means), _ptr(self.scales), _ptr(self.quats), _ptr(self.opacity),
                             _ptr(self.sh), _ptr(self.feat), self.n, self.sh_degree, self.d, self.feat_dtype, 0)


@dataclass
class Image:
    C: torch.Tensor
    F: torch.Tensor | None
    T: torch.Tensor
    n_iter: torch.Tensor

    def struct(self) -> L.FhImage:
        return L.FhImage(_ptr(self.C), _ptr(self.F), _ptr(self.T), _ptr(self.n_iter))


@dataclass
class FusionAcc:
    """Neumaier-compensated per-Gaussian fusion accumulators (running value = sum + comp)."""
    sum: torch.Tensor
    comp: torch.Tensor
    wsum: torch.Tensor
    wcomp: torch.Tensor

    @staticmethod
    def zeros(n: int, d: int, device) -> "FusionAcc":
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=device)
        return FusionAcc(z(n, d), z(n, d), z(n), z(n))

    def struct(self) -> L.FhFusion:
        return L.FhFusion(_ptr(self.sum), _ptr(self.comp), _ptr(self.wsum), _ptr(self.wcomp))


def camera_struct(cam) -> L.FhCamera:
    R = [float(x) for x in list(cam.R.reshape(-1))]
    t = [float(x) for x in list(cam.t.reshape(-1))]
    return L.FhCamera(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy),
                      (ctypes.c_float * 9)(*R), (ctypes.c_float * 3)(*t))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Rasterizer:
    """Plan + workspace for one batch of cameras and one Gaussian set size."""

    def __init__(self, cams, n: int, sh_degree: int, d: int, feat_dtype: str = "f32", form: str = "f32",
                 device="cuda", inst_capacity: int = 0, visit_capacity: int = 0, bin_rule: str = "box",
                 ndfd: bool = False, primitive: str = "gaussian"):
        self.lib = L.load()
        self.cams = list(cams)
        self.cam_arr = (L.FhCamera * len(self.cams))(*[camera_struct(c) for c in self.cams])
        self.n, self.sh_degree, self.d = int(n), int(sh_degree), int(d)
        self.feat_dtype = L.FH_BF16 if feat_dtype == "bf16" else L.FH_F32
        self.form = L.FH_FORM_BF16 if form == "bf16" else L.FH_FORM_F32
        if bin_rule not in ("box", "opacity"):
            raise L.FhError(f"bin_rule must be 'box' or 'opacity', not {bin_rule!r}")
        self.bin_rule = L.FH_BIN_OPACITY if bin_rule == "opacity" else L.FH_BIN_BOX
        self.ndfd = bool(ndfd)         # workspace storage for the NDFD gradient
        if primitive not in ("gaussian", "surfel"):
            raise L.FhError(f"primitive must be 'gaussian' or 'surfel', not {primitive!r}")
        # surfels (Section 3.1's planar primitives): no NDFD branch
        self.primitive = L.FH_PRIM_SURFEL if primitive == "surfel" else L.FH_PRIM_GAUSSIAN
        self.device = torch.device(device)
        self.plan = None
        self.ws = None
        self.tuning = None          # launch shape chosen by autotune (kept across re-plans)
        # bumped by every call that rewrites the forward state held in the
        # workspace (projection, binning, traversal lengths) or replaces the
        # workspace: a backward checks that its forward's state is still there
        self.generation = 0
        self._plan(inst_capacity, visit_capacity)

    # -- plan and workspace -------------------------------------------------
    def _plan(self, inst_cap: int, visit_cap: int) -> None:
        plan = L.FhPlan()
        L.check(self.lib.fh_plan_init(ctypes.byref(plan), self.n, self.sh_degree, self.d, self.feat_dtype, self.form,
                                      self.cam_arr, len(self.cams), int(inst_cap), int(visit_cap)), "fh_plan_init")
        if self.primitive != L.FH_PRIM_GAUSSIAN:
            L.check(self.lib.fh_plan_set_primitive(ctypes.byref(plan), self.primitive), "fh_plan_set_primitive")
        if self.tuning is not None:
            plan.tuning = self.tuning
        plan.bin_rule = self.bin_rule
        if self.ndfd:
            L.check(self.lib.fh_plan_set_ndfd(ctypes.byref(plan), 1), "fh_plan_set_ndfd")
        self.plan = plan
        self.ws = torch.empty(max(int(plan.ws_bytes), 256), dtype=torch.uint8, device=self.device)
        self.generation += 1

    def reserve(self, inst_capacity: int, visit_capacity: int) -> None:
        if inst_capacity != self.plan.inst_capacity or visit_capacity != self.plan.visit_capacity:
            self._plan(inst_capacity, visit_capacity)

    @property
    def n_pixels(self) -> int:
        return int(self.plan.n_pixels)

    @property
    def n_tiles(self) -> int:
        return int(self.plan.n_tiles)

    def ws_view(self, name: str, dtype, count: int) -> torch.Tensor:
        off = int(self.plan.off[_WS[name]])
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype)

    def counters(self) -> L.FhCounters:
        c = L.FhCounters()
        L.check(self.lib.fh_read_counters(ctypes.byref(self.plan), _ptr(self.ws), ctypes.byref(c), _stream()),
                "fh_read_counters")
        return c

    def status_async(self, out: torch.Tensor) -> None:
        """fh_get_status into `out` (int64 [4] on the device, the fh_counters
        layout: three int64 counts, then the two int32 overflow flags), on the
        current stream without synchronising."""
        check_tensor(out, "out", (4,), (torch.int64,), self.device)
        L.check(self.lib.fh_get_status(ctypes.byref(self.plan), _ptr(self.ws), _ptr(out), _stream()), "fh_get_status")

    # -- the C-ABI calls ----------------------------------------------------
    def _check_image(self, img: "Image", name: str) -> None:
        P, d, dev = self.n_pixels, self.d, self.device
        check_tensor(img.C, f"{name}.C", (P, 3), _F32, dev)
        check_tensor(img.T, f"{name}.T", (P,), _F32, dev)
        check_tensor(img.n_iter, f"{name}.n_iter", (P,), (torch.int32,), dev)
        if d:
            if img.F is None:
                raise L.FhError(f"{name}.F is required when d > 0")
            check_tensor(img.F, f"{name}.F", (P, d), _F32, dev)

    def _check_target(self, target) -> int:
        """The fusion target's dtype code; BF16 form: BF16 only (an MFMA operand)."""
        ok = (torch.bfloat16,) if self.form == L.FH_FORM_BF16 else (torch.float32, torch.bfloat16)
        check_tensor(target, "target", (self.n_pixels, self.d), ok, self.device)
        return L.FH_BF16 if target.dtype == torch.bfloat16 else L.FH_F32

    def _check_acc(self, acc: "FusionAcc") -> None:
        for nm in ("sum", "comp"):
            check_tensor(getattr(acc, nm), f"acc.{nm}", (self.n, self.d), _F32, self.device)
        for nm in ("wsum", "wcomp"):
            check_tensor(getattr(acc, nm), f"acc.{nm}", (self.n,), _F32, self.device)

    def _check_grads(self, grads: dict) -> None:
        n, nb = self.n, (self.sh_degree + 1) ** 2
        shapes = dict(means=(n, 3), scales=(n, 3), quats=(n, 4), opacity=(n,), sh=(n, nb, 3))
        for k, shp in shapes.items():
            check_tensor(grads[k], f"grads[{k!r}]", shp, _F32, self.device)

    def project(self, g: Gaussians) -> None:
        self.generation += 1
        gs = g.struct()
        L.check(self.lib.fh_project(ctypes.byref(self.plan), ctypes.byref(gs), _ptr(self.ws), _stream()), "fh_project")

    def bin_count(self) -> None:
        L.check(self.lib.fh_bin_count(ctypes.byref(self.plan), _ptr(self.ws), _stream()), "fh_bin_count")

    def bin_sort(self) -> None:
        self.generation += 1
        L.check(self.lib.fh_bin_sort(ctypes.byref(self.plan), _ptr(self.ws), _stream()), "fh_bin_sort")

    def bin_keys(self, n_inst: int):
        keys = torch.empty(n_inst, dtype=torch.int64, device=self.device)
        gids = torch.empty(n_inst, dtype=torch.int32, device=self.device)
        L.check(self.lib.fh_bin_keys(ctypes.byref(self.plan), _ptr(self.ws), _ptr(keys), _ptr(gids), n_inst,
                                     _stream()), "fh_bin_keys")
        return keys, gids

    def new_image(self) -> Image:
        P, d = self.n_pixels, self.d
        dev = self.device
        return Image(torch.empty(P, 3, dtype=torch.float32, device=dev),
                     torch.empty(P, d, dtype=torch.float32, device=dev) if d else None,
                     torch.empty(P, dtype=torch.float32, device=dev),
                     torch.empty(P, dtype=torch.int32, device=dev))

    def render_fwd(self, g: Gaussians, out: Image | None = None) -> Image:
        out = out or self.new_image()
        self._check_image(out, "out")
        self.generation += 1
        gs, im = g.struct(), out.struct()
        L.check(self.lib.fh_render_fwd(ctypes.byref(self.plan), ctypes.byref(gs), _ptr(self.ws), ctypes.byref(im),
                                       _stream()), "fh_render_fwd")
        return out

    def new_grads(self) -> dict:
        n, nb, dev = self.n, (self.sh_degree + 1) ** 2, self.device
        e = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)
        return dict(means=e(n, 3), scales=e(n, 3), quats=e(n, 4), opacity=e(n), sh=e(n, nb, 3))

    def _check_ndfd(self, g: Gaussians, gt) -> None:
        if g.feat is None or g.feat.dtype != torch.bfloat16:
            raise L.FhError("the NDFD branch needs BF16 features")
        check_tensor(gt, "gt", (self.n_pixels, self.d), (torch.bfloat16,), self.device)

    def ndfd_losses(self, g: Gaussians, fwd: Image, gt, lam: float = 0.5, k: float = 20.0):
        """(L_gt [P], L_cf [P]) of the NDFD branch for the ground-truth feature
        map gt [P, d] (BF16), after render_fwd of the same views."""
        self._check_image(fwd, "fwd")
        self._check_ndfd(g, gt)
        P, dev = self.n_pixels, self.device
        Lgt = torch.empty(P, dtype=torch.float32, device=dev)
        Lcf = torch.empty(P, dtype=torch.float32, device=dev)
        gs, im = g.struct(), fwd.struct()
        L.check(self.lib.fh_ndfd_losses(ctypes.byref(self.plan), ctypes.byref(gs), _ptr(self.ws), ctypes.byref(im),
                                        _ptr(gt), float(lam), float(k), _ptr(Lgt), _ptr(Lcf), _stream()),
                "fh_ndfd_losses")
        return Lgt, Lcf

    def render_bwd(self, g: Gaussians, fwd: Image, dC, dF=None, dT=None, target=None, acc: FusionAcc | None = None,
                   grads: dict | None = None, ndfd: dict | None = None) -> dict:
        """The adjoint (and fusion into acc when target is given).  ndfd
        (optional): dict(gt [P, d] BF16, a [P], b [P] (either may be None),
        lam, k, and optionally Lgt, Lcf [P] output tensors) adds the NDFD
        branch's gradient of sum_p (a L_gt + b L_cf) and writes its losses."""
        grads = grads or self.new_grads()
        P, d, dev = self.n_pixels, self.d, self.device
        self._check_image(fwd, "fwd")
        check_tensor(dC, "dC", (P, 3), _F32, dev)
        if dF is not None and d:
            check_tensor(dF, "dF", (P, d), _F32, dev)
        if dT is not None:
            check_tensor(dT, "dT", (P,), _F32, dev)
        self._check_grads(grads)
        tdt = L.FH_F32
        if target is not None:
            if acc is None:
                raise L.FhError("fusion needs an accumulator (acc)")
            tdt = self._check_target(target)
            self._check_acc(acc)
        gs, im = g.struct(), fwd.struct()
        up = L.FhUpstream(_ptr(dC), _ptr(dF), _ptr(dT))
        if ndfd is not None:
            if not self.ndfd:
                raise L.FhError("the NDFD gradient needs a Rasterizer made with ndfd=True (workspace storage)")
            self._check_ndfd(g, ndfd["gt"])
            for nm in ("a", "b", "Lgt", "Lcf"):
                if ndfd.get(nm) is not None:
                    check_tensor(ndfd[nm], f"ndfd[{nm!r}]", (P,), _F32, dev)
            up.ndfd_gt, up.ndfd_a, up.ndfd_b = _ptr(ndfd["gt"]), _ptr(ndfd.get("a")), _ptr(ndfd.get("b"))
            up.ndfd_Lgt, up.ndfd_Lcf = _ptr(ndfd.get("Lgt")), _ptr(ndfd.get("Lcf"))
            up.ndfd_lambda, up.ndfd_k = float(ndfd.get("lam", 0.5)), float(ndfd.get("k", 20.0))
        gr = L.FhGrads(_ptr(grads["means"]), _ptr(grads["scales"]), _ptr(grads["quats"]), _ptr(grads["opacity"]),
                       _ptr(grads["sh"]))
        fu = acc.struct() if (acc is not None and target is not None) else None
        L.check(self.lib.fh_render_bwd(ctypes.byref(self.plan), ctypes.byref(gs), _ptr(self.ws), ctypes.byref(im),
                                       ctypes.byref(up), _ptr(target), tdt,
                                       ctypes.byref(fu) if fu is not None else None, ctypes.byref(gr), _stream()),
                "fh_render_bwd")
        return grads

    def fuse_features(self, g: Gaussians, fwd: Image, target: torch.Tensor, acc: FusionAcc) -> None:
        self._check_image(fwd, "fwd")
        tdt = self._check_target(target)
        self._check_acc(acc)
        gs, im, fu = g.struct(), fwd.struct(), acc.struct()
        L.check(self.lib.fh_fuse_features(ctypes.byref(self.plan), ctypes.byref(gs), _ptr(self.ws), ctypes.byref(im),
                                          _ptr(target), tdt, ctypes.byref(fu), _stream()), "fh_fuse_features")

    # -- eager helpers with capacity management ------------------------------
    def prepare(self, g: Gaussians, margin: float = 1.05) -> L.FhCounters:
        """project + bin_sort, growing the instance capacity until it fits."""
        if self.plan.inst_capacity <= 0:
            self.project(g)
            self.bin_count()
            c = self.counters()
            self._plan(max(int(c.n_instances * margin) + 1024, 1024), self.plan.visit_capacity)
        while True:
            self.project(g)
            self.bin_sort()
            c = self.counters()
            if not c.inst_overflow:
                return c
            self._plan(int(c.n_instances * margin) + 1024, self.plan.visit_capacity)

    def capture_step(self, g: Gaussians, img: Image, dC, dF=None, dT=None, target=None,
                     acc: FusionAcc | None = None, grads: dict | None = None):
        """Capture project -> bin_sort -> render_fwd -> render_bwd (+ fusion) into
        a HIP graph on the current capacities (call `forward` or `reserve` first).
        Returns (graph, grads); graph.replay() re-runs the whole step without host
        synchronisation or launch overhead.  Overflow is checked afterwards with
        `counters()`."""
        grads = grads or self.new_grads()
        self.generation += 1
        graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            # one eager pass on the capture stream first (allocator and code objects)
            self.project(g)
            self.bin_sort()
            self.render_fwd(g, img)
            self.render_bwd(g, img, dC, dF, dT, grads=grads)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            self.project(g)
            self.bin_sort()
            self.render_fwd(g, img)
            self.render_bwd(g, img, dC, dF, dT, target=target, acc=acc, grads=grads)
        return graph, grads

    def tuning_key(self) -> str:
        """Autotune cache key: device arch, arithmetic form, feature width and
        dtype, view count, and power-of-two classes of pixels and Gaussians."""
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        return (f"{arch}|form{self.form}|d{self.d}|feat{self.feat_dtype}|bin{self.bin_rule}|views{len(self.cams)}|"
                f"px2^{max(self.n_pixels, 1).bit_length()}|n2^{max(self.n, 1).bit_length()}")

    def autotune(self, g: Gaussians, img: Image, dC=None, dF=None, dT=None, target=None, reps: int = 3,
                 cache: str | None = None) -> dict:
        """Choose the launch shape (fh_tuning) for this workload: from `cache`
        (a JSON file) when it holds this tuning_key, else by timing every
        candidate with fh_autotune (after `forward`, with the step's real
        inputs; outputs are recomputed, fusion goes to a scratch accumulator).
        Returns the chosen {"fwd_slice", "bwd_chunk", "fwd_rows", "schedule"}."""
        import json
        import os
        key = self.tuning_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            t = L.FhTuning(int(table[key]["fwd_slice"]), int(table[key]["bwd_chunk"]), int(table[key]["fwd_rows"]),
                           int(table[key].get("schedule", 0)))
        else:
            self.generation += 1
            gs, im = g.struct(), img.struct()
            up = L.FhUpstream(_ptr(dC), _ptr(dF), _ptr(dT)) if dC is not None else None
            grads = self.new_grads() if dC is not None else None
            gr = (L.FhGrads(_ptr(grads["means"]), _ptr(grads["scales"]), _ptr(grads["quats"]),
                            _ptr(grads["opacity"]), _ptr(grads["sh"])) if grads is not None else None)
            acc = FusionAcc.zeros(self.n, self.d, self.device) if (target is not None and dC is not None) else None
            fu = acc.struct() if acc is not None else None
            tdt = L.FH_BF16 if (target is not None and target.dtype == torch.bfloat16) else L.FH_F32
            L.check(self.lib.fh_autotune(ctypes.byref(self.plan), ctypes.byref(gs), _ptr(self.ws), ctypes.byref(im),
                                         ctypes.byref(up) if up is not None else None,
                                         _ptr(target) if acc is not None else None, tdt,
                                         ctypes.byref(fu) if fu is not None else None,
                                         ctypes.byref(gr) if gr is not None else None, int(reps), _stream()),
                    "fh_autotune")
            t = self.plan.tuning
            if cache:
                table[key] = {"fwd_slice": int(t.fwd_slice), "bwd_chunk": int(t.bwd_chunk), "fwd_rows": int(t.fwd_rows),
                              "schedule": int(t.schedule)}
                os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
                with open(cache, "w") as f:
                    json.dump(table, f, indent=1, sort_keys=True)
        self.tuning = L.FhTuning(int(t.fwd_slice), int(t.bwd_chunk), int(t.fwd_rows), int(t.schedule))
        self.plan.tuning = self.tuning
        return self.tuning_dict()

    def tuning_dict(self) -> dict:
        t = self.plan.tuning
        return {"fwd_slice": int(t.fwd_slice), "bwd_chunk": int(t.bwd_chunk), "fwd_rows": int(t.fwd_rows),
                "schedule": int(t.schedule)}

    def set_tuning(self, fwd_slice: int, bwd_chunk: int, fwd_rows: int = 16, schedule: int = 0) -> None:
        """Set the launch shape by hand (validated by the next call)."""
        self.tuning = L.FhTuning(int(fwd_slice), int(bwd_chunk), int(fwd_rows), int(schedule))
        self.plan.tuning = self.tuning

    def tuning_candidates(self, which: int) -> list:
        """[(fwd_slice, bwd_chunk, fwd_rows, schedule), ...] for kernel `which`."""
        out = (L.FhTuning * 32)()
        n = ctypes.c_int32()
        L.check(self.lib.fh_tuning_candidates(ctypes.byref(self.plan), int(which), out, 32, ctypes.byref(n)),
                "fh_tuning_candidates")
        return [(int(out[i].fwd_slice), int(out[i].bwd_chunk), int(out[i].fwd_rows), int(out[i].schedule))
                for i in range(n.value)]

    def forward(self, g: Gaussians, margin: float = 1.05) -> Image:
        """prepare + render_fwd, growing the visit capacity until it fits."""
        self.prepare(g, margin)
        while True:
            img = self.render_fwd(g)
            c = self.counters()
            if not c.visit_overflow and self.plan.visit_capacity > 0:
                return img
            self._plan(self.plan.inst_capacity, max(int(c.n_visited * margin) + 1024, 1024))
            self.prepare(g, margin)


def fuse_finalize(acc: FusionAcc, feat_in: torch.Tensor | None, out_dtype=torch.float32) -> torch.Tensor:
    lib = L.load()
    if out_dtype not in (torch.float32, torch.bfloat16):
        raise L.FhError("out_dtype must be float32 or bfloat16")
    n, d = acc.sum.shape
    dev = acc.sum.device
    for nm, shp in (("sum", (n, d)), ("comp", (n, d)), ("wsum", (n,)), ("wcomp", (n,))):
        check_tensor(getattr(acc, nm), f"acc.{nm}", shp, _F32, dev)
    out = torch.empty(n, d, dtype=out_dtype, device=dev)
    dt = L.FH_BF16 if out_dtype == torch.bfloat16 else L.FH_F32
    if feat_in is not None:
        check_tensor(feat_in, "feat_in", (n, d), (out_dtype,), dev)
    fu = acc.struct()
    L.check(lib.fh_fuse_finalize(ctypes.byref(fu), n, d, _ptr(feat_in), _ptr(out), dt, _stream()), "fh_fuse_finalize")
    return out
