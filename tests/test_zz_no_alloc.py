"""fh_render_fwd_static (the entry point that allocates nothing: its workspace
is a static device array) against the calls with a caller workspace, through
the C ABI: two calls in a row on the same GPU, the second with a smaller
scene, each bit for bit equal to project + bin_sort + render_fwd of the same
plan with a workspace; the counters it exports; and the size check."""
import ctypes

import numpy as np
import pytest
import torch

import scenegen
from paper_2505_19154_amd import _lib as L
from paper_2505_19154_amd.raster import Rasterizer, _ptr, _stream
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

CASES = [
    # n, half extent, SH degree, d, feature dtype, form, (width, height), primitive
    (3000, 1.5, 2, 32, "bf16", "bf16", (120, 90), "gaussian"),
    (1200, 1.2, 1, 64, "bf16", "bf16", (96, 72), "surfel"),
    (600, 1.0, 0, 16, "f32", "f32", (50, 38), "gaussian"),
]


def _static_render(r: Rasterizer, dg):
    img = r.new_image()
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")      # fh_counters: 3 int64 + 2 int32
    gs, im = dg.struct(), img.struct()
    st = r.lib.fh_render_fwd_static(ctypes.byref(r.plan), ctypes.byref(gs), ctypes.byref(im), _ptr(cnt), _stream())
    L.check(st, "fh_render_fwd_static")
    torch.cuda.synchronize()
    return img, cnt.cpu().numpy()


def test_static_entry_point_equals_the_workspace_path_on_two_calls():
    for n, h, deg, d, fdt, form, (w, hh), prim in CASES:
        g = scenegen.make_gaussians(n, h, deg, d, seed=n, feat_dtype=fdt)
        if prim == "surfel":
            g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
        cams = [scenegen.look_at_camera((0.0, -4.0, 0.0), w, hh)]
        dg = U.device_gaussians(g)
        r = Rasterizer(cams, n, deg, d, feat_dtype=fdt, form=form, primitive=prim)
        ref = r.forward(dg)                      # caller workspace; sizes the capacities
        c_ref = r.counters()
        torch.cuda.synchronize()
        assert r.plan.ws_bytes <= L.FH_STATIC_SCRATCH_BYTES
        img, cnt = _static_render(r, dg)
        for k in ("C", "F", "T", "n_iter"):
            a, b = getattr(img, k), getattr(ref, k)
            if a is None:
                continue
            assert torch.equal(a, b), (n, k)
        assert int(cnt[0]) == c_ref.n_instances and int(cnt[1]) == c_ref.n_visited
        flags = cnt[3:4].view(np.int32)
        assert flags[0] == 0 and flags[1] == 0
        print(f"[no-alloc] n={n} {w}x{hh} {prim}: equal, {int(cnt[0])} instances", flush=True)


def test_static_entry_point_rejects_a_plan_beyond_the_scratch():
    g = scenegen.make_gaussians(100, 1.0, 0, 8, seed=1)
    cams = [scenegen.look_at_camera((0.0, -4.0, 0.0), 64, 64)]
    dg = U.device_gaussians(g)
    r = Rasterizer(cams, 100, 0, 8, inst_capacity=20_000_000, visit_capacity=1000)
    assert r.plan.ws_bytes > L.FH_STATIC_SCRATCH_BYTES
    img = r.new_image()
    gs, im = dg.struct(), img.struct()
    st = r.lib.fh_render_fwd_static(ctypes.byref(r.plan), ctypes.byref(gs), ctypes.byref(im), None, _stream())
    assert st == L.FH_E_SCRATCH
