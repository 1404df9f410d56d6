"""The C-ABI library loads and exports every entry point declared in include/fhgs.h,
and the ctypes mirror matches the header's struct layout.  CPU only: no compute call."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fhgs.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fh_[a-z_0-9]+)\s*\(", src, re.M)))


def test_header_declares_the_path():
    names = _declared()
    for need in ("fh_project", "fh_bin_sort", "fh_render_fwd", "fh_render_bwd", "fh_fuse_features",
                 "fh_fuse_finalize", "fh_plan_init"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2505_19154_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.SIGNATURES), "ctypes signature table out of sync with the header"
    assert lib.fh_version() == 1


def test_struct_layout_matches_header(tmp_path):
    from paper_2505_19154_amd import _lib
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "fhgs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(fh_plan), offsetof(fh_plan, cams),
         offsetof(fh_plan, off), offsetof(fh_plan, ws_bytes), sizeof(fh_camera), sizeof(fh_gaussians),
         sizeof(fh_counters), offsetof(fh_plan, tiles_x), offsetof(fh_plan, inst_capacity),
         offsetof(fh_plan, tuning), sizeof(fh_tuning), offsetof(fh_plan, bin_rule));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include", "-I/opt/rocm/include", str(prog), "-o",
                    str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    P = _lib.FhPlan
    want = [ctypes.sizeof(P), P.cams.offset, P.off.offset, P.ws_bytes.offset, ctypes.sizeof(_lib.FhCamera),
            ctypes.sizeof(_lib.FhGaussians), ctypes.sizeof(_lib.FhCounters), P.tiles_x.offset,
            P.inst_capacity.offset, P.tuning.offset, ctypes.sizeof(_lib.FhTuning), P.bin_rule.offset]
    assert got == want


def test_plan_init_validates_on_host():
    # fh_plan_init touches no device memory
    from paper_2505_19154_amd import _lib
    lib = _lib.load()
    cam = _lib.FhCamera(64, 48, 50.0, 50.0, 32.0, 24.0, (ctypes.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1),
                        (ctypes.c_float * 3)(0, 0, 4))
    cams = (_lib.FhCamera * 1)(cam)
    plan = _lib.FhPlan()
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 16, 0, 0, cams, 1, 5000, 1000) == 0
    assert plan.n_tiles == 4 * 3 and plan.n_pixels == 64 * 48 and plan.packed_keys == 1
    assert plan.ws_bytes > 0 and plan.bin_rule == _lib.FH_BIN_BOX
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 4, 16, 0, 0, cams, 1, 0, 0) == -2   # sh degree 4


def test_workspace_regions_lie_inside_the_workspace():
    # every sub-buffer offset is recorded (none dropped past the table's end),
    # ascending, aligned, and inside ws_bytes; the Python names cover them all
    from paper_2505_19154_amd import _lib, raster
    lib = _lib.load()
    cam = _lib.FhCamera(1920, 1080, 1000.0, 1000.0, 960.0, 540.0, (ctypes.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1),
                        (ctypes.c_float * 3)(0, 0, 4))
    cams = (_lib.FhCamera * 1)(cam)
    for d, form, feat in ((256, 1, 1), (64, 0, 0), (0, 0, 0)):
        plan = _lib.FhPlan()
        assert lib.fh_plan_init(ctypes.byref(plan), 500000, 3, d, feat, form, cams, 1, 23_000_000, 1_200_000) == 0
        n = plan.n_ws
        assert 0 < n <= _lib.FH_WS_SLOTS
        assert len(raster._WS) == n
        offs = [plan.off[i] for i in range(n)]
        assert offs[0] == 0
        assert all(o % 256 == 0 for o in offs)
        assert all(b >= a for a, b in zip(offs, offs[1:]))
        assert offs[-1] <= plan.ws_bytes
        # the unit partials (the last region) are sized for the unit bound at this visit capacity
        upart = plan.ws_bytes - offs[raster._WS["upart"]]
        assert upart >= (1_200_000 * 3 // 64 + 1) * (2 * d + 2) * 4
    assert lib.fh_plan_init(ctypes.byref(plan), -1, 3, 16, 0, 0, cams, 1, 0, 0) == -1
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 16, 0, 1, cams, 1, 0, 0) == -2   # bf16 form, f32 feat
    assert lib.fh_status_string(-4) == b"capacity exceeded"


def test_tuning_defaults_and_candidates_on_host():
    from paper_2505_19154_amd import _lib
    lib = _lib.load()
    cam = _lib.FhCamera(64, 48, 50.0, 50.0, 32.0, 24.0, (ctypes.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1),
                        (ctypes.c_float * 3)(0, 0, 4))
    cams = (_lib.FhCamera * 1)(cam)

    def cands(plan, which):
        out = (_lib.FhTuning * 32)()
        n = ctypes.c_int32()
        assert lib.fh_tuning_candidates(ctypes.byref(plan), which, out, 32, ctypes.byref(n)) == 0
        return [(out[i].fwd_slice, out[i].bwd_chunk, out[i].fwd_rows) + ((out[i].schedule,) if out[i].schedule else ())
                for i in range(n.value)]

    plan = _lib.FhPlan()
    # FP32 form, d = 256, BF16-stored features: the VALU forward's slices 8..64,
    # backward chunks 16 and 32
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 256, 1, 0, cams, 1, 0, 0) == 0
    assert (plan.tuning.fwd_slice, plan.tuning.bwd_chunk, plan.tuning.fwd_rows) == (64, 32, 16)
    assert cands(plan, _lib.FH_K_RENDER_FWD) == [(8, 32, 16), (16, 32, 16), (32, 32, 16), (64, 32, 16)]
    assert cands(plan, _lib.FH_K_RENDER_BWD) == [(64, 16, 16), (64, 32, 16)]
    assert cands(plan, _lib.FH_K_PROJECT) == [(64, 32, 16)]
    # FP32 form, d = 256, FP32 features: the MFMA forward's shapes (without 16
    # rows of 128 channels)
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 256, 0, 0, cams, 1, 0, 0) == 0
    assert (plan.tuning.fwd_slice, plan.tuning.bwd_chunk, plan.tuning.fwd_rows) == (256, 32, 8)
    mf = [(32, 32, 16), (64, 32, 16), (64, 32, 8), (128, 32, 8), (256, 32, 8)]
    # (the MFMA forward in both work orders: tile index order, longest first)
    assert cands(plan, _lib.FH_K_RENDER_FWD) == mf + [c + (1,) for c in mf]
    assert cands(plan, _lib.FH_K_RENDER_BWD) == [(256, 16, 8), (256, 32, 8)]
    # BF16 form, d = 256: slices dividing d for 16-, 8- and 4-row workgroups; one backward shape
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 256, 1, 1, cams, 1, 0, 0) == 0
    assert (plan.tuning.fwd_slice, plan.tuning.fwd_rows) == (256, 8)
    bf = [(32, 32, 16), (64, 32, 16), (128, 32, 16), (64, 32, 8), (128, 32, 8), (256, 32, 8), (128, 32, 4),
          (256, 32, 4)]
    assert cands(plan, _lib.FH_K_RENDER_FWD) == bf + [c + (1,) for c in bf]
    assert cands(plan, _lib.FH_K_RENDER_BWD) == [(256, 32, 8), (256, 32, 8, 1)]
    # BF16 form, d = 96; FP32 form, d = 16; d = 1024 takes 16-Gaussian chunks
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 96, 1, 1, cams, 1, 0, 0) == 0
    assert cands(plan, _lib.FH_K_RENDER_FWD) == [(32, 32, 16), (96, 32, 16), (32, 32, 16, 1), (96, 32, 16, 1)]
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 16, 0, 0, cams, 1, 0, 0) == 0
    assert cands(plan, _lib.FH_K_RENDER_FWD) == [(8, 32, 16), (16, 32, 16)]
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 1024, 0, 0, cams, 1, 0, 0) == 0
    assert plan.tuning.bwd_chunk == 16 and cands(plan, _lib.FH_K_RENDER_BWD) == [(256, 16, 8)]
    # FP32 form at a width the MFMA forward does not take (d = 40): the VALU forward's slices
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 40, 0, 0, cams, 1, 0, 0) == 0
    assert (plan.tuning.fwd_slice, plan.tuning.fwd_rows) == (64, 16)
    assert cands(plan, _lib.FH_K_RENDER_FWD) == [(8, 32, 16), (16, 32, 16), (32, 32, 16), (64, 32, 16)]


def test_plan_set_primitive_on_host():
    # surfels: records and partials grow the workspace
    from paper_2505_19154_amd import _lib
    lib = _lib.load()
    cam = _lib.FhCamera(64, 48, 50.0, 50.0, 32.0, 24.0, (ctypes.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1),
                        (ctypes.c_float * 3)(0, 0, 4))
    cams = (_lib.FhCamera * 1)(cam)
    plan = _lib.FhPlan()
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 256, 0, 0, cams, 1, 5000, 1000) == 0
    assert plan.primitive == _lib.FH_PRIM_GAUSSIAN
    ws_gauss = plan.ws_bytes
    assert lib.fh_plan_set_primitive(ctypes.byref(plan), _lib.FH_PRIM_SURFEL) == 0
    assert plan.primitive == _lib.FH_PRIM_SURFEL and plan.ws_bytes > ws_gauss
    # the surfel density runs on the VALU forward (slices of at most 64 channels)
    assert plan.tuning.fwd_slice <= 64
    assert lib.fh_plan_set_primitive(ctypes.byref(plan), 2) == -1
    assert lib.fh_plan_set_primitive(ctypes.byref(plan), _lib.FH_PRIM_GAUSSIAN) == 0
    assert plan.ws_bytes == ws_gauss and plan.tuning.fwd_slice == 256
    # the BF16-MFMA form: surfels take the MFMA forward's shapes
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 256, 1, 1, cams, 1, 5000, 1000) == 0
    assert lib.fh_plan_set_primitive(ctypes.byref(plan), _lib.FH_PRIM_SURFEL) == 0
    assert (plan.tuning.fwd_slice, plan.tuning.fwd_rows) == (256, 8)
    # the NDFD storage: surfel partials are 16 floats per (visit, half) instead of 8
    assert lib.fh_plan_init(ctypes.byref(plan), 100, 3, 256, 1, 0, cams, 1, 5000, 1000) == 0
    ws0 = plan.ws_bytes
    assert lib.fh_plan_set_ndfd(ctypes.byref(plan), 1) == 0
    nd_gauss = plan.ws_bytes - ws0
    assert lib.fh_plan_set_primitive(ctypes.byref(plan), _lib.FH_PRIM_SURFEL) == 0
    ws_nd_s = plan.ws_bytes
    assert lib.fh_plan_set_ndfd(ctypes.byref(plan), 0) == 0
    nd_surf = ws_nd_s - plan.ws_bytes
    assert abs((nd_surf - nd_gauss) - 1000 * 2 * 8 * 4) <= 256
