"""ctypes mirror of include/fhgs.h and the loader of the in-tree libfhgs.so.

Argument marshalling only: every step of the path runs in the HIP library.
Importing this module on a machine without the built library raises at the
first call that needs it; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfhgs.so")

FH_MAX_VIEWS = 32
FH_WS_SLOTS = 48
FH_TILE = 16

FH_OK, FH_E_INVALID, FH_E_UNSUPPORTED, FH_E_HIP, FH_E_CAPACITY, FH_E_SCRATCH = 0, -1, -2, -3, -4, -5
FH_STATIC_SCRATCH_BYTES = 64 << 20
FH_F32, FH_BF16 = 0, 1
FH_FORM_F32, FH_FORM_BF16 = 0, 1
FH_BIN_BOX, FH_BIN_OPACITY = 0, 1
FH_PRIM_GAUSSIAN, FH_PRIM_SURFEL = 0, 1
(FH_K_PROJECT, FH_K_BIN, FH_K_RENDER_FWD, FH_K_RENDER_BWD, FH_K_REDUCE, FH_K_PROJECT_BWD, FH_K_NDFD) = range(7)
(FH_BUF_RECORDS, FH_BUF_DEPTH_KEY, FH_BUF_RECT, FH_BUF_DEPTH_ORDER, FH_BUF_RANGES,
 FH_BUF_TILE_NITER, FH_BUF_GRAD2D) = range(7)

_i32, _i64, _f32, _sz, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t, ctypes.c_void_p


class FhGaussians(ctypes.Structure):
    _fields_ = [("means", _vp), ("scales", _vp), ("quats", _vp), ("opacity", _vp), ("sh", _vp),
                ("feat", _vp), ("n", _i64), ("sh_degree", _i32), ("d", _i32), ("feat_dtype", _i32),
                ("reserved", _i32)]


class FhCamera(ctypes.Structure):
    _fields_ = [("width", _i32), ("height", _i32), ("fx", _f32), ("fy", _f32), ("cx", _f32), ("cy", _f32),
                ("R", _f32 * 9), ("t", _f32 * 3)]


class FhTuning(ctypes.Structure):
    _fields_ = [("fwd_slice", _i32), ("bwd_chunk", _i32), ("fwd_rows", _i32), ("schedule", _i32)]


class FhPlan(ctypes.Structure):
    _fields_ = [("n", _i64), ("n_views", _i32), ("d", _i32), ("sh_degree", _i32), ("feat_dtype", _i32),
                ("form", _i32), ("rank_bits", _i32), ("tile_bits", _i32), ("packed_keys", _i32),
                ("bin_rule", _i32), ("ndfd", _i32), ("primitive", _i32), ("inst_capacity", _i64), ("visit_capacity", _i64), ("n_pixels", _i64), ("n_tiles", _i64),
                ("cams", FhCamera * FH_MAX_VIEWS), ("pix_off", _i64 * (FH_MAX_VIEWS + 1)),
                ("tile_off", _i64 * (FH_MAX_VIEWS + 1)), ("tiles_x", _i32 * FH_MAX_VIEWS),
                ("tiles_y", _i32 * FH_MAX_VIEWS), ("tuning", FhTuning), ("n_ws", _i32), ("off", _sz * FH_WS_SLOTS),
                ("ws_bytes", _sz)]


class FhImage(ctypes.Structure):
    _fields_ = [("C", _vp), ("F", _vp), ("T", _vp), ("n_iter", _vp)]


class FhUpstream(ctypes.Structure):
    _fields_ = [("dC", _vp), ("dF", _vp), ("dT", _vp), ("ndfd_gt", _vp), ("ndfd_a", _vp), ("ndfd_b", _vp),
                ("ndfd_Lgt", _vp), ("ndfd_Lcf", _vp), ("ndfd_lambda", _f32), ("ndfd_k", _f32)]


class FhGrads(ctypes.Structure):
    _fields_ = [("means", _vp), ("scales", _vp), ("quats", _vp), ("opacity", _vp), ("sh", _vp)]


class FhFusion(ctypes.Structure):
    _fields_ = [("sum", _vp), ("comp", _vp), ("wsum", _vp), ("wcomp", _vp)]


class FhCounters(ctypes.Structure):
    _fields_ = [("n_instances", _i64), ("n_visited", _i64), ("n_culled_nonfinite", _i64),
                ("inst_overflow", _i32), ("visit_overflow", _i32)]


class FhParams(ctypes.Structure):
    _fields_ = [("means", _vp), ("log_scales", _vp), ("quats", _vp), ("logit_opacity", _vp), ("sh", _vp)]


class FhAdam(ctypes.Structure):
    _fields_ = [("lr", _f32 * 5), ("beta1", _f32), ("beta2", _f32), ("eps", _f32), ("step", _i32)]


class FhDensifyConfig(ctypes.Structure):
    _fields_ = [("grad_threshold", _f32), ("log_scale_threshold", _f32), ("prune_logit", _f32)]


_P = ctypes.POINTER
SIGNATURES = {
    "fh_plan_init": (_i32, [_P(FhPlan), _i64, _i32, _i32, _i32, _i32, _P(FhCamera), _i32, _i64, _i64]),
    "fh_plan_set_ndfd": (_i32, [_P(FhPlan), _i32]),
    "fh_plan_set_primitive": (_i32, [_P(FhPlan), _i32]),
    "fh_project": (_i32, [_P(FhPlan), _P(FhGaussians), _vp, _vp]),
    "fh_bin_count": (_i32, [_P(FhPlan), _vp, _vp]),
    "fh_bin_sort": (_i32, [_P(FhPlan), _vp, _vp]),
    "fh_bin_keys": (_i32, [_P(FhPlan), _vp, _vp, _vp, _i64, _vp]),
    "fh_render_fwd": (_i32, [_P(FhPlan), _P(FhGaussians), _vp, _P(FhImage), _vp]),
    "fh_render_bwd": (_i32, [_P(FhPlan), _P(FhGaussians), _vp, _P(FhImage), _P(FhUpstream), _vp, _i32,
                             _P(FhFusion), _P(FhGrads), _vp]),
    "fh_ndfd_losses": (_i32, [_P(FhPlan), _P(FhGaussians), _vp, _P(FhImage), _vp, _f32, _f32, _vp, _vp, _vp]),
    "fh_fuse_features": (_i32, [_P(FhPlan), _P(FhGaussians), _vp, _P(FhImage), _vp, _i32, _P(FhFusion), _vp]),
    "fh_fuse_finalize": (_i32, [_P(FhFusion), _i64, _i32, _vp, _vp, _i32, _vp]),
    "fh_read_counters": (_i32, [_P(FhPlan), _vp, _P(FhCounters), _vp]),
    "fh_get_status": (_i32, [_P(FhPlan), _vp, _vp, _vp]),
    "fh_get_buffer": (_i32, [_P(FhPlan), _vp, _i32, _P(_vp), _P(_i64)]),
    "fh_set_kernel_events": (_i32, [_i32, _vp, _vp, _i32]),
    "fh_render_fwd_static": (_i32, [_P(FhPlan), _P(FhGaussians), _P(FhImage), _vp, _vp]),
    "fh_tuning_candidates": (_i32, [_P(FhPlan), _i32, _P(FhTuning), _i32, _P(_i32)]),
    "fh_autotune": (_i32, [_P(FhPlan), _P(FhGaussians), _vp, _P(FhImage), _P(FhUpstream), _vp, _i32, _P(FhFusion),
                           _P(FhGrads), _i32, _vp]),
    "fh_adam_step": (_i32, [_i64, _i32, _P(FhParams), _P(FhParams), _P(FhParams), _P(FhGrads), _P(FhAdam), _vp, _vp,
                            _vp]),
    "fh_activate": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp]),
    "fh_densify_stats": (_i32, [_P(FhPlan), _vp, _vp, _vp, _vp]),
    "fh_densify_workspace_size": (_sz, [_i64]),
    "fh_densify_plan": (_i32, [_i64, _vp, _vp, _vp, _vp, _P(FhDensifyConfig), _vp, _vp, _vp]),
    "fh_densify_apply": (_i32, [_i64, _i32, _vp, _P(FhParams), _P(FhParams), _P(FhParams), _vp, _i64, _i64,
                                _P(FhParams),
                                _P(FhParams), _P(FhParams), _vp, _vp, _vp]),
    "fh_densify_copy_rows": (_i32, [_i64, _vp, _vp, _vp, _i64, _i64, _i64, _vp]),
    "fh_loss_workspace_size": (_sz, [_i64]),
    "fh_photometric_loss": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fh_status_string": (ctypes.c_char_p, [_i32]),
    "fh_version": (_i32, []),
}

_lib = None


class FhError(RuntimeError):
    pass


def load() -> ctypes.CDLL:
    """Load libfhgs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FhError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_19154_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, what: str) -> None:
    if status != FH_OK:
        msg = load().fh_status_string(status).decode()
        raise FhError(f"{what} failed: {msg} ({status})")
