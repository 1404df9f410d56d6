"""ctypes front end of the FP64 C compositing oracle (raster.c).

The shared object is built with gcc into oracle/_build/ (by the package's build
step, or here on first use).  Compile flags keep IEEE FP64 semantics: no
fast-math, no contraction of a*b+c into fma.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import consts

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raster.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle_raster.so")

GCC_CMD = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", _SRC, "-o", _LIB, "-lm"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(_BUILD, exist_ok=True)
        subprocess.run(GCC_CMD, check=True)
    return _LIB


_P = ctypes.c_void_p
_I = ctypes.c_int64


class _Args(ctypes.Structure):
    _fields_ = [
        ("width", _I), ("height", _I), ("tile", _I), ("tiles_x", _I), ("tiles_y", _I),
        ("d", _I), ("ambig_rel", ctypes.c_double),
        ("ranges", _P), ("list", _P),
        ("u", _P), ("v", _P), ("A", _P), ("B", _P), ("C", _P), ("opac", _P),
        ("rgb", _P), ("rgb_mag", _P), ("feat", _P),
        ("dC", _P), ("dF", _P), ("dT", _P), ("target", _P),
        ("tile_sel", _P), ("n_tile_sel", _I),
        ("out_C", _P), ("out_Cmag", _P), ("out_F", _P), ("out_Fmag", _P), ("out_T", _P), ("out_niter", _P),
        ("out_flags", _P),
        ("g2d", _P), ("g2d_mag", _P), ("fsum", _P), ("fsum_mag", _P), ("wsum", _P),
        ("dfeat", _P), ("g2d_amb", _P), ("fsum_amb", _P), ("wsum_amb", _P), ("gflags", _P), ("counts", _P),
        ("ndfd_gt", _P), ("feat_inv_norm", _P), ("ndfd_lambda", ctypes.c_double), ("ndfd_k", ctypes.c_double),
        ("ndfd_a", _P), ("ndfd_b", _P), ("out_Lgt", _P), ("out_Lcf", _P), ("out_Lcf_mag", _P), ("out_Lgt_mag", _P), ("out_FN", _P),
        ("out_WN", _P),
        ("prim", _I), ("srf", _P),
        ("den_round", ctypes.c_double), ("out_Cden", _P), ("out_Fden", _P), ("out_Tden", _P),
        ("out_Lgt_den", _P), ("out_Lcf_den", _P),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _lib.oracle_raster.argtypes = [ctypes.POINTER(_Args)]
        _lib.oracle_raster.restype = ctypes.c_int
        _lib.oracle_num_threads.restype = ctypes.c_int
        _lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib.oracle_set_num_threads.restype = None
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle_raster calls."""
    _load().oracle_set_num_threads(int(n))


def _ptr(x):
    return None if x is None else x.ctypes.data


def _f64(x):
    return None if x is None else np.ascontiguousarray(x, np.float64)


def render_view(cam, ranges, glist, proj, feat=None, dC=None, dF=None, dT=None, target=None,
                tile_sel=None, want_F=True, want_Fmag=False, want_fusion=True, want_dfeat=False,
                ndfd=None):
    """Composite one view (and its adjoint when dC is given).

    ranges [tiles, 2] and glist [M] are this view's slice of the binning (tile
    indices local to the view).  proj holds FP64 per-Gaussian u, v, A, B, C,
    opacity and rgb [N, 3] (and rgb_mag [N, 3], the magnitude companion of rgb,
    when present); for surfels (oracle.surfel) "srf" [N, 9] in place of u..C,
    and the per-Gaussian adjoint rows have 13 entries instead of 9.  Returns a
    dict of per-pixel and per-Gaussian arrays; Cden, Tden and Fden (with Fmag)
    are the surfel density's rounding allowance (zero for Gaussians).

    ndfd (optional): dict(gt=[P, d] ground-truth feature map, lam, k, and
    a, b = [P] upstream weights of L_gt and L_cf, or None); adds L_gt, L_cf,
    their companions Lgt_mag, Lcf_mag and surfel density allowances Lgt_den,
    Lcf_den, FN [P, d] and WN to the result and the NDFD terms h_k to the
    adjoint's g_k (with dC given; pass zero maps for the NDFD gradient alone).
    """
    lib = _load()
    W, H = int(cam.width), int(cam.height)
    TX = (W + consts.TILE - 1) // consts.TILE
    TY = (H + consts.TILE - 1) // consts.TILE
    P = W * H
    surf = "srf" in proj
    n = proj["opacity"].shape[0]
    gw = 13 if surf else 9
    d = 0 if feat is None else int(feat.shape[1])
    keep = {}

    def k(name, arr):
        keep[name] = arr
        return arr

    ranges = k("ranges", np.ascontiguousarray(ranges, np.int64))
    glist = k("glist", np.ascontiguousarray(glist, np.int64))
    if surf:
        u = v = A = B = C = None
        srf = k("srf", _f64(proj["srf"]))
    else:
        u, v, A, B, C = (k(nm, _f64(proj[nm])) for nm in ("u", "v", "A", "B", "C"))
        srf = None
    op = k("op", _f64(proj["opacity"]))
    rgb = k("rgb", _f64(proj["rgb"]))
    rgbm = k("rgbm", _f64(proj.get("rgb_mag")))
    featd = k("feat", _f64(feat))
    dCd, dFd, dTd, tg = (k(nm, _f64(x)) for nm, x in (("dC", dC), ("dF", dF), ("dT", dT), ("tg", target)))
    sel = k("sel", None if tile_sel is None else np.ascontiguousarray(tile_sel, np.int64))

    out = dict(C=np.zeros((P, 3)), Cmag=np.zeros((P, 3)), Cden=np.zeros((P, 3)), T=np.zeros(P),
               Tden=np.zeros(P), niter=np.zeros(P, np.int64),
               flags=np.zeros(P, np.int32), counts=np.zeros(3, np.int64))
    out["F"] = np.zeros((P, d)) if (want_F and d) else None
    out["Fmag"] = np.zeros((P, d)) if (want_Fmag and d) else None
    out["Fden"] = np.zeros((P, d)) if (want_Fmag and d) else None
    bwd = dC is not None
    out["g2d"] = np.zeros((n, gw)) if bwd else None
    out["g2d_mag"] = np.zeros((n, gw)) if bwd else None
    fus = bwd and target is not None and want_fusion and d > 0
    out["fsum"] = np.zeros((n, d)) if fus else None
    out["fsum_mag"] = np.zeros((n, d)) if fus else None
    out["wsum"] = np.zeros(n) if (bwd and target is not None) else None
    out["g2d_amb"] = np.zeros((n, gw)) if bwd else None
    out["fsum_amb"] = np.zeros((n, d)) if fus else None
    out["wsum_amb"] = np.zeros(n) if (bwd and target is not None) else None
    out["dfeat"] = np.zeros((n, d)) if (bwd and want_dfeat and d) else None
    out["gflags"] = np.zeros(n, np.int32)
    nd = {}
    if ndfd is not None:
        f64 = np.asarray(feat, np.float64)
        nrm = np.sqrt((f64 * f64).sum(1))
        nd["inv"] = k("inv", np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 0.0))
        nd["gt"] = k("gt", _f64(ndfd["gt"]))
        nd["a"] = k("na", _f64(ndfd.get("a")))
        nd["b"] = k("nb", _f64(ndfd.get("b")))
        for key, shape in (("Lgt", P), ("Lcf", P), ("Lcf_mag", P), ("Lgt_mag", P), ("WN", P), ("Lgt_den", P),
                           ("Lcf_den", P)):
            out[key] = np.zeros(shape)
        out["FN"] = np.zeros((P, d))

    args = _Args(
        width=W, height=H, tile=consts.TILE, tiles_x=TX, tiles_y=TY, d=d,
        ambig_rel=consts.AMBIG_REL,
        ranges=_ptr(ranges), list=_ptr(glist),
        u=_ptr(u), v=_ptr(v), A=_ptr(A), B=_ptr(B), C=_ptr(C), opac=_ptr(op),
        rgb=_ptr(rgb), rgb_mag=_ptr(rgbm), feat=_ptr(featd),
        dC=_ptr(dCd), dF=_ptr(dFd), dT=_ptr(dTd), target=_ptr(tg),
        tile_sel=_ptr(sel), n_tile_sel=0 if sel is None else sel.size,
        out_C=_ptr(out["C"]), out_Cmag=_ptr(out["Cmag"]), out_F=_ptr(out["F"]), out_Fmag=_ptr(out["Fmag"]),
        out_T=_ptr(out["T"]), out_niter=_ptr(out["niter"]), out_flags=_ptr(out["flags"]),
        g2d=_ptr(out["g2d"]), g2d_mag=_ptr(out["g2d_mag"]), fsum=_ptr(out["fsum"]),
        fsum_mag=_ptr(out["fsum_mag"]), wsum=_ptr(out["wsum"]), dfeat=_ptr(out["dfeat"]),
        g2d_amb=_ptr(out["g2d_amb"]), fsum_amb=_ptr(out["fsum_amb"]), wsum_amb=_ptr(out["wsum_amb"]),
        gflags=_ptr(out["gflags"]), counts=_ptr(out["counts"]),
        ndfd_gt=_ptr(nd.get("gt")), feat_inv_norm=_ptr(nd.get("inv")),
        ndfd_lambda=float(ndfd["lam"]) if ndfd else 0.0, ndfd_k=float(ndfd["k"]) if ndfd else 0.0,
        ndfd_a=_ptr(nd.get("a")), ndfd_b=_ptr(nd.get("b")), out_Lgt=_ptr(out.get("Lgt")),
        out_Lcf=_ptr(out.get("Lcf")), out_Lcf_mag=_ptr(out.get("Lcf_mag")), out_Lgt_mag=_ptr(out.get("Lgt_mag")), out_FN=_ptr(out.get("FN")),
        out_WN=_ptr(out.get("WN")),
        prim=1 if surf else 0, srf=_ptr(srf),
        den_round=consts.DEN_ROUND, out_Cden=_ptr(out["Cden"]), out_Fden=_ptr(out["Fden"]),
        out_Tden=_ptr(out["Tden"]), out_Lgt_den=_ptr(out.get("Lgt_den")), out_Lcf_den=_ptr(out.get("Lcf_den")),
    )
    rc = lib.oracle_raster(ctypes.byref(args))
    if rc != 0:
        raise MemoryError("oracle_raster: allocation failed")
    return out
