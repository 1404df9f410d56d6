"""The whole oracle path for one scene: bin (float32), project (FP64), composite
and adjoint per pixel (FP64, C), chain the adjoint back to the 3D parameters.

Algorithm 2's order: screen-space Gaussians, tile grid, duplicate with keys,
sort, tile ranges, then the per-tile, per-pixel traversal.
"""
from __future__ import annotations

import numpy as np

from . import binspec, project, raster, surfel


def view_slice(bins: dict, vi: int, cam) -> np.ndarray:
    """This view's block of the global per-tile ranges."""
    t0 = int(bins["tile_offsets"][vi])
    ntl = bins["per_view"][vi]["tiles_x"] * bins["per_view"][vi]["tiles_y"]
    return bins["ranges"][t0:t0 + ntl]


def run(g: dict, cams: list, view_tensors: list | None = None, fusion: bool = False,
        tile_sel: list | None = None, want_F: bool = True, want_dfeat: bool = False,
        want_Fmag: bool = False, magnitudes: bool = True, bin_rule: str = "box", ndfd: dict | None = None) -> dict:
    """Forward (and adjoint when view_tensors is given) for every camera.

    view_tensors[v] holds dC [P,3], dF [P,D], dT [P] and, for fusion, target [P,D].
    tile_sel[v] optionally restricts the traversal to some of view v's tiles.
    bin_rule: "box" (one KAPPA) or "opacity" (per-Gaussian kappa_i, binspec),
    or "surfel": the primitives are surfels (Section 3.1, oracle.surfel),
    binned by the image of their disc (binspec's surfel rule).
    ndfd: dict(lam, k) switches on the NDFD feature branch (Section 3.3); each
    view's tensors then hold "gt" [P, D] and, for its gradient, "ndfd_a" and
    "ndfd_b" [P] (dL/dL_gt, dL/dL_cf per pixel; dC, dF, dT may be zero maps).
    gflags: bit 0 the Gaussian decides a near-threshold skip/stop decision,
    bit 2 its colour clamp is near-threshold; grads_amb / fsum_amb / wsum_amb
    bound what near-threshold decisions of other Gaussians could change.
    Every view carries Cden, Tden and Fden: the allowance for the surfel
    density's rounding through the ray-plane intersection (zero for
    Gaussians); the adjoint's share of it is in grads_amb, fsum_amb, wsum_amb.
    """
    bins = binspec.bin_views(g, cams, bin_rule)
    feat = np.asarray(g["feat"], np.float64) if g["feat"] is not None else None
    n = g["means"].shape[0]
    views = []
    grads = None
    grads_mag = None
    grads_amb = None
    fsum = wsum = fsum_mag = dfeat = fsum_amb = wsum_amb = None
    gflags = np.zeros(n, np.int32)
    counts = np.zeros(3, np.int64)
    surf = bin_rule == "surfel"
    proj_fn = surfel.project_surfel if surf else project.project
    bwd_fn = surfel.project_surfel_bwd if surf else project.project_bwd
    unpack = _unpack_surfel if surf else _unpack
    for vi, cam in enumerate(cams):
        pr = proj_fn(g, cam)
        vt = view_tensors[vi] if view_tensors is not None else None
        out = raster.render_view(
            cam, view_slice(bins, vi, cam), bins["gids"], pr, feat=feat,
            dC=None if vt is None else vt["dC"], dF=None if vt is None else vt["dF"],
            dT=None if vt is None else vt["dT"],
            target=None if (vt is None or not fusion) else vt["target"],
            tile_sel=None if tile_sel is None else tile_sel[vi], want_F=want_F,
            want_Fmag=want_Fmag, want_fusion=fusion, want_dfeat=want_dfeat,
            ndfd=None if (ndfd is None or vt is None) else dict(
                gt=vt["gt"], lam=ndfd["lam"], k=ndfd["k"], a=vt.get("ndfd_a"), b=vt.get("ndfd_b")))
        counts += out["counts"]
        gflags |= out["gflags"]
        # bit 2: the colour clamp of a Gaussian that this view binned is ambiguous
        gflags |= np.where(pr["clamp_amb"] & bins["per_view"][vi]["binned"], 4, 0).astype(np.int32)
        rec = dict(C=out["C"], Cmag=out["Cmag"], Cden=out["Cden"], F=out["F"], Fmag=out["Fmag"], Fden=out["Fden"],
                   T=out["T"], Tden=out["Tden"], niter=out["niter"],
                   flags=out["flags"], proj=pr, g2d=out["g2d"], g2d_mag=out["g2d_mag"], g2d_amb=out["g2d_amb"])
        for key in ("Lgt", "Lcf", "Lcf_mag", "Lgt_mag", "FN", "WN", "Lgt_den", "Lcf_den"):
            if key in out:
                rec[key] = out[key]
        if vt is not None:
            up = unpack(out["g2d"])
            gv = bwd_fn(pr, up)
            grads = gv if grads is None else {k: grads[k] + gv[k] for k in grads}
            if magnitudes:
                upm = unpack(out["g2d_mag"])
                gm = bwd_fn(pr, upm, magnitude=True)
                grads_mag = gm if grads_mag is None else {k: grads_mag[k] + gm[k] for k in grads_mag}
                ga = bwd_fn(pr, unpack(out["g2d_amb"]), magnitude=True)
                grads_amb = ga if grads_amb is None else {k: grads_amb[k] + ga[k] for k in grads_amb}
            if fusion:
                fsum = out["fsum"] if fsum is None else fsum + out["fsum"]
                fsum_mag = out["fsum_mag"] if fsum_mag is None else fsum_mag + out["fsum_mag"]
                wsum = out["wsum"] if wsum is None else wsum + out["wsum"]
                fsum_amb = out["fsum_amb"] if fsum_amb is None else fsum_amb + out["fsum_amb"]
                wsum_amb = out["wsum_amb"] if wsum_amb is None else wsum_amb + out["wsum_amb"]
            if want_dfeat:
                dfeat = out["dfeat"] if dfeat is None else dfeat + out["dfeat"]
        views.append(rec)
    return dict(bins=bins, views=views, grads=grads, grads_mag=grads_mag, grads_amb=grads_amb, fsum=fsum,
                fsum_mag=fsum_mag, fsum_amb=fsum_amb, wsum=wsum, wsum_amb=wsum_amb, dfeat=dfeat, gflags=gflags,
                counts=counts)


def _unpack(g2d: np.ndarray) -> dict:
    return dict(u=g2d[:, 0], v=g2d[:, 1], A=g2d[:, 2], B=g2d[:, 3], C=g2d[:, 4],
                opacity=g2d[:, 5], rgb=g2d[:, 6:9])


def _unpack_surfel(g2d: np.ndarray) -> dict:
    return dict(srf=g2d[:, 0:9], opacity=g2d[:, 9], rgb=g2d[:, 10:13])


def finalize_fusion(fsum: np.ndarray, wsum: np.ndarray, feat_in: np.ndarray) -> np.ndarray:
    """f_hat = fsum / wsum where wsum > 0; Gaussians never blended keep their feature."""
    out = np.array(feat_in, np.float64, copy=True)
    hit = wsum > 0
    out[hit] = fsum[hit] / wsum[hit, None]
    return out
