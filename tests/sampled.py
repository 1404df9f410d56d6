"""The oracle on a sample of a large batched workload (test infrastructure).

For workloads too large for the oracle to walk every tile, the GPU tests check:
  * every tile's instance count and range, from the oracle's float32 rects
    (binspec.tile_counts / ranges_from_counts), and
  * a sample: a seeded set of small Gaussians plus, per view, every tile any
    of them touches and a few random non-empty tiles.  The oracle walks those
    tiles with their full sorted lists (binspec.tile_list), so the sampled
    Gaussians' gradient and fusion sums over all views are complete, and every
    pixel of those tiles has its forward outputs.
Only the Gaussians of the walked lists are projected, and only the rows of the
per-pixel maps at the walked pixels are read (`rows(view, key, pixels)`).
"""
from __future__ import annotations

import numpy as np

from oracle import binspec, pipeline, project, raster

GRAD_KEYS = ("means", "scales", "quats", "opacity", "sh")


def pick_gaussians(bqs: list, n: int, seed: int) -> np.ndarray:
    """n Gaussians binned in view 0 whose rect is at most 2x2 tiles in every
    view that bins them (sorted indices)."""
    small = np.ones(bqs[0]["binned"].shape, bool)
    for bq in bqs:
        w = bq["x1"] - bq["x0"] + 1
        h = bq["y1"] - bq["y0"] + 1
        small &= ~bq["binned"] | ((w <= 2) & (h <= 2))
    cand = np.nonzero(small & bqs[0]["binned"])[0]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=min(n, cand.size), replace=False))


def plan(bqs: list, counts: list, cams: list, cand: np.ndarray, extra_tiles: int, seed: int) -> list:
    """Per view: the tiles to walk, the view's global tile offset and pixel offset."""
    rng = np.random.default_rng(seed)
    tile_off = np.cumsum([0] + [bq["tiles_x"] * bq["tiles_y"] for bq in bqs])
    pix_off = np.cumsum([0] + [cam.npix for cam in cams])
    views = []
    for vi, bq in enumerate(bqs):
        tx_n = bq["tiles_x"]
        tiles = set()
        for gi in cand:
            if bq["binned"][gi]:
                for ty in range(bq["y0"][gi], bq["y1"][gi] + 1):
                    for tx in range(bq["x0"][gi], bq["x1"][gi] + 1):
                        tiles.add(int(ty * tx_n + tx))
        nonempty = np.nonzero(counts[vi] > 0)[0]
        k = min(extra_tiles, nonempty.size)
        if k:
            tiles.update(rng.choice(nonempty, size=k, replace=False).tolist())
        views.append(dict(tiles=np.array(sorted(tiles), np.int64), tile_off=int(tile_off[vi]),
                          pix_off=int(pix_off[vi])))
    return views


def tile_pixels(cam, tx_n: int, tiles: np.ndarray) -> np.ndarray:
    """View-local pixel indices of the given tiles, tile by tile, row-major inside."""
    pix = []
    for t in tiles:
        tx, ty = int(t) % tx_n, int(t) // tx_n
        ys, xs = np.mgrid[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16]
        ok = (xs < cam.width) & (ys < cam.height)
        pix.append((ys[ok] * cam.width + xs[ok]).ravel())
    return np.concatenate(pix).astype(np.int64) if pix else np.zeros(0, np.int64)


def run(g: dict, cams: list, bqs: list, cand: np.ndarray, views: list, rows, d: int, log=None) -> dict:
    """The oracle over the planned tiles of every view.

    rows(vi, key, pix) -> float rows of map `key` in ("dC", "dF", "dT", "target")
    of view vi at view-local pixels pix.  Adds to each entry of `views` its
    oracle tile lists ("lists") and forward outputs ("fwd"); returns the sampled
    Gaussians' gradient sums, magnitude companions, fusion sums and flags.
    """
    n = g["means"].shape[0]
    nb = (int(g["sh_degree"]) + 1) ** 2
    shapes = dict(means=(3,), scales=(3,), quats=(4,), opacity=(), sh=(nb, 3))
    sums = {k: np.zeros((cand.size,) + shapes[k]) for k in GRAD_KEYS}
    mags = {k: np.zeros((cand.size,) + shapes[k]) for k in GRAD_KEYS}
    fsum = np.zeros((cand.size, d))
    fsum_mag = np.zeros((cand.size, d))
    wsum = np.zeros(cand.size)
    gflag = np.zeros(cand.size, np.int32)
    for vi, (cam, bq, vw) in enumerate(zip(cams, bqs, views)):
        tx_n = bq["tiles_x"]
        lists = {int(t): binspec.tile_list(bq, int(t) % tx_n, int(t) // tx_n) for t in vw["tiles"]}
        vw["lists"] = lists
        need = np.unique(np.concatenate(list(lists.values()) + [np.zeros(0, np.int64)]))
        ranges = np.zeros((bq["tiles_x"] * bq["tiles_y"], 2), np.int64)
        glist, pos = [], 0
        for t in vw["tiles"]:
            loc = np.searchsorted(need, lists[int(t)])
            ranges[t] = (pos, pos + loc.size)
            glist.append(loc)
            pos += loc.size
        glist = np.concatenate(glist) if glist else np.zeros(0, np.int64)
        gsub = {k: (v[need] if isinstance(v, np.ndarray) and v.shape[:1] == (n,) else v) for k, v in g.items()}
        pr = project.project(gsub, cam)
        pix = tile_pixels(cam, tx_n, vw["tiles"])
        maps = {}
        for key, width in (("dC", 3), ("dF", d), ("dT", 0), ("target", d)):
            full = np.zeros((cam.npix, width) if width else cam.npix)   # rows never written stay unallocated
            full[pix] = rows(vi, key, pix)
            maps[key] = full
        out = raster.render_view(cam, ranges, glist, pr, feat=np.asarray(gsub["feat"], np.float64), dC=maps["dC"],
                                 dF=maps["dF"], dT=maps["dT"], target=maps["target"], tile_sel=vw["tiles"],
                                 want_F=True, want_Fmag=True, want_fusion=True)
        vw["fwd"] = dict(pix=pix, C=out["C"][pix], Cmag=out["Cmag"][pix], T=out["T"][pix],
                         niter=out["niter"][pix], F=out["F"][pix], Fmag=out["Fmag"][pix], flags=out["flags"][pix])
        li = np.searchsorted(need, cand)
        present = (li < need.size) & (need[np.minimum(li, max(need.size - 1, 0))] == cand) if need.size else \
            np.zeros(cand.size, bool)
        if present.any():
            sel = li[present]
            sub = {k: (v[sel] if isinstance(v, np.ndarray) and v.shape[:1] == (need.size,) else v)
                   for k, v in pr.items()}
            ref = project.project_bwd(sub, pipeline._unpack(out["g2d"][sel]))
            mag = project.project_bwd(sub, pipeline._unpack(out["g2d_mag"][sel]), magnitude=True)
            for k in GRAD_KEYS:
                sums[k][present] += ref[k]
                mags[k][present] += mag[k]
            fsum[present] += out["fsum"][sel]
            fsum_mag[present] += out["fsum_mag"][sel]
            wsum[present] += out["wsum"][sel]
            gflag[present] |= out["gflags"][sel] | np.where(pr["clamp_amb"][sel], 4, 0).astype(np.int32)
        if log:
            log(f"oracle view {vi}: {vw['tiles'].size} tiles, {need.size} Gaussians")
    return dict(sums=sums, mags=mags, fsum=fsum, fsum_mag=fsum_mag, wsum=wsum, gflag=gflag)
