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

from oracle import binspec, pipeline, project, raster, surfel

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


def pick_front(bq: dict, max_side: int, n_near: int, max_tiles: int | None = None) -> np.ndarray:
    """Gaussians of one view that the walk reaches at high density: the n_near
    nearest binned ones with a rect of at most max_side x max_side tiles,
    stopping early once the union of their rects would exceed max_tiles
    (sorted indices)."""
    small = bq["binned"] & (bq["x1"] - bq["x0"] < max_side) & (bq["y1"] - bq["y0"] < max_side)
    cand = np.nonzero(small)[0]
    cand = cand[np.argsort(bq["depth"][cand], kind="stable")[:n_near]]
    if max_tiles is not None:
        tiles, keep = set(), []
        for gi in cand:
            t = _rect_tiles(bq, int(gi))
            if len(tiles | t) > max_tiles:
                break
            tiles |= t
            keep.append(int(gi))
        cand = np.asarray(keep, np.int64)
    return np.sort(cand)


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


def run(g: dict, cams: list, bqs: list, cand: np.ndarray, views: list, rows, d: int, log=None,
        surfels: bool = False) -> dict:
    """The oracle over the planned tiles of every view (surfels: the
    primitives are surfels, bqs from binspec's surfel rule).

    rows(vi, key, pix) -> float rows of map `key` in ("dC", "dF", "dT", "target")
    of view vi at view-local pixels pix, or None for a map not given (no dT:
    zero; no target: no fusion).  Adds to each entry of `views` its
    oracle tile lists ("lists") and forward outputs ("fwd"); returns the sampled
    Gaussians' gradient sums, magnitude companions, ambiguity bounds (as
    pipeline.run's grads_amb), fusion sums and flags.
    """
    n = g["means"].shape[0]
    nb = (int(g["sh_degree"]) + 1) ** 2
    shapes = dict(means=(3,), scales=(3,), quats=(4,), opacity=(), sh=(nb, 3))
    sums = {k: np.zeros((cand.size,) + shapes[k]) for k in GRAD_KEYS}
    mags = {k: np.zeros((cand.size,) + shapes[k]) for k in GRAD_KEYS}
    ambs = {k: np.zeros((cand.size,) + shapes[k]) for k in GRAD_KEYS}
    fsum_amb = np.zeros((cand.size, d))
    wsum_amb = np.zeros(cand.size)
    fsum = np.zeros((cand.size, d))
    fsum_mag = np.zeros((cand.size, d))
    wsum = np.zeros(cand.size)
    gflag = np.zeros(cand.size, np.int32)
    for vi, (cam, bq, vw) in enumerate(zip(cams, bqs, views)):
        tx_n = bq["tiles_x"]
        given = vw.get("lists_in", {})
        lists = {int(t): given[int(t)] if int(t) in given else binspec.tile_list(bq, int(t) % tx_n, int(t) // tx_n)
                 for t in vw["tiles"]}
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
        pr = (surfel.project_surfel if surfels else project.project)(gsub, cam)
        pix = tile_pixels(cam, tx_n, vw["tiles"])
        maps = {}
        for key, width in (("dC", 3), ("dF", d), ("dT", 0), ("target", d)):
            r = rows(vi, key, pix)
            if r is None:
                maps[key] = None
                continue
            full = np.zeros((cam.npix, width) if width else cam.npix)   # rows never written stay unallocated
            full[pix] = r
            maps[key] = full
        out = raster.render_view(cam, ranges, glist, pr, feat=np.asarray(gsub["feat"], np.float64), dC=maps["dC"],
                                 dF=maps["dF"], dT=maps["dT"], target=maps["target"], tile_sel=vw["tiles"],
                                 want_F=True, want_Fmag=True, want_fusion=maps["target"] is not None)
        vw["fwd"] = dict(pix=pix, C=out["C"][pix], Cmag=out["Cmag"][pix], T=out["T"][pix],
                         niter=out["niter"][pix], F=out["F"][pix], Fmag=out["Fmag"][pix], flags=out["flags"][pix],
                         Cden=out["Cden"][pix], Tden=out["Tden"][pix], Fden=out["Fden"][pix])
        li = np.searchsorted(need, cand)
        present = (li < need.size) & (need[np.minimum(li, max(need.size - 1, 0))] == cand) if need.size else \
            np.zeros(cand.size, bool)
        if present.any():
            sel = li[present]
            sub = {k: (v[sel] if isinstance(v, np.ndarray) and v.shape[:1] == (need.size,) else v)
                   for k, v in pr.items()}
            bwd = surfel.project_surfel_bwd if surfels else project.project_bwd
            unpack = pipeline._unpack_surfel if surfels else pipeline._unpack
            ref = bwd(sub, unpack(out["g2d"][sel]))
            mag = bwd(sub, unpack(out["g2d_mag"][sel]), magnitude=True)
            amb = bwd(sub, unpack(out["g2d_amb"][sel]), magnitude=True)
            for k in GRAD_KEYS:
                sums[k][present] += ref[k]
                mags[k][present] += mag[k]
                ambs[k][present] += amb[k]
            if maps["target"] is not None:
                fsum[present] += out["fsum"][sel]
                fsum_mag[present] += out["fsum_mag"][sel]
                wsum[present] += out["wsum"][sel]
                fsum_amb[present] += out["fsum_amb"][sel]
                wsum_amb[present] += out["wsum_amb"][sel]
            gflag[present] |= out["gflags"][sel] | np.where(pr["clamp_amb"][sel], 4, 0).astype(np.int32)
        if log:
            log(f"oracle view {vi}: {vw['tiles'].size} tiles, {need.size} Gaussians")
    return dict(sums=sums, mags=mags, ambs=ambs, fsum=fsum, fsum_mag=fsum_mag, fsum_amb=fsum_amb, wsum=wsum,
                wsum_amb=wsum_amb, gflag=gflag)


def _with_rect_of(bq: dict, bq1: dict, gi: int) -> dict:
    """bq with Gaussian gi's binning replaced by that of the one-Gaussian bq1."""
    out = dict(bq)
    for k in ("binned", "x0", "x1", "y0", "y1", "depth"):
        a = np.array(bq[k], copy=True)
        a[gi] = bq1[k][0]
        out[k] = a
    return out


def _rect_tiles(bq: dict, gi: int) -> set:
    if not bq["binned"][gi]:
        return set()
    return {int(ty * bq["tiles_x"] + tx) for ty in range(bq["y0"][gi], bq["y1"][gi] + 1)
            for tx in range(bq["x0"][gi], bq["x1"][gi] + 1)}


def footprint_outputs(g: dict, cam, bq: dict, tiles: set, rows, d: int, lists: dict | None = None) -> dict:
    """FP64 oracle forward (C, F per pixel) over the pixels of `tiles` (one view;
    lists given, or from bq's float32 rects), pixels in tile order."""
    views = [dict(tiles=np.array(sorted(tiles), np.int64), tile_off=0, pix_off=0, lists_in=lists or {})]
    run(g, [cam], [bq], np.zeros(0, np.int64), views, rows, d)
    return views[0]["fwd"]


def _lists_with(bq: dict, base: dict, gi: int, rect_bq: dict) -> dict:
    """Tile lists of `base` with Gaussian gi present exactly in the tiles of its
    rect in rect_bq (its depth, and so its place in each list, unchanged)."""
    inside = _rect_tiles(rect_bq, gi)
    dbits = bq["depth"].view(np.uint32)
    out = {}
    for t, lst in base.items():
        has = bool(np.any(lst == gi))
        if (t in inside) == has:
            out[t] = lst
        elif has:
            out[t] = lst[lst != gi]
        else:
            ext = np.append(lst, gi)
            out[t] = ext[np.lexsort((ext, dbits[ext]))]
    return out


def central_difference(g: dict, cam, bq: dict, rows, d: int, gi: int, key: str, comp: int, h: float,
                       cache: dict | None = None) -> float:
    """(L(x + h) - L(x - h)) / 2h for parameter g[key][gi].flat[comp] with
    L = sum_p dC(p) . C(p) + dF(p) . F(p), over every tile Gaussian gi touches in
    either state (all other pixels are unchanged).  The two states' outputs
    are subtracted pixel by pixel before the weighted sum, so the quotient is
    not limited by the rounding of L itself.  The perturbed value is kept in
    FP64; the step must not change gi's depth (its list positions are kept).
    `cache` (a dict) keeps the unperturbed tile lists between calls."""
    n = g["means"].shape[0]
    states = []
    for sgn in (1.0, -1.0):
        arr = np.array(g[key], np.float64, copy=True)
        arr.reshape(n, -1)[gi, comp] += sgn * h
        gs = dict(g)
        gs[key] = arr
        one = {k: (v[gi:gi + 1] if isinstance(v, np.ndarray) and v.shape[:1] == (n,) else v) for k, v in gs.items()}
        states.append((gs, _with_rect_of(bq, binspec.bin_quantities(one, cam), gi)))
    tiles = _rect_tiles(bq, gi) | _rect_tiles(states[0][1], gi) | _rect_tiles(states[1][1], gi)
    cache = {} if cache is None else cache
    tx_n = bq["tiles_x"]
    for t in tiles:
        if t not in cache:
            cache[t] = binspec.tile_list(bq, t % tx_n, t // tx_n)
    base = {t: cache[t] for t in tiles}
    fp = footprint_outputs(states[0][0], cam, bq, tiles, rows, d, _lists_with(bq, base, gi, states[0][1]))
    fm = footprint_outputs(states[1][0], cam, bq, tiles, rows, d, _lists_with(bq, base, gi, states[1][1]))
    p = fp["pix"]
    dL = float(np.sum((fp["C"] - fm["C"]) * rows(0, "dC", p)))
    if d:
        dL += float(np.sum((fp["F"] - fm["F"]) * rows(0, "dF", p)))
    return dL / (2.0 * h)
