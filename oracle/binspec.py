"""Float32 binning: depth keys, tile rectangles, (tile, depth) keys and per-tile ranges.

Appendix A ("Details of the Rasterizer") and Algorithm 2 (CreateTiles,
DuplicateWithKeys, SortByKeys, IdentifyTileRanges): the image is cut into 16x16
tiles, every Gaussian is duplicated once per tile it overlaps, each copy gets a
64-bit key whose upper 32 bits hold the tile index and whose lower 32 bits hold
the depth, one radix sort orders all copies, and a second pass finds the
[start, end) range of every tile.

The keys are integers decided by float32 arithmetic, so this module fixes the
float32 operation order (every step below is one IEEE float32 operation with
round-to-nearest; no fused multiply-add) and evaluates it with numpy float32
arrays, which round every operation exactly that way:

  p_r     = ((R_r0 * mx + R_r1 * my) + R_r2 * mz) + t_r          r = x, y, z
  depth   = p_z;  visible iff depth > 0.2f
  u       = (fx * p_x) / p_z + cx;   v = (fy * p_y) / p_z + cy
  n       = ((qw*qw + qx*qx) + qy*qy) + qz*qz;  k = 2 / n
  Rq      = [[1 - k (qy qy + qz qz), k (qx qy - qw qz), k (qx qz + qw qy)],
             [k (qx qy + qw qz), 1 - k (qx qx + qz qz), k (qy qz - qw qx)],
             [k (qx qz - qw qy), k (qy qz + qw qx), 1 - k (qx qx + qy qy)]]
  M_ij    = Rq_ij * s_j
  j00 = fx / p_z;  j11 = fy / p_z;  j02 = -(j00 * p_x) / p_z;  j12 = -(j11 * p_y) / p_z
  T0_k = j00 * R_0k + j02 * R_2k;   T1_k = j11 * R_1k + j12 * R_2k     (R = camera rotation)
  W0_l = (T0_0 M_0l + T0_1 M_1l) + T0_2 M_2l;   W1_l likewise with T1
  a   = ((W0_0^2 + W0_1^2) + W0_2^2) + 0.3f;     c likewise with W1
  e_x = sqrt(KAPPA * a);  e_y = sqrt(KAPPA * c)                     (KAPPA = 11.1f)
  tx in [max(0, floor((u - e_x)/16)), min(TX-1, floor((u + e_x)/16))], ty likewise
  culled if not visible, if any of u, v, e_x, e_y is not finite, or if the rect is empty

The products inside a parenthesised pair are rounded before the add.  The box
half-extent sqrt(KAPPA Sigma2_ii) bounds every point where
-1/2 d^T Sigma2^-1 d >= -ln 255 (KAPPA > 2 ln 255 = 11.08), so no pixel where
alpha can reach 1/255 is outside the rect and tiling never changes a result.

Opacity-aware rule (rule="opacity"): alpha = o G reaches 1/255 only where
d^T Sigma2^-1 d <= 2 ln(255 o), so each Gaussian gets its own
  kappa_i = min(KAPPA, 2 ln(255 o_i) + 1/256)       (culled if 255 o_i <= 1)
in place of KAPPA, with ln evaluated in float32 by basic operations only (so
that both sides round identically):
  x = 255 * o;  x = m 2^e with m in [1, 2) (exact, from the float's bits);
  if m > sqrt2f: m = m * 0.5, e = e + 1 (exact)
  s = (m - 1) / (m + 1);  z = s * s
  p = (((z / 9 + 1/7) z + 1/5) z + 1/3) z + 1     (Horner, constants as float32:
      p = (((c9 z + c7) z + c5) z + c3) z + 1 with c_k = float32(1/k))
  ln x = float32(e) * ln2f + (s + s) * p            (the atanh series of ln m)
  kappa = min(KAPPA, (ln x + ln x) + 1/256)
|s| <= 0.1716 after the range step, so the series' remainder (s^11/11 relative)
is below float32 resolution; the 1/256 margin exceeds the float32 error of
2 ln x many times over, so the rect still holds every pixel where alpha can
reach 1/255.
"""
from __future__ import annotations

import numpy as np

from . import consts

f32 = np.float32


def _dot3(r, x, y, z):
    """((r0*x + r1*y) + r2*z) in float32, r a length-3 float32 vector."""
    return ((r[0] * x + r[1] * y) + r[2] * z)


SQRT2_F32 = f32(1.4142135)
LN2_F32 = f32(0.6931472)
C3, C5, C7, C9 = (f32(1.0 / k) for k in (3, 5, 7, 9))
KAPPA_MARGIN = f32(1.0 / 256.0)


def ln_f32(x: np.ndarray) -> np.ndarray:
    """Natural log of float32 x > 0 (finite, normal), by the fixed sequence of
    float32 operations in the module docstring."""
    x = np.asarray(x, f32)
    bits = x.view(np.uint32)
    e = (bits >> np.uint32(23)).astype(np.int64) - 127
    m = ((bits & np.uint32(0x7FFFFF)) | np.uint32(0x3F800000)).view(f32)
    big = m > SQRT2_F32
    m = np.where(big, m * f32(0.5), m).astype(f32)
    e = e + big.astype(np.int64)
    one = f32(1.0)
    s = (m - one) / (m + one)
    z = s * s
    p = (((C9 * z + C7) * z + C5) * z + C3) * z + one
    return e.astype(f32) * LN2_F32 + (s + s) * p


def opacity_kappa(o: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Per-Gaussian box factor of the opacity-aware rule, and whether the
    Gaussian can reach alpha = 1/255 at all (255 o > 1)."""
    x = f32(255.0) * np.asarray(o, f32)
    live = x > f32(1.0)
    with np.errstate(all="ignore"):
        lx = ln_f32(np.where(live, x, f32(2.0)).astype(f32))
        kap = np.minimum((lx + lx) + KAPPA_MARGIN, consts.KAPPA_F32)
    return np.where(live, kap, f32(0.0)).astype(f32), live


RULES = ("box", "opacity", "surfel")


def bin_quantities(g: dict, cam, rule: str = "box") -> dict:
    """Per-Gaussian float32 depth, rect and tile count for one camera, under the
    box rule (one KAPPA for all) or the opacity-aware rule (kappa_i)."""
    if rule not in RULES:
        raise ValueError(rule)
    mu = np.asarray(g["means"], f32)
    s = np.asarray(g["scales"], f32)
    q = np.asarray(g["quats"], f32)
    R = np.asarray(cam.R, f32)
    t = np.asarray(cam.t, f32)
    fx, fy, cx, cy = f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy)
    W, H = int(cam.width), int(cam.height)
    TX, TY = (W + consts.TILE - 1) // consts.TILE, (H + consts.TILE - 1) // consts.TILE
    mx, my, mz = mu[:, 0], mu[:, 1], mu[:, 2]

    with np.errstate(all="ignore"):
        px = _dot3(R[0], mx, my, mz) + t[0]
        py = _dot3(R[1], mx, my, mz) + t[1]
        pz = _dot3(R[2], mx, my, mz) + t[2]
        depth = pz
        visible = depth > consts.Z_NEAR_F32
        u = (fx * px) / pz + cx
        v = (fy * py) / pz + cy

        qw, qx, qy, qz = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
        n = ((qw * qw + qx * qx) + qy * qy) + qz * qz
        k = f32(2.0) / n
        one = f32(1.0)
        Rq = np.empty((mu.shape[0], 3, 3), f32)
        Rq[:, 0, 0] = one - k * (qy * qy + qz * qz)
        Rq[:, 0, 1] = k * (qx * qy - qw * qz)
        Rq[:, 0, 2] = k * (qx * qz + qw * qy)
        Rq[:, 1, 0] = k * (qx * qy + qw * qz)
        Rq[:, 1, 1] = one - k * (qx * qx + qz * qz)
        Rq[:, 1, 2] = k * (qy * qz - qw * qx)
        Rq[:, 2, 0] = k * (qx * qz - qw * qy)
        Rq[:, 2, 1] = k * (qy * qz + qw * qx)
        Rq[:, 2, 2] = one - k * (qx * qx + qy * qy)
        M = Rq * s[:, None, :]

        j00 = fx / pz
        j11 = fy / pz
        j02 = -(j00 * px) / pz
        j12 = -(j11 * py) / pz
        T0 = [j00 * R[0, kk] + j02 * R[2, kk] for kk in range(3)]
        T1 = [j11 * R[1, kk] + j12 * R[2, kk] for kk in range(3)]
        W0 = [(T0[0] * M[:, 0, l] + T0[1] * M[:, 1, l]) + T0[2] * M[:, 2, l] for l in range(3)]
        W1 = [(T1[0] * M[:, 0, l] + T1[1] * M[:, 1, l]) + T1[2] * M[:, 2, l] for l in range(3)]
        a = ((W0[0] * W0[0] + W0[1] * W0[1]) + W0[2] * W0[2]) + consts.LOWPASS_F32
        c = ((W1[0] * W1[0] + W1[1] * W1[1]) + W1[2] * W1[2]) + consts.LOWPASS_F32
        if rule == "surfel":
            return _surfel_bins(g, cam, R, s, Rq, px, py, pz, depth, visible, u, v, fx, fy, TX, TY)
        if rule == "box":
            ex = np.sqrt(consts.KAPPA_F32 * a)
            ey = np.sqrt(consts.KAPPA_F32 * c)
            live = np.ones(mu.shape[0], bool)
        else:
            kap, live = opacity_kappa(g["opacity"])
            ex = np.sqrt(kap * a)
            ey = np.sqrt(kap * c)

        ts = f32(consts.TILE)
        x0f = np.floor((u - ex) / ts)
        x1f = np.floor((u + ex) / ts)
        y0f = np.floor((v - ey) / ts)
        y1f = np.floor((v + ey) / ts)
        finite = np.isfinite(u) & np.isfinite(v) & np.isfinite(ex) & np.isfinite(ey)
        ok = visible & finite & live
        x0 = np.where(ok, np.maximum(x0f, f32(0)), f32(0))
        x1 = np.where(ok, np.minimum(x1f, f32(TX - 1)), f32(-1))
        y0 = np.where(ok, np.maximum(y0f, f32(0)), f32(0))
        y1 = np.where(ok, np.minimum(y1f, f32(TY - 1)), f32(-1))
    x0, x1, y0, y1 = (np.asarray(z, np.float64).astype(np.int64) for z in (x0, x1, y0, y1))
    nonempty = ok & (x0 <= x1) & (y0 <= y1)
    ntiles = np.where(nonempty, (x1 - x0 + 1) * (y1 - y0 + 1), 0).astype(np.int64)
    return dict(depth=depth.astype(f32), visible=visible & finite & live, binned=nonempty,
                x0=x0, x1=x1, y0=y0, y1=y1, ntiles=ntiles, tiles_x=TX, tiles_y=TY,
                u32=u.astype(f32), v32=v.astype(f32), ex=ex.astype(f32), ey=ey.astype(f32))


def surfel_frame(R, s, Rq, px, py, pz, fx, fy):
    """Float32 surfel map in pixel offsets from the projected centre (the
    surfel rule of the module docstring of oracle.surfel): camera-space scaled
    tangents T_u = s_u R_c Rq[:, 0], T_v = s_v R_c Rq[:, 1], then
      a = fx (T.x p_z - p_x T.z) / p_z^2,  b = fy (T.y p_z - p_y T.z) / p_z^2,
      c = T.z / p_z                          for T = T_u (index 0), T_v (index 1).
    Every step one float32 operation, products rounded before sums."""
    su, sv = s[:, 0], s[:, 1]
    tu = [_dot3(R[r], Rq[:, 0, 0], Rq[:, 1, 0], Rq[:, 2, 0]) * su for r in range(3)]
    tv = [_dot3(R[r], Rq[:, 0, 1], Rq[:, 1, 1], Rq[:, 2, 1]) * sv for r in range(3)]
    zz = pz * pz
    a0 = fx * ((tu[0] * pz - px * tu[2]) / zz)
    a1 = fx * ((tv[0] * pz - px * tv[2]) / zz)
    b0 = fy * ((tu[1] * pz - py * tu[2]) / zz)
    b1 = fy * ((tv[1] * pz - py * tv[2]) / zz)
    c0 = tu[2] / pz
    c1 = tv[2] / pz
    return a0, a1, b0, b1, c0, c1


def _surfel_bins(g, cam, R, s, Rq, px, py, pz, depth, visible, u, v, fx, fy, TX, TY) -> dict:
    """Tile rect of a surfel (Section 3.1): the bounding box of the image of
    its disc u^2 + v^2 <= kappa_i (the opacity-aware kappa_i, so that the disc
    holds every point where alpha can reach 1/255).  With the surfel map in
    pixel offsets from the centre, (dx w, dy w, w) = [[a0, a1, 0], [b0, b1, 0],
    [c0, c1, 1]] (u, v, 1), the disc's dual conic is
      D = kappa (a a^T, a.b, a.c; b.b, b.c; c.c) - e3 e3^T,
    the disc lies in front of the camera (its image bounded) iff D22 < 0, and
    the vertical tangents are dx = (D02 +- sqrt(D02^2 - D00 D22)) / D22 (dy
    likewise with D12, D11).  Float32, every operation rounded."""
    a0, a1, b0, b1, c0, c1 = surfel_frame(R, s, Rq, px, py, pz, fx, fy)
    kap, live = opacity_kappa(g["opacity"])
    one = f32(1.0)
    d00 = kap * (a0 * a0 + a1 * a1)
    d02 = kap * (a0 * c0 + a1 * c1)
    d11 = kap * (b0 * b0 + b1 * b1)
    d12 = kap * (b0 * c0 + b1 * c1)
    d22 = kap * (c0 * c0 + c1 * c1) - one
    front = d22 < f32(0.0)
    sx = np.sqrt(d02 * d02 - d00 * d22)
    sy = np.sqrt(d12 * d12 - d11 * d22)
    xlo = (d02 + sx) / d22
    xhi = (d02 - sx) / d22
    ylo = (d12 + sy) / d22
    yhi = (d12 - sy) / d22
    ts = f32(consts.TILE)
    x0f = np.floor((u + xlo) / ts)
    x1f = np.floor((u + xhi) / ts)
    y0f = np.floor((v + ylo) / ts)
    y1f = np.floor((v + yhi) / ts)
    finite = (np.isfinite(u) & np.isfinite(v) & np.isfinite(xlo) & np.isfinite(xhi) & np.isfinite(ylo)
              & np.isfinite(yhi))
    ok = visible & finite & live & front
    x0 = np.where(ok, np.maximum(x0f, f32(0)), f32(0))
    x1 = np.where(ok, np.minimum(x1f, f32(TX - 1)), f32(-1))
    y0 = np.where(ok, np.maximum(y0f, f32(0)), f32(0))
    y1 = np.where(ok, np.minimum(y1f, f32(TY - 1)), f32(-1))
    x0, x1, y0, y1 = (np.asarray(z, np.float64).astype(np.int64) for z in (x0, x1, y0, y1))
    nonempty = ok & (x0 <= x1) & (y0 <= y1)
    ntiles = np.where(nonempty, (x1 - x0 + 1) * (y1 - y0 + 1), 0).astype(np.int64)
    return dict(depth=depth.astype(f32), visible=ok, binned=nonempty,
                x0=x0, x1=x1, y0=y0, y1=y1, ntiles=ntiles, tiles_x=TX, tiles_y=TY,
                u32=u.astype(f32), v32=v.astype(f32), xlo=xlo.astype(f32), xhi=xhi.astype(f32),
                ylo=ylo.astype(f32), yhi=yhi.astype(f32), kappa=kap)


def duplicate_with_keys(bq_list: list) -> dict:
    """Instances of all views, in (view, Gaussian index, row-major tile) order.

    Returns keys (uint64, tile << 32 | depth bits), the Gaussian index of every
    instance, and the global tile offset of every view.
    """
    keys, gids, views = [], [], []
    tile_off = 0
    offsets = []
    for vi, bq in enumerate(bq_list):
        offsets.append(tile_off)
        idx = np.nonzero(bq["binned"])[0]
        nt = bq["ntiles"][idx]
        gid = np.repeat(idx, nt)
        # position of each instance within its Gaussian's rect, row-major
        starts = np.cumsum(nt) - nt
        local = np.arange(int(nt.sum()), dtype=np.int64) - np.repeat(starts, nt)
        wdt = (bq["x1"] - bq["x0"] + 1)[gid]
        tx = bq["x0"][gid] + local % wdt
        ty = bq["y0"][gid] + local // wdt
        tile = tile_off + ty * bq["tiles_x"] + tx
        dbits = bq["depth"].view(np.uint32)[gid].astype(np.uint64)
        keys.append((tile.astype(np.uint64) << np.uint64(32)) | dbits)
        gids.append(gid.astype(np.int64))
        views.append(np.full(gid.shape, vi, np.int64))
        tile_off += bq["tiles_x"] * bq["tiles_y"]
    return dict(keys=np.concatenate(keys) if keys else np.zeros(0, np.uint64),
                gids=np.concatenate(gids) if gids else np.zeros(0, np.int64),
                views=np.concatenate(views) if views else np.zeros(0, np.int64),
                tile_offsets=np.asarray(offsets, np.int64), num_tiles=tile_off)


def sort_and_ranges(inst: dict) -> dict:
    """Stable sort by key, then [start, end) of every tile ((0, 0) if empty)."""
    order = np.argsort(inst["keys"], kind="stable")
    skeys = inst["keys"][order]
    sgids = inst["gids"][order]
    ntl = int(inst["num_tiles"])
    tiles = (skeys >> np.uint64(32)).astype(np.int64)
    ranges = np.zeros((ntl, 2), np.int64)
    if skeys.size:
        first = np.ones(skeys.size, bool)
        first[1:] = tiles[1:] != tiles[:-1]
        last = np.ones(skeys.size, bool)
        last[:-1] = tiles[1:] != tiles[:-1]
        pos = np.arange(skeys.size)
        ranges[tiles[first], 0] = pos[first]
        ranges[tiles[last], 1] = pos[last] + 1
    return dict(keys=skeys, gids=sgids, order=order, ranges=ranges)


def tile_counts(bq: dict) -> np.ndarray:
    """Instances per tile of one view, [tiles_y * tiles_x] row-major, without
    generating the instances: each binned Gaussian adds 1 over its tile rect
    (a 2D difference array, then prefix sums along both axes)."""
    TX, TY = bq["tiles_x"], bq["tiles_y"]
    diff = np.zeros((TY + 1, TX + 1), np.int64)
    b = np.nonzero(bq["binned"])[0]
    x0, x1, y0, y1 = bq["x0"][b], bq["x1"][b], bq["y0"][b], bq["y1"][b]
    np.add.at(diff, (y0, x0), 1)
    np.add.at(diff, (y0, x1 + 1), -1)
    np.add.at(diff, (y1 + 1, x0), -1)
    np.add.at(diff, (y1 + 1, x1 + 1), 1)
    return np.cumsum(np.cumsum(diff, 0), 1)[:TY, :TX].reshape(-1)


def ranges_from_counts(counts_per_view: list) -> np.ndarray:
    """[start, end) of every global tile from per-view instance counts, in the
    order of the sorted key array ((0, 0) for an empty tile)."""
    cnt = np.concatenate(counts_per_view).astype(np.int64)
    end = np.cumsum(cnt)
    start = end - cnt
    ranges = np.stack([start, end], 1)
    ranges[cnt == 0] = 0
    return ranges


def tile_list(bq: dict, tx: int, ty: int) -> np.ndarray:
    """Gaussian indices of one tile's sorted list: every binned Gaussian whose
    rect holds the tile, ordered by (depth bits, index)."""
    hit = np.nonzero(bq["binned"] & (bq["x0"] <= tx) & (bq["x1"] >= tx) & (bq["y0"] <= ty) & (bq["y1"] >= ty))[0]
    dbits = bq["depth"].view(np.uint32)[hit]
    return hit[np.lexsort((hit, dbits))].astype(np.int64)


def bin_views(g: dict, cams: list, rule: str = "box") -> dict:
    """The whole binning step for a list of cameras."""
    bq = [bin_quantities(g, c, rule) for c in cams]
    inst = duplicate_with_keys(bq)
    srt = sort_and_ranges(inst)
    return dict(per_view=bq, tile_offsets=inst["tile_offsets"], num_tiles=inst["num_tiles"],
                keys=srt["keys"], gids=srt["gids"], ranges=srt["ranges"])
