"""Pins of the float32 binning (oracle/binspec.py): tiles, keys, sort, ranges."""
import numpy as np

import scenegen
from oracle import binspec, consts, project


def _scene(n=300, seed=0, h=1.5):
    return scenegen.make_gaussians(n, h, 0, 0, seed=seed)


def test_float32_quantities_track_fp64_projection():
    # the float32 chain computes the same depth, uv and Sigma2 diagonal as the
    # FP64 projection, to float32 accuracy (catches a dropped term or wrong index)
    g = _scene(500, 1)
    cam = scenegen.make_cameras("front96x64")[0]
    bq = binspec.bin_quantities(g, cam)
    pr = project.project(g, cam)
    vis = bq["visible"]
    assert np.allclose(bq["depth"][vis], pr["depth"][vis], rtol=2e-6)
    assert np.allclose(bq["u32"][vis], pr["u"][vis], rtol=1e-5, atol=1e-3)
    assert np.allclose(bq["v32"][vis], pr["v"][vis], rtol=1e-5, atol=1e-3)
    a32 = (bq["ex"][vis].astype(np.float64) ** 2) / consts.KAPPA
    assert np.allclose(a32, pr["a"][vis], rtol=1e-4)


def test_duplicates_match_brute_force_overlap():
    g = _scene(200, 2)
    cams = scenegen.make_cameras("front96x64")
    bins = binspec.bin_views(g, cams)
    bq = bins["per_view"][0]
    TX, TY = bq["tiles_x"], bq["tiles_y"]
    expect = set()
    for i in range(200):
        if not (bq["visible"][i]):
            continue
        for ty in range(TY):
            for tx in range(TX):
                # box [u-ex, u+ex] x [v-ey, v+ey] touches tile columns floor(./16)
                xlo = np.floor((bq["u32"][i] - bq["ex"][i]) / np.float32(16))
                xhi = np.floor((bq["u32"][i] + bq["ex"][i]) / np.float32(16))
                ylo = np.floor((bq["v32"][i] - bq["ey"][i]) / np.float32(16))
                yhi = np.floor((bq["v32"][i] + bq["ey"][i]) / np.float32(16))
                if xlo <= tx <= xhi and ylo <= ty <= yhi:
                    expect.add((ty * TX + tx, i))
    got = set(zip((bins["keys"] >> np.uint64(32)).astype(np.int64).tolist(), bins["gids"].tolist()))
    assert got == expect


def test_sort_equals_python_sorted_and_ranges():
    g = _scene(150, 3)
    cams = scenegen.make_cameras("front96x64") + scenegen.make_cameras("front40x40")
    bq = [binspec.bin_quantities(g, c) for c in cams]
    inst = binspec.duplicate_with_keys(bq)
    ref = sorted(zip(inst["keys"].tolist(), range(inst["keys"].size)))
    srt = binspec.sort_and_ranges(inst)
    assert srt["keys"].tolist() == [k for k, _ in ref]
    assert srt["order"].tolist() == [i for _, i in ref]
    tiles = (srt["keys"] >> np.uint64(32)).astype(np.int64)
    for t in range(inst["num_tiles"]):
        s, e = srt["ranges"][t]
        idx = np.nonzero(tiles == t)[0]
        if idx.size == 0:
            assert (s, e) == (0, 0)
        else:
            assert s == idx[0] and e == idx[-1] + 1 and e - s == idx.size
    # within a tile: depth ascending, ties by Gaussian index
    for t in range(inst["num_tiles"]):
        s, e = srt["ranges"][t]
        dep = (srt["keys"][s:e] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        gid = srt["gids"][s:e]
        pairs = list(zip(dep.tolist(), gid.tolist()))
        assert pairs == sorted(pairs)


def test_box_holds_every_pixel_alpha_can_reach():
    # alpha = o exp(power) >= 1/255 at a pixel centre  =>  that pixel's tile is in the rect
    g = _scene(400, 4, h=1.2)
    g["opacity"] = np.full(400, 0.999, np.float32)
    cam = scenegen.make_cameras("front128x96")[0]
    bq = binspec.bin_quantities(g, cam)
    pr = project.project(g, cam)
    ys, xs = np.mgrid[0:96, 0:128]
    x = xs.reshape(-1) + 0.5
    y = ys.reshape(-1) + 0.5
    for i in np.nonzero(bq["visible"])[0][:150]:
        dx, dy = x - pr["u"][i], y - pr["v"][i]
        power = -0.5 * (pr["A"][i] * dx * dx + 2 * pr["B"][i] * dx * dy + pr["C"][i] * dy * dy)
        hit = pr["opacity"][i] * np.exp(power) >= consts.ALPHA_MIN
        tx, ty = (x[hit] // 16).astype(int), (y[hit] // 16).astype(int)
        assert bq["binned"][i] or not hit.any()
        if hit.any():
            assert np.all((tx >= bq["x0"][i]) & (tx <= bq["x1"][i]) & (ty >= bq["y0"][i]) & (ty <= bq["y1"][i]))


def test_near_plane_and_nonfinite_culled():
    g = _scene(6, 5)
    g["means"] = g["means"].copy()
    g["means"][0] = [0.0, -3.9, 0.0]   # depth 0.1 < 0.2
    g["means"][1] = [np.nan, 0, 0]
    g["scales"] = g["scales"].copy()
    g["scales"][2] = [np.inf, 1, 1]
    cam = scenegen.make_cameras("front64x64")[0]
    bq = binspec.bin_quantities(g, cam)
    assert not bq["binned"][0] and not bq["binned"][1] and not bq["binned"][2]
    assert bq["ntiles"][:3].tolist() == [0, 0, 0]


def test_per_tile_form_equals_full_binning():
    # counts by difference array, ranges from counts and one tile's list by a
    # filter + lexsort reproduce the full duplicate/sort/ranges path on a
    # two-view scene (the form the large-batch GPU tests sample from)
    g = _scene(600, 5, 2.0)
    cams = [scenegen.look_at_camera(p, w, h) for p, w, h in (((0, -4, 0), 96, 64), ((2.5, -3, 1), 80, 72))]
    bins = binspec.bin_views(g, cams)
    counts = [binspec.tile_counts(bq) for bq in bins["per_view"]]
    assert sum(int(c.sum()) for c in counts) == bins["keys"].size
    assert np.array_equal(binspec.ranges_from_counts(counts), bins["ranges"])
    for vi, bq in enumerate(bins["per_view"]):
        off = int(bins["tile_offsets"][vi])
        for t in range(bq["tiles_x"] * bq["tiles_y"]):
            lst = binspec.tile_list(bq, t % bq["tiles_x"], t // bq["tiles_x"])
            s, e = bins["ranges"][off + t]
            assert np.array_equal(lst, bins["gids"][s:e])
