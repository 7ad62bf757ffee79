"""Pins for the oracle's tile binning (Section 2.1, "Sorting"; Section 3.2,
Comp_i as the number of tiles that use a point; Section 4.2 filtering).

Brute force in pure Python re-derives the sorted key list; the invariants
Sum hits = #keys and per-tile range length = per-tile count must hold; the
large-vs-small ellipse illustration of Section 3.1 gives rect-area closed
forms.
"""
import math
import struct

import numpy as np

import scenegen


def fbits(x):
    return struct.unpack("<I", struct.pack("<f", x))[0]


def brute_keys(mean2d, radius, depth, widths, heights, T, tile_lo=None, qbound=None):
    V = len(widths)
    n = len(radius) // V
    emitted = []
    off = 0
    for v in range(V):
        W, H = widths[v], heights[v]
        tx_n = (W + T - 1) // T
        for i in range(n):
            e = v * n + i
            r = int(radius[e])
            if r <= 0:
                continue
            mx = np.float32(mean2d[e][0])
            my = np.float32(mean2d[e][1])
            fr = np.float32(r)
            x0, x1 = math.ceil(np.float32(mx - fr)), math.floor(np.float32(mx + fr))
            y0, y1 = math.ceil(np.float32(my - fr)), math.floor(np.float32(my + fr))
            x0, y0 = max(x0, 0), max(y0, 0)
            x1, y1 = min(x1, W - 1), min(y1, H - 1)
            if x0 > x1 or y0 > y1:
                continue
            for ty in range(y0 // T, y1 // T + 1):
                for tx in range(x0 // T, x1 // T + 1):
                    g = off + ty * tx_n + tx
                    if tile_lo is not None and not tile_lo[g] <= qbound[i]:
                        continue
                    emitted.append(((g << 32) | fbits(np.float32(depth[e])), len(emitted), i))
        off += tx_n * ((H + T - 1) // T)
    emitted.sort()
    return [k for k, _, _ in emitted], [i for _, _, i in emitted], off


def test_binning_matches_brute_force_two_views(oracle_lib):
    sc = scenegen.small_scene(400, seed=11, sh_degree=0, log_scale_mu=-2.8)
    cams = [scenegen.pinhole(70, 45, 60.0, t=(0.0, 0.0, 4.0)),
            scenegen.look_at((1.0, 0.5, -3.5), (0, 0, 0), 50, 38, 60.0)]
    m2, rad, dep = [], [], []
    for c in cams:
        pr = oracle_lib.project(sc, c)
        m2.append(pr["mean2d"].astype(np.float32))
        rad.append(pr["radius"])
        dep.append(pr["depth"].astype(np.float32))
    m2, rad, dep = np.concatenate(m2), np.concatenate(rad), np.concatenate(dep)
    for T in (8, 16):
        out = oracle_lib.bin_f32(m2, rad, dep, [70, 50], [45, 38], T)
        keys, vals, ntiles = brute_keys(m2, rad, dep, [70, 50], [45, 38], T)
        np.testing.assert_array_equal(out["keys"], np.array(keys, np.uint64))
        np.testing.assert_array_equal(out["vals"], np.array(vals, np.uint32))
        assert out["hits"].sum() == out["num_keys"] == len(keys)
        lens = out["ranges"][:, 1].astype(np.int64) - out["ranges"][:, 0]
        per_tile = np.bincount((out["keys"] >> np.uint64(32)).astype(np.int64), minlength=ntiles)
        np.testing.assert_array_equal(lens, per_tile)


def test_rect_area_closed_form(oracle_lib):
    # Section 3.1's illustration: a small ellipse inside 2 tiles costs 2
    # keys, a large one spanning 4x2 tiles costs 8
    T = 16
    m2 = np.array([[15.5, 8.0], [31.5, 15.5]], np.float32)
    rad = np.array([4, 20], np.int32)     # x 11.5..19.5 -> tiles 0..1; y 4..12 -> tile 0
    dep = np.array([1.0, 2.0], np.float32)  # x 11.5..51.5 -> tiles 0..3; y -4.5..35.5 -> 0..2
    out = oracle_lib.bin_f32(m2, rad, dep, [128], [64], T)
    assert list(out["hits"][0]) == [2, 4 * 3]
    # clipping at the image border and empty rects
    m2 = np.array([[-30.0, 5.0], [2.0, 2.0], [127.9, 63.9]], np.float32)
    rad = np.array([3, 2, 5], np.int32)
    out = oracle_lib.bin_f32(m2, rad, np.ones(3, np.float32), [128], [64], T)
    assert list(out["hits"][0]) == [0, 1, 1]


def test_filter_keeps_tiles_at_or_below_bound(oracle_lib):
    # a Gaussian with quality bound m is used in tiles of level t <= m
    T = 8
    m2 = np.array([[16.0, 4.0]] * 4, np.float32)
    rad = np.array([12] * 4, np.int32)  # x 4..28 -> tiles 0..3, y 0..7 -> row 0 (+ clip)
    dep = np.arange(1, 5, dtype=np.float32)
    tile_lo = np.array([1, 2, 3, 4] + [4] * 4, np.uint8)  # 32x16 image: 4x2 tiles
    qb = np.array([1, 2, 3, 4], np.uint8)
    out = oracle_lib.bin_f32(m2, rad, dep, [32], [16], T, tile_level_lo=tile_lo, qbound=qb)
    # rows: y 0..15 -> tile rows 0..1; Gaussian m keeps tiles with level <= m
    assert list(out["hits"][0]) == [1, 2, 3, 8]
    keys, vals, _ = brute_keys(m2, rad, dep, [32], [16], T, tile_lo, qb)
    np.testing.assert_array_equal(out["keys"], np.array(keys, np.uint64))
    np.testing.assert_array_equal(out["vals"], np.array(vals, np.uint32))


def test_equal_depth_ties_go_by_index(oracle_lib):
    m2 = np.array([[8.0, 8.0]] * 5, np.float32)
    rad = np.array([3] * 5, np.int32)
    dep = np.array([2.0, 1.0, 2.0, 1.0, 2.0], np.float32)
    out = oracle_lib.bin_f32(m2, rad, dep, [16], [16], 16)
    assert list(out["vals"]) == [1, 3, 0, 2, 4]
