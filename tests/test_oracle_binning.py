"""Pins of the oracle's binning (section "Rasterizer": replicate by prefix
sum, tile id, sort by (tile id, depth), segment bounds) against library
routines and brute-force enumeration."""
import numpy as np
import pytest

import oracle


def _random_rects(rng, n, tx, ty, p_visible=0.8):
    x0 = rng.integers(0, tx, size=n)
    y0 = rng.integers(0, ty, size=n)
    x1 = np.minimum(x0 + rng.integers(1, 5, size=n), tx)
    y1 = np.minimum(y0 + rng.integers(1, 4, size=n), ty)
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    vis = rng.uniform(size=n) < p_visible
    tc = np.where(vis, (x1 - x0) * (y1 - y0), 0).astype(np.int32)
    # depths as float32 values with deliberate ties
    depth = rng.choice(rng.uniform(1, 10, size=n // 3 + 1).astype(np.float32), size=n)
    return depth.astype(np.float64), rect, tc


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_binning_against_library_sort(seed):
    rng = np.random.default_rng(seed)
    tx, ty, n = 13, 9, 500
    depth, rect, tc = _random_rects(rng, n, tx, ty)
    b = oracle.bin_pairs(depth, rect, tc, tx, ty)
    # (ii) prefix sum = cumsum
    np.testing.assert_array_equal(b["offsets"], np.concatenate([[0], np.cumsum(tc)[:-1]]))
    assert b["I"] == int(tc.sum())
    # (iii) the pair multiset is the brute-force enumeration of rect tiles
    tiles, idx = [], []
    for i in range(n):
        if tc[i] == 0:
            continue
        for y in range(rect[i, 1], rect[i, 3]):
            for x in range(rect[i, 0], rect[i, 2]):
                tiles.append(y * tx + x)
                idx.append(i)
    tiles, idx = np.array(tiles), np.array(idx)
    d32 = depth.astype(np.float32)[idx]
    # (i) library sort: lexicographic (tile, depth, index)
    order = np.lexsort((idx, d32, tiles))
    np.testing.assert_array_equal(b["vals"], idx[order])
    keys = (tiles[order].astype(np.uint64) << np.uint64(32)) | d32[order].view(np.uint32).astype(np.uint64)
    np.testing.assert_array_equal(b["keys"], keys)
    # (iv) keys non-decreasing, ranges partition [0, I)
    assert np.all(np.diff(b["keys"].astype(np.float64)) >= 0)
    r = b["ranges"]
    nonempty = r[:, 1] > r[:, 0]
    assert np.all(r[~nonempty] == 0)
    st = np.sort(r[nonempty, 0])
    en = np.sort(r[nonempty, 1])
    assert st[0] == 0 and en[-1] == b["I"]
    np.testing.assert_array_equal(st[1:], en[:-1])
    for t in range(tx * ty):
        np.testing.assert_array_equal(np.sort(idx[tiles == t]), np.sort(b["vals"][r[t, 0]:r[t, 1]]))


def test_replicated_tile_ids_follow_row_major_rect_order():
    # x = x0 + (r mod w), y = y0 + floor(r / w), t = y W' + x
    rect = np.array([[2, 1, 5, 3]], np.int32)
    tc = np.array([6], np.int32)
    b = oracle.bin_pairs(np.array([1.0]), rect, tc, 7, 4)
    tiles = (b["keys"] >> np.uint64(32)).astype(np.int64)
    assert list(tiles) == [1 * 7 + 2, 1 * 7 + 3, 1 * 7 + 4, 2 * 7 + 2, 2 * 7 + 3, 2 * 7 + 4]


def test_shuffle_invariance():
    # (v) relabelling the Gaussians keeps every per-tile list (up to the
    # relabelling) when depths are distinct.
    rng = np.random.default_rng(5)
    tx, ty, n = 8, 8, 300
    depth, rect, tc = _random_rects(rng, n, tx, ty)
    depth = rng.permutation(np.arange(1, n + 1)).astype(np.float64)
    perm = rng.permutation(n)
    a = oracle.bin_pairs(depth, rect, tc, tx, ty)
    b = oracle.bin_pairs(depth[perm], rect[perm], tc[perm], tx, ty)
    np.testing.assert_array_equal(a["ranges"], b["ranges"])
    np.testing.assert_array_equal(a["vals"], perm[b["vals"]])


def test_empty_input():
    b = oracle.bin_pairs(np.zeros(0), np.zeros((0, 4), np.int32), np.zeros(0, np.int32), 3, 2)
    assert b["I"] == 0
    assert np.all(b["ranges"] == 0)
