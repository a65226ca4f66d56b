"""Pins for the oracle's per-component statistics (area, inclusive bounding
box, coordinate sums) — checked against things other than the oracle itself:
brute-force flood fill with the statistics gathered pixel by pixel, closed
forms for images whose components are known, and invariants that hold for any
image.  Plausible slips in the statistics (swapped axes, an exclusive box
edge, an off-by-one sum) are planted in copies of its output and must fail
the brute-force pin."""
import numpy as np
import pytest

from oracle import STATS_DTYPE, oracle_label, oracle_stats
from bfs import all_images, bfs_label
from paper_1712_09789_amd import workloads as wl


def brute_stats(img, conn):
    """Statistics from a BFS labelling, gathered with plain loops."""
    lab = bfs_label(img, conn)
    H, W = img.shape
    comps = {}
    for y in range(H):
        for x in range(W):
            L = int(lab[y, x])
            if L == 0:
                continue
            c = comps.setdefault(L, [0, x, y, x, y, 0, 0])
            c[0] += 1
            c[1] = min(c[1], x)
            c[2] = min(c[2], y)
            c[3] = max(c[3], x)
            c[4] = max(c[4], y)
            c[5] += x
            c[6] += y
    out = np.zeros(len(comps), dtype=STATS_DTYPE)
    for i, L in enumerate(sorted(comps)):
        out[i] = (L, *comps[L])
    return out


def same(a, b):
    return a.shape == b.shape and all(np.array_equal(a[f], b[f]) for f in STATS_DTYPE.names)


@pytest.mark.parametrize("conn", [4, 8])
def test_exhaustive_3x3(conn):
    for img in all_images(3, 3):
        assert same(oracle_stats(img, conn), brute_stats(img, conn))


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("seed", range(6))
def test_random_vs_brute_force(conn, seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    img = wl.bernoulli(H, W, float(rng.uniform(0.2, 0.8)), seed=seed)
    assert same(oracle_stats(img, conn), brute_stats(img, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_full_image_closed_form(conn):
    H, W = 13, 21
    s = oracle_stats(np.ones((H, W), np.uint8), conn)
    assert len(s) == 1
    assert tuple(s[0]) == (1, H * W, 0, 0, W - 1, H - 1, H * W * (W - 1) // 2, W * H * (H - 1) // 2)


def test_checkerboard_4_every_pixel_alone():
    img = wl.checkerboard(9, 11)
    s = oracle_stats(img, 4)
    ys, xs = np.nonzero(img)
    assert len(s) == len(ys)
    order = np.argsort(ys * 11 + xs)
    assert np.array_equal(s["label"], (ys * 11 + xs)[order] + 1)
    assert np.all(s["area"] == 1)
    assert np.array_equal(s["x_min"], xs[order]) and np.array_equal(s["x_max"], xs[order])
    assert np.array_equal(s["y_min"], ys[order]) and np.array_equal(s["y_max"], ys[order])
    assert np.array_equal(s["sum_x"], xs[order]) and np.array_equal(s["sum_y"], ys[order])


def test_separated_rectangles_closed_form():
    H, W = 40, 50
    rects = [(2, 3, 5, 7), (10, 1, 4, 20), (20, 30, 15, 10), (36, 45, 3, 2)]  # y, x, h, w
    img = np.zeros((H, W), np.uint8)
    for y, x, h, w in rects:
        img[y:y + h, x:x + w] = 1
    for conn in (4, 8):
        s = oracle_stats(img, conn)
        assert len(s) == len(rects)
        want = sorted(rects, key=lambda r: r[0] * W + r[1])
        for row, (y, x, h, w) in zip(s, want):
            assert row["label"] == y * W + x + 1
            assert row["area"] == h * w
            assert (row["x_min"], row["y_min"], row["x_max"], row["y_max"]) == (x, y, x + w - 1, y + h - 1)
            assert row["sum_x"] == h * (w * x + w * (w - 1) // 2)
            assert row["sum_y"] == w * (h * y + h * (h - 1) // 2)


@pytest.mark.parametrize("conn", [4, 8])
def test_invariants_random(conn):
    img = wl.bernoulli(97, 131, 0.55, seed=3)
    H, W = img.shape
    s = oracle_stats(img, conn)
    lab = oracle_label(img, conn)
    assert s["area"].sum() == np.count_nonzero(img)
    assert np.all(np.diff(s["label"]) > 0)
    assert len(s) == len(np.unique(lab[lab > 0]))
    ry, rx = (s["label"] - 1) // W, (s["label"] - 1) % W
    # the smallest pixel lies on the top row of the box, inside it
    assert np.array_equal(ry, s["y_min"])
    assert np.all((s["x_min"] <= rx) & (rx <= s["x_max"]))
    assert np.all(s["x_min"] * s["area"] <= s["sum_x"]) and np.all(s["sum_x"] <= s["x_max"] * s["area"])
    assert np.all(s["y_min"] * s["area"] <= s["sum_y"]) and np.all(s["sum_y"] <= s["y_max"] * s["area"])


def _swap_axes(s):
    t = s.copy()
    t["x_min"], t["y_min"] = s["y_min"], s["x_min"]
    t["x_max"], t["y_max"] = s["y_max"], s["x_max"]
    t["sum_x"], t["sum_y"] = s["sum_y"], s["sum_x"]
    return t


def _exclusive_box(s):
    t = s.copy()
    t["x_max"] += 1
    return t


def _sum_off_by_area(s):
    t = s.copy()
    t["sum_x"] += t["area"]  # columns counted from 1
    return t


@pytest.mark.parametrize("mutant", [_swap_axes, _exclusive_box, _sum_off_by_area])
def test_planted_slips_are_caught(mutant):
    img = wl.bernoulli(23, 17, 0.5, seed=11)
    for conn in (4, 8):
        assert not same(mutant(oracle_stats(img, conn)), brute_stats(img, conn))
