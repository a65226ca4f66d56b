"""Pins of the 4x4 pattern table used by the exhaustive seam tests: every
pattern's labels equal brute-force flood fill on the pattern alone, and
patterns placed anywhere in a larger empty image keep those labels,
translated (flood fill on the whole image)."""
import numpy as np
import pytest

from bfs import bfs_label
from seam_atlas import NPAT, SIDE, expected_labels, pattern_bits, rel_table


@pytest.mark.parametrize("conn", [4, 8])
def test_table_equals_flood_fill_every_pattern(conn):
    rel = rel_table(conn)
    bits = pattern_bits()
    for p in range(NPAT):
        img = bits[p].reshape(SIDE, SIDE)
        want = bfs_label(img, conn).reshape(16)
        got = expected_labels(rel[p:p + 1], np.array([0]), np.array([0]), SIDE)[0]
        assert np.array_equal(got, want), (p, conn)


@pytest.mark.parametrize("conn", [4, 8])
def test_table_placed_in_larger_image(conn):
    rel = rel_table(conn)
    bits = pattern_bits()
    rng = np.random.default_rng(conn)
    H, W = 61, 73
    for trial in range(20):
        img = np.zeros((H, W), np.uint8)
        want = np.zeros((H, W), np.int64)
        # one pattern per 6 x 6 box at a random offset: at least one
        # background row and column between any two patterns
        for by in range(0, H - 5, 6):
            for bx in range(0, W - 5, 6):
                y0, x0 = by + int(rng.integers(0, 2)), bx + int(rng.integers(0, 2))
                p = int(rng.integers(NPAT))
                img[y0:y0 + SIDE, x0:x0 + SIDE] = bits[p].reshape(SIDE, SIDE)
                want[y0:y0 + SIDE, x0:x0 + SIDE] = expected_labels(
                    rel[p:p + 1], np.array([y0]), np.array([x0]), W)[0].reshape(SIDE, SIDE)
        assert np.array_equal(bfs_label(img, conn), want), (trial, conn)


def test_table_special_patterns():
    r4, r8 = rel_table(4), rel_table(8)
    assert (r4[0] == -1).all() and (r8[0] == -1).all()
    assert (r4[NPAT - 1] == 0).all() and (r8[NPAT - 1] == 0).all()
    # checkerboard with cell 0 set: 8 singletons under 4-connectivity, one
    # component under 8-connectivity
    cb = sum(1 << k for k in range(16) if (k // 4 + k % 4) % 2 == 0)
    fgc = [k for k in range(16) if (k // 4 + k % 4) % 2 == 0]
    assert [int(r4[cb][k]) for k in fgc] == fgc
    assert all(int(r8[cb][k]) == 0 for k in fgc)


@pytest.mark.parametrize("rows", [32, 64, 128])
@pytest.mark.parametrize("conn", [4, 8])
def test_seam_layout_assembly(conn, rows):
    """The exhaustive seam test's image assembly (run here on the CPU at a
    smaller size), for every tile height (merge groups of 256 x 256 pixels):
    the oracle's labels of each assembled image equal the expected map built
    from the pattern table, and the sites never touch."""
    import torch
    from oracle import oracle_label
    from seam_atlas import Layout
    gy = 256 // rows
    L = Layout(512 + 2 * rows, 704, rows, 64, (gy, 4), conn, "cpu")
    cells = L.pos.reshape(-1)
    assert cells.unique().numel() == cells.numel()
    for n in (0, 1, 7):
        L.assemble(n)
        img = L.img.view(L.H, 704).numpy()
        want = L.want.view(L.H, 704).numpy()
        assert np.array_equal(oracle_label(img, conn), want), (n, conn)
    assert set(k[0] for k in L.keys) == {"corner", "vseam", "hseam"}
    assert len(L.keys) == gy * 4 + 4 + gy
