"""Pins for the 3-D oracle (6- and 26-connectivity), each checked against
something other than the oracle itself: brute-force flood fill on every
2x2x2 and 1x3x3 volume and on random volumes, scipy.ndimage.label with the
3-D face / full structures, closed forms, and the 2-D oracle on one-slice
volumes.  Plausible slips planted in a copy of the C source (a dropped link
to the previous slice, a dropped diagonal) must fail the brute-force pin."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from bfs import bfs_label3d
from oracle import oracle_label, oracle_label3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def all_volumes(d, h, w):
    n = d * h * w
    codes = np.arange(1 << n, dtype=np.int64)
    bits = (codes[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1
    return bits.astype(np.uint8).reshape(-1, d, h, w)


@pytest.mark.parametrize("conn", [6, 26])
@pytest.mark.parametrize("shape", [(2, 2, 2), (1, 3, 3), (3, 1, 3), (3, 3, 1)])
def test_exhaustive_small(conn, shape):
    for v in all_volumes(*shape):
        assert np.array_equal(oracle_label3d(v, conn), bfs_label3d(v, conn))


@pytest.mark.parametrize("conn", [6, 26])
@pytest.mark.parametrize("seed", range(5))
def test_random_vs_brute_force(conn, seed):
    rng = np.random.default_rng(seed)
    D, H, W = (int(x) for x in rng.integers(1, 9, size=3))
    v = (rng.random((D, H, W)) < rng.uniform(0.2, 0.7)).astype(np.uint8)
    assert np.array_equal(oracle_label3d(v, conn), bfs_label3d(v, conn))


def canonical(lab):
    """Relabel a labelling so that each component's label is 1 + its smallest
    raster position (background stays 0)."""
    flat = lab.ravel()
    out = np.zeros(flat.shape, np.int64)
    fg = np.flatnonzero(flat)
    if len(fg):
        first = {}
        for p in fg:  # raster order: the first occurrence is the minimum
            first.setdefault(int(flat[p]), int(p))
        out[fg] = [first[int(flat[p])] + 1 for p in fg]
    return out.reshape(lab.shape)


@pytest.mark.parametrize("conn,rank", [(6, 1), (26, 3)])
@pytest.mark.parametrize("seed", range(3))
def test_scipy(conn, rank, seed):
    from scipy import ndimage
    rng = np.random.default_rng(100 + seed)
    v = (rng.random((12, 17, 23)) < 0.45).astype(np.uint8)
    lab, _ = ndimage.label(v, structure=ndimage.generate_binary_structure(3, rank))
    assert np.array_equal(oracle_label3d(v, conn), canonical(lab))


def test_closed_forms():
    D, H, W = 5, 6, 7
    full = np.ones((D, H, W), np.uint8)
    for conn in (6, 26):
        assert (oracle_label3d(full, conn) == 1).all()
        assert not oracle_label3d(np.zeros((D, H, W), np.uint8), conn).any()
    z, y, x = np.indices((D, H, W))
    cb = ((x + y + z) % 2 == 0).astype(np.uint8)
    pos = z * H * W + y * W + x + 1
    assert np.array_equal(oracle_label3d(cb, 6), np.where(cb == 1, pos, 0))  # every voxel alone
    assert np.array_equal(oracle_label3d(cb, 26), cb.astype(np.int32))      # one component, label 1
    # separated boxes: label = 1 + the box's first corner
    v = np.zeros((10, 12, 14), np.uint8)
    boxes = [(0, 0, 0, 2, 3, 4), (5, 1, 6, 3, 4, 5), (1, 8, 9, 4, 3, 4)]
    for z0, y0, x0, d, h, w in boxes:
        v[z0:z0 + d, y0:y0 + h, x0:x0 + w] = 1
    for conn in (6, 26):
        lab = oracle_label3d(v, conn)
        for z0, y0, x0, d, h, w in boxes:
            assert (lab[z0:z0 + d, y0:y0 + h, x0:x0 + w] == z0 * 168 + y0 * 14 + x0 + 1).all()


@pytest.mark.parametrize("conn2,conn3", [(4, 6), (8, 26)])
def test_one_slice_is_the_2d_labelling(conn2, conn3):
    img = (np.random.default_rng(7).random((40, 50)) < 0.5).astype(np.uint8)
    assert np.array_equal(oracle_label3d(img[None], conn3)[0], oracle_label(img, conn2))


def test_strided_volume():
    rng = np.random.default_rng(3)
    big = (rng.random((6, 9, 40)) < 0.5).astype(np.uint8)
    v = big[:, 1:8, 3:30]  # non-contiguous view
    assert np.array_equal(oracle_label3d(v, 26), bfs_label3d(np.ascontiguousarray(v), 26))


MUTANTS = {
    "no_previous_slice_link": (r"if \(z > 0 && FG\(x, y, z - 1\)\) unite\(parent, p, p - S\);", ""),
    "no_row_above_diagonals": (r"for \(int64_t dx = -1; dx <= 1; \+\+dx\) \{\n(\s+)const int64_t xx = x \+ dx;\n(\s+)if \(xx >= 0 && xx < W && FG\(xx, y - 1, z\)\)",
                               r"for (int64_t dx = 0; dx <= 0; ++dx) {\n\1const int64_t xx = x + dx;\n\2if (xx >= 0 && xx < W && FG(xx, y - 1, z))"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_slips_are_caught(tmp_path, name):
    src = open(os.path.join(ROOT, "oracle", "ccl_oracle.c")).read()
    pat, rep = MUTANTS[name]
    mutated, n = re.subn(pat, rep, src)
    assert n == 1, name
    c = tmp_path / "m.c"
    c.write_text(mutated)
    so = tmp_path / "m.so"
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-o", str(so), str(c)], check=True)
    lib = ctypes.CDLL(str(so))
    lib.oracle_label3d.restype = ctypes.c_int
    lib.oracle_label3d.argtypes = [ctypes.c_void_p] + [ctypes.c_int64] * 5 + [ctypes.c_int32,
                                                                               ctypes.c_void_p]
    caught = False
    rng = np.random.default_rng(0)
    for _ in range(20):
        v = (rng.random((4, 5, 6)) < 0.5).astype(np.uint8)
        for conn in (6, 26):
            out = np.zeros(v.shape, np.int32)
            lib.oracle_label3d(v.ctypes.data, 4, 5, 6, 6, 30, conn, out.ctypes.data)
            if not np.array_equal(out, bfs_label3d(v, conn)):
                caught = True
    assert caught, name
