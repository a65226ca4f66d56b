"""The oracle's pins are discriminating: each plausible mistake planted in a
copy of the oracle's source (compiled on the CPU into a temporary library)
makes at least one pin fail.  The real oracle is untouched."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1712_09789_amd import workloads as wl
from tests.bfs import all_images, bfs_label, stack_with_gaps, unstack_labels

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "ccl_oracle.c")

MUTANTS = {
    "drop_up_right_diagonal": (
        "if (x + 1 < W && img[(y - 1) * pitch + x + 1] != 0)\n"
        "                        unite(parent, p, p - W + 1);", ""),
    "drop_up_left_diagonal": (
        "if (x > 0 && img[(y - 1) * pitch + x - 1] != 0)\n"
        "                        unite(parent, p, p - W - 1);", ""),
    "drop_left_link": (
        "if (x > 0 && img[y * pitch + x - 1] != 0) unite(parent, p, p - 1);", ""),
    "larger_root_wins": (
        "if (ra < rb) parent[rb] = ra;", "if (ra > rb) parent[rb] = ra;"),
    "no_plus_one": (
        "(int32_t)(find_root(parent, p) + 1)", "(int32_t)(find_root(parent, p))"),
    "width_instead_of_pitch": (
        "if (img[y * pitch + x] == 0) continue;", "if (img[y * W + x] == 0) continue;"),
    "right_edge_wraps": ("x + 1 < W &&", "x + 1 <= W &&"),
    "wrong_diagonal_index": ("p - W + 1);", "p - W - 1);"),
    "background_labelled": (
        "img[y * pitch + x] != 0 ? (int32_t)(find_root(parent, p) + 1) : 0",
        "(int32_t)(find_root(parent, p) + 1)"),
    "up_row_read_with_width": (
        "if (img[(y - 1) * pitch + x] != 0) unite(parent, p, p - W);",
        "if (img[(y - 1) * W + x] != 0) unite(parent, p, p - W);"),
}


def build_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mut = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mut)
    subprocess.run(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-w", "-o",
                    str(so), str(c)], check=True)
    lib = ctypes.CDLL(str(so))
    lib.oracle_label.restype = ctypes.c_int
    lib.oracle_label.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]

    def label(img, conn):
        H, W = img.shape
        out = np.zeros((H, W), np.int32)
        rc = lib.oracle_label(img.ctypes.data, H, W, img.strides[0], conn,
                              out.ctypes.data)
        assert rc == 0
        return out
    return label


def pins_pass(label):
    """A condensed run of the oracle's pins; False as soon as one fails."""
    for conn in (4, 8):
        imgs = all_images(3, 4)
        tall = stack_with_gaps(imgs)
        got = unstack_labels(label(tall, conn), len(imgs), 3, 4)
        if not np.array_equal(got, unstack_labels(bfs_label(tall, conn), len(imgs), 3, 4)):
            return False
    img = wl.bernoulli(23, 30, 0.5, seed=1)
    padded = np.full((23, 40), 9, np.uint8)
    padded[:, :30] = img
    for conn in (4, 8):
        if not np.array_equal(label(padded[:, :30], conn), bfs_label(img, conn)):
            return False
    return True


def test_real_oracle_passes_condensed_pins():
    from oracle import oracle_label
    assert pins_pass(oracle_label)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    assert not pins_pass(build_mutant(name, tmp_path))
