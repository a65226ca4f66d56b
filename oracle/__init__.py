"""CPU oracle for connected-components labelling — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library and its Python binding never import
it; the two share no code.

``oracle_label(img, connectivity)`` returns the canonical labelling of a
binary image, as defined in the paper's problem statement (Section 3, first
paragraph: pixel position P(x, y) = x + y * W, foreground I = 1): background
pixels get 0, a foreground pixel gets 1 + the smallest position in its
4- or 8-connected component.  The arithmetic lives in ``ccl_oracle.c`` (a
plain two-pass union-find); this module only loads it and marshals numpy
arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-Wall", "-Wextra",
             "-o", tmp, _SRC],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_label.restype = ctypes.c_int
        lib.oracle_label.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int32, ctypes.c_void_p,
        ]
        lib.oracle_label3d.restype = ctypes.c_int
        lib.oracle_label3d.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
        ]
        _lib = lib
    return _lib


def oracle_label(img: np.ndarray, connectivity: int = 8) -> np.ndarray:
    """Canonical labels of a 2-D uint8 image (nonzero = foreground).

    ``img`` may be a strided view whose rows are contiguous; the row pitch in
    bytes is taken from its first stride.  Returns a dense int32 H x W array.
    """
    if img.ndim != 2 or img.dtype != np.uint8:
        raise ValueError("oracle_label expects a 2-D uint8 array")
    H, W = img.shape
    out = np.zeros((H, W), dtype=np.int32)
    if H == 0 or W == 0:
        return out
    if img.strides[1] != 1 or img.strides[0] < W:
        img = np.ascontiguousarray(img)
    pitch = img.strides[0]
    rc = _load().oracle_label(img.ctypes.data, H, W, pitch, int(connectivity),
                              out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_label failed with status {rc}")
    return out


def oracle_label3d(vol: np.ndarray, connectivity: int = 26) -> np.ndarray:
    """Canonical labels of a 3-D uint8 volume indexed [z, y, x] (nonzero =
    foreground), 6- or 26-connectivity: 0 for background, else 1 + the
    smallest position x + y * W + z * W * H in the component.  Rows must be
    contiguous; the row and slice pitches come from the strides."""
    if vol.ndim != 3 or vol.dtype != np.uint8:
        raise ValueError("oracle_label3d expects a 3-D uint8 array")
    D, H, W = vol.shape
    out = np.zeros((D, H, W), dtype=np.int32)
    if D == 0 or H == 0 or W == 0:
        return out
    if (vol.strides[2] != 1 or (H > 1 and vol.strides[1] < W)
            or (D > 1 and vol.strides[0] < (H - 1) * vol.strides[1] + W)):
        vol = np.ascontiguousarray(vol)
    pitch = vol.strides[1] if H > 1 else W
    slice_pitch = vol.strides[0] if D > 1 else H * pitch  # a length-1 axis may carry any stride
    rc = _load().oracle_label3d(vol.ctypes.data, D, H, W, pitch, slice_pitch,
                                int(connectivity), out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_label3d failed with status {rc}")
    return out


# Per-component statistics: the quantities the paper names as the use of a
# labelling (the size and the location of each connected set, Section 1),
# written out from their definitions over the labelled pixels.
STATS_DTYPE = np.dtype([("label", np.int32), ("area", np.int32),
                        ("x_min", np.int32), ("y_min", np.int32),
                        ("x_max", np.int32), ("y_max", np.int32),
                        ("sum_x", np.int64), ("sum_y", np.int64)])


def oracle_stats(img: np.ndarray, connectivity: int = 8) -> np.ndarray:
    """Statistics of every connected component, in ascending label order.

    For the component with label L (1 + its smallest raster position):
    area = number of its pixels; x_min/x_max, y_min/y_max = the smallest and
    largest column and row among them (an inclusive bounding box); sum_x,
    sum_y = the sums of their columns and rows (centroid = sum / area)."""
    lab = oracle_label(img, connectivity)
    ys, xs = np.nonzero(lab)
    labels, inv, area = np.unique(lab[ys, xs], return_inverse=True, return_counts=True)
    n = len(labels)
    out = np.zeros(n, dtype=STATS_DTYPE)
    out["label"] = labels
    out["area"] = area
    big = np.iinfo(np.int32).max
    for field, coord, fn, init in (("x_min", xs, np.minimum, big), ("y_min", ys, np.minimum, big),
                                   ("x_max", xs, np.maximum, -1), ("y_max", ys, np.maximum, -1)):
        acc = np.full(n, init, dtype=np.int64)
        fn.at(acc, inv, coord)
        out[field] = acc
    for field, coord in (("sum_x", xs), ("sum_y", ys)):
        acc = np.zeros(n, dtype=np.int64)
        np.add.at(acc, inv, coord.astype(np.int64))
        out[field] = acc
    return out
