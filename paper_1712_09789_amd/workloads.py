"""Seeded synthetic binary images shaped like the paper's workloads.

This module only draws inputs; it holds none of the labelling arithmetic.
Both the GPU path and the CPU oracle are fed the very same bytes produced
here, never two regenerations.

Contents (the paper evaluates on random-noise images of several sizes and
foreground densities, Section 4.1 and Section 4.2; its natural images are not
available, so smoothed-threshold blobs stand in for large coherent regions):

* ``bernoulli``    i.i.d. foreground with probability p;
* ``blobs``        uniform noise smoothed by a Gaussian of width sigma, then
                   thresholded at a quantile (the median by default);
* ``checkerboard`` (x + y) even is foreground, so (0, 0) is foreground;
* ``spiral``       a one-pixel-wide rectangular spiral with one-pixel gaps that
                   starts at (0, 0) and winds inwards (a single component);
* ``serpentine``   stripes of width w separated by gaps of width w, joined at
                   alternating ends (a single component);
* ``full`` / ``empty`` and ``stripes`` (k separated horizontal lines).

All generators return C-contiguous ``uint8`` arrays with values {0, 1}
(``value`` lets a test encode foreground as another nonzero byte).
"""
from __future__ import annotations

import math

import numpy as np


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def bernoulli(H: int, W: int, p: float, seed: int = 0, value: int = 1) -> np.ndarray:
    rng = rng_for(seed)
    return (rng.random((H, W)) < p).astype(np.uint8) * np.uint8(value)


def blobs(H: int, W: int, sigma: float, seed: int = 0, quantile: float = 0.5,
          value: int = 1) -> np.ndarray:
    from scipy.ndimage import gaussian_filter

    rng = rng_for(seed)
    u = rng.random((H, W), dtype=np.float32)
    s = gaussian_filter(u, sigma=sigma, mode="reflect", truncate=4.0)
    thr = np.quantile(s, quantile)
    return (s > thr).astype(np.uint8) * np.uint8(value)


def checkerboard(H: int, W: int, value: int = 1) -> np.ndarray:
    yy, xx = np.indices((H, W))
    return (((xx + yy) & 1) == 0).astype(np.uint8) * np.uint8(value)


def full(H: int, W: int, value: int = 1) -> np.ndarray:
    return np.full((H, W), value, dtype=np.uint8)


def empty(H: int, W: int) -> np.ndarray:
    return np.zeros((H, W), dtype=np.uint8)


def stripes(H: int, W: int, period: int = 2, value: int = 1) -> np.ndarray:
    """Full-width horizontal lines on rows 0, period, 2*period, ..."""
    img = np.zeros((H, W), dtype=np.uint8)
    img[::period, :] = value
    return img


def spiral(H: int, W: int, value: int = 1) -> np.ndarray:
    """One-pixel line, one-pixel gap, rectangular, starting at (0, 0).

    Layer k walks right along row 2k, down column W-1-2k, left along row
    H-1-2k and up column 2k to row 2k+2, where layer k+1 begins.  Every
    segment starts where the previous one ended, so the drawn set is one
    4-connected path.
    """
    img = np.zeros((H, W), dtype=np.uint8)
    if H == 0 or W == 0:
        return img
    y, x = 0, 0
    img[0, 0] = value
    k = 0
    while True:
        # right along row 2k
        tx = W - 1 - 2 * k
        if tx > x:
            img[y, x:tx + 1] = value
            x = tx
        else:
            break
        # down column W-1-2k
        ty = H - 1 - 2 * k
        if ty > y:
            img[y:ty + 1, x] = value
            y = ty
        else:
            break
        # left along row H-1-2k
        tx = 2 * k
        if tx < x:
            img[y, tx:x + 1] = value
            x = tx
        else:
            break
        # up column 2k to row 2k+2
        ty = 2 * k + 2
        if ty < y:
            img[ty:y + 1, x] = value
            y = ty
        else:
            break
        k += 1
    return img


def serpentine(H: int, W: int, width: int = 1, vertical: bool = False,
               value: int = 1) -> np.ndarray:
    """Stripes of ``width`` pixels with ``width``-pixel gaps, joined at
    alternating ends (right end after stripe 0, left end after stripe 1, ...).

    ``vertical=True`` draws the same pattern transposed.
    """
    if vertical:
        return np.ascontiguousarray(serpentine(W, H, width, False, value).T)
    img = np.zeros((H, W), dtype=np.uint8)
    period = 2 * width
    nstripes = (H + period - 1) // period
    for i in range(nstripes):
        y0 = i * period
        img[y0:min(y0 + width, H), :] = value
        # connector through the gap below stripe i, if a stripe follows
        g0, g1 = y0 + width, min(y0 + period, H)
        if i + 1 < nstripes and g0 < H:
            if i % 2 == 0:
                img[g0:g1, max(W - width, 0):] = value
            else:
                img[g0:g1, :min(width, W)] = value
    return img


# ---------------------------------------------------------------------------
# named workload families
# ---------------------------------------------------------------------------

DENSITIES = (0.1, 0.3, 0.5, 0.7, 0.9)
BLOB_SIGMAS = (4, 16)


def single_image_contents():
    """The 7 content kinds of the 2048^2 / 4096^2 single-image sweep:
    Bernoulli at five densities and blobs at two widths."""
    out = [("bernoulli", {"p": p}) for p in DENSITIES]
    out += [("blobs", {"sigma": s}) for s in BLOB_SIGMAS]
    return out


def make(kind: str, H: int, W: int, seed: int = 0, **kw) -> np.ndarray:
    if kind == "bernoulli":
        return bernoulli(H, W, kw.get("p", 0.5), seed, kw.get("value", 1))
    if kind == "blobs":
        return blobs(H, W, kw.get("sigma", 4), seed, kw.get("quantile", 0.5),
                     kw.get("value", 1))
    if kind == "checkerboard":
        return checkerboard(H, W, kw.get("value", 1))
    if kind == "full":
        return full(H, W, kw.get("value", 1))
    if kind == "empty":
        return empty(H, W)
    if kind == "spiral":
        return spiral(H, W, kw.get("value", 1))
    if kind == "serpentine":
        return serpentine(H, W, kw.get("width", 1), kw.get("vertical", False),
                          kw.get("value", 1))
    if kind == "stripes":
        return stripes(H, W, kw.get("period", 2), kw.get("value", 1))
    raise ValueError(f"unknown workload kind {kind!r}")


ADVERSARIAL = (
    ("spiral", {}),
    ("serpentine", {"width": 1}),
    ("serpentine", {"width": 3}),
    ("checkerboard", {}),
    ("full", {}),
)


def batch_specs(n: int = 256, seed: int = 0, lo: int = 64, hi: int = 2048):
    """Uneven batch: H and W drawn independently log-uniform in [lo, hi];
    content half Bernoulli (p ~ U[0.1, 0.9]) and half blobs (sigma 4 or 16,
    threshold quantile ~ U[0.1, 0.9])."""
    rng = rng_for(seed)
    specs = []
    for i in range(n):
        H = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        W = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        if rng.random() < 0.5:
            specs.append((H, W, "bernoulli", {"p": float(rng.uniform(0.1, 0.9))},
                          seed * 100003 + i))
        else:
            specs.append((H, W, "blobs", {"sigma": int(rng.choice(BLOB_SIGMAS)),
                                          "quantile": float(rng.uniform(0.1, 0.9))},
                          seed * 100003 + i))
    return specs


SERVING_MIX = ((480, 640, 0.5), (1080, 1920, 0.35), (2160, 3840, 0.15))


def serving_frames(n: int, seed: int = 0):
    """Frame sizes for the serving stream (640x480 / 1920x1080 / 3840x2160
    with weights 0.5 / 0.35 / 0.15), blob content with sigma 8."""
    rng = rng_for(seed)
    w = np.array([m[2] for m in SERVING_MIX])
    idx = rng.choice(len(SERVING_MIX), size=n, p=w / w.sum())
    return [(SERVING_MIX[i][0], SERVING_MIX[i][1], seed * 1000003 + k)
            for k, i in enumerate(idx)]


# ---------------------------------------------------------------------------
# volumes [z, y, x]
# ---------------------------------------------------------------------------

def bernoulli3d(D: int, H: int, W: int, p: float, seed: int = 0) -> np.ndarray:
    rng = rng_for(seed)
    return (rng.random((D, H, W)) < p).astype(np.uint8)


def blobs3d(D: int, H: int, W: int, sigma: float, seed: int = 0,
            quantile: float = 0.5) -> np.ndarray:
    """Uniform noise smoothed by a 3-D Gaussian and thresholded at a quantile
    (coherent regions, like a segmented scan)."""
    from scipy.ndimage import gaussian_filter

    rng = rng_for(seed)
    u = rng.random((D, H, W), dtype=np.float32)
    s = gaussian_filter(u, sigma=sigma, mode="reflect", truncate=4.0)
    return (s > np.quantile(s, quantile)).astype(np.uint8)


def checkerboard3d(D: int, H: int, W: int) -> np.ndarray:
    z, y, x = np.indices((D, H, W))
    return ((x + y + z) % 2 == 0).astype(np.uint8)


def make3d(kind: str, D: int, H: int, W: int, seed: int = 0, **kw) -> np.ndarray:
    if kind == "bernoulli":
        return bernoulli3d(D, H, W, kw.get("p", 0.5), seed)
    if kind == "blobs":
        return blobs3d(D, H, W, kw.get("sigma", 2.0), seed, kw.get("quantile", 0.5))
    if kind == "checkerboard":
        return checkerboard3d(D, H, W)
    if kind == "full":
        return np.ones((D, H, W), np.uint8)
    if kind == "empty":
        return np.zeros((D, H, W), np.uint8)
    if kind == "slabs":  # full even slices, empty odd ones: one component per even slice
        v = np.zeros((D, H, W), np.uint8)
        v[::2] = 1
        return v
    raise ValueError(kind)

