"""Brute-force breadth-first flood fill: the textbook definition of connected
components, used to pin the oracle on small images.

Seeds are taken in raster order, so the seed of each component is its smallest
position and its label is simply 1 + seed (background 0) — the canonical form
the oracle and the GPU path produce.
"""
from collections import deque

import numpy as np


def bfs_label(img: np.ndarray, connectivity: int) -> np.ndarray:
    H, W = img.shape
    fg = (np.asarray(img) != 0).tolist()
    out = [[0] * W for _ in range(H)]
    if connectivity == 4:
        nbrs = ((-1, 0), (1, 0), (0, -1), (0, 1))
    elif connectivity == 8:
        nbrs = tuple((dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                     if (dy, dx) != (0, 0))
    else:
        raise ValueError(connectivity)
    for y0 in range(H):
        row = fg[y0]
        for x0 in range(W):
            if not row[x0] or out[y0][x0]:
                continue
            lab = y0 * W + x0 + 1
            out[y0][x0] = lab
            q = deque([(y0, x0)])
            while q:
                y, x = q.popleft()
                for dy, dx in nbrs:
                    yy, xx = y + dy, x + dx
                    if 0 <= yy < H and 0 <= xx < W and fg[yy][xx] and not out[yy][xx]:
                        out[yy][xx] = lab
                        q.append((yy, xx))
    return np.array(out, dtype=np.int32).reshape(H, W)


def all_images(h: int, w: int) -> np.ndarray:
    """Every binary h x w image, as an array of shape (2**(h*w), h, w)."""
    n = h * w
    codes = np.arange(1 << n, dtype=np.int64)
    bits = (codes[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1
    return bits.astype(np.uint8).reshape(-1, h, w)


def stack_with_gaps(imgs: np.ndarray) -> np.ndarray:
    """Stack images vertically with one background row between them, so that
    no two images touch under either connectivity."""
    k, h, w = imgs.shape
    tall = np.zeros((k * (h + 1), w), dtype=np.uint8)
    tall.reshape(k, h + 1, w)[:, :h, :] = imgs
    return tall


def unstack_labels(labels: np.ndarray, k: int, h: int, w: int) -> np.ndarray:
    """Undo ``stack_with_gaps`` for canonical labels: image i's labels are
    offset by its first position i*(h+1)*w."""
    lab = labels.reshape(k, h + 1, w)[:, :h, :].astype(np.int64)
    base = (np.arange(k, dtype=np.int64) * (h + 1) * w)[:, None, None]
    return np.where(lab > 0, lab - base, 0).astype(np.int32)


def bfs_label3d(vol: np.ndarray, connectivity: int) -> np.ndarray:
    """Flood fill of a [z, y, x] volume, seeds in raster order (so the label
    is 1 + the seed's position x + y*W + z*W*H)."""
    D, H, W = vol.shape
    fg = (np.asarray(vol) != 0)
    out = np.zeros((D, H, W), dtype=np.int64)
    if connectivity == 6:
        nbrs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if abs(dz) + abs(dy) + abs(dx) == 1]
    elif connectivity == 26:
        nbrs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if (dz, dy, dx) != (0, 0, 0)]
    else:
        raise ValueError(connectivity)
    for z0 in range(D):
        for y0 in range(H):
            for x0 in range(W):
                if not fg[z0, y0, x0] or out[z0, y0, x0]:
                    continue
                lab = z0 * H * W + y0 * W + x0 + 1
                out[z0, y0, x0] = lab
                q = deque([(z0, y0, x0)])
                while q:
                    z, y, x = q.popleft()
                    for dz, dy, dx in nbrs:
                        zz, yy, xx = z + dz, y + dy, x + dx
                        if (0 <= zz < D and 0 <= yy < H and 0 <= xx < W and fg[zz, yy, xx]
                                and not out[zz, yy, xx]):
                            out[zz, yy, xx] = lab
                            q.append((zz, yy, xx))
    return out.astype(np.int32)
