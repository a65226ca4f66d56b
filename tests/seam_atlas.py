"""Every 4x4 binary pattern (2^16 of them) and its canonical labelling, for
the exhaustive seam tests.

The patterns are laid out on an atlas, 256 per row, each followed by a
background row and column, and the atlas is labelled by the oracle once per
connectivity.  A pattern's components then lie inside its 4x4 cell, and
because raster order inside a cell is the same wherever the cell sits, one
table per connectivity describes the labels of the pattern placed anywhere
in an otherwise empty image:

    rel[p, c] = cell index (0..15, row-major) of the smallest pixel of the
                component that holds cell c of pattern p, or -1 for background.

A pattern with its top-left cell at (y0, x0) of a W-wide image then has the
label 1 + (y0 + rel // 4) * W + (x0 + rel % 4) at cell c (0 where rel < 0).
Bit k of the pattern id is cell k.
"""
from __future__ import annotations

import functools

import numpy as np
import torch

from oracle import oracle_label

NPAT = 1 << 16
SIDE = 4
STEP_ALONG = SIDE + 1  # pattern spacing along a seam
GRID = 256          # patterns per atlas row (and rows of patterns)
STEP = SIDE + 1     # a background row / column after every pattern


@functools.lru_cache(maxsize=None)
def pattern_bits() -> np.ndarray:
    """(NPAT, 16) uint8: cell k of pattern p is bit k of p."""
    p = np.arange(NPAT, dtype=np.uint32)[:, None]
    return ((p >> np.arange(16, dtype=np.uint32)[None, :]) & 1).astype(np.uint8)


def atlas() -> np.ndarray:
    """All patterns on one (GRID * STEP)^2 image, pattern p at
    (STEP * (p // GRID), STEP * (p % GRID))."""
    cells = pattern_bits().reshape(GRID, GRID, SIDE, SIDE)
    img = np.zeros((GRID, STEP, GRID, STEP), np.uint8)
    img[:, :SIDE, :, :SIDE] = cells.transpose(0, 2, 1, 3)
    return img.reshape(GRID * STEP, GRID * STEP)


@functools.lru_cache(maxsize=None)
def rel_table(connectivity: int) -> np.ndarray:
    """(NPAT, 16) int8 table of the module docstring, from the oracle's
    labelling of the atlas."""
    A = atlas()
    Wa = A.shape[1]
    lab = oracle_label(A, connectivity).astype(np.int64)
    lab = lab.reshape(GRID, STEP, GRID, STEP)[:, :SIDE, :, :SIDE].transpose(0, 2, 1, 3)
    lab = lab.reshape(NPAT, SIDE, SIDE)
    p = np.arange(NPAT)
    oy = (STEP * (p // GRID))[:, None, None]
    ox = (STEP * (p % GRID))[:, None, None]
    pos = lab - 1
    ry, rx = pos // Wa - oy, pos % Wa - ox
    rel = np.where(lab > 0, ry * SIDE + rx, -1).reshape(NPAT, 16)
    # every label must point inside the pattern's own cell
    fg = lab.reshape(NPAT, 16) > 0
    assert ((rel >= 0) == fg).all() and (rel < 16).all()
    return rel.astype(np.int8)


def expected_labels(rel_rows: np.ndarray, y0: np.ndarray, x0: np.ndarray, W: int) -> np.ndarray:
    """Labels of patterns (rows of `rel_table`) placed at (y0, x0) in a W-wide
    image, shape (n, 16); 0 on background cells."""
    r = rel_rows.astype(np.int64)
    lab = 1 + (y0[:, None] + r // SIDE) * W + x0[:, None] + r % SIDE
    return np.where(r >= 0, lab, 0)


def sites(H, W, rows, cols, G):
    """Top-left corners of the pattern sites, by class.  G = tiles per merge
    group side, or (tiles per group column, tiles per group row)."""
    GY, GX = (G, G) if isinstance(G, int) else G
    out = {}
    nty, ntx = H // rows, W // cols
    # corners of four tiles
    for k in range(1, nty):
        for i in range(1, ntx):
            out.setdefault(("corner", k % GY, i % GX), []).append((k * rows - 2, i * cols - 2))
    # along vertical seams, between the corner patterns (gap row on each side)
    along_v = list(range(3, rows - SIDE - 3, STEP_ALONG))
    along_h = list(range(3, cols - SIDE - 3, STEP_ALONG))
    for i in range(1, ntx):
        for k in range(nty):
            for r in along_v:
                out.setdefault(("vseam", i % GX), []).append((k * rows + r, i * cols - 2))
    for k in range(1, nty):
        for i in range(ntx):
            for c in along_h:
                out.setdefault(("hseam", k % GY), []).append((k * rows - 2, i * cols + c))
    return {key: np.array(v, np.int64) for key, v in out.items()}


class Layout:
    """Sites of one image size and tile grid, and the tensors that place the
    n-th assignment of patterns on them."""

    def __init__(self, H, W, rows, cols, G, conn, device):
        self.H, self.W = H, W
        by_class = sites(H, W, rows, cols, G)
        self.keys = sorted(by_class)
        self.counts = {k: len(by_class[k]) for k in self.keys}
        self.n_images = -(-NPAT // min(self.counts.values()))
        dev = torch.device(device)
        self.bits = torch.from_numpy(pattern_bits().astype(bool)).to(dev)
        self.rel = torch.from_numpy(rel_table(conn).astype(np.int64)).to(dev)
        self.y0 = torch.from_numpy(np.concatenate([by_class[k][:, 0] for k in self.keys])).to(dev)
        self.x0 = torch.from_numpy(np.concatenate([by_class[k][:, 1] for k in self.keys])).to(dev)
        self.cls = np.concatenate([np.full(self.counts[k], j) for j, k in enumerate(self.keys)])
        local = np.concatenate([np.arange(self.counts[k]) for k in self.keys])
        cnt = np.array([self.counts[k] for k in self.keys])[self.cls]
        self.local = torch.from_numpy(local).to(dev)
        self.cnt = torch.from_numpy(cnt).to(dev)
        dy = torch.arange(16, device=dev) // SIDE
        dx = torch.arange(16, device=dev) % SIDE
        self.pos = (self.y0[:, None] + dy[None, :]) * W + self.x0[:, None] + dx[None, :]
        self.img = torch.empty(H * W, dtype=torch.uint8, device=dev)
        self.want = torch.empty(H * W, dtype=torch.int32, device=dev)

    def assemble(self, n):
        """Image n and its expected labels (flat tensors); returns the
        pattern id of every site."""
        pid = (n * self.cnt + self.local) % NPAT
        r = self.rel[pid]
        self.img.zero_()
        self.img[self.pos[self.bits[pid]]] = 1
        lab = 1 + (self.y0[:, None] + r // SIDE) * self.W + self.x0[:, None] + r % SIDE
        self.want.zero_()
        self.want[self.pos[r >= 0]] = lab[r >= 0].to(torch.int32)
        return pid

    def describe(self, pid, bad):
        hit = torch.nonzero((self.pos == bad).any(dim=1))
        if not hit.numel():
            return "outside every pattern"
        s = int(hit[0])
        return (f"site {s} class {self.keys[self.cls[s]]} at ({int(self.y0[s])}, "
                f"{int(self.x0[s])}), pattern {int(pid[s]):#06x}")
