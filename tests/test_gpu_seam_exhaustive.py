"""Exhaustive seam parity (the block merge, Section 3.2, Algorithm "Boundary
analysis", Eq. 1-2): every one of the 2^16 4x4 binary patterns is placed
centred on every kind of seam of the tile grid, and the whole image is
compared with the oracle's labels.

Kinds (tiles of 64 columns and R rows, merge groups of 256 x 256 pixels,
i.e. GX = 4 tile columns by GY = 256 / R tile rows):
  vertical seam at tile column i      (class i mod GX; 0 = merge-group seam)
  horizontal seam at tile row k       (class k mod GY; 0 = merge-group seam)
  corner of four tiles at (k, i)      (class (k mod GY, i mod GX): (0, 0) is
                                       a group corner; (k, 0) / (0, i) are the
                                       points where a tile seam meets a group
                                       seam, whose diagonals the merge between
                                       groups handles)
Every class sees all 2^16 patterns, for every tile height the library is
built for (R = 32, 64, 128).  The images are 8192 x 8192: patterns sit on
every tile corner and every fifth row (column) along each seam, each
isolated by background.  Expected labels come from the oracle through the
pattern table (tests/seam_atlas.py); the images and expected label maps are
assembled on the device with plain tensor indexing.
"""
import numpy as np
import pytest

from seam_atlas import NPAT, Layout

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZE = 8192
GROUP_PX = 256  # merge-group side in pixels


@pytest.fixture(scope="module")
def ccl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_09789_amd.ccl as c
    return c


@pytest.mark.parametrize("rows", [32, 64, 128])
@pytest.mark.parametrize("conn", [4, 8])
def test_every_pattern_on_every_seam_kind(ccl, conn, rows):
    cols = ccl.tile_shape()[1]
    L = Layout(SIZE, SIZE, rows, cols, (GROUP_PX // rows, GROUP_PX // cols), conn, "cuda")
    print(f"[seam-exhaustive] conn={conn} tile {rows}x{cols}: {len(L.keys)} classes, "
          f"{sum(L.counts.values())} sites per image, {L.n_images} images", flush=True)
    seen = {k: np.zeros(NPAT, bool) for k in L.keys}
    out = torch.empty((SIZE, SIZE), dtype=torch.int32, device="cuda")
    for n in range(L.n_images):
        pid = L.assemble(n)
        ccl.label(L.img.view(SIZE, SIZE), conn, out=out, tile_rows=rows)
        torch.cuda.synchronize()
        got = out.view(-1)
        if not torch.equal(got, L.want):
            bad = int(torch.nonzero(got != L.want)[0])
            raise AssertionError(f"conn={conn} image {n}: pixel ({bad // SIZE}, {bad % SIZE}) "
                                 f"got {int(got[bad])} want {int(L.want[bad])}; "
                                 f"{L.describe(pid, bad)}")
        pid_h = pid.cpu().numpy()
        for j, k in enumerate(L.keys):
            seen[k][pid_h[L.cls == j]] = True
    missing = {k: int((~v).sum()) for k, v in seen.items() if not v.all()}
    assert not missing, missing
    print(f"[seam-exhaustive] conn={conn}: all {NPAT} patterns exact on all "
          f"{len(L.keys)} seam classes", flush=True)
