"""The paper's local-step variants (C2FL, RC2FL, CC2FL, NC2FL) through
ccl_label_ablation: labels equal to the oracle's for every variant, and
per-tile counters that respect what the union-find must do at least: every
union that joins two trees is one successful atomic merge, so a tile needs at
least (trees after the coarse step) - (components in the tile) of them."""
import numpy as np
import pytest

from oracle import oracle_label
from paper_1712_09789_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VARIANTS = ["C2FL", "RC2FL", "CC2FL", "NC2FL"]


@pytest.fixture(scope="module")
def ccl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_09789_amd.ccl as c
    return c


def run(ccl, img, variant):
    d = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    labels, cnt = ccl.label_ablation(d, variant, counters=True)
    torch.cuda.synchronize()
    return labels.cpu().numpy(), cnt.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("H,W", [(1, 1), (5, 70), (64, 64), (65, 63), (200, 333)])
@pytest.mark.parametrize("p", [0.3, 0.6])
def test_labels_equal_oracle(ccl, variant, H, W, p):
    img = wl.bernoulli(H, W, p, seed=H + 3 * W)
    print(f"[ablation] {variant} {H}x{W} p={p}", flush=True)
    got, _ = run(ccl, img, variant)
    assert np.array_equal(got, oracle_label(img, 4))


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind,kw", [("blobs", {"sigma": 4}), ("checkerboard", {}),
                                     ("full", {}), ("empty", {}), ("spiral", {}),
                                     ("serpentine", {"width": 1}), ("bernoulli", {"p": 0.5})])
def test_contents_1024(ccl, variant, kind, kw):
    img = wl.make(kind, 1024, 1024, seed=2, **kw)
    print(f"[ablation] {variant} {kind}{kw}", flush=True)
    got, _ = run(ccl, img, variant)
    assert np.array_equal(got, oracle_label(img, 4))


def tiles(img):
    H, W = img.shape
    for ty in range(0, H, 64):
        for tx in range(0, W, 64):
            yield img[ty:ty + 64, tx:tx + 64] != 0


def lower_bounds(img):
    """Per tile: components and the trees each variant starts refinement with."""
    out = []
    for t in tiles(img):
        comps = len(np.unique(oracle_label(t.astype(np.uint8), 4))) - (1 if (~t).any() else 0)
        fg = int(t.sum())
        left = np.zeros_like(t)
        left[:, 1:] = t[:, :-1]
        up = np.zeros_like(t)
        up[1:, :] = t[:-1, :]
        row_starts = t & ~left
        runs = int(row_starts.sum())
        vruns = int((t & ~up).sum())
        # a run starts a tree after column linking iff no pixel above touches it
        trees_c2fl = 0
        for y in range(t.shape[0]):
            xs = np.flatnonzero(row_starts[y])
            for s0 in xs:
                e = s0
                while e + 1 < t.shape[1] and t[y, e + 1]:
                    e += 1
                if y == 0 or not t[y - 1, s0:e + 1].any():
                    trees_c2fl += 1
        out.append({"comps": comps, "NC2FL": fg, "RC2FL": runs, "CC2FL": vruns, "C2FL": trees_c2fl})
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_counters_respect_lower_bounds(ccl, seed):
    img = wl.bernoulli(256, 192, 0.55, seed=seed)
    bounds = lower_bounds(img)
    for v in VARIANTS:
        _, cnt = run(ccl, img, v)
        assert cnt.shape == (len(bounds), 2)
        for k, b in enumerate(bounds):
            assert cnt[k, 1] >= b[v] - b["comps"], (v, k, cnt[k], b)


def test_counters_closed_forms(ccl):
    # empty: nothing to do
    for v in VARIANTS:
        _, cnt = run(ccl, np.zeros((128, 128), np.uint8), v)
        assert not cnt.any()
    # full 128 x 128: one component per tile
    full = np.ones((128, 128), np.uint8)
    _, c = run(ccl, full, "C2FL")
    assert (c[:, 1] == 0).all()          # every run's only link is its coarse link
    _, r = run(ccl, full, "RC2FL")
    assert (r[:, 1] >= 63).all()         # 64 row runs joined by unions
    _, cc = run(ccl, full, "CC2FL")
    assert (cc[:, 1] >= 63).all()        # 64 column chains joined by unions
    _, n = run(ccl, full, "NC2FL")
    assert (n[:, 1] >= 4095).all()       # 4096 pixels joined by unions
