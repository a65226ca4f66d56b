"""The largest images the ABI accepts (H * W just under 2^31): labels near the
top of the int32 range, about half a million tiles and a billion components.
The oracle cannot label 2^31 pixels in seconds, so the inputs are images
whose labelling has a closed form, generated and checked on the device row
block by row block."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 46340  # N * N = 2147395600 < 2^31 - 1


@pytest.fixture(scope="module")
def ccl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_09789_amd.ccl as c
    return c


def check_rows(labels, expected_rows, what, step=1024):
    H = labels.shape[0]
    for y0 in range(0, H, step):
        y1 = min(H, y0 + step)
        want = expected_rows(y0, y1)
        if not torch.equal(labels[y0:y1], want):
            bad = (labels[y0:y1] != want).nonzero()[0].tolist()
            y, x = y0 + bad[0], bad[1]
            raise AssertionError(f"{what}: first mismatch at ({y},{x}): "
                                 f"got {int(labels[y, x])} want {int(want[bad[0], x])}")


def test_max_size_checkerboard_4(ccl):
    # 4-connectivity: every foreground pixel (x + y even) is its own component
    print(f"[max] checkerboard {N}x{N} conn=4", flush=True)
    ys = torch.arange(N, device="cuda", dtype=torch.int64)
    xs = torch.arange(N, device="cuda", dtype=torch.int64)
    img = torch.empty((N, N), dtype=torch.uint8, device="cuda")
    for y0 in range(0, N, 4096):
        y1 = min(N, y0 + 4096)
        img[y0:y1] = ((ys[y0:y1, None] + xs[None, :]) % 2 == 0).to(torch.uint8)
    labels = ccl.label(img, 4)
    torch.cuda.synchronize()

    def expected(y0, y1):
        pos = ys[y0:y1, None] * N + xs[None, :] + 1
        fg = (ys[y0:y1, None] + xs[None, :]) % 2 == 0
        return torch.where(fg, pos, torch.zeros_like(pos)).to(torch.int32)

    check_rows(labels, expected, "checkerboard conn 4")
    assert int(labels[N - 1, N - 1]) == N * N  # the largest label, just under 2^31
    del img, labels
    torch.cuda.empty_cache()


def test_max_size_full_and_stripes_8(ccl):
    # 8-connectivity: the full image is one component (label 1 everywhere);
    # columns of foreground one apart are separate components (label x + 1)
    print(f"[max] full {N}x{N} conn=8", flush=True)
    img = torch.ones((N, N), dtype=torch.uint8, device="cuda")
    labels = ccl.label(img, 8)
    torch.cuda.synchronize()
    check_rows(labels, lambda y0, y1: torch.ones((y1 - y0, N), dtype=torch.int32, device="cuda"),
               "full conn 8")
    print(f"[max] stripes {N}x{N} conn=8", flush=True)
    xs = torch.arange(N, device="cuda", dtype=torch.int32)
    img[:] = (xs % 2 == 0).to(torch.uint8)[None, :]
    ccl.label(img, 8, out=labels)
    torch.cuda.synchronize()
    row = torch.where(xs % 2 == 0, xs + 1, torch.zeros_like(xs))
    check_rows(labels, lambda y0, y1: row[None, :].expand(y1 - y0, N), "stripes conn 8")
    del img, labels
    torch.cuda.empty_cache()
