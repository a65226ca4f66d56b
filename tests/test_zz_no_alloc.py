"""ccl_label_noalloc, the entry point for callers that cannot allocate
device memory, through the C ABI: on two calls in a row (the second with a
smaller image) its labels equal those of ccl_label, the entry point it
varies, and the oracle's; and the library keeps no workspace for the stream
it ran on.  Labels are integers: the bar is equality."""
import ctypes

import numpy as np
import pytest

from oracle import oracle_label
from paper_1712_09789_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ccl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_09789_amd.ccl as c
    f = c.lib().ccl_label_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    return c


def noalloc(ccl, d, conn, out, stream):
    H, W = d.shape
    return ccl.lib().ccl_label_noalloc(d.data_ptr(), H, W, d.stride(0) if H > 1 else W, conn,
                                       out.data_ptr(), int(stream.cuda_stream))


def test_noalloc_equals_label_on_two_calls(ccl):
    st = torch.cuda.Stream()  # a stream the library has not seen: no workspace of its own
    cases = [(wl.bernoulli(4096, 4096, 0.5, seed=3), 8),   # the largest headline size
             (wl.blobs(1080, 1920, 4, seed=4), 4)]          # then a smaller image
    for img, conn in cases:
        print(f"[noalloc] {img.shape} conn={conn}", flush=True)
        d = torch.from_numpy(img).cuda()
        want = ccl.label(d, conn)
        torch.cuda.synchronize()
        out = torch.full(img.shape, -1, dtype=torch.int32, device="cuda")
        st.wait_stream(torch.cuda.current_stream())
        rc = noalloc(ccl, d, conn, out, st)
        assert rc == 0, ccl.lib().ccl_last_error()
        st.synchronize()
        assert torch.equal(out, want), (img.shape, conn)
        assert np.array_equal(out.cpu().numpy(), oracle_label(img, conn)), (img.shape, conn)
    assert ccl.workspace_cached(st) == 0


def test_noalloc_pitched_unaligned_view(ccl):
    """A view into a wider image (row pitch > width, first pixel off a
    16-byte boundary), after the calls above left their values in the shared
    scratch: labels equal ccl_label's and the oracle's."""
    big = wl.bernoulli(900, 1301, 0.55, seed=5)
    d = torch.from_numpy(big).cuda()[3:850, 7:1290]
    img = np.ascontiguousarray(big[3:850, 7:1290])
    assert d.stride(0) == 1301 and d.data_ptr() % 16 != 0
    for conn in (4, 8):
        print(f"[noalloc] pitched view {img.shape} conn={conn}", flush=True)
        want = ccl.label(d, conn)
        torch.cuda.synchronize()
        out = torch.full(img.shape, -1, dtype=torch.int32, device="cuda")
        st = torch.cuda.current_stream()
        assert noalloc(ccl, d, conn, out, st) == 0, ccl.lib().ccl_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, want)
        assert np.array_equal(out.cpu().numpy(), oracle_label(img, conn))


def test_noalloc_rejects_images_beyond_the_scratch(ccl):
    d = torch.zeros((8192, 8192), dtype=torch.uint8, device="cuda")
    out = torch.full((8192, 8192), -7, dtype=torch.int32, device="cuda")
    assert noalloc(ccl, d, 8, out, torch.cuda.current_stream()) == -2
    assert b"fixed scratch" in ccl.lib().ccl_last_error()
    torch.cuda.synchronize()
    assert bool((out == -7).all())
