"""The C-ABI library loads on the CPU, exports every function declared in
include/ccl.h, and rejects bad arguments on the host before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccl.h")
LIB = os.environ.get("CCL_LIBRARY") or os.path.join(ROOT, "paper_1712_09789_amd", "libccl.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(ccl_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libccl.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ccl_label", "ccl_label_batch", "ccl_last_error",
                     "ccl_release_workspace"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _label(lib, name="ccl_label"):
    f = getattr(lib, name)
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    lib.ccl_last_error.restype = ctypes.c_char_p
    return f


FAKE_IMG = 0x10000000
FAKE_OUT = 0x20000000


@pytest.mark.parametrize("name", ["ccl_label", "ccl_label_local", "ccl_label_noalloc"])
@pytest.mark.parametrize("args,status", [
    ((FAKE_IMG, -1, 4, 4, 8, FAKE_OUT), -1),       # negative height
    ((FAKE_IMG, 4, -4, 4, 8, FAKE_OUT), -1),       # negative width
    ((FAKE_IMG, 4, 4, 4, 6, FAKE_OUT), -1),        # connectivity 6
    ((None, 4, 4, 4, 8, FAKE_OUT), -1),            # null image
    ((FAKE_IMG, 4, 4, 4, 8, None), -1),            # null labels
    ((FAKE_IMG, 4, 8, 7, 8, FAKE_OUT), -1),        # pitch < W
    ((FAKE_IMG, 4, 4, 4, 8, FAKE_IMG + 8), -1),    # overlap
    ((FAKE_IMG, 65536, 65536, 65536, 8, FAKE_OUT), -2),  # > 2^31 - 1 pixels
    ((None, 0, 5, 5, 8, None), 0),                 # empty image: no-op
    ((None, 5, 0, 0, 4, None), 0),
])
def test_validation(lib, name, args, status):
    f = _label(lib, name)
    assert f(*args, None) == status
    if status != 0:
        assert len(lib.ccl_last_error()) > 0


FAKE_CNT = 0x30000000
FAKE_COMPS = 0x40000000


@pytest.mark.parametrize("args,status", [
    ((FAKE_IMG, -1, 4, 4, 8, FAKE_OUT, FAKE_COMPS, 10, FAKE_CNT), -1),  # negative height
    ((FAKE_IMG, 4, 4, 4, 6, FAKE_OUT, FAKE_COMPS, 10, FAKE_CNT), -1),   # connectivity 6
    ((FAKE_IMG, 4, 4, 4, 8, None, FAKE_COMPS, 10, FAKE_CNT), -1),       # null labels
    ((FAKE_IMG, 4, 4, 4, 8, FAKE_OUT, FAKE_COMPS, 10, None), -1),       # null count
    ((FAKE_IMG, 4, 4, 4, 8, FAKE_OUT, FAKE_COMPS, -1, FAKE_CNT), -1),   # negative capacity
    ((FAKE_IMG, 4, 4, 4, 8, FAKE_OUT, None, 10, FAKE_CNT), -1),         # null comps
    ((FAKE_IMG, 1 << 16, 1 << 16, 1 << 16, 8, FAKE_OUT, FAKE_COMPS, 10, FAKE_CNT), -2),
])
def test_stats_validation(lib, args, status):
    f = lib.ccl_label_stats
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p]
    lib.ccl_last_error.restype = ctypes.c_char_p
    assert f(*args, None) == status
    assert b"ccl_label_stats" in lib.ccl_last_error()


@pytest.mark.parametrize("args,status", [
    ((FAKE_IMG, 4, 4, 4, 4, FAKE_OUT, None), -1),       # variant 4 does not exist
    ((FAKE_IMG, 4, 4, 4, -1, FAKE_OUT, None), -1),      # negative variant
    ((FAKE_IMG, -1, 4, 4, 0, FAKE_OUT, None), -1),      # negative height
    ((FAKE_IMG, 4, 4, 4, 0, None, None), -1),           # null labels
])
def test_ablation_validation(lib, args, status):
    f = lib.ccl_label_ablation
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.ccl_last_error.restype = ctypes.c_char_p
    assert f(*args, None) == status
    assert b"ccl_label_ablation" in lib.ccl_last_error()


@pytest.mark.parametrize("args,status", [
    ((FAKE_IMG, -1, 4, 4, 4, 16, 26, FAKE_OUT), -1),          # negative depth
    ((FAKE_IMG, 2, 4, 4, 4, 16, 8, FAKE_OUT), -1),            # connectivity 8 is 2-D only
    ((None, 2, 4, 4, 4, 16, 6, FAKE_OUT), -1),                # null volume
    ((FAKE_IMG, 2, 4, 4, 4, 16, 6, None), -1),                # null labels
    ((FAKE_IMG, 2, 4, 8, 7, 32, 6, FAKE_OUT), -1),            # pitch < W
    ((FAKE_IMG, 2, 4, 4, 4, 8, 26, FAKE_OUT), -1),            # slice pitch < slice
    ((FAKE_IMG, 2, 4, 4, 4, 16, 26, FAKE_IMG + 8), -1),       # overlap
    ((FAKE_IMG, 1024, 2048, 2048, 2048, 1 << 22, 26, FAKE_OUT), -2),  # > 2^31 voxels
    ((FAKE_IMG, 65536, 32768, 1, 1, 32768, 6, FAKE_OUT), -2),  # 2^31 voxels exactly
    ((FAKE_IMG, 2, 4, 4, 4, 16, 0, FAKE_OUT), -1),            # connectivity 0
    ((FAKE_IMG, 0, 4, 4, 4, 16, 26, FAKE_OUT), 0),            # empty volume
])
def test_volume_validation(lib, args, status):
    f = lib.ccl_label_3d
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_void_p]
    lib.ccl_last_error.restype = ctypes.c_char_p
    assert f(*args, None) == status
    if status:
        assert b"ccl_label_3d" in lib.ccl_last_error()


def test_batch_validation(lib):
    import paper_1712_09789_amd.ccl as c  # the binding loads on CPU too
    descs = (c.ImageDesc * 3)()
    descs[0] = c.ImageDesc(FAKE_IMG, 4, 4, 4, 8, FAKE_OUT)
    descs[1] = c.ImageDesc(FAKE_IMG + 4096, 4, 4, 4, 5, FAKE_OUT + 4096)
    descs[2] = c.ImageDesc(FAKE_IMG + 8192, 4, 4, 4, 8, FAKE_OUT + 8192)
    assert c.lib().ccl_label_batch(descs, 3, None) == -1
    assert b"[1]" in c.lib().ccl_last_error()
    assert c.lib().ccl_label_batch(descs, 0, None) == 0
    assert c.lib().ccl_label_batch(None, 2, None) == -1


def test_sizes_and_shape(lib):
    import paper_1712_09789_amd.ccl as c
    rows, cols = c.tile_shape()
    assert (rows, cols) == (64, 64)
    assert c.tile_shapes() == [32, 64, 128]
    assert c.workspace_bytes(0, 10) == 0
    assert c.workspace_bytes(-1, 10) == -1
    assert c.workspace_bytes(8192, 8192) > 0
    # the largest need over the tile heights: 32-row tiles have the most
    # border slots per pixel
    assert c.workspace_bytes(1000, 1000) >= c.workspace_bytes(1000, 999)


def test_tiled_entry_points_validate(lib):
    import paper_1712_09789_amd.ccl as c
    L = c.lib()
    for rows in (1, 16, 48, 96, 256, -32):
        assert L.ccl_label_tiled(FAKE_IMG, 4, 4, 4, 8, FAKE_OUT, rows, None) == -1, rows
        assert b"tile height" in L.ccl_last_error()
        descs = (c.ImageDesc * 1)()
        descs[0] = c.ImageDesc(FAKE_IMG, 4, 4, 4, 8, FAKE_OUT)
        assert L.ccl_label_batch_tiled(descs, 1, rows, None) == -1, rows
    # argument errors are found before any launch, whatever the height
    for rows in (0, 32, 64, 128):
        assert L.ccl_label_tiled(FAKE_IMG, 4, 4, 3, 8, FAKE_OUT, rows, None) == -1
        assert L.ccl_label_tiled(FAKE_IMG, 4, 4, 4, 6, FAKE_OUT, rows, None) == -1
        assert L.ccl_label_tiled(FAKE_IMG, 0, 4, 4, 8, FAKE_OUT, rows, None) == 0
        # one pixel row per tile row of a 2^31-wide image: too many tiles
        assert L.ccl_label_tiled(FAKE_IMG, 1, (1 << 31) - 1, (1 << 31) - 1, 8,
                                 FAKE_OUT + (1 << 33), rows, None) == -2


def test_noalloc_size_limit(lib):
    """Images whose workspace exceeds the fixed scratch are rejected on the
    host, before any device call; the 4096^2 headline size fits."""
    f = _label(lib, "ccl_label_noalloc")
    assert f(FAKE_IMG, 8192, 8192, 8192, 8, FAKE_OUT + (1 << 30), None) == -2
    assert b"fixed scratch" in lib.ccl_last_error()
    assert f(FAKE_IMG, 1, (1 << 31) - 1, (1 << 31) - 1, 8, FAKE_OUT + (1 << 33), None) == -2


def test_replay_and_segment_copy_validation(lib):
    import paper_1712_09789_amd.ccl as c
    L = c.lib()
    for kind in (-1, 1, 3, 4, 5, 6):
        assert L.ccl_replay_last(kind, 1, None) == -1
    assert L.ccl_replay_last(0, -1, None) == -1
    # no labelling call has been made on this thread
    assert L.ccl_replay_last(0, 1, None) == -1
    assert b"no labelling call" in L.ccl_last_error()
    assert L.ccl_copy_segments(FAKE_IMG, FAKE_OUT, 4096, 48, 256, None) == -1  # 48 % 16 ok, 4096 % 48
    assert L.ccl_copy_segments(FAKE_IMG, FAKE_OUT, 4096, 64, 32, None) == -1   # stride < segment
    assert L.ccl_copy_segments(FAKE_IMG + 8, FAKE_OUT, 4096, 64, 256, None) == -1
    assert L.ccl_copy_segments(None, None, 0, 64, 256, None) == 0


def test_copy_validation(lib):
    import paper_1712_09789_amd.ccl as c
    assert c.lib().ccl_copy_bytes(FAKE_IMG, FAKE_OUT, 15, None) == -1
    assert c.lib().ccl_copy_bytes(FAKE_IMG + 1, FAKE_OUT, 16, None) == -1
    assert c.lib().ccl_copy_bytes(None, None, 0, None) == 0


def test_product_path_does_not_touch_the_oracle():
    # the library sources and the binding never import, load or include it
    pkg = os.path.join(ROOT, "paper_1712_09789_amd")
    bad = re.compile(r"(import\s+oracle|from\s+oracle|liboracle|ccl_oracle|oracle_label)")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not bad.search(text), fn


def test_launch_policy_validation(lib):
    import paper_1712_09789_amd.ccl as c
    L = c.lib()
    n = L.ccl_launch_buckets(None, 0)
    assert n >= 2
    arr = (ctypes.c_int64 * n)()
    assert L.ccl_launch_buckets(arr, n) == n
    assert list(arr) == sorted(arr) and arr[n - 1] == (1 << 63) - 1
    for args in ((2, 0, 8, 0, 0, 0), (-1, 0, 8, 0, 0, 0), (0, n, 8, 0, 0, 0),
                 (0, -1, 8, 0, 0, 0), (0, 0, 6, 0, 0, 0), (0, 0, 8, 48, 0, 0),
                 (0, 0, 8, 0, 2, 0), (1, 0, 4, 0, 0, -2)):
        assert L.ccl_set_launch_policy(*args) == -1, args
        assert b"ccl_set_launch_policy" in L.ccl_last_error()
    try:
        for batch in (0, 1):
            for b in range(n):
                for conn in (4, 8):
                    for rows in (32, 64, 128):
                        assert L.ccl_set_launch_policy(batch, b, conn, rows, 1, 0) == 0
                        px = arr[b] if b < n - 1 else arr[n - 2] + 1
                        assert c.policy_tile_rows(batch, px, conn) == rows
                    assert L.ccl_set_launch_policy(batch, b, conn, 0, -1, -1) == 0
                    assert c.policy_tile_rows(batch, arr[0], conn) == 64
        assert c.policy_tile_rows(2, 100, 8) == -1
        assert c.policy_tile_rows(0, 100, 5) == -1
    finally:
        c.reset_launch_policy()


def test_launch_policy_cache_loader(tmp_path):
    """A tuner cache is applied only on the architecture it names, and an
    out-of-range entry is rejected by the library."""
    import json
    import paper_1712_09789_amd.ccl as c
    n = len(c.launch_buckets())
    choices = [{"batch": b, "bucket": k, "connectivity": conn, "tile_rows": 128, "local": 1,
                "final": 0} for b in (0, 1) for k in range(n) for conn in (4, 8)]
    path = tmp_path / "policy.json"
    path.write_text(json.dumps({"arch": "gfxTEST", "choices": choices}))
    try:
        assert not c.apply_launch_policy(str(path), arch="gfxOTHER")
        assert c.policy_tile_rows(0, 1000, 8) == 64
        assert c.apply_launch_policy(str(path), arch="gfxTEST")
        assert c.policy_tile_rows(0, 1000, 8) == 128
        assert c.policy_tile_rows(1, 1 << 40, 4) == 128
        bad = tmp_path / "bad.json"
        bad.write_text(json.dumps({"arch": "gfxTEST", "choices": [
            {"batch": 0, "bucket": 0, "connectivity": 8, "tile_rows": 96, "local": 0,
             "final": 0}]}))
        with pytest.raises(c.CCLError):
            c.apply_launch_policy(str(bad), arch="gfxTEST")
    finally:
        c.reset_launch_policy()


def test_packaged_policy_is_well_formed():
    """The packaged cache names an architecture, one entry per (class,
    bucket, connectivity), and only heights and grids the library accepts."""
    import json
    import paper_1712_09789_amd.ccl as c
    with open(c.LAUNCH_POLICY_PATH) as fh:
        cache = json.load(fh)
    assert cache["arch"].startswith("gfx")
    n = len(c.launch_buckets())
    keys = {(e["batch"], e["bucket"], e["connectivity"]) for e in cache["choices"]}
    assert keys == {(b, k, conn) for b in (0, 1) for k in range(n) for conn in (4, 8)}
    for e in cache["choices"]:
        assert e["tile_rows"] in (0, 32, 64, 128)
        assert e["local"] in (-1, 0, 1) and e["final"] in (-1, 0, 1)
