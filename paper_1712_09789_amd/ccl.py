"""Python binding of the C ABI in include/ccl.h (argument marshalling only).

Every labelling step runs in the HIP kernels of ``libccl.so``; this module
passes device pointers, sizes and the stream handle, and turns status codes
into exceptions.  torch is used for device memory and streams only.  There is
no fallback: if the library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# CCL_LIBRARY names another build of the library (the sanitized host build)
LIB_PATH = os.environ.get("CCL_LIBRARY") or os.path.join(_HERE, "libccl.so")

CCL_OK = 0
STATUS_NAMES = {0: "CCL_OK", -1: "CCL_ERR_INVALID_ARG", -2: "CCL_ERR_TOO_LARGE",
                -3: "CCL_ERR_OUT_OF_MEMORY", -4: "CCL_ERR_HIP"}
KERNEL_KINDS = ("local", "seam", "final", "copy", "block", "stats", "vmerge", "vfinal",
                "vlocal")
# Layout of ccl_component (include/ccl.h), 40 bytes per component.
COMPONENT_DTYPE = np.dtype([("label", np.int32), ("area", np.int32),
                            ("x_min", np.int32), ("y_min", np.int32),
                            ("x_max", np.int32), ("y_max", np.int32),
                            ("sum_x", np.int64), ("sum_y", np.int64)])
assert COMPONENT_DTYPE.itemsize == 40
# Variants of ccl_label_ablation (the paper's C2FL, RC2FL, CC2FL, NC2FL).
ABLATIONS = {"C2FL": 0, "RC2FL": 1, "CC2FL": 2, "NC2FL": 3}


class CCLError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class ImageDesc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("pitch_bytes", ctypes.c_int64), ("connectivity", ctypes.c_int32),
                ("labels", ctypes.c_void_p)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run "
                          "`python -m paper_1712_09789_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    for name in ("ccl_label", "ccl_label_local"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [vp, i32, i32, i64, i32, vp, vp]
    lib.ccl_label_stats.restype = ctypes.c_int
    lib.ccl_label_stats.argtypes = [vp, i32, i32, i64, i32, vp, vp, i64, vp, vp]
    lib.ccl_label_3d.restype = ctypes.c_int
    lib.ccl_label_3d.argtypes = [vp, i32, i32, i32, i64, i64, i32, vp, vp]
    lib.ccl_label_ablation.restype = ctypes.c_int
    lib.ccl_label_ablation.argtypes = [vp, i32, i32, i64, i32, vp, vp, vp]
    lib.ccl_label_tiled.restype = ctypes.c_int
    lib.ccl_label_tiled.argtypes = [vp, i32, i32, i64, i32, vp, i32, vp]
    lib.ccl_label_batch.restype = ctypes.c_int
    lib.ccl_label_batch.argtypes = [ctypes.POINTER(ImageDesc), i32, vp]
    lib.ccl_label_batch_tiled.restype = ctypes.c_int
    lib.ccl_label_batch_tiled.argtypes = [ctypes.POINTER(ImageDesc), i32, i32, vp]
    lib.ccl_tile_cols.restype = i32
    lib.ccl_tile_rows.restype = i32
    lib.ccl_workspace_bytes.restype = i64
    lib.ccl_workspace_bytes.argtypes = [i32, i32]
    lib.ccl_workspace_cached.restype = i64
    lib.ccl_workspace_cached.argtypes = [vp]
    lib.ccl_last_error.restype = ctypes.c_char_p
    lib.ccl_release_workspace.restype = ctypes.c_int
    lib.ccl_release_workspace.argtypes = [i32]
    lib.ccl_timing_enable.restype = ctypes.c_int
    lib.ccl_timing_enable.argtypes = [i32]
    lib.ccl_timing_read.restype = ctypes.c_int
    lib.ccl_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), i32]
    lib.ccl_copy_segments.restype = ctypes.c_int
    lib.ccl_copy_segments.argtypes = [vp, vp, i64, i32, i64, vp]
    lib.ccl_replay_last.restype = ctypes.c_int
    lib.ccl_replay_last.argtypes = [i32, i32, vp]
    lib.ccl_copy_bytes.restype = ctypes.c_int
    lib.ccl_copy_bytes.argtypes = [vp, vp, i64, vp]
    lib.ccl_plan_create.restype = ctypes.c_int
    lib.ccl_plan_create.argtypes = [ctypes.POINTER(ImageDesc), i32, vp, ctypes.POINTER(vp)]
    lib.ccl_plan_run.restype = ctypes.c_int
    lib.ccl_plan_run.argtypes = [vp, vp]
    lib.ccl_plan_destroy.restype = ctypes.c_int
    lib.ccl_plan_destroy.argtypes = [vp]
    lib.ccl_set_launch_policy.restype = ctypes.c_int
    lib.ccl_set_launch_policy.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.ccl_launch_buckets.restype = i32
    lib.ccl_launch_buckets.argtypes = [ctypes.POINTER(ctypes.c_int64), i32]
    lib.ccl_policy_tile_rows.restype = i32
    lib.ccl_policy_tile_rows.argtypes = [i32, i64, i32]
    lib.ccl_tile_shapes.restype = i32
    lib.ccl_tile_shapes.argtypes = [ctypes.POINTER(ctypes.c_int32), i32]
    return lib


_lib = _load()

# Launch-shape choices measured by paper_1712_09789_amd.tune on a device of
# the architecture they name; applied at import when the device matches.
# CCL_LAUNCH_POLICY names another cache file, or "builtin" to keep the
# library's built-in choices.
LAUNCH_POLICY_PATH = os.path.join(_HERE, "launch_policy.json")
launch_policy_applied: str | None = None


def lib() -> ctypes.CDLL:
    return _lib


def _check(status: int) -> None:
    if status != CCL_OK:
        raise CCLError(status, _lib.ccl_last_error().decode(errors="replace"))


def launch_buckets() -> list[int]:
    """Upper pixel-count bound of each launch-policy bucket (the last is
    2**63 - 1)."""
    n = _lib.ccl_launch_buckets(None, 0)
    arr = (ctypes.c_int64 * n)()
    _lib.ccl_launch_buckets(arr, n)
    return list(arr)


def tile_shapes() -> list[int]:
    """Tile heights built into the library (tiles are 64 columns wide)."""
    n = _lib.ccl_tile_shapes(None, 0)
    arr = (ctypes.c_int32 * n)()
    _lib.ccl_tile_shapes(arr, n)
    return list(arr)


def set_launch_policy(batch: int, bucket: int, connectivity: int, tile_rows: int = 0,
                      local: int = -1, final: int = -1) -> None:
    """Tile height (0 = built-in) and the grids of the local step and the
    final relabel (-1 = built-in choice, 0 = persistent, 1 = one workgroup
    per tile) for one launch class (0 = one image, 1 = several), pixel bucket
    and connectivity (ccl_set_launch_policy in ccl.h)."""
    _check(_lib.ccl_set_launch_policy(int(batch), int(bucket), int(connectivity),
                                      int(tile_rows), int(local), int(final)))


def reset_launch_policy() -> None:
    """Every policy entry back to the built-in choices."""
    for batch in (0, 1):
        for bucket in range(len(launch_buckets())):
            for conn in (4, 8):
                set_launch_policy(batch, bucket, conn)


def policy_tile_rows(batch: int, pixels: int, connectivity: int) -> int:
    """Tile height the current policy picks for a launch class."""
    return int(_lib.ccl_policy_tile_rows(int(batch), int(pixels), int(connectivity)))


def apply_launch_policy(path: str, arch: str | None = None) -> bool:
    """Apply a cache written by paper_1712_09789_amd.tune; returns False
    (and changes nothing) if the cache was tuned on another architecture."""
    import json
    with open(path) as fh:
        cache = json.load(fh)
    if arch is None:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    if cache.get("arch") != arch:
        return False
    for c in cache["choices"]:
        set_launch_policy(c["batch"], c["bucket"], c["connectivity"], c["tile_rows"],
                          c["local"], c["final"])
    return True


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _image_args(img: torch.Tensor):
    """(H, W, pitch in bytes) of a 2-D uint8 image.  Rows must be contiguous
    and must not overlap (row stride >= W); expanded or overlapping views are
    rejected here, before anything reaches the device."""
    if img.dim() != 2 or img.dtype != torch.uint8:
        raise ValueError("image must be a 2-D torch.uint8 tensor")
    H, W = img.shape
    if H > 0 and W > 1 and img.stride(1) != 1:
        raise ValueError("image rows must be contiguous (stride(1) == 1)")
    if H > 1 and W > 0 and img.stride(0) < W:
        raise ValueError(f"image rows overlap: row stride {img.stride(0)} < width {W} "
                         "(an expanded or overlapping view; pass a contiguous copy)")
    if not img.is_cuda:
        raise ValueError("image must be a device (cuda) tensor")
    return H, W, (img.stride(0) if H > 1 else W)


def _out_for(img: torch.Tensor, out: torch.Tensor | None) -> torch.Tensor:
    H, W = img.shape
    if out is None:
        return torch.empty((H, W), dtype=torch.int32, device=img.device)
    if out.shape != (H, W) or out.dtype != torch.int32 or not out.is_contiguous() \
            or out.device != img.device:
        raise ValueError("out must be a contiguous int32 tensor of the image's shape "
                         "on the image's device")
    return out


def label(img: torch.Tensor, connectivity: int = 8, out: torch.Tensor | None = None,
          stream=None, tile_rows: int = 0) -> torch.Tensor:
    """Canonical connected-component labels of a uint8 device image
    (0 = background, else 1 + smallest raster position of the component).
    tile_rows: 32, 64 or 128 fixes the tile height (ccl_label_tiled); 0 lets
    the launch policy choose (ccl_label)."""
    H, W, pitch = _image_args(img)
    out = _out_for(img, out)
    if tile_rows:
        _check(_lib.ccl_label_tiled(img.data_ptr(), H, W, pitch, int(connectivity),
                                    out.data_ptr(), int(tile_rows), _stream_handle(stream)))
    else:
        _check(_lib.ccl_label(img.data_ptr(), H, W, pitch, int(connectivity), out.data_ptr(),
                              _stream_handle(stream)))
    return out


def max_components(H: int, W: int, connectivity: int = 8) -> int:
    """Most components an H x W image can have (isolated pixels on a
    checkerboard for 4-connectivity, on every other row and column for 8)."""
    if connectivity == 4:
        return (H * W + 1) // 2
    return ((H + 1) // 2) * ((W + 1) // 2)


def label_stats(img: torch.Tensor, connectivity: int = 8, out: torch.Tensor | None = None,
                capacity: int | None = None, stream=None):
    """Labels plus the statistics of every component (ccl_label_stats).

    Returns (labels, comps, count): comps is a uint8 device tensor holding
    `capacity` ccl_component records (sorted by label; default capacity =
    the most components the image can have), count a one-element int64
    device tensor.  ``components_to_numpy`` copies the valid records out."""
    H, W, pitch = _image_args(img)
    out = _out_for(img, out)
    if capacity is None:
        capacity = max_components(H, W, connectivity)
    comps = torch.empty(capacity * COMPONENT_DTYPE.itemsize, dtype=torch.uint8,
                        device=img.device)
    count = torch.empty(1, dtype=torch.int64, device=img.device)
    _check(_lib.ccl_label_stats(img.data_ptr(), H, W, pitch, int(connectivity), out.data_ptr(),
                                comps.data_ptr(), int(capacity), count.data_ptr(),
                                _stream_handle(stream)))
    return out, comps, count


def components_to_numpy(comps: torch.Tensor, count: torch.Tensor) -> np.ndarray:
    """The valid records of a label_stats result as a numpy structured array
    (synchronises with the device)."""
    total = int(count.item())
    if total < 0:
        raise CCLError(-4, f"ccl_label_stats: the device reported an internal consistency "
                           f"failure (count {total}); labels and statistics are invalid")
    n = min(total, comps.numel() // COMPONENT_DTYPE.itemsize)
    raw = comps[:n * COMPONENT_DTYPE.itemsize].cpu().numpy()
    return raw.view(COMPONENT_DTYPE).copy()


def label_3d(vol: torch.Tensor, connectivity: int = 26, out: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
    """Canonical labels of a uint8 device volume indexed [z, y, x]
    (ccl_label_3d; 6- or 26-connectivity)."""
    if vol.dim() != 3 or vol.dtype != torch.uint8:
        raise ValueError("volume must be a 3-D torch.uint8 tensor")
    D, H, W = vol.shape
    if D > 0 and H > 0 and W > 1 and vol.stride(2) != 1:
        raise ValueError("volume rows must be contiguous (stride(2) == 1)")
    pitch = vol.stride(1) if H > 1 else W
    if H > 1 and W > 0 and pitch < W:
        raise ValueError(f"volume rows overlap: row stride {pitch} < width {W}")
    slice_pitch = vol.stride(0) if D > 1 else H * pitch
    if D > 1 and H > 0 and W > 0 and slice_pitch < (H - 1) * pitch + W:
        raise ValueError(f"volume slices overlap: slice stride {slice_pitch} < "
                         f"{(H - 1) * pitch + W}")
    if not vol.is_cuda:
        raise ValueError("volume must be a device (cuda) tensor")
    if out is None:
        out = torch.empty((D, H, W), dtype=torch.int32, device=vol.device)
    elif out.shape != (D, H, W) or out.dtype != torch.int32 or not out.is_contiguous() \
            or out.device != vol.device:
        raise ValueError("out must be a contiguous int32 tensor of the volume's shape "
                         "on the volume's device")
    _check(_lib.ccl_label_3d(vol.data_ptr(), D, H, W, pitch, slice_pitch, int(connectivity),
                             out.data_ptr(), _stream_handle(stream)))
    return out


def label_ablation(img: torch.Tensor, variant: str = "C2FL", out: torch.Tensor | None = None,
                   counters: bool = False, stream=None):
    """4-connected labels through one of the paper's local-step variants
    (ccl_label_ablation).  With counters=True also returns a (tiles, 2) int32
    device tensor of per-tile find-loop steps and atomic merge attempts
    (tiles in row-major order; the C side writes them as uint32)."""
    H, W, pitch = _image_args(img)
    out = _out_for(img, out)
    cnt = None
    if counters:
        tc, tr = tile_shape()
        ntiles = ((W + tc - 1) // tc) * ((H + tr - 1) // tr)
        cnt = torch.zeros((max(ntiles, 1), 2), dtype=torch.int32, device=img.device)
    _check(_lib.ccl_label_ablation(img.data_ptr(), H, W, pitch, ABLATIONS[variant],
                                   out.data_ptr(), cnt.data_ptr() if cnt is not None else None,
                                   _stream_handle(stream)))
    return (out, cnt) if counters else out


def label_local(img: torch.Tensor, connectivity: int = 8, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """Local step only: every tile labelled as a separate image."""
    H, W, pitch = _image_args(img)
    out = _out_for(img, out)
    _check(_lib.ccl_label_local(img.data_ptr(), H, W, pitch, int(connectivity),
                                out.data_ptr(), _stream_handle(stream)))
    return out


def make_descs(imgs: Sequence[torch.Tensor], outs: Sequence[torch.Tensor],
               connectivity) -> ctypes.Array:
    n = len(imgs)
    conns = connectivity if isinstance(connectivity, (list, tuple)) else [connectivity] * n
    arr = (ImageDesc * max(n, 1))()
    for i, (im, o) in enumerate(zip(imgs, outs)):
        H, W, pitch = _image_args(im)
        arr[i] = ImageDesc(im.data_ptr(), H, W, pitch, int(conns[i]), o.data_ptr())
    return arr


def label_batch(imgs: Sequence[torch.Tensor], connectivity=8,
                outs: Sequence[torch.Tensor] | None = None, stream=None, tile_rows: int = 0):
    """Label several independent images in one call; returns the label
    tensors.  tile_rows as in label()."""
    if outs is None:
        outs = [_out_for(im, None) for im in imgs]
    else:
        outs = [_out_for(im, o) for im, o in zip(imgs, outs)]
    descs = make_descs(imgs, outs, connectivity)
    if tile_rows:
        _check(_lib.ccl_label_batch_tiled(descs, len(imgs), int(tile_rows),
                                          _stream_handle(stream)))
    else:
        _check(_lib.ccl_label_batch(descs, len(imgs), _stream_handle(stream)))
    return list(outs)


def tile_shape() -> tuple[int, int]:
    """(rows, cols) of the built-in tile shape (the statistics, ablation,
    volume and local-step paths always use it)."""
    return int(_lib.ccl_tile_rows()), int(_lib.ccl_tile_cols())


def workspace_bytes(H: int, W: int) -> int:
    return int(_lib.ccl_workspace_bytes(H, W))


def workspace_cached(stream=None) -> int:
    """Bytes of the library workspace kept for `stream` (current device)."""
    return int(_lib.ccl_workspace_cached(_stream_handle(stream)))


def release_workspace(device: int = 0) -> None:
    _check(_lib.ccl_release_workspace(device))


def timing_enable(on: bool = True, kinds=None) -> None:
    """Record HIP events around the kernels named in `kinds` (all when None)."""
    if not on:
        mask = 0
    elif kinds is None:
        mask = (1 << len(KERNEL_KINDS)) - 1
    else:
        mask = sum(1 << KERNEL_KINDS.index(k) for k in kinds)
    _check(_lib.ccl_timing_enable(mask))


def timing_read() -> dict:
    nk = len(KERNEL_KINDS)
    ms = (ctypes.c_double * nk)()
    n = (ctypes.c_int64 * nk)()
    k = _lib.ccl_timing_read(ms, n, nk)
    if k < 0:
        _check(k)
    return {KERNEL_KINDS[i]: (float(ms[i]), int(n[i])) for i in range(nk)}


def copy_segments(src: torch.Tensor, dst: torch.Tensor, segment_bytes: int,
                  src_stride_bytes: int, stream=None) -> None:
    """Gather dst.nbytes bytes from segments of src (ccl_copy_segments)."""
    nbytes = dst.numel() * dst.element_size()
    if (nbytes // segment_bytes) * src_stride_bytes > src.numel() * src.element_size():
        raise ValueError("src is too small for the segments")
    _check(_lib.ccl_copy_segments(src.data_ptr(), dst.data_ptr(), nbytes, int(segment_bytes),
                                  int(src_stride_bytes), _stream_handle(stream)))


def replay_last(kind: str, reps: int, stream=None) -> None:
    """Launch one kernel ("local" or "final") of this thread's most recent
    labelling call `reps` more times, back to back (ccl_replay_last; after
    "local" the labels are valid again only once the call is repeated)."""
    _check(_lib.ccl_replay_last(KERNEL_KINDS.index(kind), int(reps), _stream_handle(stream)))


def copy_bytes(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _check(_lib.ccl_copy_bytes(src.data_ptr(), dst.data_ptr(), nbytes,
                               _stream_handle(stream)))


class Plan:
    """A prepared batch (ccl_plan_*): the images and label buffers are bound
    at creation; run() only launches kernels, so it can be captured into a
    graph (torch.cuda.graph) and replayed after new pixels are written into
    the same input tensors."""

    def __init__(self, imgs: Sequence[torch.Tensor], connectivity=8,
                 outs: Sequence[torch.Tensor] | None = None, stream=None):
        if outs is None:
            outs = [_out_for(im, None) for im in imgs]
        else:
            outs = [_out_for(im, o) for im, o in zip(imgs, outs)]
        self.imgs, self.outs = list(imgs), list(outs)
        self._descs = make_descs(self.imgs, self.outs, connectivity)
        h = ctypes.c_void_p()
        _check(_lib.ccl_plan_create(self._descs, len(self.imgs), _stream_handle(stream),
                                    ctypes.byref(h)))
        self._h = h

    def run(self, stream=None) -> list:
        _check(_lib.ccl_plan_run(self._h, _stream_handle(stream)))
        return self.outs

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.ccl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _apply_packaged_policy() -> None:
    global launch_policy_applied
    path = os.environ.get("CCL_LAUNCH_POLICY", LAUNCH_POLICY_PATH)
    if path == "builtin" or not os.path.exists(path) or not torch.cuda.is_available():
        return
    if apply_launch_policy(path):
        launch_policy_applied = path


_apply_packaged_policy()
