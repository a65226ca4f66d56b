"""Host-side checks of the Python binding that need no GPU: views whose rows
overlap (an expanded tensor, a row stride below the width) are rejected
before any pointer reaches the library, so the kernels can never read past
a smaller allocation."""
import pytest
import torch

import paper_1712_09789_amd.ccl as ccl


def test_expanded_image_rejected_before_launch():
    img = torch.zeros(1, 300, dtype=torch.uint8).expand(200, 300)
    assert img.stride(0) == 0
    with pytest.raises(ValueError, match="overlap"):
        ccl.label(img, 8)
    with pytest.raises(ValueError, match="overlap"):
        ccl.label_local(img, 4)
    with pytest.raises(ValueError, match="overlap"):
        ccl.label_stats(img, 8)


def test_overlapping_rows_rejected_before_launch():
    base = torch.zeros(4096, dtype=torch.uint8)
    img = base.as_strided((10, 64), (32, 1))  # rows overlap by half
    with pytest.raises(ValueError, match="overlap"):
        ccl.label(img, 4)
    one_col = torch.zeros(1, 1, dtype=torch.uint8).expand(50, 1)
    with pytest.raises(ValueError, match="overlap"):
        ccl.label(one_col, 4)


def test_volume_overlap_rejected_before_launch():
    vol = torch.zeros(1, 1, 64, dtype=torch.uint8).expand(8, 16, 64)
    with pytest.raises(ValueError, match="overlap"):
        ccl.label_3d(vol, 6)
    slab = torch.zeros(1, 16, 64, dtype=torch.uint8).expand(8, 16, 64)
    with pytest.raises(ValueError, match="slices overlap"):
        ccl.label_3d(slab, 26)


def test_host_tensors_rejected():
    with pytest.raises(ValueError, match="device"):
        ccl.label(torch.zeros(8, 8, dtype=torch.uint8), 8)
    with pytest.raises(ValueError, match="device"):
        ccl.label_3d(torch.zeros(2, 8, 8, dtype=torch.uint8), 6)


def test_inconsistent_count_raises():
    """A negative component count is the device's report that a label could
    not belong to its pixel: the records must not be handed out."""
    comps = torch.zeros(4 * ccl.COMPONENT_DTYPE.itemsize, dtype=torch.uint8)
    with pytest.raises(ccl.CCLError, match="consistency"):
        ccl.components_to_numpy(comps, torch.tensor([-1], dtype=torch.int64))
    # a valid count hands out that many records (fewer if the array is shorter)
    assert len(ccl.components_to_numpy(comps, torch.tensor([3], dtype=torch.int64))) == 3
    assert len(ccl.components_to_numpy(comps, torch.tensor([9], dtype=torch.int64))) == 4
