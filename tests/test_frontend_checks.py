"""Argument checks of the PyTorch front end that run without a GPU: the
target-size rule that decides the stride the kernels read targets with."""

import pytest

from paper_2208_12737_amd.drr import target_stride


def test_target_stride_shared_or_per_pose():
    assert target_stride(64, 5, 64) == 0          # one image for every pose
    assert target_stride(5 * 64, 5, 64) == 64     # one image per pose
    assert target_stride(64, 1, 64) == 0


@pytest.mark.parametrize("numel", [0, 63, 65, 2 * 64, 4 * 64, 6 * 64])
def test_target_of_any_other_size_is_rejected(numel):
    # 1 < k < n images (or more than n) would make the kernels read past the
    # end of the tensor or mix up poses
    with pytest.raises(ValueError):
        target_stride(numel, 5, 64)
