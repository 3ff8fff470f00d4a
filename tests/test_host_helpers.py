"""Host-side helpers of the landscape sweep and the registration report
(no GPU): offset generators and the pose-error metric."""

import math

import numpy as np

from paper_2208_12737_amd.landscape import PAPER_RANGES, grid_offsets, random_offsets
from paper_2208_12737_amd.register import pose_errors


def test_random_offsets_cover_the_box():
    off = random_offsets(20000, seed=3)
    assert off.shape == (20000, 7) and off.dtype == np.float32
    assert np.all(off[:, 6] == 0.0)                       # SDD is never displaced
    for j, r in enumerate(PAPER_RANGES):
        assert np.all(np.abs(off[:, j]) <= 0.5 * r + 1e-6)
        # uniform over the full width: the extremes come close to the edges
        assert off[:, j].max() > 0.49 * r and off[:, j].min() < -0.49 * r
    np.testing.assert_array_equal(off, random_offsets(20000, seed=3))
    assert not np.array_equal(off, random_offsets(20000, seed=4))


def test_grid_offsets_layout():
    k = 5
    off = grid_offsets(1, 4, 2.0, 8.0, k)
    assert off.shape == (k * k, 7)
    others = [c for c in range(7) if c not in (1, 4)]
    assert np.all(off[:, others] == 0.0)
    grid = off.reshape(k, k, 7)
    np.testing.assert_allclose(grid[:, 0, 1], np.linspace(-1.0, 1.0, k))   # rows: param i
    np.testing.assert_allclose(grid[0, :, 4], np.linspace(-4.0, 4.0, k))   # columns: param j
    assert np.all(grid[k // 2, k // 2] == 0.0)            # centre sample is the ground truth


def test_pose_errors_geodesic_and_translation():
    base = np.array([0.3, -0.2, 0.1, 5.0, -3.0, 2.0, 1020.0])
    r, t = pose_errors(base[None], base[None])
    assert abs(r[0]) < 1e-6 and t[0] == 0.0
    # a rotation about the z axis composed on the left: the geodesic angle
    # between R and Rz(d) R is |d| whatever R is
    for d in (0.05, -0.4, 1.2):
        moved = base.copy()
        moved[0] += d                                        # Rz(theta + d) = Rz(d) Rz(theta)
        r, _ = pose_errors(moved[None], base[None])
        assert abs(r[0] - math.degrees(abs(d))) < 1e-9
    shifted = base.copy()
    shifted[3:6] += (3.0, 4.0, 12.0)
    _, t = pose_errors(shifted[None], base[None])
    assert abs(t[0] - 13.0) < 1e-12
