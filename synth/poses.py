"""Seeded pose batches.

A pose is seven float32 numbers (theta, phi, gamma, bx, by, bz, sdd): three
rotation angles in radians, a translation in mm and the source-to-detector
distance in mm.  Draw order from ``numpy.random.default_rng(seed)``:
angles = uniform(-max_angle, max_angle, (n, 3)), then
translations = uniform(-max_shift, max_shift, (n, 3)).
"""

from __future__ import annotations

import numpy as np


def random_poses(n: int, max_angle: float, max_shift: float, sdd: float,
                 seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    ang = rng.uniform(-max_angle, max_angle, (n, 3))
    sh = rng.uniform(-max_shift, max_shift, (n, 3))
    out = np.empty((n, 7), dtype=np.float32)
    out[:, 0:3] = ang
    out[:, 3:6] = sh
    out[:, 6] = sdd
    return out
