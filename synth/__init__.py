"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This package generates inputs only: CT-like phantom volumes, detector
descriptions and pose batches.  It holds none of the ray-tracing method's
arithmetic (no plane crossings, no line integrals, no gradients), so the
oracle and the GPU path can both consume its arrays without sharing any part
of the computation under test.
"""

from .phantom import Phantom, make_phantom, ellipsoid_phantom
from .poses import random_poses

__all__ = [
    "Phantom",
    "make_phantom",
    "ellipsoid_phantom",
    "random_poses",
]
