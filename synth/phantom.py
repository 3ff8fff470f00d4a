"""Seeded ellipsoid phantoms standing in for the paper's chest CT.

The paper renders a chest CT of about 360 x 360 x 332.5 mm whose voxel grid
is not given (Section 3, registration experiment); it is not available here.
These phantoms stand in for it with the same physical size and a CT-like
structure: soft tissue (a background ellipsoid), an optional dense shell that
mimics bone, and random interior ellipsoids of varying attenuation.

Layout: the volume is a C-order float32 array of shape (nx, ny, nz); element
[i, j, k] is the attenuation of the voxel whose centre is
origin + (i + 0.5, j + 0.5, k + 0.5) * spacing, with origin = -n * spacing / 2
so that the grid is centred on the world origin.

Draw order from ``numpy.random.default_rng(seed)`` (PCG64), per interior
ellipsoid k = 0..n-1, in this order:
  centre   = uniform(-1, 1, 3) * 0.5 * background_semi_axes
  semi     = uniform(3, 20, 3) * scale          (mm)
  q        = normal(size=4), normalised          (uniform random rotation)
  mu       = uniform(0, 2)
Ellipsoids are painted in that order, later ones overwriting earlier ones.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Phantom:
    volume: np.ndarray          # float32, C-order (nx, ny, nz)
    spacing: tuple              # (dX, dY, dZ) in mm
    origin: tuple               # position of plane 0 on each axis, mm

    @property
    def shape(self):
        return self.volume.shape


def _quat_to_matrix(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
            [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
            [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
        ]
    )


def _centres(n: int, d: float, o: float) -> np.ndarray:
    return o + (np.arange(n, dtype=np.float64) + 0.5) * d


def _paint_ellipsoid(vol, spacing, origin, centre, semi, rot, mu):
    """Set voxels whose centre lies inside the rotated ellipsoid to mu."""
    # half-extent of the rotated ellipsoid along each world axis
    half = np.sqrt(((rot * semi[None, :]) ** 2).sum(axis=1))
    lo_hi = []
    for c in range(3):
        n = vol.shape[c]
        lo = int(np.floor((centre[c] - half[c] - origin[c]) / spacing[c] - 0.5))
        hi = int(np.ceil((centre[c] + half[c] - origin[c]) / spacing[c] - 0.5)) + 1
        lo, hi = max(lo, 0), min(hi, n)
        if lo >= hi:
            return
        lo_hi.append((lo, hi))
    xs = _centres(vol.shape[0], spacing[0], origin[0])[lo_hi[0][0]:lo_hi[0][1]] - centre[0]
    ys = _centres(vol.shape[1], spacing[1], origin[1])[lo_hi[1][0]:lo_hi[1][1]] - centre[1]
    zs = _centres(vol.shape[2], spacing[2], origin[2])[lo_hi[2][0]:lo_hi[2][1]] - centre[2]
    # body-frame coordinates r = rot^T (x - centre), evaluated one x-slab at
    # a time to keep temporaries small
    sub = vol[lo_hi[0][0]:lo_hi[0][1], lo_hi[1][0]:lo_hi[1][1], lo_hi[2][0]:lo_hi[2][1]]
    for ii, x in enumerate(xs):
        q = np.zeros((ys.size, zs.size))
        for a in range(3):
            r = (rot[0, a] * x + rot[1, a] * ys[:, None] + rot[2, a] * zs[None, :]) / semi[a]
            q += r * r
        sub[ii][q <= 1.0] = mu


def _axis_ellipsoid_mask(shape, spacing, origin, semi):
    r = [(_centres(n, spacing[c], origin[c]) / semi[c]) ** 2 for c, n in enumerate(shape)]
    out = np.empty(shape, dtype=bool)
    for i in range(shape[0]):
        out[i] = (r[0][i] + r[1][:, None] + r[2][None, :]) <= 1.0
    return out


def ellipsoid_phantom(shape, spacing, n_ellipsoids, seed, shell_mm=0.0,
                      background_mu=0.2, shell_mu=1.8, semi_range=(3.0, 20.0),
                      scale=None) -> Phantom:
    """Build a seeded phantom (see the module docstring for the recipe)."""
    shape = tuple(int(s) for s in shape)
    spacing = tuple(float(s) for s in spacing)
    extent = np.array([shape[c] * spacing[c] for c in range(3)])
    origin = tuple(float(-e / 2.0) for e in extent)
    if scale is None:
        scale = float(extent.min()) / 64.0
    vol = np.zeros(shape, dtype=np.float32)
    bg_semi = 0.45 * extent
    vol[_axis_ellipsoid_mask(shape, spacing, origin, bg_semi)] = background_mu
    if shell_mm > 0.0:
        inner = bg_semi - shell_mm
        shell = _axis_ellipsoid_mask(shape, spacing, origin, bg_semi) & ~_axis_ellipsoid_mask(
            shape, spacing, origin, inner)
        vol[shell] = shell_mu
    rng = np.random.default_rng(seed)
    for _ in range(n_ellipsoids):
        centre = rng.uniform(-1.0, 1.0, 3) * 0.5 * bg_semi
        semi = rng.uniform(semi_range[0], semi_range[1], 3) * scale
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        mu = rng.uniform(0.0, 2.0)
        _paint_ellipsoid(vol, spacing, origin, centre, semi, _quat_to_matrix(q), np.float32(mu))
    return Phantom(volume=vol, spacing=spacing, origin=origin)


def make_phantom(kind: str, seed: int = 0) -> Phantom:
    """Named phantoms of the benchmark workloads.

    small  : 64^3 at 1.0 mm, 8 interior ellipsoids (no shell)
    ct512  : 512 x 512 x 133 at 0.7 x 0.7 x 2.5 mm, 32 ellipsoids + 5 mm shell
    ct128  : 128^3 at 2 mm; ct256: 256^3 at 1 mm;
    ct512x300 : 512 x 512 x 300 at 0.7 x 0.7 x 1.25 mm (serving mix volumes)
    """
    if kind == "small":
        return ellipsoid_phantom((64, 64, 64), (1.0, 1.0, 1.0), 8, seed)
    if kind == "ct512":
        return ellipsoid_phantom((512, 512, 133), (0.7, 0.7, 2.5), 32, seed, shell_mm=5.0)
    if kind == "ct128":
        return ellipsoid_phantom((128, 128, 128), (2.0, 2.0, 2.0), 32, seed, shell_mm=5.0)
    if kind == "ct256":
        return ellipsoid_phantom((256, 256, 256), (1.0, 1.0, 1.0), 32, seed, shell_mm=5.0)
    if kind == "ct512x300":
        return ellipsoid_phantom((512, 512, 300), (0.7, 0.7, 1.25), 32, seed, shell_mm=5.0)
    raise ValueError(f"unknown phantom kind {kind!r}")
