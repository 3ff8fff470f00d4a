"""Independent brute-force line integrals that pin the oracle.

TEST INFRASTRUCTURE ONLY.  None of these share a formula with the oracle's
Siddon implementation: there is no slab min/max bound, no merged crossing
list and no midpoint-floor voxel rule here.

  chord_face_clip   length of a segment inside an axis-aligned box, found by
                    intersecting the segment with the six face planes and
                    testing which pieces lie inside the box.
  per_voxel_sum     sum over every voxel of attenuation x chord through that
                    voxel's box -- the exact radiological path of Eq. 1 for a
                    piecewise-constant volume, computed voxel by voxel.
  fine_step_integral  a Riemann sum of Eq. 1 with point samples of the
                    volume, exact for axis-aligned rays whose sample points
                    avoid the voxel planes.
"""

from __future__ import annotations

import numpy as np


def chord_face_clip(s, p, lo, hi):
    """Length of the part of segment s->p inside the box [lo, hi]."""
    s, p = np.asarray(s, float), np.asarray(p, float)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    d = p - s
    ts = [0.0, 1.0]
    for c in range(3):
        if d[c] != 0.0:
            for plane in (lo[c], hi[c]):
                t = (plane - s[c]) / d[c]
                if 0.0 < t < 1.0:
                    ts.append(t)
    ts = np.sort(np.array(ts))
    total = 0.0
    for a, b in zip(ts[:-1], ts[1:]):
        if b <= a:
            continue
        m = s + 0.5 * (a + b) * d
        if np.all(m >= lo) and np.all(m <= hi):
            total += (b - a)
    return total * float(np.linalg.norm(d))


def per_voxel_chords(dims, spacing, origin, s, p):
    """Chord of segment s->p through every voxel box, shape dims (vectorised)."""
    nx, ny, nz = dims
    s, p = np.asarray(s, float), np.asarray(p, float)
    d = p - s
    L = float(np.linalg.norm(d))
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    idx = np.stack([ii, jj, kk], axis=-1).reshape(-1, 3).astype(float)
    lo = np.asarray(origin, float) + idx * np.asarray(spacing, float)
    hi = lo + np.asarray(spacing, float)
    nvox = idx.shape[0]
    cand = [np.zeros(nvox), np.ones(nvox)]
    for c in range(3):
        for plane in (lo[:, c], hi[:, c]):
            if d[c] != 0.0:
                t = (plane - s[c]) / d[c]
                t = np.where((t > 0.0) & (t < 1.0), t, 0.0)
            else:
                t = np.zeros(nvox)
            cand.append(t)
    ts = np.sort(np.stack(cand, axis=1), axis=1)          # [nvox, 8]
    a, b = ts[:, :-1], ts[:, 1:]
    mid = s[None, None, :] + (0.5 * (a + b))[:, :, None] * d[None, None, :]
    inside = np.all((mid >= lo[:, None, :]) & (mid <= hi[:, None, :]), axis=2)
    seg = np.where(inside & (b > a), b - a, 0.0).sum(axis=1)
    return (seg * L).reshape(dims)


def per_voxel_sum(volume, spacing, origin, s, p):
    """Sum over voxels of attenuation x chord, and the count of voxels crossed."""
    ch = per_voxel_chords(volume.shape, spacing, origin, s, p)
    return float((np.asarray(volume, float) * ch).sum()), int((ch > 0).sum())


def fine_step_integral(volume, spacing, origin, s, p, n_steps):
    """Midpoint Riemann sum of Eq. 1 with nearest-cell point sampling."""
    s, p = np.asarray(s, float), np.asarray(p, float)
    d = p - s
    t = (np.arange(n_steps) + 0.5) / n_steps
    pts = s[None, :] + t[:, None] * d[None, :]
    f = (pts - np.asarray(origin, float)[None, :]) / np.asarray(spacing, float)[None, :]
    idx = np.floor(f).astype(np.int64)
    dims = np.asarray(volume.shape)
    inside = np.all((idx >= 0) & (idx < dims[None, :]), axis=1)
    vals = np.zeros(n_steps)
    ii = idx[inside]
    vals[inside] = np.asarray(volume, float)[ii[:, 0], ii[:, 1], ii[:, 2]]
    return float(vals.sum() * np.linalg.norm(d) / n_steps)
