"""Loss-landscape sweeps of the registration objective (Sec. 3.2).

The negative ZNCC (or, with ``loss="l2"``, the mean squared difference, for
which the paper reports similar landscapes) between the DRR at a displaced
pose and the DRR at the ground-truth pose is evaluated for many
displacements: random samples drawn
uniformly over ranges of 90 deg for theta and phi, 45 deg for gamma and
30 mm for each translation (centred on the ground truth, as in the paper's
convexity study), and regular 2-D grids over pairs of parameters.  Each
batch is one fused tracing launch that reduces only the loss moments per
tile (drr_render_ncc_loss, or drr_render_l2 without a gradient): no image,
Jacobian or gradient is stored.
"""

from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from .drr import Detector, Volume, render, render_l2, render_ncc_loss

# full widths of the sampled ranges (theta, phi, gamma in rad; shifts in mm)
PAPER_RANGES = (math.radians(90.0), math.radians(90.0), math.radians(45.0), 30.0, 30.0, 30.0)


def random_offsets(n: int, seed: int, ranges=PAPER_RANGES) -> np.ndarray:
    """[n, 7] offsets, uniform in +-range/2 per parameter (SDD fixed)."""
    rng = np.random.default_rng(seed)
    off = np.zeros((n, 7), np.float32)
    for j, r in enumerate(ranges):
        off[:, j] = rng.uniform(-0.5 * r, 0.5 * r, n)
    return off


def grid_offsets(i: int, j: int, span_i: float, span_j: float, k: int) -> np.ndarray:
    """[k*k, 7] offsets on a regular k x k grid over parameters i and j
    (+-span/2 each, the centre sample exactly zero when k is odd)."""
    a = np.linspace(-0.5 * span_i, 0.5 * span_i, k)
    b = np.linspace(-0.5 * span_j, 0.5 * span_j, k)
    off = np.zeros((k * k, 7), np.float32)
    off[:, i] = np.repeat(a, k)
    off[:, j] = np.tile(b, k)
    return off


def sweep(volume: Volume, det: Detector, gt_pose, offsets: np.ndarray,
          chunk: int = 4096, target: torch.Tensor | None = None,
          loss: str = "zncc") -> np.ndarray:
    """Loss (-ZNCC, or mean squared difference for loss="l2") at
    gt_pose + offsets, for every offset row."""
    if loss not in ("zncc", "l2"):
        raise ValueError(f"unknown loss {loss!r}")
    dev = volume.device
    gt = torch.as_tensor(np.asarray(gt_pose, np.float32).reshape(1, 7), device=dev)
    if target is None:
        target = render(volume, gt, det)[0]
    out = np.empty(len(offsets), np.float32)
    lib = _lib.load()
    ws_fn = lib.drr_ncc_loss_workspace_bytes if loss == "zncc" else lib.drr_l2_workspace_bytes
    need = ws_fn(ctypes.byref(det.desc), min(chunk, len(offsets)))
    ws = torch.empty(max(need, 8), dtype=torch.uint8, device=dev)
    off_t = torch.as_tensor(np.asarray(offsets, np.float32), device=dev)
    for s in range(0, len(offsets), chunk):
        poses = (gt + off_t[s:s + chunk]).contiguous()
        if loss == "zncc":
            val = render_ncc_loss(volume, poses, det, target, workspace=ws)
        else:
            val = render_l2(volume, poses, det, target, grad=False, workspace=ws)[0]
        out[s:s + len(poses)] = val.cpu().numpy()
    return out


def radial_monotonicity(volume: Volume, det: Detector, gt_pose, n_dirs: int, n_steps: int,
                        ranges=PAPER_RANGES, seed: int = 0, radius: float = 1.0,
                        loss: str = "zncc"):
    """Fraction of random directions (in the offset box, scaled by `radius`)
    along which the loss never decreases when moving away from the ground
    truth, sampled at n_steps points -- a convexity indicator."""
    rng = np.random.default_rng(seed)
    dirs = rng.uniform(-1, 1, (n_dirs, 6)) * (0.5 * np.asarray(ranges) * radius)
    t = np.linspace(0.0, 1.0, n_steps)
    off = np.zeros((n_dirs * n_steps, 7), np.float32)
    off[:, :6] = (dirs[:, None, :] * t[None, :, None]).reshape(-1, 6)
    vals = sweep(volume, det, gt_pose, off, loss=loss).reshape(n_dirs, n_steps)
    mono = np.all(np.diff(vals, axis=1) >= -1e-6 * max(1.0, float(np.abs(vals).max())), axis=1)
    return float(mono.mean()), vals
