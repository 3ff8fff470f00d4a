"""Batched 6-DoF slice-to-volume registration on the GPU (Sec. 3.2).

Each problem moves a pose so that its DRR matches a fixed target image,
minimising the negative zero-normalised cross-correlation by gradient
descent with momentum (heavy ball), with separate step sizes for the
rotations and the translations and the source-to-detector distance held
fixed.  All problems advance together: one step is one fused tracing launch
(image, loss and pose gradient for every problem, drr_render_ncc_grad)
followed by one momentum update (drr_pose_momentum_step).  With
``use_graph`` every step of the run is captured once into a single HIP graph
and replayed, so a whole registration is one graph launch.  The problems can
be split into ``chains`` groups that advance on streams of their own (in the
graph: independent branches), so that one group's launches fill the GPU while
another's finish; each problem's arithmetic is the same in any grouping.
"""

from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from .drr import (Detector, Volume, _stream, render, drr, ncc_loss, momentum_step,
                  target_stride)

# Step sizes of Sec. 3.2 (rotations in rad, translations in mm); SDD fixed.
PAPER_RATE_ROT = 5.3e-2
PAPER_RATE_XYZ = 75.0
PAPER_MOMENTUM = 0.9
CONVERGED_LOSS = -0.999


def default_rates(n: int, rot: float = PAPER_RATE_ROT, xyz: float = PAPER_RATE_XYZ,
                  device="cuda") -> torch.Tensor:
    r = torch.zeros((n, 7), dtype=torch.float32, device=device)
    r[:, 0:3] = rot
    r[:, 3:6] = xyz
    return r


class BatchedRegistration:
    """Registers n problems on one volume and detector at once.

    targets: [n, H, W] fixed images; init: [n, 7] starting poses;
    rates: [n, 7] per-problem, per-parameter step sizes; chains: number of
    independent problem groups (two measured fastest for 32 problems of
    256 x 256 pixels: one group's launch tail overlaps the other's work);
    record: keep every step's poses and pose gradients (eager runs only) in
    ``pose_history`` / ``grad_history`` [steps + 1, n, 7]."""

    def __init__(self, volume: Volume, det: Detector, targets: torch.Tensor,
                 init: torch.Tensor, rates: torch.Tensor, steps: int = 200,
                 momentum: float = PAPER_MOMENTUM, use_graph: bool = True, chains: int = 2,
                 record: bool = False):
        self.volume, self.det = volume, det
        self.n = init.shape[0]
        self.steps = steps
        self.momentum = float(momentum)
        dev = init.device
        if init.ndim != 2 or init.shape[1] != 7:
            raise ValueError(f"init must be [n, 7], got {tuple(init.shape)}")
        if tuple(rates.shape) != tuple(init.shape):
            raise ValueError(f"rates must be [n, 7] like init, got {tuple(rates.shape)}")
        # one target per problem, or one shared by all (stride 0)
        self.target_stride = target_stride(targets.numel(), self.n, det.pixels)
        self.targets = targets.contiguous().to(device=dev, dtype=torch.float32)
        self.init = init.detach().clone().contiguous()
        self.rates = rates.contiguous().to(torch.float32)
        self.poses = self.init.clone()
        self.vel = torch.zeros_like(self.poses)
        self.loss = torch.empty((self.n,), dtype=torch.float32, device=dev)   # warm-up only
        self.grad = torch.empty((self.n, 7), dtype=torch.float32, device=dev)
        self.history = torch.empty((steps + 1, self.n), dtype=torch.float32, device=dev)
        if record and use_graph:
            raise ValueError("record=True needs use_graph=False (the graph holds only the "
                             "library's kernels)")
        self.record = record
        if record:
            self.pose_history = torch.empty((steps + 1, self.n, 7), dtype=torch.float32,
                                            device=dev)
            self.grad_history = torch.empty_like(self.pose_history)
        self.use_graph = use_graph
        self.graph = None
        # problem ranges of the chains, and one workspace per chain
        k = max(1, min(int(chains), self.n))
        cuts = [self.n * c // k for c in range(k + 1)]
        self.groups = [(a, b) for a, b in zip(cuts[:-1], cuts[1:])]
        self.ws = []
        for a, b in self.groups:
            nbytes = _lib.load().drr_ncc_grad_workspace_bytes(ctypes.byref(det.desc), b - a)
            self.ws.append(torch.empty(max(nbytes, 8), dtype=torch.uint8, device=dev))
        self.streams = [torch.cuda.Stream() for _ in self.groups] if k > 1 else []

    def _objective(self, g: int, loss_out: torch.Tensor):
        a, b = self.groups[g]
        ws = self.ws[g]
        _lib.call("drr_render_ncc_grad", self.volume.packed.data_ptr(),
                  ctypes.byref(self.volume.desc), ctypes.byref(self.det.desc),
                  self.poses[a:b].data_ptr(), b - a,
                  self.targets.data_ptr() + 4 * a * self.target_stride,
                  self.target_stride, None, loss_out[a:b].data_ptr(), self.grad[a:b].data_ptr(),
                  ws.data_ptr(), ws.numel(), _stream())

    def _update(self, g: int):
        a, b = self.groups[g]
        _lib.call("drr_pose_momentum_step", self.poses[a:b].data_ptr(), self.vel[a:b].data_ptr(),
                  self.grad[a:b].data_ptr(), self.rates[a:b].data_ptr(), self.momentum, b - a,
                  _stream())

    def _keep(self, g: int, i: int):
        if self.record:
            a, b = self.groups[g]
            self.pose_history[i, a:b].copy_(self.poses[a:b])
            self.grad_history[i, a:b].copy_(self.grad[a:b])

    def _chain(self, g: int):
        # the loss of step i is written straight into history row i: the
        # graph holds only the library's kernels (no copy or fill nodes)
        for i in range(self.steps):
            self._objective(g, self.history[i])
            self._keep(g, i)
            self._update(g)
        self._objective(g, self.history[self.steps])
        self._keep(g, self.steps)

    def _all_steps(self):
        if not self.streams:
            self._chain(0)
            return
        main = torch.cuda.current_stream()
        for st in self.streams:
            st.wait_stream(main)
        for g, st in enumerate(self.streams):
            with torch.cuda.stream(st):
                self._chain(g)
        for st in self.streams:
            main.wait_stream(st)

    def _reset(self):
        self.poses.copy_(self.init)
        self.vel.zero_()

    def capture(self):
        """Capture the whole run (all steps) into one HIP graph."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._reset()
            for g in range(len(self.groups)):
                self._objective(g, self.loss)     # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._all_steps()
        self.graph = g

    def run(self):
        """Runs the registration from the initial poses; returns final poses
        [n, 7] and the loss history [steps + 1, n] (device tensors)."""
        self._reset()
        if self.use_graph:
            if self.graph is None:
                self.capture()
                self._reset()
            self.graph.replay()
        else:
            self._all_steps()
        return self.poses, self.history


def register_one_at_a_time(volume: Volume, det: Detector, targets: torch.Tensor,
                           init: torch.Tensor, rates: torch.Tensor, steps: int = 200,
                           momentum: float = PAPER_MOMENTUM):
    """Comparison path: each problem alone, one DRR per step through the plain
    autograd route (render with a stored Jacobian, NCC loss, backward), then
    the same momentum update."""
    out = init.detach().clone()
    final_loss = torch.empty((init.shape[0],), dtype=torch.float32, device=init.device)
    for k in range(init.shape[0]):
        p = init[k:k + 1].detach().clone()
        v = torch.zeros_like(p)
        r = rates[k:k + 1].contiguous()
        for _ in range(steps):
            q = p.clone().requires_grad_(True)
            loss = ncc_loss(drr(volume, q, det), targets[k])
            loss.sum().backward()
            momentum_step(p, v, q.grad.contiguous(), r, momentum)
        with torch.no_grad():
            final_loss[k] = ncc_loss(render(volume, p, det), targets[k])[0]
        out[k] = p[0]
    return out, final_loss


def _rot(p):
    """Rotation matrix Rz(theta) Ry(phi) Rx(gamma) of a pose (host, FP64):
    used only to report pose errors."""
    t, f, g = (float(v) for v in p[:3])
    cz, sz, cy, sy, cx, sx = math.cos(t), math.sin(t), math.cos(f), math.sin(f), math.cos(g), math.sin(g)
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    return Rz @ Ry @ Rx


def pose_errors(est: np.ndarray, gt: np.ndarray):
    """(rotation error in degrees (geodesic), translation error in mm) per problem."""
    rot, tr = [], []
    for a, b in zip(np.asarray(est, float), np.asarray(gt, float)):
        m = _rot(a).T @ _rot(b)
        c = np.clip((np.trace(m) - 1.0) / 2.0, -1.0, 1.0)
        rot.append(math.degrees(math.acos(c)))
        tr.append(float(np.linalg.norm(a[3:6] - b[3:6])))
    return np.array(rot), np.array(tr)
