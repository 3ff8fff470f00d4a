"""Pose gradients at clinical size: the 512 x 512 x 133 CT, a 200 x 200
detector at 1.4 mm (SDD 1020 mm) and a batch of 64 poses, with the negative
ZNCC against a target rendered at a seeded ground-truth pose.

The whole batch runs in one launch; sampled poses are checked against the
FP64 oracle's image and frozen-index Jacobian over every pixel, and the
fused loss gradient against FP64 central differences of the oracle's loss
(steps 1e-4 rad / 1e-3 mm) over the kink-free pixels.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from synth import make_phantom, random_poses
from tests._parity import (assert_gradient_close, assert_image_close, column_errors,
                           oracle_image)

pytestmark = pytest.mark.gpu

DEV = "cuda"
H = W = 200
PITCH = 1.4
SDD = 1020.0
JAC_RTOL = 2e-4
FD_RTOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


@pytest.fixture(scope="module")
def batch():
    import paper_2208_12737_amd as P
    ph = make_phantom("ct512", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    det = P.Detector(H, W, PITCH, PITCH)
    gt = random_poses(1, math.pi / 6, 30.0, SDD, seed=40)[0].astype(np.float64)
    rng = np.random.default_rng(41)
    off = np.zeros((64, 7))
    off[:, :3] = rng.uniform(-math.radians(15), math.radians(15), (64, 3))
    off[:, 3:6] = rng.uniform(-25.0, 25.0, (64, 3))
    poses = (gt[None] + off).astype(np.float32)
    target = torch.from_numpy(oracle_image(grid, gt, H, W, PITCH, PITCH, nthreads=16)).to(DEV)
    pt = torch.from_numpy(poses).to(DEV)
    loss, grad, img = P.render_ncc_grad(vol, pt, det, target, return_image=True)
    _, jac = P.render(vol, pt, det, jacobian=True)
    return P, vol, grid, det, gt, poses, target, loss, grad, img, jac


@pytest.mark.parametrize("b", [5, 50])
def test_sampled_poses_match_oracle_image_and_jacobian(batch, b):
    P, vol, grid, det, gt, poses, target, loss, grad, img, jac = batch
    rimg, rjac = oracle.render_jacobian(grid, poses[b:b + 1].astype(np.float64), H, W, PITCH,
                                        PITCH, nthreads=8)
    assert_image_close(img[b:b + 1].cpu().numpy(), rimg)
    errs = column_errors(jac[b].cpu().numpy().astype(np.float64), rjac[0])
    assert max(errs) <= JAC_RTOL, errs
    # the fused gradient equals the oracle's chain of d(-ZNCC)/dI and J
    T = target.cpu().numpy().astype(np.float64)
    z, gz = oracle.zncc_grad(rimg[0], T)
    assert loss[b].item() == pytest.approx(-z, abs=2e-6)
    ref = -np.einsum("hw,hwj->j", gz, rjac[0])
    assert_gradient_close(grad[b].cpu().numpy(), ref, gz, rjac[0], f"fused -ZNCC, pose {b}")
    # retraced backward of the same image gradient
    gr = P.render_backward_retrace(vol, torch.from_numpy(poses[b:b + 1]).to(DEV), det,
                                   torch.from_numpy((-gz).astype(np.float32)).to(DEV)[None])
    assert_gradient_close(gr[0].cpu().numpy(), ref, gz, rjac[0], f"retrace, pose {b}")


@pytest.mark.parametrize("b", [12, 40])
def test_fused_l2_at_clinical_size(batch, b):
    """The L2 objective (mean squared difference) fused over the same 64-pose
    launch: sampled poses' loss and pose gradient against the oracle's image,
    Jacobian and L2 gradient."""
    P, vol, grid, det, gt, poses, target, loss, grad, img, jac = batch
    pt = torch.from_numpy(poses).to(DEV)
    l2, g2 = P.render_l2(vol, pt, det, target)
    rimg, rjac = oracle.render_jacobian(grid, poses[b:b + 1].astype(np.float64), H, W, PITCH,
                                        PITCH, nthreads=8)
    T = target.cpu().numpy().astype(np.float64)
    v, gi = oracle.l2_grad(rimg[0], T)
    assert l2[b].item() == pytest.approx(v, rel=1e-5)
    ref = np.einsum("hw,hwj->j", gi, rjac[0])
    assert_gradient_close(g2[b].cpu().numpy(), ref, gi, rjac[0], f"fused L2, pose {b}")


def test_detector_jacobian_at_clinical_size(batch):
    """d image / d (delta_x, delta_y, offset_u, offset_v) of one pose of the
    batch, every pixel, against the oracle's frozen-index derivative."""
    P, vol, grid, det, gt, poses, target, loss, grad, img, jac = batch
    b = 21
    dimg, djac = P.render_detector_jacobian(vol, torch.from_numpy(poses[b:b + 1]).to(DEV), det)
    rimg, rjac = oracle.render_detector_jacobian(grid, poses[b:b + 1].astype(np.float64), H, W,
                                                 PITCH, PITCH, nthreads=8)
    assert_image_close(dimg.cpu().numpy(), rimg)
    errs = column_errors(djac[0].cpu().numpy().astype(np.float64), rjac[0])
    assert max(errs) <= JAC_RTOL, errs


def test_batch_gradient_equals_unfused_path(batch):
    """Fused objective = render -> NCC loss -> stored-Jacobian backward, on
    all 64 poses of the launch."""
    P, vol, grid, det, gt, poses, target, loss, grad, img, jac = batch
    pt = torch.from_numpy(poses).to(DEV).requires_grad_(True)
    l2 = P.ncc_loss(P.drr(vol, pt, det), target)
    l2.sum().backward()
    torch.testing.assert_close(l2.detach(), loss, rtol=1e-5, atol=1e-6)
    for b in range(64):
        tol = 1e-4 * grad[b].abs().max().item()
        torch.testing.assert_close(pt.grad[b], grad[b], rtol=1e-4, atol=tol)


@pytest.mark.parametrize("b", [9, 33, 58])
def test_masked_gradient_vs_central_differences(batch, b):
    """At this size a 1e-4 rad rotation reorders some plane crossings of
    most rays (only ~0.04-2 % of pixels stay kink-free for the angles,
    ~17-52 % for the shifts), so both checks run on the kink-free pixels of
    each parameter: the per-pixel Jacobian against the oracle's difference
    quotients, and the gradient of the masked loss against its difference
    quotient.  At least 10 pixels must be kink-free (a rotation about the
    principal axis leaves as few as ~15 of the 40 000 for some poses)."""
    P, vol, grid, det, gt, poses, target, loss, grad, img, jac = batch
    pose = poses[b].astype(np.float64)
    J = jac[b].cpu().numpy().astype(np.float64)
    T = target.cpu().numpy().astype(np.float64)
    I0, _, h0 = oracle.render(grid, pose, H, W, PITCH, PITCH, nthreads=8)
    steps = [1e-4] * 3 + [1e-3] * 3 + [1e-3]
    for j in range(7):
        pp, pm = pose.copy(), pose.copy()
        pp[j] += steps[j]
        pm[j] -= steps[j]
        Ip, _, hp = oracle.render(grid, pp, H, W, PITCH, PITCH, nthreads=8)
        Im, _, hm = oracle.render(grid, pm, H, W, PITCH, PITCH, nthreads=8)
        m = ((hp == h0) & (hm == h0))[0]
        assert m.sum() >= 10, (j, int(m.sum()))
        fdpix = (Ip[0] - Im[0])[m] / (pp[j] - pm[j])
        colscale = np.abs(J[:, :, j]).max()
        assert np.abs(J[:, :, j][m] - fdpix).max() <= FD_RTOL * colscale, j
        fd = (-oracle.zncc(Ip[0][m], T[m]) + oracle.zncc(Im[0][m], T[m])) / (pp[j] - pm[j])
        _, gz = oracle.zncc_grad(I0[0][m], T[m])
        an = -(gz * J[:, :, j][m]).sum()
        floor = 1e-3 * np.abs(gz).sum() * np.abs(J[:, :, j][m]).max()
        assert abs(an - fd) <= FD_RTOL * max(abs(fd), floor), (j, an, fd)


def test_fused_gradient_in_the_benchmark_configuration():
    """The benchmark's forward + backward batch exactly as timed: 256 moving
    poses (ground truth +-5 deg / +-5 mm) on the 512 x 512 x 133 CT, 256 x 256
    detector at 1.4 mm, one target per pose, one fused launch.  Two sampled
    poses are checked against the oracle's image, Jacobian and ZNCC gradient
    over every pixel."""
    import ctypes
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd import _lib
    ph = make_phantom("ct512", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    det = P.Detector(256, 256, 1.4, 1.4)
    nb = 256
    gt_np = random_poses(nb, math.pi / 6, 30.0, SDD, seed=2)
    off = np.random.default_rng(3).uniform(-1, 1, (nb, 7)).astype(np.float32)
    off[:, :3] *= math.radians(5.0)
    off[:, 3:6] *= 5.0
    off[:, 6] = 0.0
    moving_np = gt_np + off
    targets = P.render(vol, torch.from_numpy(gt_np).to(DEV), det)
    # the sampled poses' targets come from the oracle (they are oracle inputs)
    for b in (31, 200):
        targets[b] = torch.from_numpy(oracle_image(grid, gt_np[b], 256, 256, 1.4, 1.4,
                                                   nthreads=16)).to(DEV)
    moving = torch.from_numpy(moving_np).to(DEV)
    ws = torch.empty(_lib.load().drr_ncc_grad_workspace_bytes(ctypes.byref(det.desc), nb),
                     dtype=torch.uint8, device=DEV)
    loss, grad = P.render_ncc_grad(vol, moving, det, targets, workspace=ws)
    torch.cuda.synchronize()
    assert torch.isfinite(loss).all() and torch.isfinite(grad).all()
    for b in (31, 200):
        rimg, rjac = oracle.render_jacobian(grid, moving_np[b:b + 1].astype(np.float64), 256,
                                            256, 1.4, 1.4, nthreads=16)
        T = targets[b].cpu().numpy().astype(np.float64)
        z, gz = oracle.zncc_grad(rimg[0], T)
        assert loss[b].item() == pytest.approx(-z, abs=2e-6)
        ref = -np.einsum("hw,hwj->j", gz, rjac[0])
        assert_gradient_close(grad[b].cpu().numpy(), ref, gz, rjac[0], f"fused -ZNCC, pose {b}")
