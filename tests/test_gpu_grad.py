"""GPU pose gradients and the NCC loss against the FP64 oracle.

Jacobians are compared with the oracle's frozen-index Jacobian (itself pinned
to central differences), and with FP64 central differences of the oracle on
pixels whose voxel sequence does not change within the step (kink-free).
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
# FP32 per-ray sums against the FP64 frozen-index Jacobian, relative to each
# parameter's largest entry.
JAC_RTOL = 2e-4
# Tolerance against central differences on kink-free pixels.
FD_RTOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


@pytest.fixture(scope="module")
def small():
    import paper_2208_12737_amd as P
    ph = make_phantom("small", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    return ph, vol, oracle.Grid(ph.volume, ph.spacing, ph.origin)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@pytest.mark.parametrize("seed", [0, 3])
def test_jacobian_matches_oracle(small, seed):
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    poses = random_poses(2, math.pi / 8, 10.0, 1000.0, seed=seed)
    det = P.Detector(48, 40, 2.5, 2.5)
    img, jac = P.render(vol, _gpu(poses), det, jacobian=True)
    rimg, rjac = oracle.render_jacobian(grid, poses.astype(np.float64), 48, 40, 2.5, 2.5,
                                        nthreads=4)
    assert_image_close(img.cpu().numpy(), rimg)
    err = column_errors(jac.cpu().numpy(), rjac)
    assert np.all(err <= JAC_RTOL), err


def _near_parallel_pose(axis, H, W, pitch, rho):
    """A pose for which one detector ray runs almost parallel to the planes of
    `axis` (|d_axis| of order 1e-4 mm or less against |d| ~ 2 rho)."""
    if axis == 2:      # row H/2 - 1: d_z = 2 rho sin(phi) - (pitch / 2) cos(phi)
        return np.array([0.2, math.atan(pitch / (4 * rho)), 0.0, 1.0, -2.0, 0.5, 2 * rho],
                        np.float32)
    if axis == 1:      # column W/2 - 1: d_y = -2 rho sin(theta) - (pitch / 2) cos(theta)
        return np.array([-math.atan(pitch / (4 * rho)), 0.0, 0.0, 1.0, -2.0, 0.5, 2 * rho],
                        np.float32)
    # column W/2 - 1 with the central ray along y: d_x = -2 rho cos(theta) + (pitch / 2) sin(theta)
    return np.array([math.atan2(2 * rho, -pitch / 2), 0.1, 0.0, 1.0, -2.0, 0.5, 2 * rho],
                    np.float32)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_jacobian_rays_parallel_to_planes(small, axis):
    """Rays almost parallel to one family of planes: the tail divides that
    axis's sums by d_c, so their rounding error is multiplied by |d| / d_c
    (here ~1e7); every axis is summed explicitly to keep that error relative
    to the axis's own terms."""
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    H = W = 64
    pitch, rho = 2.0, 500.0
    pose = _near_parallel_pose(axis, H, W, pitch, rho)
    p64 = pose.astype(np.float64)
    dmin = min(abs((lambda sp: (sp[1] - sp[0])[axis])(oracle.ray_endpoints(p64, H, W, pitch, pitch, h, w)))
               for h in range(H) for w in range(W))
    assert dmin < 1e-3, dmin
    det = P.Detector(H, W, pitch, pitch)
    img, jac = P.render(vol, _gpu(pose[None]), det, jacobian=True)
    rimg, rjac = oracle.render_jacobian(grid, p64[None], H, W, pitch, pitch, nthreads=4)
    assert_image_close(img.cpu().numpy(), rimg)
    errs = column_errors(jac.cpu().numpy()[0], rjac[0])
    assert max(errs) <= JAC_RTOL, errs


def test_folded_and_masked_exits_agree():
    """The detector plane cuts the grid, so some rays end inside it (alpha =
    1, traced by the masked loop) and the rest leave through a face (their
    exit crossing folded into the loop, unless their wave also holds a ray
    that ends inside).  The same rays on a detector three pixels larger on
    every side (so each wave holds other neighbours, and face-exit rays next
    to the boundary change loop) give bitwise the same image and Jacobian;
    the image mode gives the same image; all against the oracle.  The grid is
    non-zero up to its faces, so every exit term counts."""
    import paper_2208_12737_amd as P
    rng = np.random.default_rng(77)
    dims, spacing = (40, 36, 44), (1.0, 1.2, 0.9)
    ext = np.asarray(dims) * np.asarray(spacing)
    origin = tuple(float(v) for v in -0.5 * ext)
    data = rng.uniform(0.2, 2.0, dims).astype(np.float32)
    vol = P.Volume(torch.from_numpy(data), spacing, origin, device=DEV)
    grid = oracle.Grid(data, spacing, origin)
    # source at x ~ +44 mm (outside), detector plane at x ~ -16 mm (inside)
    pose = np.array([[0.05, -0.04, 0.03, 14.0, 0.5, -0.7, 60.0]], np.float32)
    H = W = 30
    small_det, big_det = P.Detector(H, W, 2.0, 2.0), P.Detector(H + 6, W + 6, 2.0, 2.0)
    p64 = pose[0].astype(np.float64)
    inside = np.array([[np.all((oracle.ray_endpoints(p64, H, W, 2.0, 2.0, h, w)[1] > origin)
                               & (oracle.ray_endpoints(p64, H, W, 2.0, 2.0, h, w)[1]
                                  < np.asarray(origin) + ext))
                        for w in range(W)] for h in range(H)])
    assert 100 < inside.sum() < H * W - 100, inside.sum()
    ia, ja = P.render(vol, _gpu(pose), small_det, jacobian=True)
    ib, jb = P.render(vol, _gpu(pose), big_det, jacobian=True)
    assert torch.equal(ia[0], ib[0, 3:3 + H, 3:3 + W])
    assert torch.equal(ja[0], jb[0, 3:3 + H, 3:3 + W])
    assert torch.equal(P.render(vol, _gpu(pose), small_det), ia)
    rimg, rjac = oracle.render_jacobian(grid, p64[None], H, W, 2.0, 2.0, nthreads=4)
    assert_image_close(ia.cpu().numpy(), rimg)
    errs = column_errors(ja.cpu().numpy()[0], rjac[0])
    assert max(errs) <= JAC_RTOL, errs


def test_jacobian_with_clamped_ends(small):
    """Source and detector inside the volume (SDD 40 mm in a 64 mm cube): the
    ray ends are clamped to alpha = 0 and 1 and belong to no plane.  GPU
    Jacobian against the oracle's, and both against FP64 central differences
    on kink-free pixels."""
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    H = W = 24
    pitch = 1.5
    pose = np.array([0.3, 0.2, 0.1, 1.0, 2.0, 3.0, 40.0], np.float32)
    det = P.Detector(H, W, pitch, pitch)
    img, jac = P.render(vol, _gpu(pose[None]), det, jacobian=True)
    p64 = pose.astype(np.float64)
    rimg, rjac = oracle.render_jacobian(grid, p64[None], H, W, pitch, pitch)
    assert_image_close(img.cpu().numpy(), rimg)
    errs = column_errors(jac.cpu().numpy()[0], rjac[0])
    assert max(errs) <= JAC_RTOL, errs
    fd, ok = oracle.render_fd(grid, p64, H, W, pitch, pitch, [1e-4] * 3 + [1e-3] * 4)
    J = jac.cpu().numpy()[0].astype(np.float64)
    for j in range(7):
        m = ok[:, :, j]
        assert m.sum() > 50, (j, int(m.sum()))
        scale = np.abs(J[:, :, j]).max()
        assert np.abs(J[:, :, j][m] - fd[:, :, j][m]).max() <= FD_RTOL * scale, j
        assert np.abs(rjac[0, :, :, j][m] - fd[:, :, j][m]).max() <= 1e-4 * scale, j


def test_jacobian_vs_central_differences(small):
    """Per-pixel d image / d pose against FP64 central differences of the
    oracle with steps 1e-4 rad / 1e-3 mm, on kink-free pixels."""
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    pose = random_poses(1, math.pi / 8, 10.0, 1000.0, seed=4)
    det = P.Detector(32, 32, 4.0, 4.0)
    _, jac = P.render(vol, _gpu(pose), det, jacobian=True)
    jac = jac.cpu().numpy()[0]
    steps = [1e-4] * 3 + [1e-3] * 3 + [1e-3]
    fd, ok = oracle.render_fd(grid, pose[0].astype(np.float64), 32, 32, 4.0, 4.0, steps,
                              nthreads=4)
    for j in range(7):
        m = ok[:, :, j]
        assert m.mean() > 0.3
        scale = np.abs(fd[:, :, j][m]).max()
        err = np.abs(jac[:, :, j][m] - fd[:, :, j][m]).max() / scale
        assert err <= FD_RTOL, (j, err)


def test_backward_stored_and_retrace(small):
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    poses = random_poses(3, math.pi / 8, 10.0, 1000.0, seed=5)
    det = P.Detector(40, 44, 2.0, 2.0)
    rng = np.random.default_rng(1)
    g = rng.normal(size=(3, 40, 44)).astype(np.float32)
    _, jac = P.render(vol, _gpu(poses), det, jacobian=True)
    gp = P.render_backward(det, jac, _gpu(g)).cpu().numpy()
    gr = P.render_backward_retrace(vol, _gpu(poses), det, _gpu(g)).cpu().numpy()
    _, rjac = oracle.render_jacobian(grid, poses.astype(np.float64), 40, 44, 2.0, 2.0,
                                     nthreads=4)
    ref = np.einsum("bhw,bhwj->bj", g.astype(np.float64), rjac)
    for b in range(3):
        assert_gradient_close(gp[b], ref[b], g[b], rjac[b], f"stored-J backward, pose {b}")
        assert_gradient_close(gr[b], ref[b], g[b], rjac[b], f"retrace backward, pose {b}")
    np.testing.assert_allclose(gp, gr, rtol=1e-5, atol=1e-6 * np.abs(gp).max())


def test_autograd_function(small):
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    poses = _gpu(random_poses(2, math.pi / 8, 10.0, 1000.0, seed=6))
    det = P.Detector(32, 32, 4.0, 4.0)
    g = torch.randn((2, 32, 32), device=DEV)
    for retrace in (False, True):
        p = poses.clone().requires_grad_(True)
        img = P.drr(vol, p, det, retrace=retrace)
        (img * g).sum().backward()
        _, jac = P.render(vol, poses, det, jacobian=True)
        ref = P.render_backward(det, jac, g)
        torch.testing.assert_close(p.grad, ref, rtol=1e-5, atol=1e-5 * ref.abs().max().item())


def test_ncc_forward_backward():
    import paper_2208_12737_amd as P
    rng = np.random.default_rng(2)
    I = rng.uniform(0, 5, (3, 37, 29))
    T = rng.uniform(0, 5, (3, 37, 29))
    It, Tt = _gpu(I), _gpu(T).requires_grad_(False)
    x = It.clone().requires_grad_(True)
    loss = P.ncc_loss(x, Tt)
    gl = torch.tensor([1.0, -2.0, 0.5], device=DEV)
    (loss * gl).sum().backward()
    for b in range(3):
        z, gz = oracle.zncc_grad(It[b].cpu().numpy().astype(np.float64), T[b].astype(np.float32))
        assert loss[b].item() == pytest.approx(-z, abs=1e-6)
        np.testing.assert_allclose(x.grad[b].cpu().numpy(), -gl[b].item() * gz, rtol=1e-4,
                                   atol=1e-5 * np.abs(gz).max())
    # one target shared by all images
    loss2 = P.ncc_loss(It, Tt[0])
    for b in range(3):
        z = oracle.zncc(It[b].cpu().numpy(), T[0].astype(np.float32))
        assert loss2[b].item() == pytest.approx(-z, abs=1e-6)


def test_fused_ncc_gradient_matches_oracle(small):
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    det = P.Detector(40, 40, 3.0, 3.0)
    gt = random_poses(1, math.pi / 8, 10.0, 1000.0, seed=8)
    moving = random_poses(3, math.pi / 8, 10.0, 1000.0, seed=9)
    target = _gpu(oracle_image(grid, gt[0], 40, 40, 3.0, 3.0))[None]
    loss, grad, img = P.render_ncc_grad(vol, _gpu(moving), det, target[0], return_image=True)
    T = target.cpu().numpy()[0].astype(np.float64)
    rimg, rjac = oracle.render_jacobian(grid, moving.astype(np.float64), 40, 40, 3.0, 3.0,
                                        nthreads=4)
    assert_image_close(img.cpu().numpy(), rimg)
    for b in range(3):
        z, gz = oracle.zncc_grad(rimg[b], T)
        assert loss[b].item() == pytest.approx(-z, abs=2e-6)
        ref = -np.einsum("hw,hwj->j", gz, rjac[b])
        assert_gradient_close(grad[b].cpu().numpy(), ref, gz, rjac[b], f"fused -ZNCC, pose {b}")
    # the fused path equals render -> ncc_loss -> autograd
    p = _gpu(moving).requires_grad_(True)
    l2 = P.ncc_loss(P.drr(vol, p, det), target[0])
    l2.sum().backward()
    torch.testing.assert_close(l2, loss, rtol=1e-5, atol=1e-6)
    torch.testing.assert_close(p.grad, grad, rtol=1e-4, atol=1e-4 * grad.abs().max().item())


def test_fused_l2_matches_oracle(small):
    """Mean squared difference and its pose gradient, fused, against the
    oracle's image, Jacobian and L2 gradient; the loss-only form gives the
    same loss, and the gradient equals the stored-Jacobian contraction of
    2 (I - T) / N."""
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    H, W = 36, 44
    det = P.Detector(H, W, 3.0, 3.0)
    gt = random_poses(1, math.pi / 8, 10.0, 1000.0, seed=18)
    moving = random_poses(4, math.pi / 8, 10.0, 1000.0, seed=19)
    target = _gpu(oracle_image(grid, gt[0], H, W, 3.0, 3.0))[None]
    loss, grad, img = P.render_l2(vol, _gpu(moving), det, target[0], return_image=True)
    T = target.cpu().numpy()[0].astype(np.float64)
    rimg, rjac = oracle.render_jacobian(grid, moving.astype(np.float64), H, W, 3.0, 3.0,
                                        nthreads=4)
    assert_image_close(img.cpu().numpy(), rimg)
    for b in range(4):
        v, gl = oracle.l2_grad(rimg[b], T)
        assert loss[b].item() == pytest.approx(v, rel=1e-5)
        ref = np.einsum("hw,hwj->j", gl, rjac[b])
        assert_gradient_close(grad[b].cpu().numpy(), ref, gl, rjac[b], f"fused L2, pose {b}")
    only, none = P.render_l2(vol, _gpu(moving), det, target[0], grad=False)
    assert none is None
    torch.testing.assert_close(only, loss, rtol=1e-6, atol=0.0)
    # per-pose targets give the same result as one shared target
    per = target.expand(4, H, W).contiguous()
    l4, g4 = P.render_l2(vol, _gpu(moving), det, per)
    torch.testing.assert_close(l4, loss, rtol=0.0, atol=0.0)
    torch.testing.assert_close(g4, grad, rtol=0.0, atol=0.0)
    gimg = (2.0 / (H * W)) * (img - target[0])
    g2 = P.render_backward_retrace(vol, _gpu(moving), det, gimg)
    torch.testing.assert_close(g2, grad, rtol=1e-4, atol=1e-4 * grad.abs().max().item())
    # at the target pose the loss and gradient vanish, up to the difference
    # of the GPU's and the oracle's image (within the image tolerance)
    l0, g0 = P.render_l2(vol, _gpu(gt), det, target[0])
    assert l0.item() <= 1e-10 * float((target[0].double() ** 2).mean())
    assert g0.abs().max().item() <= 1e-4 * grad.abs().max().item()


def test_occupancy_settings_give_identical_results(small):
    """Every residency setting of the direct launches (1, 2, 8 workgroups per
    CU, unlimited, default) yields bitwise the same image and fused gradient;
    the LDS reserved to cap residency stays within the per-workgroup limit."""
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd import _lib
    ph, vol, grid = small
    det = P.Detector(40, 36, 3.0, 3.0)
    gt = random_poses(1, math.pi / 8, 10.0, 1000.0, seed=21)
    moving = _gpu(random_poses(5, math.pi / 8, 10.0, 1000.0, seed=22))
    target = P.render(vol, _gpu(gt), det)[0]
    img0 = P.render(vol, moving, det)
    loss0, grad0 = P.render_ncc_grad(vol, moving, det, target)
    try:
        for occ in (1, 2, 8, 0, -1):
            _lib.call("drr_set_launch_occupancy", occ)
            assert torch.equal(P.render(vol, moving, det), img0), occ
            loss, grad = P.render_ncc_grad(vol, moving, det, target)
            torch.cuda.synchronize()
            assert torch.equal(loss, loss0) and torch.equal(grad, grad0), occ
    finally:
        _lib.call("drr_set_launch_occupancy", -1)


def test_masked_ncc_gradient_vs_central_differences(small):
    """d(-ZNCC)/d pose over the pixels that are kink-free for a parameter,
    with the GPU Jacobian, against FP64 central differences of the oracle's
    masked loss (steps 1e-4 rad / 1e-3 mm)."""
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    H = W = 32
    det = P.Detector(H, W, 4.0, 4.0)
    gt = random_poses(1, math.pi / 8, 10.0, 1000.0, seed=12)[0].astype(np.float64)
    pose = gt + np.array([0.03, -0.02, 0.04, 1.5, -1.0, 2.0, 0.0])
    T, _, _ = oracle.render(grid, gt, H, W, 4.0, 4.0)
    _, jac = P.render(vol, _gpu(pose[None]), det, jacobian=True)
    jac = jac.cpu().numpy()[0].astype(np.float64)
    steps = [1e-4] * 3 + [1e-3] * 3 + [1e-3]
    I0, _, h0 = oracle.render(grid, pose, H, W, 4.0, 4.0)
    for j in range(7):
        pp, pm = pose.copy(), pose.copy()
        pp[j] += steps[j]
        pm[j] -= steps[j]
        Ip, _, hp = oracle.render(grid, pp, H, W, 4.0, 4.0)
        Im, _, hm = oracle.render(grid, pm, H, W, 4.0, 4.0)
        m = ((hp == h0) & (hm == h0))[0]
        fd = (-oracle.zncc(Ip[0][m], T[0][m]) + oracle.zncc(Im[0][m], T[0][m])) / (2 * steps[j])
        _, gz = oracle.zncc_grad(I0[0][m], T[0][m])
        an = -(gz * jac[:, :, j][m]).sum()
        assert abs(an - fd) <= FD_RTOL * max(abs(fd), 1e-3 * np.abs(gz).sum() * np.abs(jac[:, :, j][m]).max()), (j, an, fd)


def test_momentum_step():
    import paper_2208_12737_amd as P
    rng = np.random.default_rng(3)
    p = rng.normal(size=(5, 7)).astype(np.float32)
    v = rng.normal(size=(5, 7)).astype(np.float32)
    g = rng.normal(size=(5, 7)).astype(np.float32)
    r = rng.uniform(0, 1, (5, 7)).astype(np.float32)
    pt, vt = _gpu(p), _gpu(v)
    P.momentum_step(pt, vt, _gpu(g), _gpu(r), 0.9)
    v2 = 0.9 * v + g
    np.testing.assert_allclose(vt.cpu().numpy(), v2, rtol=1e-6)
    np.testing.assert_allclose(pt.cpu().numpy(), p - r * v2, rtol=1e-5, atol=1e-6)


def test_detector_jacobian_matches_oracle_and_differences(small):
    """d image / d (delta_x, delta_y, offset_u, offset_v) at a non-zero
    principal-point offset: against the oracle's analytic derivative and
    against FP64 central differences of the oracle on kink-free pixels."""
    import paper_2208_12737_amd as P
    ph, vol, grid = small
    poses = random_poses(2, math.pi / 8, 10.0, 1000.0, seed=13)
    H, W, dx, dy, ou, ov = 33, 29, 3.0, 2.5, 4.2, -2.9
    det = P.Detector(H, W, dx, dy, ou, ov)
    img, jd = P.render_detector_jacobian(vol, _gpu(poses), det)
    rimg, rjd = oracle.render_detector_jacobian(grid, poses.astype(np.float64), H, W, dx, dy,
                                                offset=(ou, ov))
    assert_image_close(img.cpu().numpy(), rimg)
    jd = jd.cpu().numpy()
    scale = np.abs(rjd).max(axis=(0, 1, 2))
    assert np.all(np.abs(jd - rjd).max(axis=(0, 1, 2)) <= JAC_RTOL * scale)
    e = 1e-3
    p0 = poses[0].astype(np.float64)
    base = np.array([dx, dy, ou, ov])
    _, _, h0 = oracle.render(grid, p0, H, W, dx, dy, offset=(ou, ov))
    for j in range(4):
        a, b = base.copy(), base.copy()
        a[j] += e
        b[j] -= e
        ip, _, hp = oracle.render(grid, p0, H, W, a[0], a[1], offset=(a[2], a[3]))
        im, _, hm = oracle.render(grid, p0, H, W, b[0], b[1], offset=(b[2], b[3]))
        ok = ((hp == h0) & (hm == h0))[0]
        fd = (ip - im)[0] / (2 * e)
        err = np.abs(jd[0, :, :, j][ok] - fd[ok]).max() / np.abs(fd[ok]).max()
        assert err <= FD_RTOL, (j, err)
    # pose Jacobian and the fused gradient with the offset detector
    _, jac = P.render(vol, _gpu(poses), det, jacobian=True)
    _, rjac = oracle.render_jacobian(grid, poses.astype(np.float64), H, W, dx, dy,
                                     offset=(ou, ov))
    errs = column_errors(jac.cpu().numpy(), rjac)
    assert max(errs) <= JAC_RTOL, errs
