"""The PyTorch front end rejects tensors whose sizes or devices would make a
kernel read or write past a buffer, before anything is launched."""

import math

import numpy as np
import pytest
import torch

from synth import make_phantom, random_poses

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


@pytest.fixture(scope="module")
def setup():
    import paper_2208_12737_amd as P
    ph = make_phantom("small", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    det = P.Detector(16, 12, 4.0, 4.0)
    poses = torch.from_numpy(random_poses(4, math.pi / 8, 10.0, 1000.0, seed=0)).to(DEV)
    return P, vol, det, poses


@pytest.mark.parametrize("fn", ["render_ncc_grad", "render_ncc_loss", "render_l2"])
@pytest.mark.parametrize("k", [2, 3, 5])
def test_fused_objectives_reject_target_sizes(setup, fn, k):
    P, vol, det, poses = setup
    bad = torch.zeros((k, det.height, det.width), device=DEV)
    with pytest.raises(ValueError):
        getattr(P, fn)(vol, poses, det, bad)


def test_fused_objectives_accept_shared_and_per_pose_targets(setup):
    P, vol, det, poses = setup
    shared = P.render(vol, poses[:1], det)[0]
    per = shared.expand(4, det.height, det.width).contiguous()
    a, ga = P.render_ncc_grad(vol, poses, det, shared)
    b, gb = P.render_ncc_grad(vol, poses, det, per)
    assert torch.equal(a, b) and torch.equal(ga, gb)


def test_ncc_loss_rejects_target_sizes(setup):
    P, vol, det, poses = setup
    img = P.render(vol, poses, det)
    with pytest.raises(ValueError):
        P.ncc_loss(img, torch.zeros((2, det.height, det.width), device=DEV))


def test_backward_rejects_mismatched_shapes(setup):
    P, vol, det, poses = setup
    img, jac = P.render(vol, poses, det, jacobian=True)
    g = torch.ones_like(img)
    with pytest.raises(ValueError):
        P.render_backward(det, jac, g[:3])                        # grad_image too small
    with pytest.raises(ValueError):
        P.render_backward(det, jac[..., :6].contiguous(), g)      # jac of 6 columns
    with pytest.raises(ValueError):
        P.render_backward(P.Detector(16, 13, 4.0, 4.0), jac, g)   # jac for another detector
    with pytest.raises(ValueError):
        P.render_backward_retrace(vol, poses, det, g[:3])


def test_momentum_step_rejects_mismatched_shapes(setup):
    P, vol, det, poses = setup
    p = poses.clone()
    v = torch.zeros_like(p)
    g = torch.zeros_like(p)
    r = torch.zeros_like(p)
    with pytest.raises(ValueError):
        P.momentum_step(p, v[:3].contiguous(), g, r, 0.9)
    with pytest.raises(ValueError):
        P.momentum_step(p, v, g, r[:, :6].contiguous(), 0.9)
    with pytest.raises(ValueError):
        P.momentum_step(p.reshape(-1), v.reshape(-1), g.reshape(-1), r.reshape(-1), 0.9)
    P.momentum_step(p, v, g, r, 0.9)                                # the valid call runs


def test_registration_rejects_target_sizes(setup):
    P, vol, det, poses = setup
    from paper_2208_12737_amd.register import BatchedRegistration, default_rates
    rates = default_rates(4)
    with pytest.raises(ValueError):
        BatchedRegistration(vol, det, torch.zeros((2, det.height, det.width), device=DEV),
                            poses, rates, steps=2, use_graph=False)
    # one shared target is accepted (stride 0) and equals four copies of it
    shared = P.render(vol, poses[:1], det)[0]
    a = BatchedRegistration(vol, det, shared, poses, rates, steps=2, use_graph=False)
    b = BatchedRegistration(vol, det, shared.expand(4, det.height, det.width).contiguous(),
                            poses, rates, steps=2, use_graph=False)
    pa, ha = a.run()
    pb, hb = b.run()
    torch.cuda.synchronize()
    assert torch.equal(pa, pb) and torch.equal(ha, hb)


def test_plan_items_reject_short_jacobian_and_counts(setup):
    P, vol, det, poses = setup
    from paper_2208_12737_amd.plan import Item, Plan
    plan = Plan([vol], max_items=4, use_graph=False)
    img = torch.empty((det.height, det.width), device=DEV)
    with pytest.raises(ValueError):
        plan.execute([Item(0, det, poses[0], img,
                           jac=torch.empty((det.height, det.width, 6), device=DEV))])
    with pytest.raises(ValueError):
        plan.execute([Item(0, det, poses[0], img,
                           counts=torch.empty(det.pixels - 1, dtype=torch.int32, device=DEV))])
    with pytest.raises(TypeError):
        plan.execute([Item(0, det, poses[0], img,
                           counts=torch.empty(det.pixels, dtype=torch.float32, device=DEV))])
    plan.close()
