"""Batched registration on the GPU: every step's loss and pose gradient
equal the FP64 oracle's at that step's pose and every update is the
heavy-ball step of Sec. 3.2, graph replays equal the eager run, and the loss
falls from the initial poses."""

import math

import numpy as np
import pytest
import torch

import oracle
from synth import make_phantom, random_poses
from tests._parity import assert_gradient_close, oracle_image

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


def _problem(n=4, seed=0, oracle_targets=False):
    import paper_2208_12737_amd as P
    ph = make_phantom("small", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    det = P.Detector(64, 64, 2.0, 2.0)
    gt = random_poses(n, math.pi / 8, 10.0, 1000.0, seed=seed)
    rng = np.random.default_rng(seed + 100)
    off = np.zeros((n, 7), np.float32)
    off[:, :3] = rng.uniform(-1, 1, (n, 3)) * math.radians(4.0)
    off[:, 3:6] = rng.uniform(-1, 1, (n, 3)) * 3.0
    gt_t = torch.from_numpy(gt).to(DEV)
    if oracle_targets:
        targets = torch.from_numpy(np.stack([oracle_image(grid, g, 64, 64, 2.0, 2.0)
                                             for g in gt])).to(DEV)
    else:
        targets = P.render(vol, gt_t, det)
    init = torch.from_numpy(gt + off).to(DEV)
    if oracle_targets:
        return vol, det, gt, targets, init, grid
    return vol, det, gt, targets, init


def test_trajectory_follows_the_oracle():
    """Eager single chain, 6 steps, 3 problems: at every step the loss is the
    oracle's -ZNCC of the DRR at that step's pose, the pose gradient is the
    oracle's ZNCC gradient chained with its frozen-index Jacobian (per
    component), and the next pose is the heavy-ball update of Sec. 3.2 from
    that gradient (v <- 0.9 v + g, pose <- pose - rate * v, FP32)."""
    from paper_2208_12737_amd.register import BatchedRegistration, default_rates
    vol, det, gt, targets, init, grid = _problem(n=3, seed=2, oracle_targets=True)
    rates = default_rates(3, rot=2e-2, xyz=20.0)
    steps = 6
    reg = BatchedRegistration(vol, det, targets, init, rates, steps=steps, use_graph=False,
                              chains=1, record=True)
    _, hist = reg.run()
    torch.cuda.synchronize()
    P_h = reg.pose_history.cpu().numpy()
    G_h = reg.grad_history.cpu().numpy()
    L_h = hist.cpu().numpy()
    T = targets.cpu().numpy().astype(np.float64)
    r = rates.cpu().numpy()
    assert np.array_equal(P_h[0], init.cpu().numpy())
    vel = np.zeros((3, 7), np.float32)
    for i in range(steps + 1):
        rimg, rjac = oracle.render_jacobian(grid, P_h[i].astype(np.float64), 64, 64, 2.0, 2.0,
                                            nthreads=8)
        for k in range(3):
            z, gz = oracle.zncc_grad(rimg[k], T[k])
            assert abs(L_h[i, k] + z) <= 2e-6, (i, k, L_h[i, k], -z)
            ref = -np.einsum("hw,hwj->j", gz, rjac[k])
            assert_gradient_close(G_h[i, k], ref, gz, rjac[k], f"step {i}, problem {k}")
        if i < steps:
            vel = np.float32(0.9) * vel + G_h[i]
            nxt = P_h[i] - r * vel
            np.testing.assert_allclose(P_h[i + 1], nxt, rtol=1e-6,
                                       atol=1e-6 * np.abs(P_h[i]).max())


def test_graph_replays_equal_eager():
    from paper_2208_12737_amd.register import BatchedRegistration, default_rates
    vol, det, gt, targets, init = _problem()
    rates = default_rates(4, rot=2e-2, xyz=20.0)
    eager = BatchedRegistration(vol, det, targets, init, rates, steps=30, use_graph=False)
    pe, he = eager.run()
    pe, he = pe.clone(), he.clone()
    graph = BatchedRegistration(vol, det, targets, init, rates, steps=30, use_graph=True)
    for rep in range(3):
        # unrelated eager work between the replays
        junk = torch.randn(1000, device=DEV).sum()
        pg, hg = graph.run()
        torch.cuda.synchronize()
        assert torch.equal(pg, pe), rep
        assert torch.equal(hg, he), rep
        del junk


@pytest.mark.parametrize("chains", [2, 3])
def test_chains_give_identical_results(chains):
    """Problems split over independent streams (graph branches) follow
    exactly the trajectories of the single chain, eager and replayed."""
    from paper_2208_12737_amd.register import BatchedRegistration, default_rates
    vol, det, gt, targets, init = _problem(n=5, seed=7)
    rates = default_rates(5, rot=2e-2, xyz=20.0)
    one = BatchedRegistration(vol, det, targets, init, rates, steps=12, use_graph=False,
                              chains=1)
    p1, h1 = one.run()
    p1, h1 = p1.clone(), h1.clone()
    for use_graph in (False, True):
        reg = BatchedRegistration(vol, det, targets, init, rates, steps=12, use_graph=use_graph,
                                  chains=chains)
        for rep in range(2):
            pc, hc = reg.run()
            torch.cuda.synchronize()
            assert torch.equal(pc, p1), (use_graph, rep)
            assert torch.equal(hc, h1), (use_graph, rep)


def test_loss_decreases():
    from paper_2208_12737_amd.register import BatchedRegistration, default_rates
    vol, det, gt, targets, init = _problem(seed=3)
    reg = BatchedRegistration(vol, det, targets, init, default_rates(4, rot=2e-2, xyz=20.0),
                              steps=80)
    poses, hist = reg.run()
    h = hist.cpu().numpy()
    assert np.all(np.isfinite(h))
    assert np.all(h[-1] < h[0])
    assert h[-1].mean() < -0.95


def test_one_at_a_time_path_tracks_batched_path():
    """The plain per-problem autograd route follows the same trajectory over
    a few steps (different kernels, same mathematics)."""
    from paper_2208_12737_amd.register import (BatchedRegistration, default_rates,
                                               register_one_at_a_time)
    vol, det, gt, targets, init = _problem(n=2, seed=5)
    rates = default_rates(2, rot=2e-2, xyz=20.0)
    reg = BatchedRegistration(vol, det, targets, init, rates, steps=5, use_graph=False)
    pb, _ = reg.run()
    po, _ = register_one_at_a_time(vol, det, targets, init, rates, steps=5)
    torch.testing.assert_close(po, pb, rtol=1e-4, atol=1e-4)


def test_registration_in_the_benchmark_configuration():
    """The benchmark's problems (32 on the 512 x 512 x 133 CT, 256 x 256
    detector, starts up to 15 deg / 25 mm off) for 20 steps: the captured
    two-chain graph follows the eager single chain bit for bit, and the mean
    loss falls."""
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.register import BatchedRegistration, default_rates
    ph = make_phantom("ct512", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    det = P.Detector(256, 256, 1.4, 1.4)
    n = 32
    gt = random_poses(n, math.pi / 6, 30.0, 1020.0, seed=11)
    rng = np.random.default_rng(12)
    off = np.zeros((n, 7), np.float32)
    off[:, :3] = rng.uniform(-1, 1, (n, 3)) * math.radians(15.0)
    off[:, 3:6] = rng.uniform(-1, 1, (n, 3)) * 25.0
    targets = P.render(vol, torch.from_numpy(gt).to(DEV), det)
    init = torch.from_numpy(gt + off).to(DEV)
    rates = default_rates(n)
    eager = BatchedRegistration(vol, det, targets, init, rates, steps=20, use_graph=False,
                                chains=1)
    pe, he = eager.run()
    pe, he = pe.clone(), he.clone()
    graph = BatchedRegistration(vol, det, targets, init, rates, steps=20, use_graph=True,
                                chains=2)
    pg, hg = graph.run()
    torch.cuda.synchronize()
    assert torch.equal(pg, pe) and torch.equal(hg, he)
    h = he.cpu().numpy()
    assert np.all(np.isfinite(h))
    assert h[-1].mean() < h[0].mean() - 0.05
