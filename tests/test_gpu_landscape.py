"""Loss-only fused ZNCC (landscape sweeps) against the image + NCC path and
the oracle."""

import math

import numpy as np
import pytest
import torch

import oracle
from synth import make_phantom, random_poses
from tests._parity import oracle_image

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
    return P, ph, vol


def test_loss_only_matches_image_path_and_oracle(setup):
    P, ph, vol = setup
    det = P.Detector(48, 40, 2.5, 2.5)
    gt = random_poses(1, math.pi / 8, 10.0, 1000.0, seed=2)
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    target = torch.from_numpy(oracle_image(grid, gt[0], 48, 40, 2.5, 2.5)).to(DEV)
    poses = torch.from_numpy(random_poses(9, math.pi / 8, 10.0, 1000.0, seed=3)).to(DEV)
    a = P.render_ncc_loss(vol, poses, det, target)
    b = P.ncc_loss(P.render(vol, poses, det), target)
    torch.testing.assert_close(a, b, rtol=1e-6, atol=1e-6)
    img, _, _ = oracle.render(grid, poses.cpu().numpy().astype(np.float64), 48, 40, 2.5, 2.5)
    T = target.cpu().numpy().astype(np.float64)
    for k in range(9):
        assert a[k].item() == pytest.approx(-oracle.zncc(img[k], T), abs=2e-6)


def test_landscape_minimum_at_ground_truth(setup):
    P, ph, vol = setup
    from paper_2208_12737_amd.landscape import grid_offsets, radial_monotonicity, sweep
    det = P.Detector(48, 48, 2.5, 2.5)
    gt = random_poses(1, math.pi / 8, 5.0, 1000.0, seed=4)[0]
    off = grid_offsets(0, 3, math.radians(20.0), 10.0, 9)          # theta x t_x
    loss = sweep(vol, det, gt, off, chunk=32)
    centre = 4 * 9 + 4
    assert loss[centre] == pytest.approx(-1.0, abs=1e-5)
    assert np.argmin(loss) == centre
    frac, _ = radial_monotonicity(vol, det, gt, n_dirs=16, n_steps=6, radius=0.1)
    assert frac >= 0.75


def test_l2_landscape_minimum_at_ground_truth(setup):
    P, ph, vol = setup
    from paper_2208_12737_amd.landscape import grid_offsets, radial_monotonicity, sweep
    det = P.Detector(40, 40, 3.0, 3.0)
    gt = random_poses(1, math.pi / 8, 5.0, 1000.0, seed=5)[0]
    off = grid_offsets(1, 4, math.radians(20.0), 10.0, 7)          # phi x t_y
    loss = sweep(vol, det, gt, off, chunk=16, loss="l2")
    centre = 3 * 7 + 3
    assert np.argmin(loss) == centre and loss[centre] <= 1e-9 * loss.max()
    # loss-only values equal the fused loss-and-gradient values
    poses = torch.from_numpy(gt[None] + off).to(DEV)
    target = P.render(vol, torch.from_numpy(gt[None]).to(DEV), det)[0]
    full, _ = P.render_l2(vol, poses, det, target)
    np.testing.assert_allclose(loss, full.cpu().numpy(), rtol=1e-6, atol=0)
    frac, _ = radial_monotonicity(vol, det, gt, n_dirs=16, n_steps=6, radius=0.1, loss="l2")
    assert frac >= 0.75


def test_landscape_in_the_benchmark_configuration():
    """The sweep as benchmarked: the 512 x 512 x 133 CT, a 256 x 256 detector
    at 1.4 mm, 8192 offsets of the paper's box in one launch; sampled poses'
    -ZNCC against the oracle's DRR and the same target."""
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.landscape import random_offsets, sweep
    ph = make_phantom("ct512", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    det = P.Detector(256, 256, 1.4, 1.4)
    gt = random_poses(1, math.pi / 6, 30.0, 1020.0, seed=21)[0]
    off = random_offsets(8192, seed=22)
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    target = torch.from_numpy(oracle_image(grid, gt, 256, 256, 1.4, 1.4, nthreads=16)).to(DEV)
    loss = sweep(vol, det, gt, off, chunk=8192, target=target)
    assert np.all(np.isfinite(loss)) and np.all(np.abs(loss) <= 1.0 + 1e-6)
    T = target.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(6)
    for k in rng.choice(8192, 4, replace=False):
        pose = (gt + off[k]).astype(np.float32).astype(np.float64)
        img, _, _ = oracle.render(grid, pose, 256, 256, 1.4, 1.4, nthreads=8)
        assert loss[k] == pytest.approx(-oracle.zncc(img[0], T), abs=2e-6), k
