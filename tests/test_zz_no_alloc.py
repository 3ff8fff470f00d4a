"""The allocation-free fused objective (drr_render_ncc_grad_noalloc), called
through the C ABI, equals drr_render_ncc_grad with a caller workspace bit for
bit, on two calls in a row (the second smaller, on the scratch the first
left behind); a batch larger than the fixed scratch is rejected."""

import ctypes
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


def _both(P, lib, vol, det, poses, target, tstride):
    n = poses.shape[0]
    stream = torch.cuda.current_stream().cuda_stream
    out = []
    for noalloc in (True, False):
        img = torch.full((n, det.height, det.width), float("nan"), device=DEV)
        loss = torch.full((n,), float("nan"), device=DEV)
        grad = torch.full((n, 7), float("nan"), device=DEV)
        if noalloc:
            lib.call("drr_render_ncc_grad_noalloc", vol.packed.data_ptr(), ctypes.byref(vol.desc),
                     ctypes.byref(det.desc), poses.data_ptr(), n, target.data_ptr(), tstride,
                     img.data_ptr(), loss.data_ptr(), grad.data_ptr(), stream)
        else:
            need = lib.load().drr_ncc_grad_workspace_bytes(ctypes.byref(det.desc), n)
            ws = torch.empty(need, dtype=torch.uint8, device=DEV)
            lib.call("drr_render_ncc_grad", vol.packed.data_ptr(), ctypes.byref(vol.desc),
                     ctypes.byref(det.desc), poses.data_ptr(), n, target.data_ptr(), tstride,
                     img.data_ptr(), loss.data_ptr(), grad.data_ptr(), ws.data_ptr(), need,
                     stream)
        out.append((img, loss, grad))
    torch.cuda.synchronize()
    return out


def test_noalloc_equals_workspace_call_twice():
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd import _lib
    ph = make_phantom("small", seed=0)
    grid = oracle.Grid(ph.volume, ph.spacing, ph.origin)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    cases = [(P.Detector(40, 44, 3.0, 3.0), 6, 0), (P.Detector(24, 20, 4.0, 4.0), 2, 1)]
    for det, n, seed in cases:
        print(f"noalloc case: detector {det.height}x{det.width}, {n} poses", flush=True)
        gt = random_poses(n, math.pi / 8, 10.0, 1000.0, seed=50 + seed)
        poses = torch.from_numpy(random_poses(n, math.pi / 8, 10.0, 1000.0, seed=60 + seed)).to(DEV)
        if seed == 0:      # one target per pose
            target = torch.from_numpy(np.stack([oracle_image(grid, g, det.height, det.width,
                                                             det.delta_x, det.delta_y)
                                                for g in gt])).to(DEV)
            tstride = det.pixels
        else:              # one shared target
            target = torch.from_numpy(oracle_image(grid, gt[0], det.height, det.width,
                                                   det.delta_x, det.delta_y)).to(DEV)
            tstride = 0
        (ia, la, ga), (ib, lb, gb) = _both(P, _lib, vol, det, poses, target, tstride)
        assert torch.isfinite(la).all() and torch.isfinite(ga).all()
        assert torch.equal(ia, ib) and torch.equal(la, lb) and torch.equal(ga, gb), (det, n)


def test_noalloc_rejects_batches_beyond_the_scratch():
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd import _lib
    ph = make_phantom("small", seed=0)
    vol = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    det = P.Detector(256, 256, 1.0, 1.0)
    per_pose = _lib.load().drr_ncc_grad_workspace_bytes(ctypes.byref(det.desc), 1)
    n = _lib.DRR_NOALLOC_SCRATCH_BYTES // per_pose + 1
    poses = torch.zeros((n, 7), device=DEV)
    target = torch.zeros((256, 256), device=DEV)
    loss = torch.empty((n,), device=DEV)
    grad = torch.empty((n, 7), device=DEV)
    st = _lib.load().drr_render_ncc_grad_noalloc(
        vol.packed.data_ptr(), ctypes.byref(vol.desc), ctypes.byref(det.desc), poses.data_ptr(),
        n, target.data_ptr(), 0, None, loss.data_ptr(), grad.data_ptr(),
        torch.cuda.current_stream().cuda_stream)
    assert st == _lib.DRR_ENOMEM
    assert b"scratch" in _lib.load().drr_last_error()
