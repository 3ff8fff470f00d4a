"""Batched plans: persistent tile-queue launches, graph replay and the
autotuner give the same results as the plain per-call renders."""

import math
import os

import numpy as np
import pytest
import torch

import oracle
from synth import make_phantom, random_poses
from tests._parity import assert_image_close

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


@pytest.fixture(scope="module")
def vols():
    import paper_2208_12737_amd as P
    ph = make_phantom("small", seed=0)
    rng = np.random.default_rng(9)
    odd = rng.uniform(0, 2, (17, 9, 23)).astype(np.float32)
    v0 = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    v1 = P.Volume(torch.from_numpy(odd), (0.7, 2.1, 1.3), (2.0, -7.0, -20.0), device=DEV)
    return [v0, v1], [oracle.Grid(ph.volume, ph.spacing, ph.origin),
                      oracle.Grid(odd, (0.7, 2.1, 1.3), (2.0, -7.0, -20.0))]


def _mixed_items(P, vols, seed):
    from paper_2208_12737_amd.plan import Item
    rng = np.random.default_rng(seed)
    dets = [P.Detector(64, 64, 2.0, 2.0), P.Detector(37, 53, 1.7, 2.3), P.Detector(1, 1, 1.0, 1.0),
            P.Detector(20, 100, 0.9, 0.9)]
    items = []
    for k in range(12):
        vi = int(rng.integers(0, 2))
        det = dets[int(rng.integers(0, len(dets)))]
        sdd = 1000.0 if vi == 0 else 300.0
        pose = random_poses(1, math.pi / 8, 5.0, sdd, seed=1000 * seed + k)[0]
        mode = k % 3
        img = torch.empty((det.height, det.width), device=DEV)
        jac = torch.empty((det.height, det.width, 7), device=DEV) if mode == 1 else None
        cnt = torch.empty((det.height, det.width), dtype=torch.int32, device=DEV) if mode == 2 else None
        items.append(Item(vi, det, torch.from_numpy(pose).to(DEV), img, jac, cnt))
    return items


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("strategy", [0, 1])
def test_plan_matches_plain_render(vols, use_graph, strategy):
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.plan import Plan
    vs, grids = vols
    plan = Plan(vs, max_items=64, use_graph=use_graph, strategy=strategy)
    for rep in range(3):            # replays with new poses and outputs
        items = _mixed_items(P, vs, seed=rep)
        plan.execute(items)
        torch.cuda.synchronize()
        for it in items:
            if it.jac is not None:
                ref_i, ref_j = P.render(vs[it.volume], it.pose[None], it.det, jacobian=True)
                torch.testing.assert_close(it.jac, ref_j[0], rtol=1e-6, atol=1e-6 * ref_j.abs().max().item())
            elif it.counts is not None:
                ref_i, ref_c = P.render_count(vs[it.volume], it.pose[None], it.det)
                assert torch.equal(it.counts, ref_c[0])
            else:
                ref_i = P.render(vs[it.volume], it.pose[None], it.det)
            torch.testing.assert_close(it.image, ref_i[0], rtol=1e-6, atol=1e-6)
        # and against the oracle for a few items
        for it in items[:4]:
            ref, _, _ = oracle.render(grids[it.volume], it.pose.cpu().numpy().astype(np.float64),
                                      it.det.height, it.det.width, it.det.delta_x, it.det.delta_y)
            assert_image_close(it.image.cpu().numpy()[None], ref)
    plan.close()


@pytest.mark.parametrize("strategy", [0, 1])
def test_plan_is_deterministic(vols, strategy):
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.plan import Plan
    vs, _ = vols
    plan = Plan(vs, max_items=64, use_graph=True, strategy=strategy)
    a = _mixed_items(P, vs, seed=5)
    b = _mixed_items(P, vs, seed=5)
    plan.execute(a)
    plan.execute(b)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x.image, y.image)
    plan.close()


def test_autotune_and_cache(vols, tmp_path):
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.plan import Plan
    vs, _ = vols
    cache = str(tmp_path / "tune.txt")
    items = _mixed_items(P, vs, seed=7)
    plan = Plan(vs, max_items=64, use_graph=True, autotune=True, tune_items=items,
                cache_path=cache)
    cfg = plan.config
    assert os.path.exists(cache)
    plan2 = Plan(vs, max_items=64, use_graph=True, autotune=True, tune_items=items,
                 cache_path=cache)
    assert plan2.config == cfg
    out = _mixed_items(P, vs, seed=8)
    plan2.execute(out)
    torch.cuda.synchronize()
    for it in out:
        if it.jac is None and it.counts is None:
            ref = P.render(vs[it.volume], it.pose[None], it.det)
            torch.testing.assert_close(it.image, ref[0], rtol=1e-6, atol=1e-6)
    plan.close()
    plan2.close()


def test_plan_rejects_bad_items(vols):
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd import _lib
    from paper_2208_12737_amd.plan import Item, Plan
    vs, _ = vols
    plan = Plan(vs, max_items=4, use_graph=False)
    det = P.Detector(8, 8, 1.0, 1.0)
    ok = Item(0, det, torch.zeros(7, device=DEV), torch.empty((8, 8), device=DEV))
    with pytest.raises(_lib.DrrError):
        plan.execute([ok] * 5)                       # over capacity
    with pytest.raises(_lib.DrrError):
        plan.execute([Item(5, det, ok.pose, ok.image)])   # bad volume index
    plan.close()
