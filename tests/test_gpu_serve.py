"""Serving on the GPU: each result equals the same request served alone and
the plain single-DRR path, whatever mix it was batched with."""

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
def volumes():
    import paper_2208_12737_amd as P
    a = make_phantom("small", seed=0)
    b = make_phantom("small", seed=1)
    rng = np.random.default_rng(4)
    c = rng.uniform(0, 1, (40, 30, 20)).astype(np.float32)
    return {"a": P.Volume(torch.from_numpy(a.volume), a.spacing, a.origin, device=DEV),
            "b": P.Volume(torch.from_numpy(b.volume), b.spacing, b.origin, device=DEV,
                          layout="input"),
            "c": P.Volume(torch.from_numpy(c), (1.5, 2.0, 2.5), None, device=DEV)}


def _requests(volumes, n, seed):
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.serve import FWD, FWDBWD, Request
    rng = np.random.default_rng(seed)
    sizes = [(32, 32, 2.0), (48, 40, 1.5), (64, 64, 1.0), (17, 23, 3.0)]
    reqs = []
    for i in range(n):
        v = ["a", "b", "c"][int(rng.integers(0, 3))]
        H, W, px = sizes[int(rng.integers(0, len(sizes)))]
        pose = random_poses(1, math.pi / 8, 5.0, 400.0, seed=seed * 1000 + i)[0]
        kind = FWD if rng.uniform() < 0.7 else FWDBWD
        target = None
        if kind == FWDBWD:
            gt = pose.copy()
            gt[:3] += 0.02
            target = P.render(volumes[v], torch.from_numpy(gt).to(DEV)[None],
                              P.Detector(H, W, px, px))[0]
        reqs.append(Request(v, H, W, px, px, pose, kind, target))
    return reqs


def _same(a, b):
    if isinstance(a, tuple):
        return all(torch.equal(x, y) for x, y in zip(a, b))
    return torch.equal(a, b)


def test_alone_vs_mix_and_plain(volumes):
    from paper_2208_12737_amd.serve import FWD, GpuBackend, Server, plain_forward
    reqs = _requests(volumes, 40, seed=1)
    be = GpuBackend(volumes, n_streams=3)
    # a small budget forces many ticks with overlapping batches
    srv = Server(be, hbm_budget_bytes=6 * 64 * 64 * 4 * 3, n_streams=3, max_batch=8)
    tickets = []
    for i, r in enumerate(reqs):
        tickets.append(srv.submit(r))
        if i % 5 == 4:
            srv.tick()                       # arrivals interleaved with scheduling
    srv.run_until_idle()
    torch.cuda.synchronize()
    assert srv.batches >= 5
    for r, t in zip(reqs, tickets):
        mixed = t.wait(0)
        solo_srv = Server(GpuBackend(volumes, n_streams=1), hbm_budget_bytes=1 << 30)
        st = solo_srv.submit(r)
        solo_srv.run_until_idle()
        torch.cuda.synchronize()
        assert _same(mixed, st.wait(0))
        if r.kind == FWD:
            assert torch.equal(mixed, plain_forward(volumes, r))
        else:
            img, loss, grad = mixed
            assert torch.isfinite(grad).all() and loss.item() < 0


def test_bad_requests_fail_at_submission(volumes):
    from paper_2208_12737_amd.serve import FWD, FWDBWD, GpuBackend, Request, Server
    srv = Server(GpuBackend(volumes, n_streams=1), hbm_budget_bytes=1 << 30)
    pose = np.zeros(7, np.float32)
    pose[6] = 400.0
    with pytest.raises(KeyError):
        srv.submit(Request("missing", 8, 8, 1.0, 1.0, pose, FWD))
    with pytest.raises(ValueError):       # target of the wrong size
        srv.submit(Request("a", 8, 8, 1.0, 1.0, pose, FWDBWD, torch.zeros(9, device=DEV)))
    with pytest.raises(ValueError):       # target on the host
        srv.submit(Request("a", 8, 8, 1.0, 1.0, pose, FWDBWD, torch.zeros(64)))
    with pytest.raises(ValueError):       # invalid detector
        srv.submit(Request("a", 0, 8, 1.0, 1.0, pose, FWD))
    assert srv.pending() == 0


def test_serving_mix_in_the_benchmark_configuration():
    """The benchmark's four resident volumes (128^3 at 2 mm, 256^3 at 1 mm,
    512 x 512 x 133 and 512 x 512 x 300) and four detector sizes (pitch
    358.4 mm / N): every volume and detector pair as a forward request, half
    of them also as forward + backward requests, served under a small budget;
    forward results equal the plain single-DRR path and fwd+bwd results equal
    the fused call, bit for bit."""
    import paper_2208_12737_amd as P
    from paper_2208_12737_amd.serve import FWD, FWDBWD, GpuBackend, Request, Server, plain_forward
    names = ["ct128", "ct256", "ct512", "ct512x300"]
    vols = {}
    for nm in names:
        ph = make_phantom(nm, seed=0)
        vols[nm] = P.Volume(torch.from_numpy(ph.volume), ph.spacing, ph.origin, device=DEV)
    reqs = []
    for i, nm in enumerate(names):
        for j, N in enumerate((128, 200, 256, 512)):
            px = 358.4 / N
            pose = random_poses(1, math.pi / 6, 30.0, 1020.0, seed=100 + 4 * i + j)[0]
            reqs.append(Request(nm, N, N, px, px, pose, FWD))
            if (i + j) % 2 == 0:
                gt = pose.copy()
                gt[:3] += 0.03
                tg = P.render(vols[nm], torch.from_numpy(gt).to(DEV)[None],
                              P.Detector(N, N, px, px))[0]
                reqs.append(Request(nm, N, N, px, px, pose, FWDBWD, tg))
    srv = Server(GpuBackend(vols, n_streams=3), hbm_budget_bytes=8 << 20, n_streams=3,
                 max_batch=6)
    tickets = [srv.submit(r) for r in reqs]
    srv.run_until_idle()
    torch.cuda.synchronize()
    assert srv.batches >= 4
    for r, t in zip(reqs, tickets):
        got = t.wait(0)
        det = P.Detector(r.height, r.width, r.delta_x, r.delta_y)
        if r.kind == FWD:
            assert torch.equal(got, plain_forward(vols, r))
        else:
            img, loss, grad = got
            pose = torch.from_numpy(np.asarray(r.pose, np.float32)).to(DEV)[None]
            l_ref, g_ref, i_ref = P.render_ncc_grad(vols[r.volume], pose, det, r.target,
                                                    return_image=True)
            assert torch.equal(img, i_ref[0])
            assert torch.equal(loss.reshape(1), l_ref) and torch.equal(grad, g_ref[0])
