"""The C ABI used from plain C (tests/c/render_from_c.c: no Python, no torch
in the process): volume packing, forward DRRs and the fused -ZNCC gradient
equal the Python front end's results bit for bit."""

import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from synth import random_poses

pytestmark = pytest.mark.gpu
DEV = "cuda"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


def test_c_program_matches_python_front_end(tmp_path):
    import paper_2208_12737_amd as P
    gcc = shutil.which("gcc")
    assert gcc is not None, "gcc is needed to build the C consumer"
    libdir = os.path.join(ROOT, "paper_2208_12737_amd")
    exe = tmp_path / "render_from_c"
    build = subprocess.run(
        [gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
         "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "c", "render_from_c.c"),
         "-L", libdir, "-ldrr", "-L", "/opt/rocm/lib", "-lamdhip64",
         f"-Wl,-rpath,{libdir}", "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)],
        capture_output=True, text=True)
    assert build.returncode == 0, build.stderr

    rng = np.random.default_rng(8)
    v = rng.uniform(0, 2, (17, 9, 23)).astype(np.float32)
    spacing, origin = (0.7, 2.1, 1.3), (2.0, -7.0, -20.0)
    H, W, dx, dy = 37, 53, 1.7, 2.3
    poses = random_poses(5, 0.4, 5.0, 300.0, seed=9)
    vol = P.Volume(torch.from_numpy(v), spacing, origin, device=DEV)
    det = P.Detector(H, W, dx, dy)
    gt = poses[0].copy()
    gt[:3] += 0.02
    target = P.render(vol, torch.from_numpy(gt).to(DEV)[None], det)[0].contiguous()

    (tmp_path / "meta.txt").write_text(
        " ".join(str(x) for x in (*v.shape, *spacing, *origin, H, W, dx, dy, len(poses))))
    v.tofile(tmp_path / "volume.f32")
    poses.astype(np.float32).tofile(tmp_path / "poses.f32")
    target.cpu().numpy().astype(np.float32).tofile(tmp_path / "target.f32")
    print(f"running the C consumer on {len(poses)} poses, {H}x{W}", flush=True)
    run = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True,
                         timeout=120)
    assert run.returncode == 0, (run.returncode, run.stderr)

    img_c = np.fromfile(tmp_path / "image.f32", np.float32).reshape(len(poses), H, W)
    loss_c = np.fromfile(tmp_path / "loss.f32", np.float32)
    grad_c = np.fromfile(tmp_path / "grad.f32", np.float32).reshape(len(poses), 7)
    pt = torch.from_numpy(poses).to(DEV)
    img_py = P.render(vol, pt, det).cpu().numpy()
    loss_py, grad_py = P.render_ncc_grad(vol, pt, det, target)
    np.testing.assert_array_equal(img_c, img_py)
    np.testing.assert_array_equal(loss_c, loss_py.cpu().numpy())
    np.testing.assert_array_equal(grad_c, grad_py.cpu().numpy())
    assert np.all(np.isfinite(grad_c)) and (img_c > 0).any()
