"""Shared helpers of the GPU parity tests (no method arithmetic here)."""

import numpy as np

# Image tolerance: FP32 images against the FP64 oracle.
IMAGE_RTOL = 1e-5


def image_errors(gpu, ref, floor=1e-3):
    """(max relative error over pixels with |ref| >= floor * max|ref|,
        max absolute error elsewhere divided by max|ref|)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    m = np.abs(ref).max()
    if m == 0:
        return 0.0, float(np.abs(gpu).max())
    big = np.abs(ref) >= floor * m
    rel = (np.abs(gpu - ref)[big] / np.abs(ref[big])).max() if big.any() else 0.0
    small = (np.abs(gpu - ref)[~big]).max() / m if (~big).any() else 0.0
    return float(rel), float(small)


def assert_image_close(gpu, ref, rtol=IMAGE_RTOL, what="image"):
    rel, small = image_errors(gpu, ref)
    assert rel <= rtol and small <= rtol, f"{what}: max rel {rel:.3e}, small-pixel abs {small:.3e}"


def column_errors(gpu, ref):
    """Per-parameter error of Jacobians [..., k] (k = 7 pose parameters, or 4
    detector parameters) relative to each column's largest magnitude."""
    k = np.shape(ref)[-1]
    gpu = np.asarray(gpu, dtype=np.float64).reshape(-1, k)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, k)
    scale = np.abs(ref).max(axis=0) + 1e-300
    return np.abs(gpu - ref).max(axis=0) / scale


# Pose gradients dL/d pose = sum_i (dL/dI_i) J_ij against the oracle's chain
# of its FP64 image gradient and frozen-index Jacobian: every component
# within GRAD_RTOL of its own value, plus a floor for components near zero.
# The floor is GRAD_FLOOR * sum_i |dL/dI_i| * max_i |J_ij|: the GPU's
# per-pixel Jacobian is formed from FP32 sums over the ray's crossings and
# stored in FP32, an error of a few ulps (2^-24 ~ 6e-8) of the column scale
# per pixel, so 16 ulps of that scale in every pixel, all of one sign, bound
# what it can add to the contraction.
GRAD_RTOL = 1e-3
GRAD_FLOOR = 1e-6


def gradient_errors(got, ref, gimg, jac):
    """Per-component |got - ref| divided by the allowed error
    GRAD_RTOL |ref_j| + GRAD_FLOOR sum|gimg| max|J_j| (<= 1 passes), for one
    pose: got, ref [7]; gimg [H, W] (or [n_pixels]); jac [H, W, 7]."""
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    k = ref.shape[0]
    floor = GRAD_FLOOR * np.abs(np.asarray(gimg, dtype=np.float64)).sum() * \
        np.abs(np.asarray(jac, dtype=np.float64).reshape(-1, k)).max(axis=0)
    return np.abs(got - ref) / (GRAD_RTOL * np.abs(ref) + floor + 1e-300)


def assert_gradient_close(got, ref, gimg, jac, what="gradient"):
    r = gradient_errors(got, ref, gimg, jac)
    assert np.all(r <= 1.0), (f"{what}: error / allowed per component {np.array2string(r, precision=3)}; "
                              f"got {np.asarray(got).reshape(-1)}, oracle {np.asarray(ref).reshape(-1)}")
    return r


def oracle_image(grid, pose, H, W, delta_x, delta_y, offset=(0.0, 0.0), nthreads=8):
    """A DRR from the FP64 oracle, rounded to FP32 [H, W]: targets that both
    the GPU path and the oracle take as input are made this way, so no oracle
    input comes from the GPU path."""
    import oracle
    p = np.asarray(pose, dtype=np.float32).astype(np.float64).reshape(1, 7)
    img, _, _ = oracle.render(grid, p, H, W, delta_x, delta_y, offset=offset, nthreads=nthreads)
    return np.ascontiguousarray(img[0], dtype=np.float32)
