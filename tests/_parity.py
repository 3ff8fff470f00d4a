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
