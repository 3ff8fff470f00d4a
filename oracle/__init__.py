"""FP64 CPU oracle for Siddon DRRs, their pose derivatives and the NCC loss.

TEST INFRASTRUCTURE ONLY: the GPU path is checked against these functions.
Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package; the product path never does.

The arithmetic lives in ``drr_oracle.c`` (plain C, FP64, a full sort of each
ray's plane crossings, following Eq. 2-4 and Sec. 2.3-2.4 of the paper); this
module only marshals numpy arrays.  ``brute`` holds independent algorithms
(per-voxel chord sums, fine-step integration, a face-clipping chord) that pin
the oracle without sharing its formulas.

Parity status per function:
  render / trace_rays        pinned (closed forms, brute force, invariants)
  trace_rays_grad            pinned (central differences of trace_rays)
  ray_endpoint_derivs        pinned (central differences of ray_endpoints)
  render_jacobian            pinned (central differences of render)
  render_detector_jacobian   pinned (central differences of render in the pitch and
                             the principal-point offsets; offset = whole pixels shifts
                             the image)
  zncc / zncc_grad           pinned (closed forms, invariances, differences)
  l2 / l2_grad               pinned (closed forms, invariances, differences)
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DRR_ORACLE_LIB may point the tests at another build of drr_oracle.c (used to
# check that planted mistakes in the oracle make its pins fail).
_LIB_PATH = os.environ.get("DRR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_up = ctypes.POINTER(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_rotation.argtypes = [ctypes.c_double] * 3 + [ctypes.c_int, _dp]
    lib.orc_ray_endpoints.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.orc_ray_endpoint_derivs.argtypes = lib.orc_ray_endpoints.argtypes
    lib.orc_trace_rays.argtypes = [_dp, _ip, _dp, _dp, _dp, _dp, ctypes.c_int64, _dp, _lp,
                                   _up, ctypes.c_int]
    lib.orc_render.argtypes = [_dp, _ip, _dp, _dp, _dp, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double,
                               ctypes.c_int32, ctypes.c_int32, _dp, _lp, _up, ctypes.c_int]
    lib.orc_trace_rays_grad.argtypes = [_dp, _ip, _dp, _dp, _dp, _dp, ctypes.c_int64, _dp,
                                        _dp, _dp, ctypes.c_int]
    lib.orc_render_jacobian.argtypes = [_dp, _ip, _dp, _dp, _dp, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        _dp, _dp, ctypes.c_int]
    lib.orc_render_detector_jacobian.argtypes = lib.orc_render_jacobian.argtypes
    lib.orc_zncc.argtypes = [_dp, _dp, ctypes.c_int64, _dp]
    lib.orc_zncc.restype = ctypes.c_double
    lib.orc_l2.argtypes = [_dp, _dp, ctypes.c_int64, _dp]
    lib.orc_l2.restype = ctypes.c_double
    lib.orc_openmp_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


class Grid:
    """A CT grid for the oracle: FP64 copy of the volume plus its geometry."""

    def __init__(self, volume, spacing, origin=None):
        self.vol = _d(volume)
        self.dims = np.ascontiguousarray(self.vol.shape, dtype=np.int32)
        self.spacing = _d(spacing)
        if origin is None:
            origin = -0.5 * self.dims * self.spacing
        self.origin = _d(origin)

    def args(self):
        return (_ptr(self.vol), _ptr(self.dims, _ip), _ptr(self.spacing), _ptr(self.origin))


def max_threads() -> int:
    return int(_load().orc_openmp_max_threads())


def rotation(theta, phi, gamma, which=-1):
    """R = Rz(theta) Ry(phi) Rx(gamma), or its derivative (which = 0, 1, 2)."""
    out = np.zeros(9)
    _load().orc_rotation(theta, phi, gamma, which, _ptr(out))
    return out.reshape(3, 3)


def ray_endpoints(pose, H, W, delta_x, delta_y, h, w, offset=(0.0, 0.0)):
    s, p = np.zeros(3), np.zeros(3)
    _load().orc_ray_endpoints(_ptr(_d(pose)), H, W, delta_x, delta_y, offset[0], offset[1], h, w,
                              _ptr(s), _ptr(p))
    return s, p


def ray_endpoint_derivs(pose, H, W, delta_x, delta_y, h, w, offset=(0.0, 0.0)):
    ds, dp = np.zeros(21), np.zeros(21)
    _load().orc_ray_endpoint_derivs(_ptr(_d(pose)), H, W, delta_x, delta_y, offset[0],
                                    offset[1], h, w, _ptr(ds), _ptr(dp))
    return ds.reshape(3, 7), dp.reshape(3, 7)


def trace_rays(grid: Grid, src, dst, nthreads=1):
    """E, positive-segment count and voxel-sequence hash for arbitrary rays."""
    src, dst = _d(src).reshape(-1, 3), _d(dst).reshape(-1, 3)
    n = src.shape[0]
    E = np.zeros(n)
    cnt = np.zeros(n, dtype=np.int64)
    hsh = np.zeros(n, dtype=np.uint64)
    _load().orc_trace_rays(*grid.args(), _ptr(src), _ptr(dst), n, _ptr(E), _ptr(cnt, _lp),
                           _ptr(hsh, _up), nthreads)
    return E, cnt, hsh


def trace_rays_grad(grid: Grid, src, dst, nthreads=1):
    """E and its frozen-index derivatives with respect to s and p."""
    src, dst = _d(src).reshape(-1, 3), _d(dst).reshape(-1, 3)
    n = src.shape[0]
    E, gs, gp = np.zeros(n), np.zeros((n, 3)), np.zeros((n, 3))
    _load().orc_trace_rays_grad(*grid.args(), _ptr(src), _ptr(dst), n, _ptr(E), _ptr(gs),
                                _ptr(gp), nthreads)
    return E, gs, gp


def render(grid: Grid, poses, H, W, delta_x, delta_y, rows=None, nthreads=1,
           offset=(0.0, 0.0)):
    """DRR images [B, H, W] (float64) with segment counts and sequence hashes.

    ``rows = (r0, r1)`` evaluates only detector rows r0..r1-1 (others stay 0);
    ``offset`` is the detector's principal point (offset_u, offset_v) in mm.
    """
    poses = _d(poses).reshape(-1, 7)
    B = poses.shape[0]
    r0, r1 = (0, H) if rows is None else rows
    img = np.zeros((B, H, W))
    cnt = np.zeros((B, H, W), dtype=np.int64)
    hsh = np.zeros((B, H, W), dtype=np.uint64)
    _load().orc_render(*grid.args(), _ptr(poses), B, H, W, delta_x, delta_y, offset[0],
                       offset[1], r0, r1, _ptr(img), _ptr(cnt, _lp), _ptr(hsh, _up), nthreads)
    return img, cnt, hsh


def render_jacobian(grid: Grid, poses, H, W, delta_x, delta_y, nthreads=1,
                    offset=(0.0, 0.0)):
    """Images [B, H, W] and frozen-index Jacobians [B, H, W, 7] (float64)."""
    poses = _d(poses).reshape(-1, 7)
    B = poses.shape[0]
    img = np.zeros((B, H, W))
    jac = np.zeros((B, H, W, 7))
    _load().orc_render_jacobian(*grid.args(), _ptr(poses), B, H, W, delta_x, delta_y,
                                offset[0], offset[1], _ptr(img), _ptr(jac), nthreads)
    return img, jac


def render_detector_jacobian(grid: Grid, poses, H, W, delta_x, delta_y, nthreads=1,
                             offset=(0.0, 0.0)):
    """Images [B, H, W] and d image / d (delta_x, delta_y, offset_u, offset_v)
    [B, H, W, 4]."""
    poses = _d(poses).reshape(-1, 7)
    B = poses.shape[0]
    img = np.zeros((B, H, W))
    jac = np.zeros((B, H, W, 4))
    _load().orc_render_detector_jacobian(*grid.args(), _ptr(poses), B, H, W, delta_x,
                                         delta_y, offset[0], offset[1], _ptr(img), _ptr(jac),
                                         nthreads)
    return img, jac


def render_fd(grid: Grid, pose, H, W, delta_x, delta_y, steps, nthreads=1, offset=(0.0, 0.0)):
    """Central differences of the image with respect to each pose parameter.

    Returns (fd [H, W, 7], kink_free [H, W, 7]): a pixel is kink-free for
    parameter j when its voxel sequence is the same at pose - h_j, pose and
    pose + h_j, i.e. the difference quotient does not straddle a voxel-index
    change.
    """
    pose = _d(pose).reshape(7)
    steps = np.broadcast_to(np.asarray(steps, dtype=np.float64), (7,))
    _, _, h0 = render(grid, pose, H, W, delta_x, delta_y, nthreads=nthreads, offset=offset)
    fd = np.zeros((H, W, 7))
    ok = np.zeros((H, W, 7), dtype=bool)
    for j in range(7):
        if steps[j] == 0.0:
            continue
        pp, pm = pose.copy(), pose.copy()
        pp[j] += steps[j]
        pm[j] -= steps[j]
        ip, _, hp = render(grid, pp, H, W, delta_x, delta_y, nthreads=nthreads, offset=offset)
        im, _, hm = render(grid, pm, H, W, delta_x, delta_y, nthreads=nthreads, offset=offset)
        fd[:, :, j] = (ip[0] - im[0]) / (pp[j] - pm[j])
        ok[:, :, j] = (hp[0] == h0[0]) & (hm[0] == h0[0])
    return fd, ok


def zncc(I, T):
    I, T = _d(I).ravel(), _d(T).ravel()
    return float(_load().orc_zncc(_ptr(I), _ptr(T), I.size, None))


def zncc_grad(I, T):
    """ZNCC(I, T) and dZNCC/dI (same shape as I)."""
    shape = np.shape(I)
    I, T = _d(I).ravel(), _d(T).ravel()
    g = np.zeros_like(I)
    z = float(_load().orc_zncc(_ptr(I), _ptr(T), I.size, _ptr(g)))
    return z, g.reshape(shape)


def l2(I, T):
    """Mean squared difference (1/N) sum (I - T)^2."""
    I, T = _d(I).ravel(), _d(T).ravel()
    return float(_load().orc_l2(_ptr(I), _ptr(T), I.size, None))


def l2_grad(I, T):
    """L2(I, T) and dL2/dI (same shape as I)."""
    shape = np.shape(I)
    I, T = _d(I).ravel(), _d(T).ravel()
    g = np.zeros_like(I)
    v = float(_load().orc_l2(_ptr(I), _ptr(T), I.size, _ptr(g)))
    return v, g.reshape(shape)
