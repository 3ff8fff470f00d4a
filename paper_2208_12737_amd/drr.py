"""PyTorch front end of libdrr: resident volumes, renders, autograd, NCC.

PyTorch provides device memory and the current HIP stream; every step of
the computation runs in the HIP kernels behind the C ABI (include/drr.h).
Nothing here computes pixels, gradients or losses.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    return t.contiguous()


def _poses(poses: torch.Tensor) -> torch.Tensor:
    p = _dev_f32(poses, "poses")
    if p.ndim == 1:
        p = p.reshape(1, -1)
    if p.ndim != 2 or p.shape[1] != 7:
        raise ValueError(f"poses must be [n, 7], got {tuple(poses.shape)}")
    return p


def target_stride(numel: int, n: int, hw: int) -> int:
    """Element stride between the per-pose targets of a batch of n images of
    hw pixels: 0 when one image is shared by every pose, hw when there is
    one per pose.  Any other size would make the kernels read past the
    tensor, so it is rejected."""
    if numel == hw:
        return 0
    if numel == n * hw:
        return hw
    raise ValueError(f"target must hold one image ({hw} elements) or one per pose "
                     f"({n} x {hw}); got {numel} elements")


def _expect_numel(t: torch.Tensor, name: str, numel: int) -> None:
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()} "
                         f"(shape {tuple(t.shape)})")


def _same_device(device, *named) -> None:
    for name, t in named:
        if t is not None and t.device != device:
            raise ValueError(f"{name} is on {t.device}, expected {device}")


def _check_volume(volume: "Volume", p: torch.Tensor) -> None:
    _same_device(p.device, ("volume", volume.packed))


@dataclass(frozen=True)
class Detector:
    """Detector of height x width pixels; delta_x / delta_y are the column /
    row pitches in mm, offset_u / offset_v the principal-point offset in mm
    (pixel (h, w) sits at ((w + 1/2 - W/2) delta_x + offset_u,
    (h + 1/2 - H/2) delta_y + offset_v) on the detector plane)."""
    height: int
    width: int
    delta_x: float
    delta_y: float
    offset_u: float = 0.0
    offset_v: float = 0.0

    @property
    def desc(self) -> _lib.DetectorDesc:
        return _lib.detector_desc(self.height, self.width, self.delta_x, self.delta_y,
                                  self.offset_u, self.offset_v)

    @property
    def pixels(self) -> int:
        return self.height * self.width


LAYOUTS = {"input": _lib.DRR_LAYOUT_INPUT, "per_axis": _lib.DRR_LAYOUT_PER_AXIS}


class Volume:
    """A CT volume packed into the renderer's layout and kept in HBM.

    data: float32 tensor of shape (nx, ny, nz) (C-order, any device);
    spacing: voxel size in mm; origin: position of plane 0 per axis (default
    centres the grid on the world origin); layout: "per_axis" (three copies,
    one per principal ray axis, fastest) or "input" (one copy).  Renders are
    bitwise identical for both layouts.
    """

    def __init__(self, data: torch.Tensor, spacing, origin=None, device=None,
                 layout: str = "per_axis"):
        if data.ndim != 3:
            raise ValueError("volume data must be 3-D (nx, ny, nz)")
        device = torch.device(device) if device is not None else (
            data.device if data.is_cuda else torch.device("cuda"))
        src = data.to(device=device, dtype=torch.float32).contiguous()
        self.shape = tuple(int(v) for v in src.shape)
        self.spacing = tuple(float(v) for v in spacing)
        if origin is None:
            origin = tuple(-0.5 * n * s for n, s in zip(self.shape, self.spacing))
        self.origin = tuple(float(v) for v in origin)
        if layout not in LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
        self.layout = layout
        self.desc = _lib.volume_desc(self.shape, self.spacing, self.origin, LAYOUTS[layout])
        nbytes = _lib.load().drr_volume_packed_bytes(ctypes.byref(self.desc))
        if nbytes == 0:
            _lib.check("drr_volume_packed_bytes", _lib.DRR_EINVAL)
        self.packed = torch.empty(nbytes // 4, dtype=torch.float32, device=device)
        _lib.call("drr_volume_pack", src.data_ptr(), self.packed.data_ptr(),
                  ctypes.byref(self.desc), _stream())
        self.device = device

    @property
    def nbytes(self) -> int:
        return self.packed.numel() * 4


def choose_layout(data: torch.Tensor, spacing, det: "Detector", poses: torch.Tensor, origin=None,
                  device=None, max_bytes: int | None = None, reps: int = 5):
    """Pack `data` in each layout whose packed size fits `max_bytes`, time the
    forward render of `poses` on `det` from each (median of `reps` launches
    after two warm-ups, HIP events on the current stream), and return the
    Volume in the fastest layout and the times {layout: ms}.  The layouts give
    bitwise the same images; they differ in speed (each copy has the
    principal axis of the rays that read it slowest in memory) and in size
    (three copies or one)."""
    p = _poses(poses)
    times = {}
    best = None
    for name in ("per_axis", "input"):
        if max_bytes is not None:
            shape = tuple(int(v) for v in data.shape)
            org = origin if origin is not None else tuple(-0.5 * n * float(s)
                                                          for n, s in zip(shape, spacing))
            desc = _lib.volume_desc(shape, spacing, org, LAYOUTS[name])
            if _lib.load().drr_volume_packed_bytes(ctypes.byref(desc)) > max_bytes:
                continue
        vol = Volume(data, spacing, origin, device=device, layout=name)
        for _ in range(2):
            render(vol, p, det)
        out = []
        for _ in range(max(1, int(reps))):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            render(vol, p, det)
            b.record()
            b.synchronize()
            out.append(a.elapsed_time(b))
        out.sort()
        times[name] = out[len(out) // 2]
        if best is None or times[name] < times[best.layout]:
            best = vol
        del vol
    if best is None:
        raise ValueError(f"no volume layout fits in {max_bytes} bytes")
    return best, times


def render(volume: Volume, poses: torch.Tensor, det: Detector, jacobian: bool = False):
    """DRRs [n, H, W] (and, if asked, Jacobians [n, H, W, 7])."""
    p = _poses(poses)
    _check_volume(volume, p)
    n = p.shape[0]
    img = torch.empty((n, det.height, det.width), dtype=torch.float32, device=p.device)
    jac = torch.empty((n, det.height, det.width, 7), dtype=torch.float32,
                      device=p.device) if jacobian else None
    _lib.call("drr_render", volume.packed.data_ptr(), ctypes.byref(volume.desc),
              ctypes.byref(det.desc), p.data_ptr(), n, img.data_ptr(),
              jac.data_ptr() if jac is not None else None, _stream())
    return (img, jac) if jacobian else img


def render_detector_jacobian(volume: Volume, poses: torch.Tensor, det: Detector):
    """DRRs [n, H, W] and d image / d (delta_x, delta_y, offset_u, offset_v)
    [n, H, W, 4]."""
    p = _poses(poses)
    _check_volume(volume, p)
    n = p.shape[0]
    img = torch.empty((n, det.height, det.width), dtype=torch.float32, device=p.device)
    jac = torch.empty((n, det.height, det.width, 4), dtype=torch.float32, device=p.device)
    _lib.call("drr_render_detector_jacobian", volume.packed.data_ptr(), ctypes.byref(volume.desc),
              ctypes.byref(det.desc), p.data_ptr(), n, img.data_ptr(), jac.data_ptr(),
              _stream())
    return img, jac


def render_count(volume: Volume, poses: torch.Tensor, det: Detector):
    """DRRs and per-pixel counts of voxel gathers (positive-length segments)."""
    p = _poses(poses)
    _check_volume(volume, p)
    n = p.shape[0]
    img = torch.empty((n, det.height, det.width), dtype=torch.float32, device=p.device)
    cnt = torch.empty((n, det.height, det.width), dtype=torch.int32, device=p.device)
    _lib.call("drr_render_count", volume.packed.data_ptr(), ctypes.byref(volume.desc),
              ctypes.byref(det.desc), p.data_ptr(), n, img.data_ptr(), cnt.data_ptr(),
              _stream())
    return img, cnt


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 8), dtype=torch.uint8, device=device)


def _reuse_workspace(ws: torch.Tensor | None, need: int, device):
    """(pointer owner, size in bytes) of the caller's workspace when it is a
    contiguous tensor on `device` of at least `need` bytes, else of a fresh
    one."""
    if (ws is not None and ws.is_cuda and ws.device == device and ws.is_contiguous()
            and ws.numel() * ws.element_size() >= need):
        return ws, ws.numel() * ws.element_size()
    fresh = _workspace(need, device)
    return fresh, fresh.numel()


def render_backward(det: Detector, jac: torch.Tensor, grad_image: torch.Tensor) -> torch.Tensor:
    """grad_pose[n, 7] = sum over pixels of grad_image * jac."""
    jac = _dev_f32(jac, "jac")
    g = _dev_f32(grad_image, "grad_image")
    if jac.ndim != 4 or tuple(jac.shape[1:]) != (det.height, det.width, 7):
        raise ValueError(f"jac must be [n, {det.height}, {det.width}, 7], got {tuple(jac.shape)}")
    n = jac.shape[0]
    _expect_numel(g, "grad_image", n * det.pixels)
    _same_device(jac.device, ("grad_image", g))
    out = torch.empty((n, 7), dtype=torch.float32, device=jac.device)
    ws_n = _lib.load().drr_backward_workspace_bytes(ctypes.byref(det.desc), n)
    ws = _workspace(ws_n, jac.device)
    _lib.call("drr_render_backward", ctypes.byref(det.desc), n, jac.data_ptr(), g.data_ptr(),
              out.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    return out


def render_backward_retrace(volume: Volume, poses: torch.Tensor, det: Detector,
                            grad_image: torch.Tensor) -> torch.Tensor:
    """Same gradient as render_backward, tracing the rays again instead of
    reading a stored Jacobian."""
    p = _poses(poses)
    _check_volume(volume, p)
    g = _dev_f32(grad_image, "grad_image")
    n = p.shape[0]
    _expect_numel(g, "grad_image", n * det.pixels)
    _same_device(p.device, ("grad_image", g))
    out = torch.empty((n, 7), dtype=torch.float32, device=p.device)
    ws_n = _lib.load().drr_backward_workspace_bytes(ctypes.byref(det.desc), n)
    ws = _workspace(ws_n, p.device)
    _lib.call("drr_render_backward_retrace", volume.packed.data_ptr(), ctypes.byref(volume.desc),
              ctypes.byref(det.desc), p.data_ptr(), n, g.data_ptr(), out.data_ptr(),
              ws.data_ptr(), ws.numel(), _stream())
    return out


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, poses, volume, det, retrace):
        ctx.det, ctx.volume, ctx.retrace = det, volume, retrace
        if ctx.needs_input_grad[0] and not retrace:
            img, jac = render(volume, poses, det, jacobian=True)
            ctx.save_for_backward(jac)
        else:
            img = render(volume, poses, det)
            ctx.save_for_backward(poses.detach())
        return img

    @staticmethod
    def backward(ctx, grad_image):
        (saved,) = ctx.saved_tensors
        if ctx.retrace:
            grad = render_backward_retrace(ctx.volume, saved, ctx.det, grad_image)
        else:
            grad = render_backward(ctx.det, saved, grad_image)
        return grad, None, None, None


def drr(volume: Volume, poses: torch.Tensor, det: Detector, retrace: bool = False) -> torch.Tensor:
    """Differentiable DRR: images [n, H, W]; gradients flow to poses [n, 7].

    retrace=False stores the per-pixel Jacobian in the forward pass;
    retrace=True stores nothing and traces the rays again in backward."""
    return _RenderFn.apply(poses, volume, det, retrace)


class _NCCFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image, target):
        img = _dev_f32(image, "image")
        tgt = _dev_f32(target, "target")
        if img.ndim < 2:
            raise ValueError(f"image must be [n, ...], got {tuple(img.shape)}")
        n = img.shape[0]
        hw = img[0].numel()
        tstride = target_stride(tgt.numel(), n, hw)
        _same_device(img.device, ("target", tgt))
        stats = torch.empty((n, 5), dtype=torch.float64, device=img.device)
        loss = torch.empty((n,), dtype=torch.float32, device=img.device)
        ws = _workspace(_lib.load().drr_ncc_workspace_bytes(n, hw), img.device)
        _lib.call("drr_ncc_forward", img.data_ptr(), tgt.data_ptr(), tstride, n, hw,
                  stats.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
        ctx.save_for_backward(img, tgt, stats)
        ctx.tstride, ctx.hw = tstride, hw
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        img, tgt, stats = ctx.saved_tensors
        gl = _dev_f32(grad_loss, "grad_loss")
        n = img.shape[0]
        _expect_numel(gl, "grad_loss", n)
        out = torch.empty_like(img)
        _lib.call("drr_ncc_backward", img.data_ptr(), tgt.data_ptr(), ctx.tstride,
                  stats.data_ptr(), gl.data_ptr(), n, ctx.hw, out.data_ptr(), _stream())
        return out, None


def ncc_loss(image: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Negative zero-normalised cross-correlation per image: [n]."""
    return _NCCFn.apply(image, target)


def render_ncc_grad(volume: Volume, poses: torch.Tensor, det: Detector, target: torch.Tensor,
                    return_image: bool = False, workspace: torch.Tensor | None = None):
    """Fused registration objective: (loss [n], grad_pose [n, 7][, image])."""
    p = _poses(poses)
    _check_volume(volume, p)
    tgt = _dev_f32(target, "target")
    n = p.shape[0]
    hw = det.pixels
    tstride = target_stride(tgt.numel(), n, hw)
    _same_device(p.device, ("target", tgt))
    loss = torch.empty((n,), dtype=torch.float32, device=p.device)
    grad = torch.empty((n, 7), dtype=torch.float32, device=p.device)
    img = torch.empty((n, det.height, det.width), dtype=torch.float32,
                      device=p.device) if return_image else None
    need = _lib.load().drr_ncc_grad_workspace_bytes(ctypes.byref(det.desc), n)
    ws, ws_bytes = _reuse_workspace(workspace, need, p.device)
    _lib.call("drr_render_ncc_grad", volume.packed.data_ptr(), ctypes.byref(volume.desc),
              ctypes.byref(det.desc), p.data_ptr(), n, tgt.data_ptr(), tstride,
              img.data_ptr() if img is not None else None, loss.data_ptr(), grad.data_ptr(),
              ws.data_ptr(), ws_bytes, _stream())
    return (loss, grad, img) if return_image else (loss, grad)


def render_ncc_loss(volume: Volume, poses: torch.Tensor, det: Detector, target: torch.Tensor,
                    workspace: torch.Tensor | None = None) -> torch.Tensor:
    """-ZNCC of each pose's DRR against `target` (one shared image or one per
    pose), without storing images or gradients: [n]."""
    p = _poses(poses)
    _check_volume(volume, p)
    tgt = _dev_f32(target, "target")
    n = p.shape[0]
    hw = det.pixels
    tstride = target_stride(tgt.numel(), n, hw)
    _same_device(p.device, ("target", tgt))
    loss = torch.empty((n,), dtype=torch.float32, device=p.device)
    need = _lib.load().drr_ncc_loss_workspace_bytes(ctypes.byref(det.desc), n)
    ws, ws_bytes = _reuse_workspace(workspace, need, p.device)
    _lib.call("drr_render_ncc_loss", volume.packed.data_ptr(), ctypes.byref(volume.desc),
              ctypes.byref(det.desc), p.data_ptr(), n, tgt.data_ptr(), tstride, None,
              loss.data_ptr(), ws.data_ptr(), ws_bytes, _stream())
    return loss


def render_l2(volume: Volume, poses: torch.Tensor, det: Detector, target: torch.Tensor,
              grad: bool = True, return_image: bool = False,
              workspace: torch.Tensor | None = None):
    """Fused mean-squared-difference objective: loss [n] = mean (I - T)^2 per
    pose, and with ``grad`` its pose gradient [n, 7]; returns
    (loss, grad_pose or None[, image])."""
    p = _poses(poses)
    _check_volume(volume, p)
    tgt = _dev_f32(target, "target")
    n = p.shape[0]
    hw = det.pixels
    tstride = target_stride(tgt.numel(), n, hw)
    _same_device(p.device, ("target", tgt))
    loss = torch.empty((n,), dtype=torch.float32, device=p.device)
    g = torch.empty((n, 7), dtype=torch.float32, device=p.device) if grad else None
    img = torch.empty((n, det.height, det.width), dtype=torch.float32,
                      device=p.device) if return_image else None
    need = _lib.load().drr_l2_workspace_bytes(ctypes.byref(det.desc), n)
    ws, ws_bytes = _reuse_workspace(workspace, need, p.device)
    _lib.call("drr_render_l2", volume.packed.data_ptr(), ctypes.byref(volume.desc),
              ctypes.byref(det.desc), p.data_ptr(), n, tgt.data_ptr(), tstride,
              img.data_ptr() if img is not None else None, loss.data_ptr(),
              g.data_ptr() if g is not None else None, ws.data_ptr(), ws_bytes, _stream())
    return (loss, g, img) if return_image else (loss, g)


def momentum_step(poses: torch.Tensor, velocity: torch.Tensor, grad: torch.Tensor,
                  rate: torch.Tensor, momentum: float) -> None:
    """In place: velocity = momentum * velocity + grad; poses -= rate * velocity."""
    if poses.ndim != 2 or poses.shape[1] != 7:
        raise ValueError(f"poses must be [n, 7], got {tuple(poses.shape)}")
    for t, name in ((poses, "poses"), (velocity, "velocity"), (grad, "grad"), (rate, "rate")):
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        _dev_f32(t, name)
        if t.shape != poses.shape:
            raise ValueError(f"{name} must have the shape of poses {tuple(poses.shape)}, "
                             f"got {tuple(t.shape)}")
        _same_device(poses.device, (name, t))
    n = poses.shape[0]
    _lib.call("drr_pose_momentum_step", poses.data_ptr(), velocity.data_ptr(), grad.data_ptr(),
              rate.data_ptr(), float(momentum), n, _stream())
