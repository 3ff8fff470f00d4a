"""Batched render plans (persistent tile-queue kernels, HIP graph replay,
autotuned launch shape) -- a thin wrapper of drr_plan_* in include/drr.h."""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _lib
from .drr import Detector, Volume, _stream


@dataclass
class Item:
    """One render: volume index, detector, a device pose [7] and outputs.

    An objective item (``target`` given) computes the fused -ZNCC against
    ``target`` into ``loss`` [1] and its pose gradient into ``grad`` [7],
    using ``partials`` (float64, ``item_workspace_bytes(det)`` bytes) as
    scratch; its ``image`` is optional.  ``objective_item`` allocates these."""
    volume: int
    det: Detector
    pose: torch.Tensor
    image: Optional[torch.Tensor]
    jac: Optional[torch.Tensor] = None
    counts: Optional[torch.Tensor] = None
    target: Optional[torch.Tensor] = None
    loss: Optional[torch.Tensor] = None
    grad: Optional[torch.Tensor] = None
    partials: Optional[torch.Tensor] = None

    def flags(self) -> int:
        f = 0
        if self.jac is not None:
            f |= _lib.DRR_ITEM_JAC
        if self.counts is not None:
            f |= _lib.DRR_ITEM_COUNT
        if self.target is not None:
            f |= _lib.DRR_ITEM_NCC
        return f


def item_workspace_bytes(det: Detector) -> int:
    """Scratch bytes of one objective item on detector `det`."""
    n = int(_lib.load().drr_plan_item_workspace_bytes(ctypes.byref(det.desc)))
    if n == 0:
        raise ValueError(f"invalid detector {det}")
    return n


def objective_item(volume: int, det: Detector, pose: torch.Tensor, target: torch.Tensor,
                   image: Optional[torch.Tensor] = None) -> Item:
    """An objective item with freshly allocated loss, gradient and scratch."""
    dev = pose.device
    return Item(volume, det, pose, image, target=target,
                loss=torch.empty(1, dtype=torch.float32, device=dev),
                grad=torch.empty(7, dtype=torch.float32, device=dev),
                partials=torch.empty(item_workspace_bytes(det) // 8, dtype=torch.float64,
                                     device=dev))


def _check(k, name, t, numel, dtype=torch.float32):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"item {k}: {name} must be a contiguous {dtype} GPU tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"item {k}: {name} has {t.numel()} elements, expected {numel}")


def _items_array(items: Sequence[Item]):
    arr = (_lib.WorkItem * max(len(items), 1))()
    for k, it in enumerate(items):
        _check(k, "pose", it.pose, 7)
        if it.image is not None:
            _check(k, "image", it.image, it.det.pixels)
        elif it.target is None:
            raise ValueError(f"item {k}: image is required")
        if it.jac is not None:
            _check(k, "jac", it.jac, 7 * it.det.pixels)
        if it.counts is not None:
            _check(k, "counts", it.counts, it.det.pixels, torch.int32)
        if it.target is not None:
            _check(k, "target", it.target, it.det.pixels)
            for name in ("loss", "grad", "partials"):
                if getattr(it, name) is None:
                    raise ValueError(f"item {k}: objective item needs {name}")
            _check(k, "loss", it.loss, 1)
            _check(k, "grad", it.grad, 7)
            _check(k, "partials", it.partials, None, torch.float64)
            if it.partials.numel() * 8 < item_workspace_bytes(it.det):
                raise ValueError(f"item {k}: partials smaller than item_workspace_bytes")
        w = arr[k]
        w.volume = it.volume
        w.flags = it.flags()
        w.det = it.det.desc
        w.pose = it.pose.data_ptr()
        w.image = it.image.data_ptr() if it.image is not None else None
        w.jac = it.jac.data_ptr() if it.jac is not None else None
        w.counts = it.counts.data_ptr() if it.counts is not None else None
        if it.target is not None:
            w.target = it.target.data_ptr()
            w.loss = it.loss.data_ptr()
            w.grad = it.grad.data_ptr()
            w.partials = it.partials.data_ptr()
    return arr


class Plan:
    """Renders lists of heterogeneous items in one persistent launch.

    Results equal rendering each item alone.  `autotune` times candidate
    launch shapes on `tune_items` at creation (results cached in
    `cache_path` when given)."""

    def __init__(self, volumes: Sequence[Volume], max_items: int = 1024, use_graph: bool = True,
                 autotune: bool = False, tune_items: Optional[Sequence[Item]] = None,
                 cache_path: Optional[str] = None, strategy: int = -1, tile_code: int = -1,
                 wg_per_cu: int = -1):
        self.volumes = list(volumes)
        self._descs = (_lib.VolumeDesc * len(self.volumes))(*[v.desc for v in self.volumes])
        self._packed = (ctypes.c_void_p * len(self.volumes))(
            *[v.packed.data_ptr() for v in self.volumes])
        d = _lib.PlanDesc()
        d.max_items = max_items
        d.n_volumes = len(self.volumes)
        d.volumes = self._descs
        d.packed = self._packed
        d.use_graph = 1 if use_graph else 0
        d.autotune = 1 if autotune else 0
        self._cache = cache_path.encode() if cache_path else None
        d.tune_cache_path = self._cache
        d.strategy = strategy
        d.tile_code = tile_code
        d.wg_per_cu = wg_per_cu
        self._desc = d
        tune = list(tune_items or [])
        arr = _items_array(tune) if tune else None
        h = ctypes.c_void_p()
        _lib.call("drr_plan_create", ctypes.byref(d), arr, len(tune), _stream(), ctypes.byref(h))
        self._h = h
        self.max_items = max_items

    def execute(self, items: Sequence[Item]) -> None:
        if len(items) == 0:
            return
        arr = _items_array(items)
        _lib.call("drr_plan_execute", self._h, arr, len(items), _stream())

    @property
    def config(self):
        s, t, w, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.call("drr_plan_config", self._h, ctypes.byref(s), ctypes.byref(t), ctypes.byref(w),
                  ctypes.byref(g))
        names = {_lib.DRR_PLAN_PERSISTENT: "persistent", _lib.DRR_PLAN_FLAT: "flat",
                 _lib.DRR_PLAN_AUTO: "auto"}
        return {"strategy": names[s.value],
                "tile_code": t.value, "wg_per_cu": w.value, "use_graph": bool(g.value)}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().drr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
