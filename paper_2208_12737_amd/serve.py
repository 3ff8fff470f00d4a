"""Continuous-batching request loop over CT volumes resident in HBM.

Requests (a volume, a detector, a pose, forward or forward + backward)
arrive at any time.  Each scheduler tick
  1. completes the batches whose device work has finished (non-blocking
     event queries), releasing their memory and slots,
  2. admits queued requests in arrival order while the in-flight memory
     stays within the HBM budget and a slot is free (a request larger than
     the whole budget is rejected at submission),
  3. launches the admitted requests as one batch on the next of a few
     streams: one plan execute renders every request (any mix of volumes
     and detector sizes); forward + backward requests are objective items of
     that execute, which also reduce -ZNCC against their target and its pose
     gradient.
Batches on different streams overlap on the device, so requests that arrive
while others run are admitted as soon as memory and slots free up.  Every
result is computed by the same per-ray and per-pose kernels as a request
served alone, with fixed-order reductions, so it is bitwise independent of
the mix it was batched with.

The scheduling logic is independent of the GPU: ``Server`` drives a backend
object (``GpuBackend`` here, or a stand-in in tests).
"""

from __future__ import annotations

import collections
import ctypes
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

import numpy as np

FWD = "fwd"
FWDBWD = "fwdbwd"


class RequestRejected(RuntimeError):
    pass


@dataclass
class Request:
    volume: str
    height: int
    width: int
    delta_x: float
    delta_y: float
    pose: np.ndarray                  # 7 floats (host)
    kind: str = FWD                   # FWD or FWDBWD
    target: Any = None                # device image [H, W] for FWDBWD
    arrival: float = field(default_factory=time.perf_counter)


class Ticket:
    """Handle of a submitted request."""

    def __init__(self, req: Request, nbytes: int):
        self.request = req
        self.nbytes = nbytes
        self.done_at: Optional[float] = None
        self.result: Any = None
        self.error: Optional[BaseException] = None
        self._event = threading.Event()

    def done(self) -> bool:
        return self._event.is_set()

    def wait(self, timeout: Optional[float] = None):
        if not self._event.wait(timeout):
            raise TimeoutError("request not finished")
        if self.error is not None:
            raise self.error
        return self.result

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_at is None else self.done_at - self.request.arrival

    def _finish(self, result=None, error=None):
        self.result, self.error = result, error
        self.done_at = time.perf_counter()
        self._event.set()


class Server:
    """Scheduler: admission by memory budget and slots, continuous batching.

    backend must provide
      bytes_for(req) -> int           device bytes the request holds in flight
      launch(tickets, stream) -> h    enqueue the batch, return a handle
      poll(h) -> bool                 True once the device work is complete
      collect(h) -> list              one result per ticket, in order
    """

    def __init__(self, backend, hbm_budget_bytes: int, max_inflight: int = 1024,
                 n_streams: int = 2, max_batch: int = 512):
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.max_inflight = int(max_inflight)
        self.n_streams = int(n_streams)
        self.max_batch = int(max_batch)
        self.queue: collections.deque = collections.deque()
        self.inflight: List[tuple] = []        # (handle, tickets)
        self.used_bytes = 0
        self.used_slots = 0
        self.next_stream = 0
        self.completed: List[Ticket] = []
        self.batches = 0
        self._lock = threading.Lock()

    # ------------------------------------------------------------ client side
    def submit(self, req: Request) -> Ticket:
        nbytes = int(self.backend.bytes_for(req))
        t = Ticket(req, nbytes)
        if nbytes > self.budget:
            t._finish(error=RequestRejected(
                f"request needs {nbytes} bytes, more than the whole budget {self.budget}"))
            return t
        with self._lock:
            self.queue.append(t)
        return t

    def cancel(self, ticket: Ticket) -> bool:
        """Removes a request that has not been admitted yet."""
        with self._lock:
            try:
                self.queue.remove(ticket)
            except ValueError:
                return False
        ticket._finish(error=RequestRejected("cancelled"))
        return True

    # ------------------------------------------------------------ scheduler
    def _complete(self) -> int:
        n = 0
        still = []
        for h, tickets in self.inflight:
            if self.backend.poll(h):
                try:
                    results = self.backend.collect(h)
                    for t, r in zip(tickets, results):
                        t._finish(result=r)
                except BaseException as e:   # the batch failed: fail its requests only
                    for t in tickets:
                        if not t.done():
                            t._finish(error=e)
                for t in tickets:
                    self.used_bytes -= t.nbytes
                    self.used_slots -= 1
                    self.completed.append(t)
                n += len(tickets)
            else:
                still.append((h, tickets))
        self.inflight = still
        return n

    def _admit(self) -> List[Ticket]:
        batch: List[Ticket] = []
        with self._lock:
            while self.queue and len(batch) < self.max_batch:
                t = self.queue[0]
                if self.used_slots + 1 > self.max_inflight:
                    break
                if self.used_bytes + t.nbytes > self.budget:
                    break
                self.queue.popleft()
                self.used_bytes += t.nbytes
                self.used_slots += 1
                batch.append(t)
        return batch

    def tick(self) -> int:
        """One scheduling round; returns the number of requests completed."""
        n = self._complete()
        batch = self._admit()
        if batch:
            stream = self.next_stream
            self.next_stream = (self.next_stream + 1) % self.n_streams
            try:
                h = self.backend.launch(batch, stream)
                self.inflight.append((h, batch))
                self.batches += 1
            except BaseException as e:
                for t in batch:
                    self.used_bytes -= t.nbytes
                    self.used_slots -= 1
                    t._finish(error=e)
                    self.completed.append(t)
        return n

    def pending(self) -> int:
        with self._lock:
            return len(self.queue) + sum(len(t) for _, t in self.inflight)

    def run_until_idle(self, idle_sleep: float = 0.0):
        while self.pending():
            self.tick()
            if idle_sleep:
                time.sleep(idle_sleep)


# ---------------------------------------------------------------- GPU backend

class GpuBackend:
    """Runs each batch as one execute of a plan over the resident volumes.

    The work-item table is filled here directly from the requests (the
    buffers are allocated here, so the per-item checks of ``Plan.execute``
    are not repeated); the library still validates every item."""

    def __init__(self, volumes: Dict[str, Any], n_streams: int = 2, max_items: int = 2048):
        import torch
        from .plan import Plan
        self.torch = torch
        self.names = list(volumes)
        self.volumes = volumes
        self.index = {n: i for i, n in enumerate(self.names)}
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.plan = Plan([volumes[n] for n in self.names], max_items=max_items, use_graph=False)
        self.dev = volumes[self.names[0]].packed.device
        self._dets: Dict[tuple, tuple] = {}   # (H, W, dx, dy) -> (desc, scratch doubles)

    def _det(self, r: Request):
        key = (r.height, r.width, r.delta_x, r.delta_y)
        d = self._dets.get(key)
        if d is None:
            from . import _lib
            desc = _lib.detector_desc(r.height, r.width, r.delta_x, r.delta_y)
            ws = int(_lib.load().drr_plan_item_workspace_bytes(ctypes.byref(desc)))
            if ws == 0:
                raise ValueError(f"invalid detector {key}")
            d = self._dets[key] = (desc, ws // 8)
        return d

    def bytes_for(self, req: Request) -> int:
        if req.volume not in self.index:
            raise KeyError(f"unknown volume {req.volume!r}")
        _, ws = self._det(req)
        px = req.height * req.width
        if req.kind == FWD:
            return 4 * px + 64
        t = req.target
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.device == self.dev and
                t.dtype == torch.float32 and t.is_contiguous() and t.numel() == px):
            raise ValueError("target must be a contiguous float32 tensor of height x width "
                             "pixels on the volumes' device")
        return 4 * px + 8 * ws + 32 + 64

    def launch(self, tickets: List[Ticket], stream_idx: int):
        """One plan execute for the whole batch: forward items render an
        image, fwd+bwd items also reduce -ZNCC against their target and its
        pose gradient in the same launch.

        Results are allocated on the caller's current stream (the stream
        the client will use them on), scratch on the batch's own stream, so
        that memory a client frees is never handed to a later batch while
        the client's own work may still read it."""
        torch = self.torch
        from . import _lib
        stream = self.streams[stream_idx]
        n = len(tickets)
        reqs = [t.request for t in tickets]
        host = torch.empty((n, 7), dtype=torch.float32, pin_memory=True)
        host.numpy()[:] = np.stack([np.asarray(r.pose, np.float32) for r in reqs])
        dets = [self._det(r) for r in reqs]
        obj = [k for k, r in enumerate(reqs) if r.kind != FWD]
        imgs = [torch.empty((r.height, r.width), dtype=torch.float32, device=self.dev)
                for r in reqs]
        # loss and gradient of objective item j at lg[j, 0] and lg[j, 1:8]
        lg = torch.empty((len(obj), 8), dtype=torch.float32, device=self.dev) if obj else None
        stream.wait_stream(torch.cuda.current_stream())
        out = [None] * n
        arr = (_lib.WorkItem * n)()
        with torch.cuda.stream(stream):
            poses = host.to(self.dev, non_blocking=True)
            parts = None
            if obj:
                parts = torch.empty(sum(dets[k][1] for k in obj), dtype=torch.float64,
                                    device=self.dev)
            pbase = poses.data_ptr()
            j = poff = 0
            for k, r in enumerate(reqs):
                img = imgs[k]
                w = arr[k]
                w.volume = self.index[r.volume]
                w.det = dets[k][0]
                w.pose = pbase + 28 * k
                w.image = img.data_ptr()
                if r.kind == FWD:
                    out[k] = img
                    continue
                w.flags = _lib.DRR_ITEM_NCC
                w.target = r.target.data_ptr()
                w.loss = lg.data_ptr() + 32 * j
                w.grad = w.loss + 4
                w.partials = parts.data_ptr() + 8 * poff
                out[k] = (img, lg[j, 0], lg[j, 1:])
                j += 1
                poff += dets[k][1]
            _lib.call("drr_plan_execute", self.plan._h, arr, n, stream.cuda_stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        # the host pose buffer, the pose copy, the scratch and the requests
        # (their targets) stay referenced until the batch completes
        return (ev, out, (host, poses, parts, reqs))

    def poll(self, h) -> bool:
        return h[0].query()

    def collect(self, h):
        return h[1]


def plain_forward(volumes: Dict[str, Any], req: Request):
    """Comparison path: one request, one plain drr_render call, synchronous."""
    import torch
    from .drr import Detector, render
    det = Detector(req.height, req.width, req.delta_x, req.delta_y)
    pose = torch.from_numpy(np.asarray(req.pose, np.float32)).to(volumes[req.volume].device)
    return render(volumes[req.volume], pose[None], det)[0]
