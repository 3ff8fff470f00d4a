"""Request-loop scheduling on the CPU with a stand-in backend (no GPU):
admission by memory budget and slots, continuous batching across ticks,
failure isolation and cancellation."""

import numpy as np
import pytest

from paper_2208_12737_amd.serve import FWD, FWDBWD, Request, RequestRejected, Server


class FakeBackend:
    """Completes a batch `delay` polls after its launch; result = a value
    derived from the request only (so it is independent of the batch)."""

    def __init__(self, delay=2, fail_volume=None):
        self.delay = delay
        self.fail_volume = fail_volume
        self.launched = []
        self.live_bytes = 0
        self.max_live_bytes = 0

    def bytes_for(self, req):
        return req.height * req.width * (2 if req.kind == FWDBWD else 1)

    def launch(self, tickets, stream):
        if any(t.request.volume == self.fail_volume for t in tickets):
            raise RuntimeError("backend failure")
        self.launched.append(([t.request for t in tickets], stream))
        b = sum(t.nbytes for t in tickets)
        self.live_bytes += b
        self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)
        return {"left": self.delay, "tickets": tickets, "bytes": b}

    def poll(self, h):
        h["left"] -= 1
        return h["left"] < 0

    def collect(self, h):
        self.live_bytes -= h["bytes"]
        return [float(np.sum(t.request.pose)) * t.request.height for t in h["tickets"]]


def _req(i, vol="a", hw=8, kind=FWD):
    return Request(vol, hw, hw, 1.0, 1.0, np.full(7, float(i)), kind)


def test_all_requests_complete_in_order_with_correct_results():
    be = FakeBackend()
    srv = Server(be, hbm_budget_bytes=10_000)
    tickets = [srv.submit(_req(i)) for i in range(20)]
    srv.run_until_idle()
    for i, t in enumerate(tickets):
        assert t.wait(0) == pytest.approx(7.0 * i * 8)
        assert t.latency is not None and t.latency >= 0
    # admission was FIFO
    order = [r.pose[0] for batch, _ in be.launched for r in batch]
    assert order == sorted(order)


def test_budget_bounds_inflight_memory_and_queues_the_rest():
    be = FakeBackend(delay=3)
    budget = 3 * 64 + 10                       # three 8x8 forward requests
    srv = Server(be, hbm_budget_bytes=budget)
    tickets = [srv.submit(_req(i)) for i in range(10)]
    srv.tick()
    assert srv.used_bytes <= budget and len(srv.queue) == 7
    srv.run_until_idle()
    assert be.max_live_bytes <= budget
    assert all(t.done() and t.error is None for t in tickets)
    assert len(be.launched) >= 4               # needed several batches


def test_oversized_request_rejected_immediately():
    srv = Server(FakeBackend(), hbm_budget_bytes=100)
    t = srv.submit(_req(0, hw=64))
    assert t.done()
    with pytest.raises(RequestRejected):
        t.wait(0)
    assert srv.pending() == 0


def test_slot_limit():
    be = FakeBackend(delay=5)
    srv = Server(be, hbm_budget_bytes=1 << 30, max_inflight=4)
    for i in range(10):
        srv.submit(_req(i))
    srv.tick()
    assert srv.used_slots == 4
    srv.run_until_idle()
    assert srv.used_slots == 0 and srv.used_bytes == 0


def test_continuous_batching_admits_late_arrivals_while_others_run():
    be = FakeBackend(delay=4)
    srv = Server(be, hbm_budget_bytes=1 << 20, n_streams=3)
    first = [srv.submit(_req(i)) for i in range(3)]
    srv.tick()                                  # batch 1 in flight
    late = [srv.submit(_req(10 + i, kind=FWDBWD)) for i in range(2)]
    srv.tick()                                  # batch 2 launched while batch 1 runs
    assert len(srv.inflight) == 2
    streams = [s for _, s in be.launched]
    assert streams[0] != streams[1]             # they overlap on different streams
    srv.run_until_idle()
    assert all(t.done() for t in first + late)


def test_result_independent_of_batch_mix():
    alone = Server(FakeBackend(), hbm_budget_bytes=1 << 20)
    t0 = alone.submit(_req(5, hw=16, kind=FWDBWD))
    alone.run_until_idle()
    mixed = Server(FakeBackend(), hbm_budget_bytes=1 << 20)
    ts = [mixed.submit(_req(i, hw=8 + 8 * (i % 2), kind=FWD if i % 3 else FWDBWD))
          for i in range(12)]
    t1 = mixed.submit(_req(5, hw=16, kind=FWDBWD))
    mixed.run_until_idle()
    assert t0.wait(0) == t1.wait(0)


def test_backend_failure_fails_only_that_batch():
    be = FakeBackend(fail_volume="bad")
    srv = Server(be, hbm_budget_bytes=1 << 20, max_batch=1)
    good1 = srv.submit(_req(1))
    bad = srv.submit(_req(2, vol="bad"))
    good2 = srv.submit(_req(3))
    srv.run_until_idle()
    assert good1.wait(0) is not None and good2.wait(0) is not None
    with pytest.raises(RuntimeError):
        bad.wait(0)
    assert srv.used_bytes == 0 and srv.used_slots == 0


def test_cancel_queued_request():
    be = FakeBackend(delay=3)
    srv = Server(be, hbm_budget_bytes=64)
    a = srv.submit(_req(1))
    b = srv.submit(_req(2))
    srv.tick()                                  # a admitted, b queued (budget)
    assert srv.cancel(b)
    assert not srv.cancel(a)
    srv.run_until_idle()
    assert a.wait(0) is not None
    with pytest.raises(RequestRejected):
        b.wait(0)
