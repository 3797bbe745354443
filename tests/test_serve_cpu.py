"""Scheduling logic of the continuous-batching server, on the CPU with a fake
executor that simulates device time and memory."""
import threading
import time

import pytest

from paper_1901_02492_amd.serve import Request, Server, footprint_bytes


class FakeExecutor:
    """Simulated device: a batch takes the sum of its requests' costs; memory is
    accounted independently of the server to check its budget."""

    def __init__(self, cost_s=0.002, fail_prepare=(), fail_launch_with=()):
        self.cost_s = cost_s
        self.fail_prepare = set(fail_prepare)
        self.fail_launch_with = set(fail_launch_with)
        self.lock = threading.Lock()
        self.live = 0
        self.peak_live = 0
        self.order = []
        self.busy_until = 0.0

    def footprint(self, req):
        n, h, w = req.shape
        return n * h * w

    def prepare(self, req):
        if req.rid in self.fail_prepare:
            raise RuntimeError(f"prepare failed for {req.rid}")
        with self.lock:
            self.live += self.footprint(req)
            self.peak_live = max(self.peak_live, self.live)
            self.order.append(req.rid)
        return {"req": req}

    def launch(self, handles):
        if any(h["req"].rid in self.fail_launch_with for h in handles):
            raise RuntimeError("launch failed")
        now = time.perf_counter()
        start = max(now, self.busy_until)
        self.busy_until = start + self.cost_s * len(handles)
        return self.busy_until

    def done(self, token):
        return time.perf_counter() >= token

    def result(self, h):
        return ("result", h["req"].rid)

    def release(self, h):
        with self.lock:
            self.live -= self.footprint(h["req"])


def _req(rid, shape=(2, 4, 4), arrival=0.0, n_vel=10):
    return Request(rid=rid, shape=shape, t=None, vel=[0] * n_vel, psf=None, k=1, make=None,
                   arrival=arrival)


def test_all_requests_complete_in_order_within_budget():
    ex = FakeExecutor()
    srv = Server(ex, budget_bytes=3 * 32).start()   # three 2x4x4 requests fit at once
    futs = [srv.submit(_req(i)) for i in range(20)]
    res = [f.result(timeout=10) for f in futs]
    srv.stop()
    assert [r.result for r in res] == [("result", i) for i in range(20)]
    assert ex.order == list(range(20))               # admitted in arrival order
    assert ex.peak_live <= 3 * 32 and srv.peak_bytes <= 3 * 32
    assert ex.live == 0 and srv.bytes_in_use == 0
    assert all(r.latency >= 0 and r.finished >= r.admitted >= r.arrival for r in res)


def test_requests_are_batched_when_they_queue_up():
    ex = FakeExecutor(cost_s=0.01)
    srv = Server(ex, budget_bytes=10 ** 9, max_batch=8, max_inflight=1)
    futs = [srv.submit(_req(i)) for i in range(16)]  # queued before the loop starts
    srv.start()
    for f in futs:
        f.result(timeout=10)
    srv.stop()
    assert max(srv.batches) == 8 and sum(srv.batches) == 16


def test_batches_respect_the_work_cap():
    # Work per request: n * h * w * V.  Small ones (320) pack up to the cap of
    # 1000; a large one (4000) runs alone; order stays FIFO.
    ex = FakeExecutor(cost_s=0.005)
    srv = Server(ex, budget_bytes=10 ** 9, max_inflight=1, batch_work=1000)
    sizes = [(2, 4, 4)] * 3 + [(10, 20, 2)] + [(2, 4, 4)] * 4
    futs = [srv.submit(_req(i, shape=sh)) for i, sh in enumerate(sizes)]
    srv.start()
    for f in futs:
        f.result(timeout=10)
    srv.stop()
    assert srv.batches == [3, 1, 3, 1]
    assert ex.order == list(range(len(sizes)))


def test_oversized_request_fails_alone():
    ex = FakeExecutor()
    srv = Server(ex, budget_bytes=100).start()
    big = srv.submit(_req(0, shape=(10, 10, 10)))
    small = srv.submit(_req(1))
    with pytest.raises(MemoryError):
        big.result(timeout=5)
    assert small.result(timeout=5).result == ("result", 1)
    srv.stop()


def test_failing_prepare_is_isolated():
    ex = FakeExecutor(fail_prepare={3})
    srv = Server(ex, budget_bytes=10 ** 6).start()
    futs = [srv.submit(_req(i)) for i in range(6)]
    for i, f in enumerate(futs):
        if i == 3:
            with pytest.raises(RuntimeError):
                f.result(timeout=5)
        else:
            assert f.result(timeout=5).result == ("result", i)
    srv.stop()
    assert srv.bytes_in_use == 0


def test_failing_launch_fails_only_its_batch():
    ex = FakeExecutor(fail_launch_with={2})
    srv = Server(ex, budget_bytes=32, max_batch=1).start()   # one request per batch
    futs = [srv.submit(_req(i)) for i in range(5)]
    for i, f in enumerate(futs):
        if i == 2:
            with pytest.raises(RuntimeError):
                f.result(timeout=5)
        else:
            assert f.result(timeout=5).result == ("result", i)
    srv.stop()
    assert srv.bytes_in_use == 0 and ex.live == 0


def test_late_arrivals_are_admitted_while_others_run():
    ex = FakeExecutor(cost_s=0.02)
    srv = Server(ex, budget_bytes=2 * 32, max_inflight=2).start()
    first = [srv.submit(_req(i)) for i in range(2)]
    time.sleep(0.005)                                 # both running now
    late = [srv.submit(_req(10 + i)) for i in range(3)]
    for f in first + late:
        f.result(timeout=10)
    srv.stop()
    assert ex.peak_live <= 2 * 32
    assert ex.order == [0, 1, 10, 11, 12]


def test_footprint_counts_every_buffer():
    # 15 x 4096^2, 600 velocities, K = 50: inputs 2.26 GB + planes 2.01 GB +
    # candidates 11.7 GB, ordered in place (no separate results).
    b = footprint_bytes(15, 4096, 4096, 600, 50, 50)
    assert 15.9e9 < b < 16.1e9
    # 16-bit planes: their copy, and results apart from the candidates.
    assert (footprint_bytes(15, 4096, 4096, 600, 50, 50, lp="f16") - b
            == 15 * 4096 * 4096 * 4 + 4096 * 4096 * 50 * 14)
    # more candidates than results: results apart from the candidates.
    assert (footprint_bytes(15, 4096, 4096, 600, 50, 64) - b
            == 4096 * 4096 * (64 + 50 - 50) * 14)
