"""Serving scheduler on the CPU with a fake executor: admission by memory
budget, FIFO back-pressure, capacity, rejection, cancellation, failure
isolation and latency accounting.  No GPU is involved."""
import math

import numpy as np
import pytest

import oracle
from paper_1405_1020_amd import serve, synth


class FakeClock:
    """Advances by `dt` seconds on every reading."""

    def __init__(self, dt=0.001):
        self.t = 0.0
        self.dt = dt

    def __call__(self):
        self.t += self.dt
        return self.t


class FakeExecutor:
    """Completes a request after `polls` polls, computing its output with the
    CPU oracle; can be told to fail given request ids at submit or poll."""

    def __init__(self, polls=3, fail_submit=(), fail_poll=()):
        self.polls = polls
        self.fail_submit = set(fail_submit)
        self.fail_poll = set(fail_poll)
        self.running = 0
        self.max_running = 0
        self.order = []

    def submit(self, req):
        if req.rid in self.fail_submit:
            raise RuntimeError("submit failed")
        self.running += 1
        self.max_running = max(self.max_running, self.running)
        self.order.append(req.rid)
        return {"req": req, "left": self.polls}

    def poll(self, h):
        req = h["req"]
        if req.rid in self.fail_poll:
            self.running -= 1
            raise RuntimeError("device error")
        h["left"] -= 1
        if h["left"] > 0:
            return False
        req.dst[...] = oracle.oilpaint_ref(req.src, req.radius, req.levels)
        self.running -= 1
        return True


class FakeCollectExecutor(FakeExecutor):
    """Reports completions in bulk through collect(); poll must not be used."""

    def __init__(self, polls=3):
        super().__init__(polls=polls)
        self.live = {}
        self.next = 1

    def submit(self, req):
        h = super().submit(req)
        t = self.next
        self.next += 1
        self.live[t] = h
        return t

    def poll(self, ticket):
        raise AssertionError("poll used although collect exists")

    def collect(self):
        done = {t for t, h in self.live.items() if FakeExecutor.poll(self, h)}
        for t in done:
            del self.live[t]
        return done


def reqs(sizes, arrivals=None, r=2, L=20):
    out = []
    for i, (w, h) in enumerate(sizes):
        img = synth.make_random(w, h, seed=i)
        a = arrivals[i] if arrivals else 0.0
        out.append(serve.ServeRequest(i, a, w, h, r, L, src=img))
    return out


def np_alloc(req):
    return np.zeros((req.height, req.width, 3), np.uint8)


def drain(server, requests):
    for q in requests:
        server.submit(q)
    for _ in range(10000):
        server.step()
        if server.idle():
            return
    raise AssertionError("server did not drain")


def test_budget_back_pressure_and_results():
    rs = reqs([(20, 10)] * 6)
    per = serve.request_bytes(rs[0])
    ex = FakeExecutor()
    s = serve.Server(ex, budget_bytes=2 * per, allocate=np_alloc, clock=FakeClock())
    s.start()
    drain(s, rs)
    st = s.stats()
    assert st["completed"] == 6
    assert ex.max_running == 2
    assert s.peak_used <= 2 * per
    assert s.used == 0
    for q in rs:
        assert np.array_equal(q.dst, oracle.oilpaint_ref(q.src, q.radius, q.levels))


def test_bulk_completion_collect():
    rs = reqs([(20, 10), (7, 9), (33, 4), (5, 5), (16, 16)])
    ex = FakeCollectExecutor(polls=2)
    s = serve.Server(ex, budget_bytes=3 * serve.request_bytes(rs[0]), allocate=np_alloc, clock=FakeClock())
    s.start()
    drain(s, rs)
    assert s.stats()["completed"] == 5 and s.used == 0 and not ex.live
    for q in rs:
        assert np.array_equal(q.dst, oracle.oilpaint_ref(q.src, q.radius, q.levels))


def test_fifo_head_is_not_overtaken():
    # a large request at the head waits for memory; smaller ones behind it
    # do not overtake it
    rs = reqs([(40, 40), (50, 50), (5, 5), (5, 5)])
    budget = serve.request_bytes(rs[0]) + serve.request_bytes(rs[2]) + serve.request_bytes(rs[3])
    ex = FakeExecutor(polls=2)
    s = serve.Server(ex, budget_bytes=budget, allocate=np_alloc, clock=FakeClock())
    s.start()
    drain(s, rs)
    assert ex.order == [0, 1, 2, 3]


def test_capacity_limit():
    rs = reqs([(8, 8)] * 10)
    ex = FakeExecutor(polls=4)
    s = serve.Server(ex, budget_bytes=1 << 30, capacity=3, allocate=np_alloc, clock=FakeClock())
    s.start()
    drain(s, rs)
    assert ex.max_running == 3 and s.stats()["completed"] == 10


def test_reject_request_larger_than_budget():
    rs = reqs([(100, 100), (5, 5)])
    s = serve.Server(FakeExecutor(), budget_bytes=serve.request_bytes(rs[1]) + 10, allocate=np_alloc,
                     clock=FakeClock())
    s.start()
    drain(s, rs)
    st = s.stats()
    assert st["completed"] == 1 and st["failed"] == 1
    assert rs[0].status == "failed" and "budget" in rs[0].error


def test_cancel_waiting_request():
    rs = reqs([(30, 30), (30, 30), (30, 30)])
    per = serve.request_bytes(rs[0])
    s = serve.Server(FakeExecutor(polls=5), budget_bytes=per, allocate=np_alloc, clock=FakeClock())
    s.start()
    for q in rs:
        s.submit(q)
    s.step()  # admits request 0 only
    assert s.cancel(2) is True
    assert s.cancel(0) is False  # already running
    while not s.idle():
        s.step()
    st = s.stats()
    assert st["completed"] == 2 and st["cancelled"] == 1 and rs[2].status == "cancelled"


def test_executor_failures_are_isolated():
    rs = reqs([(12, 9)] * 6)
    ex = FakeExecutor(fail_submit={1}, fail_poll={4})
    freed = []
    s = serve.Server(ex, budget_bytes=1 << 30, allocate=np_alloc, free=lambda q: freed.append(q.rid),
                     clock=FakeClock())
    s.start()
    drain(s, rs)
    st = s.stats()
    assert st["completed"] == 4 and st["failed"] == 2
    assert s.used == 0 and sorted(freed) == list(range(6))
    for q in rs:
        if q.status == "done":
            assert np.array_equal(q.dst, oracle.oilpaint_ref(q.src, q.radius, q.levels))


class FakeStatusCollectExecutor(FakeCollectExecutor):
    """collect() returns {ticket: error message}, as QueueExecutor does: the
    requests in `fail` are reported complete with an error."""

    def __init__(self, fail=(), polls=2):
        super().__init__(polls=polls)
        self.fail = set(fail)

    def collect(self):
        done = FakeCollectExecutor.collect(self)
        return {t: ("launch failed" if self.rid_of[t] in self.fail else "") for t in done}

    def submit(self, req):
        t = super().submit(req)
        self.rid_of = getattr(self, "rid_of", {})
        self.rid_of[t] = req.rid
        return t


def test_collect_status_fails_only_the_failed_requests():
    rs = reqs([(10, 7)] * 5)
    ex = FakeStatusCollectExecutor(fail={1, 3})
    freed = []
    s = serve.Server(ex, budget_bytes=1 << 30, allocate=np_alloc, free=lambda q: freed.append(q.rid),
                     clock=FakeClock())
    s.start()
    drain(s, rs)
    st = s.stats()
    assert st["completed"] == 3 and st["failed"] == 2
    assert [q.status for q in rs] == ["done", "failed", "done", "failed", "done"]
    assert rs[1].error == "launch failed" and s.used == 0 and sorted(freed) == list(range(5))


def test_latency_accounting_open_loop():
    arrivals = [0.0, 0.05, 0.05, 0.2]
    rs = reqs([(6, 6)] * 4, arrivals=arrivals)
    clock = FakeClock(dt=0.001)
    s = serve.Server(FakeExecutor(polls=3), budget_bytes=1 << 30, allocate=np_alloc, clock=clock)
    st = serve.run_open_loop(s, rs)
    assert st["completed"] == 4
    for q in rs:
        assert q.done_s >= q.arrival_s and q.admitted_s >= q.arrival_s
        assert 0 < q.latency_s < 0.05
    lat = sorted(q.latency_s for q in rs)
    assert math.isclose(st["p50_ms"], lat[1] * 1e3) and math.isclose(st["p99_ms"], lat[3] * 1e3)
    assert st["megapixels"] == pytest.approx(4 * 36 / 1e6)
