"""Serving loop: filter requests admitted by a device-memory budget and run
with continuous batching.

The paper filters one image per call (Section 4, the program around
ApplyOilPaintOnBuffer); serving many requests is this project's addition.

A `Server` holds:
  * an admission queue (arrival order).  A request is admitted when its
    device bytes (its output buffer plus a fixed per-request allowance) fit
    the remaining budget and fewer than `capacity` requests are in flight;
    otherwise it waits (back-pressure).  A waiting request may be cancelled.
  * an executor that runs admitted requests.  `QueueExecutor` pushes them
    into the library's continuous-batching queue (oilpaint_queue_*): work of
    requests that arrive while others are on the GPU joins the next
    persistent launch.  `PlainExecutor` is the baseline: one plain kernel
    launch per request, in arrival order, on one stream.
  * per-request timestamps: latency = completion seen by the host - arrival.

Executors only need submit(req) -> handle and poll(handle) -> bool (raising
for a failed request), so the scheduling is testable on the CPU with a fake
executor.  An executor may also offer collect() -> the handles completed
since the last call (a set, or a dict handle -> error message, empty for
success); the server then makes one such call per step instead of a poll per
running request.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Callable, Optional


@dataclass
class ServeRequest:
    rid: int
    arrival_s: float          # scheduled arrival, seconds from the start of the run
    width: int
    height: int
    radius: int
    levels: int
    src: Any = None           # device image view (uint8 [H, W, 3])
    dst: Any = None           # output buffer, allocated at admission
    admitted_s: float = math.nan
    done_s: float = math.nan
    status: str = "new"       # new -> waiting -> running -> done | cancelled | failed
    error: str = ""
    handle: Any = None

    @property
    def pixels(self) -> int:
        return self.width * self.height

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


PER_REQUEST_OVERHEAD = 4096  # descriptor and bookkeeping bytes counted per request


def request_bytes(req: ServeRequest) -> int:
    """Device bytes a request holds while admitted: its output (3 bytes per
    pixel) plus a fixed allowance.  Its source is a view of an image already
    resident on the device."""
    return 3 * req.pixels + PER_REQUEST_OVERHEAD


class Server:
    def __init__(self, executor, budget_bytes: int, capacity: int = 4096,
                 allocate: Optional[Callable[[ServeRequest], Any]] = None,
                 free: Optional[Callable[[ServeRequest], None]] = None,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.capacity = int(capacity)
        self.allocate = allocate
        self.free = free
        self.clock = clock
        self.t0 = None
        self.used = 0
        self.peak_used = 0
        self.waiting: deque[ServeRequest] = deque()
        self.running: list[ServeRequest] = []
        self.finished: list[ServeRequest] = []
        self.rejected: list[ServeRequest] = []

    # -- time -------------------------------------------------------------
    def start(self):
        self.t0 = self.clock()

    def now(self) -> float:
        return self.clock() - self.t0

    # -- requests ---------------------------------------------------------
    def submit(self, req: ServeRequest):
        """A request arrives.  Requests that can never fit the budget are
        rejected at once."""
        if request_bytes(req) > self.budget:
            req.status = "failed"
            req.error = "larger than the memory budget"
            self.rejected.append(req)
            return
        req.status = "waiting"
        self.waiting.append(req)

    def cancel(self, rid: int) -> bool:
        """Cancel a request that is still waiting for admission."""
        for r in self.waiting:
            if r.rid == rid:
                self.waiting.remove(r)
                r.status = "cancelled"
                self.finished.append(r)
                return True
        return False

    def _admit(self):
        while self.waiting and len(self.running) < self.capacity:
            req = self.waiting[0]
            need = request_bytes(req)
            if self.used + need > self.budget:
                break  # FIFO: the head waits for memory, nobody overtakes it
            self.waiting.popleft()
            self.used += need
            self.peak_used = max(self.peak_used, self.used)
            req.admitted_s = self.now()
            if self.allocate is not None:
                req.dst = self.allocate(req)
            try:
                req.handle = self.ex.submit(req)
                req.status = "running"
                self.running.append(req)
            except Exception as e:  # a failed submission fails this request only
                self._finish(req, failed=str(e))

    def _finish(self, req: ServeRequest, failed: str = ""):
        req.done_s = self.now()
        req.status = "failed" if failed else "done"
        req.error = failed
        self.used -= request_bytes(req)
        if self.free is not None:
            self.free(req)
        self.finished.append(req)

    def step(self) -> int:
        """Admit what fits, then collect completions.  Returns the number of
        requests completed in this step."""
        self._admit()
        n = 0
        still = []
        collect = getattr(self.ex, "collect", None)
        completed = None
        if collect is not None:
            try:
                completed = collect()
            except Exception:  # fall back to polling: failures stay per request
                completed = None
        for req in self.running:
            err = ""
            try:
                if completed is not None:
                    done = req.handle in completed
                    if done and isinstance(completed, dict):
                        err = completed[req.handle] or ""
                else:
                    done = self.ex.poll(req.handle)
            except Exception as e:
                self._finish(req, failed=str(e))
                n += 1
                continue
            if done:
                self._finish(req, failed=err)
                n += 1
            else:
                still.append(req)
        self.running = still
        if n:
            self._admit()
        return n

    def idle(self) -> bool:
        return not self.waiting and not self.running

    # -- statistics -------------------------------------------------------
    def stats(self) -> dict:
        done = [r for r in self.finished if r.status == "done"]
        lat = sorted(r.latency_s for r in done)

        def pct(p):
            if not lat:
                return math.nan
            k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
            return lat[k]
        mp = sum(r.pixels for r in done) / 1e6
        span = (max(r.done_s for r in done) - min(r.arrival_s for r in done)) if done else math.nan
        return {
            "completed": len(done),
            "failed": sum(1 for r in self.finished if r.status == "failed") + len(self.rejected),
            "cancelled": sum(1 for r in self.finished if r.status == "cancelled"),
            "megapixels": mp,
            "span_s": span,
            "mp_per_s": mp / span if done and span > 0 else math.nan,
            "p50_ms": pct(50) * 1e3,
            "p99_ms": pct(99) * 1e3,
            "mean_ms": (sum(lat) / len(lat) * 1e3) if lat else math.nan,
            "peak_bytes": self.peak_used,
        }


def run_open_loop(server: Server, requests: list[ServeRequest], spin_sleep_s: float = 0.0,
                  deadline_s: float = 600.0) -> dict:
    """Deliver `requests` at their scheduled arrival times (open loop: the
    arrival schedule does not wait for the server) and run the server until
    every request has finished.  Returns server.stats()."""
    pending = deque(sorted(requests, key=lambda r: r.arrival_s))
    server.start()
    while pending or not server.idle():
        now = server.now()
        if now > deadline_s:
            raise TimeoutError("serving run exceeded %.0f s" % deadline_s)
        while pending and pending[0].arrival_s <= now:
            server.submit(pending.popleft())
        progressed = server.step()
        if not progressed and spin_sleep_s > 0:
            time.sleep(spin_sleep_s)
    return server.stats()


# ---------------------------------------------------------------------------
# GPU executors
# ---------------------------------------------------------------------------

class QueueExecutor:
    """Continuous batching through the library's request queue."""

    def __init__(self, capacity: int = 4096, step_pixels: int = 0):
        from . import binding
        self.B = binding
        self.q = binding.Queue(capacity=capacity, step_pixels=step_pixels)

    def submit(self, req: ServeRequest):
        return self.q.push(self.B.Item(req.src, req.dst, req.radius, req.levels))

    def poll(self, ticket) -> bool:
        return self.q.poll(ticket)

    def collect(self) -> dict:
        """{ticket: error message or ""} of the requests completed since the
        last call."""
        done = {}
        while True:
            got = self.q.completed_status()
            for t, st in got:
                done[t] = "" if st == self.B.OK else "%s (%d)" % (self.B.strerror(st), st)
            if len(got) < 4096:
                return done

    def close(self):
        self.q.close()


class PlainExecutor:
    """Baseline: one plain kernel launch per request, in admission order, on
    one stream; completion is observed through an event per request."""

    def __init__(self):
        import torch
        from . import binding
        self.torch = torch
        self.B = binding
        self.stream = torch.cuda.Stream()

    def submit(self, req: ServeRequest):
        ev = self.torch.cuda.Event()
        self.B.run(self.B.Item(req.src, req.dst, req.radius, req.levels), stream=self.stream)
        ev.record(self.stream)
        return ev

    def poll(self, ev) -> bool:
        return ev.query()

    def close(self):
        self.stream.synchronize()


def make_requests(workload) -> list[ServeRequest]:
    """ServeRequests for a synth.ServeWorkload (device canvases)."""
    out = []
    for r in workload.requests:
        out.append(ServeRequest(r.rid, r.arrival_s, r.width, r.height, r.radius, r.levels,
                                src=workload.image(r)))
    return out


def device_allocator(keep: bool, preallocate=None):
    """allocate/free callbacks that give each admitted request a dense
    [H, W, 3] output buffer; with keep=True outputs stay alive in the request
    after completion (for verification).  With `preallocate` (the requests
    of a run) every output is allocated up front, so that no allocation
    falls inside the served run."""
    import torch
    pool = {}
    if preallocate is not None:
        for req in preallocate:
            pool[req.rid] = torch.empty((req.height, req.width, 3), dtype=torch.uint8, device=req.src.device)

    def allocate(req: ServeRequest):
        if req.rid in pool:
            return pool.pop(req.rid)
        return torch.empty((req.height, req.width, 3), dtype=torch.uint8, device=req.src.device)

    def free(req: ServeRequest):
        if not keep:
            req.dst = None
    return allocate, free
