"""GPU parity of the served form: serve.Server admitting a seeded Poisson
stream of requests by a device-memory budget and running them through the
library's continuous-batching queue (QueueExecutor).

Requests arrive while others are on the GPU (a burst at t = 0 larger than the
budget, then Poisson arrivals), so they are admitted as memory frees up and
their work shares launches.  Every result must equal the same request filtered
alone by the plain kernel, and whole outputs of every request up to 0.5 MP plus
a seeded sample of the larger ones must equal the oracle (the Section 4
definition, clipped window) byte for byte."""
import numpy as np
import pytest

from paper_1405_1020_amd import binding as B
from paper_1405_1020_amd import serve, synth
from gpu_util import ref, first_mismatch, torch_mod

pytestmark = pytest.mark.gpu


class CountingExecutor(serve.QueueExecutor):
    """QueueExecutor that records, at each submission, how many admitted
    requests had not yet been seen complete."""

    def __init__(self, server_ref, **kw):
        super().__init__(**kw)
        self.server_ref = server_ref
        self.in_flight_at_submit = []

    def submit(self, req):
        self.in_flight_at_submit.append(len(self.server_ref[0].running))
        return super().submit(req)


def test_server_queue_executor_poisson_stream():
    torch = torch_mod()
    wl = synth.serve_workload(n=160, rate=4000.0, seed=55, mp_range=(0.01, 3.0), n_canvas=3,
                              canvas_wh=(2400, 1800))
    reqs = serve.make_requests(wl)
    burst = 24
    for q in reqs[:burst]:
        q.arrival_s = 0.0
    burst_bytes = sum(serve.request_bytes(q) for q in reqs[:burst])
    budget = 24 << 20
    assert burst_bytes > budget  # the burst cannot be admitted at once: back-pressure
    holder = [None]
    ex = CountingExecutor(holder, capacity=64, step_pixels=1 << 20)
    alloc, free = serve.device_allocator(keep=True)
    server = serve.Server(ex, budget_bytes=budget, capacity=16, allocate=alloc, free=free)
    holder[0] = server
    st = serve.run_open_loop(server, reqs, deadline_s=120.0)
    ex.close()
    torch.cuda.synchronize()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert server.peak_used <= budget
    # requests were submitted while earlier ones were still on the GPU
    assert max(ex.in_flight_at_submit) >= 2
    # each result equals the same request run alone by the plain kernel
    for q in reqs:
        alone = torch.empty_like(q.dst)
        B.run(B.Item(q.src, alone, q.radius, q.levels))  # a crop: src and dst strides differ
        torch.cuda.synchronize()
        assert torch.equal(alone, q.dst), (q.rid, q.width, q.height, q.radius, q.levels)
    # whole outputs against the oracle: every request <= 0.5 MP, and a seeded
    # quarter of the larger ones
    rng = np.random.default_rng(56)
    checked = 0
    for q in reqs:
        if q.pixels > 500_000 and rng.random() >= 0.25:
            continue
        img = q.src.contiguous().cpu().numpy()
        mm = first_mismatch(q.dst.cpu().numpy(), ref(img, q.radius, q.levels))
        assert mm is None, (q.rid, q.width, q.height, q.radius, q.levels, mm)
        checked += 1
    assert checked >= 60
