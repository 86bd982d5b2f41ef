"""Scheduler logic of the request server on the CPU: a fake executor stands
in for the GPU batch (it completes render requests in one tick and counts
down track iterations), so admission by slots and memory budget, FIFO order,
retirement and the latency report are checked without a device."""
import numpy as np

from paper_2506_02741_amd import serve


class FakeServer(serve.Server):
    def __init__(self, sizes, **kw):
        super().__init__(keyframes=[], sections=[(0, 1)] * 4, device="cpu", **kw)
        self.sizes = sizes
        self.launched = []

    def estimate_bytes(self, req):
        return self.sizes[req.rid]

    def _view_for(self, req):
        return None

    def _execute(self, rend, trk):
        assert self.mem_used <= self.budget
        assert len(rend) + len(trk) <= self.max_active
        self.launched.append(([r.rid for r in rend], [r.rid for r in trk]))
        for r in rend:
            r._left = 0
            r.result = dict(ok=True)
        for r in trk:
            r._left -= 1
            if r._left == 0:
                r.result = dict(ok=True)


def trace(n, seed=0):
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for i in range(n):
        t += rng.exponential(0.005)
        kind = "render" if rng.uniform() < 0.6 else "track"
        out.append(serve.Request(i, kind, int(rng.integers(0, 4)), (1, 1, 0, 0, 8, 8),
                                 np.eye(3, 4), arrival=t, iters=int(rng.integers(1, 6))))
    return out


def test_admission_budget_and_completion():
    reqs = trace(200)
    sizes = {r.rid: int(s) for r, s in zip(reqs, np.random.default_rng(1).integers(1, 10, len(reqs)))}
    srv = FakeServer(sizes, budget_bytes=25, max_active=6)
    rep = srv.run_trace(reqs, realtime=False)
    assert rep["requests"] == 200 and not srv.queue and not srv.active
    assert srv.peak_mem <= 25 and srv.mem_used == 0
    for r in srv.finished:
        assert r.result == dict(ok=True)
        assert r.done >= r.admitted >= r.arrival
    # a track request of n iterations stays exactly n ticks in the batches
    for r in reqs:
        if r.kind == "track":
            assert sum(r.rid in t for _, t in srv.launched) == r.iters
        else:
            assert sum(r.rid in rr for rr, _ in srv.launched) == 1
    assert rep["p50_ms"] is not None and rep["p99_ms"] >= rep["p50_ms"]


def test_fifo_admission_no_starvation():
    reqs = trace(50, seed=3)
    sizes = {r.rid: (20 if r.rid == 5 else 1) for r in reqs}   # one large request
    srv = FakeServer(sizes, budget_bytes=20, max_active=8)
    srv.run_trace(reqs, realtime=False)
    by_rid = sorted(srv.finished, key=lambda r: r.rid)
    # FIFO: a request is never admitted before one that arrived earlier
    assert all(a.admitted <= b.admitted for a, b in zip(by_rid, by_rid[1:]))
    # the large request waited for the budget but was served (no starvation)
    assert any(r.rid == 5 for r in srv.finished)
