"""Request loop logic on the CPU with a fake backend: admission by memory and
slots, arrival order, overlap of concurrent requests, reuse and eviction of
resident problems, isolation of failing requests."""
import threading
import time

import numpy as np
import pytest

from paper_1605_04521_amd.serve import Plan, Request, Server, latency_stats, medium_key, poisson_arrivals


class FakeBackend:
    def __init__(self, sizes, delay=0.05, fail=()):
        self.sizes = sizes
        self.delay = delay
        self.fail = set(fail)
        self.allocated = 0
        self.max_allocated = 0
        self.idle = []
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.started = []
        self.evicted = []

    def footprint(self, req):
        return self.sizes[req.mesh]

    def plan(self, req):
        key = medium_key(req.eps, 1.0)
        with self.lock:
            for i, e in enumerate(self.idle):
                if e[0] == req.mesh:
                    return Plan("reuse", handle=self.idle.pop(i))
        return Plan("new", nbytes=self.sizes[req.mesh])

    def evict_idle(self, nbytes):
        freed = 0
        with self.lock:
            while self.idle and freed < nbytes:
                e = self.idle.pop(0)
                self.evicted.append(e[0])
                freed += e[2]
                self.allocated -= e[2]
        return freed

    def run(self, req, plan):
        key = medium_key(req.eps, 1.0)
        with self.lock:
            self.max_allocated = max(self.max_allocated, self.allocated)
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.started.append(req.rid)
        if plan.kind == "reuse":
            req.reused = "factors" if plan.handle[1] == key else "buffers"
            nbytes = plan.handle[2]
        else:
            req.reused = "new"
            nbytes = plan.nbytes
        try:
            time.sleep(self.delay)
            if req.rid in self.fail:
                raise RuntimeError("forced failure")
            req.result = np.full(3, float(req.rid))
        finally:
            with self.lock:
                self.active -= 1
                self.idle.append((req.mesh, key, nbytes))


def make(rid, mesh="a", arrival=0.0, eps=0.0):
    return Request(rid=rid, arrival=arrival, mesh=mesh, eps=np.array([eps + 1j]), sources=[object()])


def test_budget_and_slots_respected():
    be = FakeBackend({"a": 40, "b": 70})
    reqs = [make(i, "a" if i % 2 else "b", 0.0, eps=i) for i in range(10)]
    Server(be, budget=120, slots=3, use_streams=False).run(reqs, realtime=False)
    assert be.max_allocated <= 120
    assert be.max_active <= 3
    assert all(r.error is None for r in reqs)


def test_concurrent_requests_overlap_and_keep_order():
    be = FakeBackend({"a": 10}, delay=0.1)
    reqs = [make(i, "a", 0.0, eps=i) for i in range(4)]
    t = Server(be, budget=100, slots=4, use_streams=False).run(reqs, realtime=False)
    assert be.max_active >= 2
    assert t < 4 * 0.1
    assert be.started == sorted(be.started)


def test_reuse_and_eviction():
    be = FakeBackend({"a": 60, "b": 60}, delay=0.01)
    r1 = make(1, "a", 0.00, eps=1)
    r2 = make(2, "a", 0.05, eps=1)      # same mesh, same medium -> factors reused
    r3 = make(3, "a", 0.10, eps=2)      # same mesh, new medium -> buffers reused
    r4 = make(4, "b", 0.15, eps=1)      # other mesh: needs room -> evicts 'a'
    Server(be, budget=100, slots=1, use_streams=False).run([r1, r2, r3, r4], realtime=True)
    assert [r.reused for r in (r1, r2, r3, r4)] == ["new", "factors", "buffers", "new"]
    assert be.evicted == ["a"]


def test_failing_request_does_not_stop_the_loop():
    be = FakeBackend({"a": 10}, delay=0.01, fail={2})
    reqs = [make(i, "a", 0.0, eps=i) for i in range(5)]
    Server(be, budget=100, slots=2, use_streams=False).run(reqs, realtime=False)
    assert reqs[2].error is not None
    assert all(r.error is None for r in reqs if r.rid != 2)
    st = latency_stats(reqs)
    assert st["failed"] == 1 and st["requests"] == 4


def test_request_larger_than_budget_rejected():
    be = FakeBackend({"a": 500})
    with pytest.raises(ValueError):
        Server(be, budget=100, slots=1, use_streams=False).run([make(0)], realtime=False)


def test_poisson_arrivals_mean_gap():
    a = poisson_arrivals(4000, 4.0, 0)
    assert np.all(np.diff(a) > 0)
    assert abs(np.mean(np.diff(a)) - 0.25) < 0.02
