"""Request loop logic on the CPU with a fake backend: admission by memory and
slots, arrival order, overlap of concurrent requests, reuse and eviction of
resident problems, growth of a reused problem's workspace, isolation of
failing requests (also when the problem cannot be created)."""
import time

import numpy as np
import pytest

from paper_1605_04521_amd.serve import Plan, Request, Resident, Scheduler, Server, latency_stats, medium_key, \
    poisson_arrivals


class FakeBackend:
    """Problem bytes = base[mesh] + per_src * sources (held after the solve);
    a solve takes `delay` seconds of wall time."""

    def __init__(self, base, per_src=0, temp=0, delay=0.05, fail=(), fail_create=()):
        self.base, self.per_src, self.temp = base, per_src, temp
        self.delay = delay
        self.fail = set(fail)
        self.fail_create = set(fail_create)
        self.allocated = 0
        self.max_allocated = 0
        self.true_max = 0          # what the fake device really held at most
        self.held_now = 0
        self.idle = []
        self.active = 0
        self.max_active = 0
        self.started = []
        self.evicted = []
        self.clock = 0

    def held_for(self, req, old=0):
        return max(old, self.base[req.mesh] + self.per_src * len(req.sources))

    def footprint(self, req):
        return self.held_for(req) + self.temp

    def plan(self, req):
        key = medium_key(req.eps, 1.0)
        cand = [e for e in self.idle if e.mesh == req.mesh]
        same = [e for e in cand if e.key == key]
        pick = same[0] if same else (cand[0] if cand else None)
        if pick is None:
            return Plan("new", nbytes=self.footprint(req))
        return Plan("reuse", entry=pick, nbytes=max(0, self.held_for(req) - pick.held) + self.temp)

    def take(self, plan):
        if plan.entry is not None:
            self.idle.remove(plan.entry)

    def evict_idle(self, nbytes, keep=None):
        freed = 0
        self.idle.sort(key=lambda e: e.last_use)
        for e in [e for e in self.idle if e is not keep]:
            if freed >= nbytes:
                break
            self.idle.remove(e)
            self.evicted.append(e.mesh)
            freed += e.held
            self.allocated -= e.held
            self.held_now -= e.held
        return freed

    def start(self, req, run):
        plan = run["plan"]
        run["key"] = medium_key(req.eps, 1.0)
        self.active += 1
        self.max_active = max(self.max_active, self.active)
        self.started.append(req.rid)
        if plan.kind == "reuse":
            run["P"], run["old"] = plan.entry.problem, plan.entry.held
            req.reused = "factors" if plan.entry.key == run["key"] else "partial"
        else:
            if req.rid in self.fail_create:
                self.active -= 1
                raise RuntimeError("forced failure at creation")
            run["P"], run["old"] = object(), 0
            req.reused = "new"
        run["held"] = self.held_for(req, run["old"])
        self.held_now += run["held"] - run["old"] + self.temp
        self.true_max = max(self.true_max, self.held_now)
        run["end"] = time.perf_counter() + self.delay

    def poll(self, run):
        return time.perf_counter() >= run["end"]

    def finish(self, req, run):
        self.active -= 1
        self.held_now -= self.temp
        if req.rid in self.fail:
            raise RuntimeError("forced failure")
        req.result = np.full(3, float(req.rid))

    def release(self, req, run):
        plan = run["plan"]
        held = run.get("held", 0) if run.get("P") is not None else 0
        self.allocated += held - run.get("old", 0) - (plan.nbytes - plan.copy_bytes)
        if run.get("P") is not None:
            self.clock += 1
            self.idle.append(Resident(req.mesh, 0, run["key"] if req.error is None else "", run["P"], held,
                                      self.clock))


def make(rid, mesh="a", arrival=0.0, eps=0.0, nsrc=1):
    return Request(rid=rid, arrival=arrival, mesh=mesh, eps=np.array([eps + 1j]), sources=[object()] * nsrc)


def test_budget_and_slots_respected():
    be = FakeBackend({"a": 40, "b": 70})
    reqs = [make(i, "a" if i % 2 else "b", 0.0, eps=i) for i in range(10)]
    Server(be, budget=120, slots=3).run(reqs, realtime=False)
    assert be.max_allocated <= 120 and be.true_max <= 120
    assert be.max_active <= 3
    assert all(r.error is None for r in reqs)


def test_concurrent_requests_overlap_and_keep_order():
    be = FakeBackend({"a": 10}, delay=0.1)
    reqs = [make(i, "a", 0.0, eps=i) for i in range(4)]
    t = Server(be, budget=100, slots=4).run(reqs, realtime=False)
    assert be.max_active >= 2
    assert t < 4 * 0.1
    assert be.started == sorted(be.started)


def test_reuse_and_eviction():
    be = FakeBackend({"a": 60, "b": 60}, delay=0.01)
    r1 = make(1, "a", 0.00, eps=1)
    r2 = make(2, "a", 0.05, eps=1)      # same mesh, same medium -> factors reused
    r3 = make(3, "a", 0.10, eps=2)      # same mesh, new medium -> partly re-factorised in place
    r4 = make(4, "b", 0.15, eps=1)      # other mesh: needs room -> evicts 'a'
    Server(be, budget=100, slots=1).run([r1, r2, r3, r4], realtime=True)
    assert [r.reused for r in (r1, r2, r3, r4)] == ["new", "factors", "partial", "new"]
    assert be.evicted == ["a"]
    assert be.true_max <= 100


def test_reused_problem_growing_workspace_is_charged():
    """A problem made for 1 source and reused by a 32-source request grows its
    Krylov workspace: the growth is charged at admission, so under a tight
    budget the 32-source request waits for an eviction instead of exceeding
    the budget, and the idle entry then records the larger size."""
    be = FakeBackend({"a": 50, "b": 50}, per_src=2, temp=4, delay=0.01)
    r1 = make(1, "a", 0.00, eps=1, nsrc=1)       # holds 52
    r2 = make(2, "b", 0.00, eps=1, nsrc=1)       # holds 52
    r3 = make(3, "a", 0.10, eps=1, nsrc=32)      # reuse of 'a' needs 114: 62 more + 4 temporaries
    Server(be, budget=160, slots=2).run([r1, r2, r3], realtime=True)
    assert all(r.error is None for r in (r1, r2, r3))
    assert r3.reused == "factors"
    assert be.true_max <= 160 and be.max_allocated <= 160
    assert be.evicted == ["b"]
    held = {e.mesh: e.held for e in be.idle}
    assert held == {"a": 114}
    assert be.allocated == 114


def test_failing_request_does_not_stop_the_loop():
    be = FakeBackend({"a": 10}, delay=0.01, fail={2})
    reqs = [make(i, "a", 0.0, eps=i) for i in range(5)]
    Server(be, budget=100, slots=2).run(reqs, realtime=False)
    assert reqs[2].error is not None
    assert all(r.error is None for r in reqs if r.rid != 2)
    st = latency_stats(reqs)
    assert st["failed"] == 1 and st["requests"] == 4


def test_failed_creation_releases_its_reservation():
    be = FakeBackend({"a": 30, "b": 40}, delay=0.01, fail_create={0})
    reqs = [make(0, "b", 0.0), make(1, "a", 0.0)]
    Server(be, budget=100, slots=2).run(reqs, realtime=False)
    assert reqs[0].error is not None and "creation" in reqs[0].error
    assert reqs[1].error is None
    # only the successful request's problem is held
    assert be.allocated == 30 and [e.mesh for e in be.idle] == ["a"]


def test_request_larger_than_budget_rejected():
    be = FakeBackend({"a": 500})
    with pytest.raises(ValueError):
        Server(be, budget=100, slots=1).run([make(0)], realtime=False)


def test_poisson_arrivals_mean_gap():
    a = poisson_arrivals(4000, 4.0, 0)
    assert np.all(np.diff(a) > 0)
    assert abs(np.mean(np.diff(a)) - 0.25) < 0.02
