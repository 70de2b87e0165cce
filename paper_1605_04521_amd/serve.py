"""Continuous-batching request loop for streams of forward solves.

An imaging inversion issues forward solves one after another, each with its
own permittivity map and a set of transmitting antennas (right-hand sides),
often on a handful of meshes, and with media that differ mostly inside the
imaged head (Sec. 6: slowly varying systems).  The loop:

* admits a request when a slot is free and its device memory fits the HBM
  budget.  A new problem is charged its exact footprint (operator, factors,
  Krylov workspace for the request's sources, solve temporaries, plus the
  mesh's shared device copy the first time); a resident idle problem on the
  same mesh is charged only what the request needs beyond the bytes it
  already holds (a larger source count grows its Krylov workspace).  Idle
  problems are evicted, least recently used first, to make room.  Admission
  is re-evaluated at every arrival and every completion;
* keeps problems (device operator, LU factors, Krylov workspace) resident per
  mesh: a request with the resident medium reuses every factor; a new medium
  is assembled in place and only the subdomains whose local data changed are
  factorised again (the library keeps the others);
* runs every admitted request's solve as an asynchronous library call (a
  ticket) on its own HIP stream, so the kernels of concurrent requests overlap
  on the device; all right-hand sides of a request share one block Krylov
  space (at most 32 of them);
* records arrival, start and completion times and, once a request has
  finished, corrects the budget with the bytes its problem really holds.

The scheduling core (`Scheduler`, `Server`) does not touch the GPU, so it is
tested on the CPU with a fake backend.
"""
from __future__ import annotations

import hashlib
import heapq
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float               # seconds since the start of the run
    mesh: str                    # key into the mesh catalogue
    eps: np.ndarray              # complex128 [n_tets]
    sources: list
    precision: int = 0
    # filled by the server
    start: float = None
    finish: float = None
    result: object = None
    iters: object = None
    relres: object = None
    error: str = None
    reused: str = ""             # "factors" (same medium), "partial" (new medium, some factors kept) or "new"
    refactored: tuple = None     # (subdomains factorised for this request, subdomains)


def medium_key(eps: np.ndarray, k0: float) -> str:
    h = hashlib.sha256(np.ascontiguousarray(eps).tobytes())
    h.update(np.float64(k0).tobytes())
    return h.hexdigest()


@dataclass
class Resident:
    """A problem kept on the device between requests."""
    mesh: str
    precision: int
    key: str                     # medium key its factors were made for
    problem: object
    held: int                    # device bytes it holds (operator, factors, workspaces)
    last_use: int = 0


@dataclass
class Plan:
    kind: str                    # "reuse" or "new"
    entry: Resident = None       # the idle problem to reuse
    nbytes: int = 0              # bytes to reserve on admission
    copy_bytes: int = 0          # part of nbytes that is the mesh's shared device copy


class Scheduler:
    """Slots + device-memory admission; requests start in arrival order."""

    def __init__(self, backend, budget: int, slots: int):
        self.backend = backend
        self.budget = budget
        self.slots = slots
        self.running = 0
        self.waiting = []          # heap of (arrival, rid, request)

    def submit(self, req):
        if self.backend.footprint(req) > self.budget:
            raise ValueError(f"request {req.rid} can never fit the budget of {self.budget} bytes")
        heapq.heappush(self.waiting, (req.arrival, req.rid, req))

    def admit(self):
        out = []
        while self.waiting and self.running < self.slots:
            req = self.waiting[0][2]
            plan = self.backend.plan(req)
            over = self.backend.allocated + plan.nbytes - self.budget
            if over > 0:
                self.backend.evict_idle(over, keep=plan.entry)
            if self.backend.allocated + plan.nbytes > self.budget:
                break                              # wait for a completion
            self.backend.take(plan)
            self.backend.allocated += plan.nbytes  # reserved
            self.backend.max_allocated = max(self.backend.max_allocated, self.backend.allocated)
            heapq.heappop(self.waiting)
            self.running += 1
            out.append((req, plan))
        return out

    def done(self):
        self.running -= 1


class GpuBackend:
    """Resident problems per mesh on one GPU, all allocated through one
    library context whose budget is the loop's (the library refuses what
    admission would have let through by mistake), straight from hipMalloc."""

    def __init__(self, catalogue, budget: int = 0, slots: int = 4):
        import torch
        from .api import Context, Layout
        self.catalogue = catalogue       # mesh key -> gen.Problem (mesh, partition, k0, degree)
        self.layouts = {k: Layout.from_problem(p) for k, p in catalogue.items()}
        # hipMalloc / hipFree per allocation: problems of very different sizes
        # come and go, and memory returned to a caching allocator stays split
        # among its cached segments (a later large request then fails although
        # the budget has room)
        self.ctx = Context(budget=budget, allocator="hip")
        self.idle = []                   # Resident
        self.copies = set()              # meshes whose shared device copy is counted
        self.allocated = 0
        self.max_allocated = 0
        self.lock = threading.Lock()
        self.clock = 0
        self.streams = [torch.cuda.Stream() for _ in range(max(1, slots))]
        self.free_streams = list(self.streams)

    @staticmethod
    def _krylov(req):
        from . import _lib as B
        return B.MXW_KRYLOV_BLOCK if len(req.sources) <= 32 else B.MXW_KRYLOV_PSEUDOBLOCK

    def need(self, req) -> int:
        """Bytes of a problem for this request, without the mesh's copy."""
        return self.layouts[req.mesh].footprint(req.precision, len(req.sources), krylov=self._krylov(req),
                                                with_layout_copy=False)

    def temp_bytes(self, req) -> int:
        """The solve's temporaries inside need(req): right-hand sides, the
        solution, face integrals (see mxw_layout_footprint)."""
        info = self.layouts[req.mesh].info()
        nfloc = {1: 3, 2: 8, 3: 15}[self.catalogue[req.mesh].degree]
        return 2 * 16 * info.ndof * len(req.sources) + 16 * max(1, info.n_imp_faces * nfloc)

    def copy_bytes(self, mesh) -> int:
        lay = self.layouts[mesh]
        return lay.footprint(0, 1) - lay.footprint(0, 1, with_layout_copy=False)

    def footprint(self, req) -> int:
        return self.need(req) + self.copy_bytes(req.mesh)

    def plan(self, req) -> Plan:
        key = medium_key(req.eps, self.catalogue[req.mesh].k0)
        with self.lock:
            cand = [e for e in self.idle if e.mesh == req.mesh and e.precision == req.precision]
            same = [e for e in cand if e.key == key]
            pick = same[0] if same else (cand[0] if cand else None)
        if pick is None:
            copy = 0 if req.mesh in self.copies else self.copy_bytes(req.mesh)
            return Plan("new", nbytes=self.need(req) + copy, copy_bytes=copy)
        # what the resident problem lacks (a larger Krylov workspace), plus the
        # solve's temporaries
        temp = self.temp_bytes(req)
        return Plan("reuse", entry=pick, nbytes=max(0, self.need(req) - temp - pick.held) + temp)

    def take(self, plan: Plan):
        with self.lock:
            if plan.entry is not None:
                self.idle.remove(plan.entry)

    def evict_idle(self, nbytes: int, keep=None) -> int:
        freed = 0
        with self.lock:
            self.idle.sort(key=lambda e: e.last_use)
            for e in [e for e in self.idle if e is not keep]:
                if freed >= nbytes:
                    break
                self.idle.remove(e)
                e.problem.close()
                freed += e.held
                self.allocated -= e.held
        return freed

    def start(self, req, run: dict):
        """Acquire the problem (reuse, new medium in place, or create) and start
        the request's solve as a ticket on a stream of its own.  run (made by
        the server with the plan) records what was acquired, also when this
        raises."""
        from .api import Problem
        plan = run["plan"]
        base = self.catalogue[req.mesh]
        key = medium_key(req.eps, base.k0)
        run["key"] = key
        if plan.kind == "new":
            self.copies.add(req.mesh)
            run["P"] = Problem.from_layout(self.layouts[req.mesh], eps=req.eps, k0=base.k0,
                                           precision=req.precision, ctx=self.ctx)
            req.reused = "new"
            n_sub = base.n_sub
            req.refactored = (n_sub, n_sub)
        else:
            P = plan.entry.problem
            run["P"], run["old"] = P, plan.entry.held
            if plan.entry.key == key:
                req.reused = "factors"
                req.refactored = (0, base.n_sub)
            else:
                P.set_medium(req.eps, base.k0)
                req.reused = "partial"
                req.refactored = (P.factor_stats()["refactored_last"], base.n_sub)
        run["stream"] = self.free_streams.pop() if self.free_streams else self.streams[0]
        run["ticket"] = run["P"].solve_async(req.sources, krylov=self._krylov(req), stream=run["stream"])

    def poll(self, run) -> bool:
        return run["ticket"].done()

    def release(self, req, run):
        """Return the problem to the idle pool and settle the reservation with
        the bytes it really holds now."""
        P, plan = run.get("P"), run["plan"]
        held = P.device_bytes() if P is not None else 0
        with self.lock:
            # the mesh copy stays counted (it lives as long as the layout)
            self.allocated += held - run.get("old", 0) - (plan.nbytes - plan.copy_bytes)
            if P is not None:
                self.clock += 1
                key = run["key"] if req.error is None else ""     # a failed request's medium is not trusted
                self.idle.append(Resident(req.mesh, req.precision, key, P, held, self.clock))
        if run.get("stream") is not None and run["stream"] not in self.free_streams:
            self.free_streams.append(run["stream"])

    def finish(self, req, run):
        x, it, rr, st = run["ticket"].wait(allow_notconv=True)
        req.result, req.iters, req.relres = x.cpu().numpy(), it, rr


class Server:
    """Replays a request stream against a backend with continuous batching:
    one host loop admits requests, starts their solves asynchronously and
    collects them as they complete."""

    def __init__(self, backend, budget: int, slots: int = 4, poll_s: float = 0.002, on_finish=None):
        self.backend = backend
        self.sched = Scheduler(backend, budget, slots)
        self.poll_s = poll_s
        self.on_finish = on_finish       # called with each request as it completes (or fails)

    def run(self, requests, realtime: bool = True, deadline: float = None):
        """Returns the wall time of the run.  deadline (seconds): requests not
        started by then are left unserved (error set); running ones finish."""
        t0 = time.perf_counter()
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        if not realtime:
            for r in pending:
                r.arrival = 0.0
        running = []
        i = 0
        while True:
            now = time.perf_counter() - t0
            if deadline is not None and now > deadline:
                for r in pending[i:]:
                    r.error = "arrived after the end of the run"
                for _, _, r in self.sched.waiting:
                    r.error = "not started before the end of the run"
                i = len(pending)
                self.sched.waiting = []
            while i < len(pending) and pending[i].arrival <= now:
                self.sched.submit(pending[i])
                i += 1
            for req, plan in self.sched.admit():
                req.start = time.perf_counter() - t0
                run = {"plan": plan}
                try:
                    self.backend.start(req, run)
                    running.append((req, run))
                except Exception as e:          # one failing request must not stop the loop
                    req.error = repr(e)
                    req.finish = time.perf_counter() - t0
                    self.backend.release(req, run)
                    self.sched.done()
                    if self.on_finish:
                        self.on_finish(req)
            still = []
            for req, run in running:
                if not self.backend.poll(run):
                    still.append((req, run))
                    continue
                try:
                    self.backend.finish(req, run)
                except Exception as e:
                    req.error = repr(e)
                req.finish = time.perf_counter() - t0
                self.backend.release(req, run)
                self.sched.done()
                if self.on_finish:
                    self.on_finish(req)
            running = still
            if i >= len(pending) and not self.sched.waiting and not running:
                break
            wait = self.poll_s
            if i < len(pending) and not running:
                wait = max(wait, pending[i].arrival - (time.perf_counter() - t0))
            time.sleep(min(wait, 0.05))
        return time.perf_counter() - t0


def latency_stats(requests):
    ok = [r for r in requests if r.error is None]
    lat = np.array([r.finish - r.arrival for r in ok])
    nrhs = sum(len(r.sources) for r in ok)
    span = max(r.finish for r in requests) - min(r.arrival for r in requests)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "solves_per_s": nrhs / span, "requests": len(ok), "failed": len(requests) - len(ok),
            "span_s": span}


def poisson_arrivals(n: int, rate: float, seed: int):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
