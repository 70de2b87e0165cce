"""Continuous-batching request loop for streams of forward solves.

An imaging inversion issues forward solves one after another, each with its
own permittivity map and a set of transmitting antennas (right-hand sides),
often on a handful of meshes.  The loop:

* admits a request when a slot is free and its device memory fits the HBM
  budget: a resident idle problem for the same mesh costs nothing, a new one
  costs its footprint; idle problems of other meshes are evicted (least
  recently used first) to make room.  Admission is re-evaluated at every
  arrival and every completion, so requests that arrive while others run
  start as soon as memory and a slot free up;
* keeps problems (device operator, LU factors, Krylov workspace) resident per
  mesh: a request whose medium equals the resident one reuses the factors
  outright; otherwise the resident problem is re-assembled and re-factorised
  in place (no device allocation);
* runs every admitted request on its own HIP stream in a worker thread, so the
  kernels of concurrent requests overlap on the device; all right-hand sides of
  a request are solved together (block GMRES, one Krylov space per request);
* records arrival, start and completion times.

The scheduling core (`Scheduler`) does not touch the GPU, so it is tested on
the CPU with a fake backend.
"""
from __future__ import annotations

import hashlib
import heapq
import threading
import time
from dataclasses import dataclass

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
    reused: str = ""             # "factors", "buffers" or "new"


def medium_key(eps: np.ndarray, k0: float) -> str:
    h = hashlib.sha256(np.ascontiguousarray(eps).tobytes())
    h.update(np.float64(k0).tobytes())
    return h.hexdigest()


@dataclass
class Plan:
    kind: str            # "reuse" or "new"
    handle: object = None
    nbytes: int = 0


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
            if plan.kind == "new":
                over = self.backend.allocated + plan.nbytes - self.budget
                if over > 0:
                    self.backend.evict_idle(over)
                if self.backend.allocated + plan.nbytes > self.budget:
                    break                          # wait for a completion
                self.backend.allocated += plan.nbytes   # reserved
            heapq.heappop(self.waiting)
            self.running += 1
            out.append((req, plan))
        return out

    def done(self):
        self.running -= 1


class GpuBackend:
    """Resident problems per mesh on one GPU (one catalogue of layouts)."""

    def __init__(self, catalogue):
        from .api import Layout
        self.catalogue = catalogue       # mesh key -> gen.Problem (mesh, partition, k0, degree)
        self.layouts = {k: Layout.from_problem(p) for k, p in catalogue.items()}
        self.idle = []                   # (last use, mesh, precision, medium key, problem, nbytes)
        self.allocated = 0
        self.lock = threading.Lock()
        self.clock = 0

    def footprint(self, req) -> int:
        return self.layouts[req.mesh].footprint(req.precision, len(req.sources))

    def plan(self, req) -> Plan:
        key = medium_key(req.eps, self.catalogue[req.mesh].k0)
        with self.lock:
            cand = [i for i, e in enumerate(self.idle) if e[1] == req.mesh and e[2] == req.precision]
            same = [i for i in cand if self.idle[i][3] == key]
            pick = same[0] if same else (cand[0] if cand else None)
            if pick is None:
                return Plan("new", nbytes=self.footprint(req))
            e = self.idle.pop(pick)
            return Plan("reuse", handle=e)

    def evict_idle(self, nbytes: int) -> int:
        freed = 0
        with self.lock:
            self.idle.sort(key=lambda e: e[0])
            while self.idle and freed < nbytes:
                e = self.idle.pop(0)
                e[4].close()
                freed += e[5]
                self.allocated -= e[5]
        return freed

    def run(self, req, plan: Plan):
        """Acquire (reuse / re-factorise / create), solve, return to the pool."""
        import torch
        from . import _lib as B
        from .api import Problem
        base = self.catalogue[req.mesh]
        key = medium_key(req.eps, base.k0)
        if plan.kind == "reuse":
            _, _, _, mkey, P, nbytes = plan.handle
            if mkey == key:
                req.reused = "factors"
            else:
                P.set_medium(req.eps, base.k0)
                req.reused = "buffers"
        else:
            nbytes = plan.nbytes
            req.reused = "new"
            P = Problem.from_layout(self.layouts[req.mesh], eps=req.eps, k0=base.k0, precision=req.precision)
        try:
            # one shared block Krylov space for the request's sources (at most
            # 32; the block method needs fewer steps than one space per source)
            krylov = B.MXW_KRYLOV_BLOCK if len(req.sources) <= 32 else B.MXW_KRYLOV_PSEUDOBLOCK
            x, it, rr, st = P.solve(req.sources, allow_notconv=True, krylov=krylov)
            torch.cuda.current_stream().synchronize()
            req.result, req.iters, req.relres = x.cpu().numpy(), it, rr
        finally:
            with self.lock:
                self.clock += 1
                self.idle.append((self.clock, req.mesh, req.precision, key, P, nbytes))


class Server:
    """Replays a request stream against a backend with continuous batching."""

    def __init__(self, backend, budget: int, slots: int = 4, use_streams: bool = True):
        self.backend = backend
        self.sched = Scheduler(backend, budget, slots)
        self.use_streams = use_streams
        self.cv = threading.Condition()

    def _worker(self, req, plan, t0):
        req.start = time.perf_counter() - t0
        try:
            if self.use_streams:
                import torch
                with torch.cuda.stream(torch.cuda.Stream()):
                    self.backend.run(req, plan)
            else:
                self.backend.run(req, plan)
        except Exception as e:     # one failing request must not stop the loop
            req.error = repr(e)
        req.finish = time.perf_counter() - t0
        with self.cv:
            self.sched.done()
            self.cv.notify_all()

    def run(self, requests, realtime: bool = True):
        """Returns the wall time of the run."""
        t0 = time.perf_counter()
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        if not realtime:
            for r in pending:
                r.arrival = 0.0
        threads = []
        i = 0
        with self.cv:
            while True:
                now = time.perf_counter() - t0
                while i < len(pending) and pending[i].arrival <= now:
                    self.sched.submit(pending[i])
                    i += 1
                for req, plan in self.sched.admit():
                    th = threading.Thread(target=self._worker, args=(req, plan, t0), daemon=True)
                    th.start()
                    threads.append(th)
                if i >= len(pending) and not self.sched.waiting and self.sched.running == 0:
                    break
                wait = 0.05
                if i < len(pending):
                    wait = min(wait, max(0.0, pending[i].arrival - (time.perf_counter() - t0)))
                self.cv.wait(timeout=wait)
        for th in threads:
            th.join()
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
