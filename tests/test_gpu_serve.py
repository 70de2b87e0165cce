"""Serving on the GPU: concurrent requests as asynchronous solves on their
own streams, problem reuse (same medium: every factor; new medium: in-place
re-factorisation of the changed subdomains only), the budget never exceeded
by the library context, and each result the same alone and in the mix."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1605_04521_amd import _lib as B
from paper_1605_04521_amd import gen
from paper_1605_04521_amd.serve import GpuBackend, Request, Server

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def catalogue():
    return {"a": gen.chamber_problem(n=5, degree=2, n_sub=6, overlap=2),
            "b": gen.chamber_problem(n=6, degree=1, n_sub=5, overlap=1)}


def requests(cat):
    ring = gen.ring_dipoles(32, 0.14, 0.196)
    out = []
    for i in range(8):
        key = "a" if i % 3 else "b"
        eps = gen.chamber_eps(cat[key].mesh, 10 + i % 2)[0]
        srcs = ring[i:i + 1 + i % 4]
        out.append(Request(rid=i, arrival=0.02 * i, mesh=key, eps=eps, sources=srcs,
                           precision=B.MXW_MIXED if i % 2 else B.MXW_FP64))
    return out


def test_results_same_alone_and_in_the_mix():
    say("[gpu] serving: mix of 8 requests on 3 slots, then each alone")
    cat = catalogue()
    mix = requests(cat)
    budget = int(50e9)
    be = GpuBackend(cat, budget=budget, slots=3)
    Server(be, budget=budget, slots=3).run(mix, realtime=True)
    assert all(r.error is None for r in mix), [r.error for r in mix]
    assert all(np.max(r.relres) <= 1e-8 for r in mix)
    assert {"factors", "partial", "new"} >= {r.reused for r in mix}
    assert any(r.reused in ("factors", "partial") for r in mix)
    # admission's exact accounting never fell below what the library holds
    u = be.ctx.usage()
    say(f"   context peak {u['peak'] / 1e9:.2f} GB, admission max {be.max_allocated / 1e9:.2f} GB")
    assert u["peak"] <= be.max_allocated <= budget
    for r in requests(cat):
        be = GpuBackend(cat, budget=budget, slots=1)
        Server(be, budget=budget, slots=1).run([r], realtime=False)
        m = mix[r.rid]
        assert np.array_equal(r.iters, m.iters), r.rid
        assert np.array_equal(r.result, m.result), r.rid
