"""Contexts (device memory through the caller's allocator, HBM budget),
exact device footprints and asynchronous solves with tickets, through the
C ABI.

The serving loop admits forward solves by their device footprint, so the
footprint must be exact: every allocation of a problem goes through its
context, which counts the bytes in use and their peak; the peak over
create + solve must equal the footprint up to the plane-wave face-integral
buffer that dipole sources do not need.
"""
import gc
import sys
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1605_04521_amd import _lib as B
from paper_1605_04521_amd import gen
from paper_1605_04521_amd.api import Context, Layout, Problem

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision,krylov,nrhs,variant", [
    (B.MXW_MIXED, B.MXW_KRYLOV_BLOCK, 32, B.MXW_PREC_ORAS),
    (B.MXW_FP64, B.MXW_KRYLOV_PSEUDOBLOCK, 32, B.MXW_PREC_ORAS),
    (B.MXW_MIXED, B.MXW_KRYLOV_PSEUDOBLOCK, 3, B.MXW_PREC_ORAS),
    (B.MXW_FP64, B.MXW_KRYLOV_PSEUDOBLOCK, 2, B.MXW_PREC_OAS),
])
def test_footprint_equals_measured_peak(precision, krylov, nrhs, variant):
    prob = gen.chamber_problem(n=6, degree=2, n_sub=9, overlap=2, n_sources=nrhs)
    say(f"[gpu] footprint vs measured peak precision={precision} krylov={krylov} nrhs={nrhs} variant={variant}")
    lay = Layout.from_problem(prob)
    ctx = Context()
    torch.cuda.synchronize()
    alloc0 = torch.cuda.memory_allocated()
    P = Problem.from_layout(lay, eps=prob.eps, k0=prob.k0, precision=precision, variant=variant, ctx=ctx)
    E, it, rr, st = P.solve_host(prob.sources, krylov=krylov)
    torch.cuda.synchronize()
    u = ctx.usage()
    fp = lay.footprint(precision, nrhs, krylov=krylov, variant=variant)
    face = max(1, lay.info().n_imp_faces * {1: 3, 2: 8, 3: 15}[prob.degree]) * 16
    say(f"   footprint {fp} B, peak {u['peak']} B, in use after {u['in_use']} B, torch {torch.cuda.max_memory_allocated() - alloc0} B")
    assert np.all(rr <= 1e-8)
    # exact: the dipole sources need no face-integral buffer
    assert u["peak"] == fp - face
    # held after the solve: everything but the solve's temporaries (right-hand
    # sides and solution staging); the problem itself holds all but the
    # layout's shared copy
    assert u["in_use"] == fp - 2 * 16 * nrhs * P.ndof - face
    copy = fp - lay.footprint(precision, nrhs, krylov=krylov, variant=variant, with_layout_copy=False)
    assert P.device_bytes() == u["in_use"] - copy
    # the same memory seen by PyTorch's allocator (512-byte blocks)
    held = torch.cuda.memory_allocated() - alloc0
    assert u["in_use"] <= held <= 1.05 * u["in_use"]
    P.close()
    del P, lay          # the layout's device copy goes with the last of them
    gc.collect()
    torch.cuda.synchronize()
    assert ctx.usage()["in_use"] == 0 and ctx.usage()["live"] == 0
    ctx.close()


def test_budget_rejects_before_allocating():
    prob = gen.chamber_problem(n=6, degree=2, n_sub=9, overlap=2, n_sources=4)
    say("[gpu] context budget")
    lay = Layout.from_problem(prob)
    need = lay.footprint(B.MXW_MIXED, 4, krylov=B.MXW_KRYLOV_BLOCK)
    op = need - (lay.footprint(B.MXW_MIXED, 4, krylov=B.MXW_KRYLOV_BLOCK, with_layout_copy=False)
                 - lay.footprint(B.MXW_MIXED, 1, with_layout_copy=False))
    # not even the operator fits: nothing is allocated
    small = Context(budget=op // 4)
    with pytest.raises(B.MxwError) as e:
        Problem.from_layout(lay, precision=B.MXW_MIXED, ctx=small)
    assert e.value.status == B.MXW_ENOMEM
    assert small.usage()["in_use"] == 0
    # the operator and a pseudo-block solve of the 4 sources fit, the block
    # workspace does not: the block solve fails with MXW_ENOMEM and the
    # problem stays usable
    mid = Context(budget=lay.footprint(B.MXW_MIXED, 4))
    assert lay.footprint(B.MXW_MIXED, 4) < need
    P = Problem.from_layout(lay, precision=B.MXW_MIXED, ctx=mid)
    with pytest.raises(B.MxwError) as e:
        P.solve_host(prob.sources, krylov=B.MXW_KRYLOV_BLOCK)
    assert e.value.status == B.MXW_ENOMEM
    assert mid.usage()["peak"] <= lay.footprint(B.MXW_MIXED, 4)
    E, it, rr, st = P.solve_host(prob.sources)
    assert np.all(rr <= 1e-8)
    # a context with memory still held cannot be destroyed
    with pytest.raises(B.MxwError) as e:
        mid.close()
    assert e.value.status == B.MXW_EBUSY
    P.close()
    del P, lay
    gc.collect()
    mid.close()


def test_async_tickets_overlap_and_match_sync():
    """Two problems on one layout (different media), each solving on its own
    stream through a ticket, a third ticket queued behind the first on the
    same problem: every result equals the synchronous solve bit for bit."""
    p1 = gen.chamber_problem(n=6, degree=2, n_sub=9, overlap=2, n_sources=4, seed=1)
    p2 = gen.chamber_problem(n=6, degree=2, n_sub=9, overlap=2, n_sources=4, seed=2)
    say("[gpu] asynchronous solves")
    lay = Layout.from_problem(p1)
    A = Problem.from_layout(lay, eps=p1.eps, k0=p1.k0, precision=B.MXW_MIXED)
    Bp = Problem.from_layout(lay, eps=p2.eps, k0=p2.k0, precision=B.MXW_MIXED)
    ref_a = A.solve(p1.sources, krylov=B.MXW_KRYLOV_BLOCK)
    ref_b = Bp.solve(p2.sources[:2])
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ta = A.solve_async(p1.sources, krylov=B.MXW_KRYLOV_BLOCK, stream=sa)
    tb = Bp.solve_async(p2.sources[:2], stream=sb)
    tc = A.solve_async(p1.sources[:1], stream=sb)       # waits for ta (same problem)
    polls = 0
    while not (ta.done() and tb.done() and tc.done()):
        polls += 1
        threading.Event().wait(0.005)
    xa, ita, rra, _ = ta.wait()
    xb, itb, rrb, _ = tb.wait()
    xc, itc, rrc, _ = tc.wait()
    torch.cuda.synchronize()
    say(f"   polled {polls} times; steps {ita[0]} / {itb.tolist()} / {itc[0]}")
    assert torch.equal(xa, ref_a[0]) and np.array_equal(ita, ref_a[1])
    assert torch.equal(xb, ref_b[0]) and np.array_equal(itb, ref_b[1])
    ref_c = A.solve(p1.sources[:1])
    assert torch.equal(xc, ref_c[0])
    # an invalid request fails at once, without a ticket
    with pytest.raises(B.MxwError):
        A.solve_async([], stream=sa)
