"""Pins of the oracle's Block GCRO-DR (the combination of block and
recycling strategies Sec. 6 names for the many transmitting antennas of the
imaging loop): with one column it is GCRO-DR, without a recycled space its
first cycle is block FGMRES, the recycled space keeps its invariants, a
block of right-hand sides inside range(C) needs no block step, one cycle
gives the minimal residual over its search space (dense least squares), and
a slowly varying sequence needs fewer block steps than block FGMRES.  A
planted mistake (the recycled part of the update dropped) fails."""
import numpy as np
import pytest

import oracle.recycle as rc
from oracle.krylov import block_fgmres
from oracle.recycle import RecycleSpace, block_gcrodr, gcrodr


def rand_system(n, p, seed, shift=2.0):
    """A = shift I + G / sqrt(n) (G complex Gaussian): eigenvalues in a disc of
    radius about sqrt(2) around shift; Mi close to the identity."""
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n) + shift * np.eye(n)
    Mi = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    B = rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))
    return A, Mi, B


def ops(A, Mi):
    return (lambda V: A @ V), (lambda V: Mi @ V)


def test_one_column_is_gcrodr():
    """p = 1 over a sequence of three nearby systems: the same block steps as
    GCRO-DR's Arnoldi steps, the same solutions and the same recycled space."""
    A0, Mi, _ = rand_system(80, 1, 2)
    rng = np.random.default_rng(5)
    s1, s2 = RecycleSpace(5), RecycleSpace(5)
    for i in range(3):
        A = A0 + 0.05 * i * np.diag(rng.standard_normal(80))
        b = rng.standard_normal(80) + 1j * rng.standard_normal(80)
        mv, pc = ops(A, Mi)
        X1, it1, rr1, ok1 = block_gcrodr(mv, pc, b[:, None], s1, tol=1e-10, restart=14)
        x2, it2, rr2, ok2 = gcrodr(mv, pc, b, s2, tol=1e-10, restart=14)
        assert ok1 and ok2 and it1 == it2, (i, it1, it2)
        assert np.linalg.norm(X1[:, 0] - x2) <= 1e-9 * np.linalg.norm(x2)
        P1, P2 = s1.C @ s1.C.conj().T, s2.C @ s2.C.conj().T
        assert np.linalg.norm(P1 - P2) <= 1e-5   # eigenvector conditioning of the pencil


def test_first_cycle_is_block_fgmres():
    A, Mi, B = rand_system(90, 4, 3)
    mv, pc = ops(A, Mi)
    sp = RecycleSpace(6)
    X1, it1, _, _ = block_gcrodr(mv, pc, B, sp, tol=1e-14, restart=20, max_iters=5)
    X2, it2, _, _ = block_fgmres(mv, pc, B, tol=1e-14, restart=5, max_iters=5)
    assert it1 == it2 == 5
    assert np.linalg.norm(X1 - X2) <= 1e-11 * np.linalg.norm(X2)
    assert sp.dim == 6


def recycled_invariants(A, Mi, sp):
    C, U, Ub = sp.C, sp.U, sp.Ubar
    return (np.linalg.norm(C.conj().T @ C - np.eye(C.shape[1])),
            np.linalg.norm(A @ Ub - C) / np.linalg.norm(C),
            np.linalg.norm(Mi @ U - Ub) / np.linalg.norm(Ub))


def test_recycled_space_invariants_and_exact_range():
    A, Mi, B = rand_system(100, 3, 4)
    mv, pc = ops(A, Mi)
    sp = RecycleSpace(8)
    X, it, rr, ok = block_gcrodr(mv, pc, B, sp, tol=1e-10, restart=17)
    assert ok and np.all(rr <= 1e-10)
    e1, e2, e3 = recycled_invariants(A, Mi, sp)
    assert e1 < 1e-12 and e2 < 1e-10 and e3 < 1e-10
    # right-hand sides in range(C): solved by the projection alone
    rng = np.random.default_rng(9)
    B2 = sp.C @ (rng.standard_normal((8, 2)) + 1j * rng.standard_normal((8, 2)))
    X2, it2, rr2, ok2 = block_gcrodr(mv, pc, B2, sp, fresh_operator=False, tol=1e-10, restart=17)
    assert ok2 and it2 == 0
    assert np.linalg.norm(B2 - A @ X2) <= 1e-10 * np.linalg.norm(B2)


def one_cycle_minimal_residual_gap(monkeypatch=None):
    """After a first solve, one cycle of a second solve: its residual against
    the dense least-squares minimum over range(Ubar) + span of the cycle's
    preconditioned blocks (captured from the run)."""
    A, Mi, B = rand_system(120, 3, 6)
    mv, pc = ops(A, Mi)
    sp = RecycleSpace(6)
    block_gcrodr(mv, pc, B, sp, tol=1e-8, restart=18)
    Ub0 = sp.Ubar.copy()
    rng = np.random.default_rng(11)
    B2 = rng.standard_normal((120, 3)) + 1j * rng.standard_normal((120, 3))
    seen = []
    pc_rec = lambda V: (seen.append(Mi @ V), seen[-1])[1]
    X, it, rr, ok = block_gcrodr(mv, pc_rec, B2, sp, fresh_operator=False, tol=1e-14, restart=18, max_iters=4)
    assert it == 4
    S = np.concatenate([Ub0] + seen[:4], axis=1)
    AS = A @ S
    best = np.linalg.norm(B2 - AS @ np.linalg.lstsq(AS, B2, rcond=None)[0])
    return np.linalg.norm(B2 - A @ X) / best - 1.0


def test_one_cycle_minimal_residual():
    assert abs(one_cycle_minimal_residual_gap()) < 1e-9


def test_planted_mistake_fails_minimal_residual(monkeypatch):
    """Dropping the recycled part of the update (X += Z Y without the
    -Ubar B Y term) breaks the minimal residual property."""
    assert abs(one_cycle_minimal_residual_gap()) < 1e-9
    # the oracle's own source with the update's recycled term removed
    src = open(rc.__file__).read()
    marker = "            X = X - space.Ubar @ (Bm[:, :jd * p] @ Y)\n"
    assert marker in src
    ns = {}
    code = src.replace(marker, "            pass\n")
    exec(compile(code, rc.__file__, "exec"), rc.__dict__.copy() | {"__name__": "planted"}, ns)
    monkeypatch.setattr(rc, "block_gcrodr", ns["block_gcrodr"])
    monkeypatch.setattr(__import__(__name__), "block_gcrodr", ns["block_gcrodr"])
    assert abs(one_cycle_minimal_residual_gap()) > 1e-6


def test_fewer_block_steps_over_a_sequence():
    A0, Mi, _ = rand_system(150, 4, 7, shift=2.0)
    rng = np.random.default_rng(13)
    sp = RecycleSpace(10)
    tot_r, tot_b = 0, 0
    for i in range(4):
        A = A0 + 0.02 * i * np.diag(rng.standard_normal(150))
        B = rng.standard_normal((150, 4)) + 1j * rng.standard_normal((150, 4))
        mv, pc = ops(A, Mi)
        _, itr, rrr, okr = block_gcrodr(mv, pc, B, sp, tol=1e-9, restart=26)
        _, itb, rrb, okb = block_fgmres(mv, pc, B, tol=1e-9, restart=6)
        assert okr and okb
        if i:
            tot_r += itr
            tot_b += itb
    assert tot_r < tot_b
