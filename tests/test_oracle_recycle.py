"""Pins of the recycling oracle (GCRO-DR over a sequence of systems, the
method Sec. 6 proposes for the slowly varying systems of the imaging loop):
the first cycle is GMRES, the harmonic Ritz selection against the textbook
formula and against exact eigenvectors, the invariants of the recycled space,
exact solves inside its range, minimal residual of a cycle by brute force,
and fewer iterations over a slowly varying sequence."""
import numpy as np
import pytest
import scipy.linalg

from oracle.krylov import fgmres
from oracle.recycle import RecycleSpace, cycle_matrices, gcrodr, harmonic_ritz
from oracle.solve import OracleSolver
from paper_1605_04521_amd import gen


def rand_system(n, seed, shift=4.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + shift * np.eye(n)
    Mi = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, Mi, b


def test_first_cycle_is_gmres():
    """Without a recycled space the first cycle runs m Arnoldi steps of
    GMRES: after exactly one cycle both give the same iterate."""
    A, Mi, b = rand_system(60, 1)
    mv, pc = (lambda v: A @ v), (lambda v: Mi @ v)
    sp = RecycleSpace(4)
    x1, it1, rr1, _ = gcrodr(mv, pc, b, sp, tol=1e-14, restart=12, max_iters=12)
    x2, it2, rr2, _ = fgmres(mv, pc, b, tol=1e-14, restart=12, max_iters=12)
    assert it1 == it2 == 12
    assert np.linalg.norm(x1 - x2) <= 1e-11 * np.linalg.norm(x2)
    assert abs(rr1 - rr2) <= 1e-10 * rr2
    assert sp.dim == 4


def test_harmonic_ritz_textbook_formula():
    """With no recycled space, Gbar = Hbar and W^H Vhat = [I; 0]: the pencil's
    eigenvalues are those of H_m + |h_{m+1,m}|^2 H_m^{-H} e_m e_m^T."""
    rng = np.random.default_rng(3)
    m = 9
    Hb = np.triu(rng.standard_normal((m + 1, m)) + 1j * rng.standard_normal((m + 1, m)), -1)
    sp = RecycleSpace(3)
    V = np.zeros((m + 1, 5), complex)
    G, WV = cycle_matrices(sp, 0, m, V, Hb, np.zeros((0, m)))
    _, theta = harmonic_ritz(G, WV, 3)
    Hm = Hb[:m, :m]
    em = np.zeros(m)
    em[-1] = 1.0
    T = Hm + abs(Hb[m, m - 1]) ** 2 * np.linalg.solve(Hm.conj().T, em)[:, None] * em[None, :]
    ref = np.linalg.eigvals(T)
    assert np.allclose(np.sort_complex(theta), np.sort_complex(ref), rtol=1e-9, atol=1e-9)


def test_full_krylov_space_recycles_exact_eigenvectors():
    """With m >= n the Krylov space is the whole space, harmonic Ritz pairs
    are exact: the recycled space spans the eigenvectors of A M^{-1} of the
    k smallest eigenvalues (principal angles ~ 0)."""
    n, k = 14, 3
    rng = np.random.default_rng(5)
    lam = np.concatenate([[0.05, 0.1j, -0.2], 3 + rng.standard_normal(n - 3)])
    X = np.eye(n) + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    Ap = X @ np.diag(lam) @ np.linalg.inv(X)          # the preconditioned operator
    Mi = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    A = Ap @ np.linalg.inv(Mi)                        # so that A M^{-1} = Ap
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    sp = RecycleSpace(k)
    x, it, rr, ok = gcrodr(lambda v: A @ v, lambda v: Mi @ v, b, sp, tol=1e-13, restart=n + 1)
    assert ok and it <= n
    Qu, _ = np.linalg.qr(sp.U)
    Qx, _ = np.linalg.qr(X[:, :3])
    s = scipy.linalg.svdvals(Qu.conj().T @ Qx)
    assert np.all(s > 1 - 1e-8), s


def test_recycled_space_invariants():
    """After solves on a Maxwell ORAS system: C^H C = I, A Ubar = C and
    Ubar = M^{-1} U."""
    prob = gen.cube_planewave_problem(n=4, degree=1, box=2)
    orc = OracleSolver.from_problem(prob)
    b = orc.rhs(prob.sources[0])
    sp = RecycleSpace(6)
    x, it, rr, ok = gcrodr(lambda v: orc.A @ v, orc.prec.apply, b, sp, restart=20)
    assert ok and rr <= 1e-8
    assert np.linalg.norm(sp.C.conj().T @ sp.C - np.eye(6)) <= 1e-12
    assert np.linalg.norm(orc.A @ sp.Ubar - sp.C) <= 1e-10
    MU = np.stack([orc.prec.apply(sp.U[:, i]) for i in range(6)], axis=1)
    assert np.linalg.norm(MU - sp.Ubar) <= 1e-10 * np.linalg.norm(sp.Ubar)
    assert np.linalg.norm(orc.A @ x - b) <= 1.01e-8 * np.linalg.norm(b)


def test_rhs_in_recycled_range_needs_no_iterations():
    """b = A Ubar c lies in range(C): the projection at the start of the
    solve is the exact solution, with no Arnoldi step."""
    A, Mi, b = rand_system(50, 7)
    mv, pc = (lambda v: A @ v), (lambda v: Mi @ v)
    sp = RecycleSpace(5)
    gcrodr(mv, pc, b, sp, restart=15)
    c = np.arange(1, 6) + 1j
    b2 = A @ (sp.Ubar @ c)
    x, it, rr, ok = gcrodr(mv, pc, b2, sp, fresh_operator=False, restart=15)
    assert ok and it == 0
    assert np.linalg.norm(x - sp.Ubar @ c) <= 1e-10 * np.linalg.norm(x)


def test_cycle_minimises_residual_over_recycled_and_krylov_space():
    """One cycle with a recycled space returns the minimal residual over
    range(Ubar) + M^{-1} K_j((I - C C^H) A M^{-1}, (I - C C^H) b), the space
    built here by brute force (dense least squares)."""
    n, m, k = 40, 10, 3
    A, Mi, b0 = rand_system(n, 11, shift=2.0)
    mv, pc = (lambda v: A @ v), (lambda v: Mi @ v)
    sp = RecycleSpace(k)
    gcrodr(mv, pc, b0, sp, tol=1e-12, restart=m, max_iters=m)   # one cycle: a space
    rng = np.random.default_rng(12)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Ubar, C = sp.Ubar.copy(), sp.C.copy()
    x, it, rr, _ = gcrodr(mv, pc, b, sp, fresh_operator=False, tol=1e-14, restart=m, max_iters=m - k)
    assert it == m - k
    Pc = np.eye(n) - C @ C.conj().T
    Ap = A @ Mi
    K = [Pc @ b]
    for _ in range(m - k - 1):
        K.append(Pc @ (Ap @ K[-1]))
    S = np.concatenate([Ubar, Mi @ np.stack(K, axis=1)], axis=1)
    coef = np.linalg.lstsq(A @ S, b, rcond=None)[0]
    rmin = np.linalg.norm(b - A @ (S @ coef)) / np.linalg.norm(b)
    assert abs(rr - rmin) <= 1e-8 * rmin + 1e-14


def test_recycling_cuts_iterations_over_a_slowly_varying_sequence():
    """Three chamber systems whose media differ by 1 %: with a recycled space
    the second and third solves take fewer Arnoldi steps than GMRES with the
    same vector storage, and all reach the tolerance."""
    base = gen.chamber_problem(n=4, degree=2, n_sub=6, overlap=1)
    sp = RecycleSpace(8)
    for step in range(3):
        eps = base.eps * (1.0 + 0.01 * step)
        orc = OracleSolver(base.mesh.xyz, base.mesh.tets, eps, base.mesh.bfaces, base.mesh.bface_kind,
                           base.part, base.n_sub, base.overlap, base.k0, base.degree)
        b = orc.rhs(base.sources[0])
        mv = lambda v: orc.A @ v
        x, it, rr, ok = gcrodr(mv, orc.prec.apply, b, sp, restart=20)
        _, it_g, _, ok_g = fgmres(mv, orc.prec.apply, b, restart=20)
        assert ok and ok_g and rr <= 1e-8
        if step > 0:
            assert it < it_g, (step, it, it_g)


@pytest.mark.parametrize("k", [1, 5])
def test_same_operator_needs_no_refresh(k):
    """Solving again with the same operator without recomputing C gives the
    same result as recomputing it (the space is already consistent)."""
    A, Mi, b = rand_system(40, 21)
    mv, pc = (lambda v: A @ v), (lambda v: Mi @ v)
    sp1, sp2 = RecycleSpace(k), RecycleSpace(k)
    gcrodr(mv, pc, b, sp1, restart=10)
    gcrodr(mv, pc, b, sp2, restart=10)
    b2 = np.roll(b, 3)
    x1, it1, _, _ = gcrodr(mv, pc, b2, sp1, fresh_operator=False, restart=10)
    x2, it2, _, _ = gcrodr(mv, pc, b2, sp2, fresh_operator=True, restart=10)
    assert abs(it1 - it2) <= 1
    assert np.linalg.norm(x1 - x2) <= 1e-7 * np.linalg.norm(x2)


def test_full_space_cycle_with_recycled_vectors_is_exact():
    """A cycle that starts from a recycled space and whose Arnoldi steps fill
    the rest of the space (k + j = n) yields exact harmonic Ritz pairs: the
    new space spans the eigenvectors of the k smallest eigenvalues.  This
    exercises the pencil with the recycled blocks (D, B_j, C^H U D,
    V^H U D), which the first cycle does not."""
    n, k = 14, 3
    rng = np.random.default_rng(6)
    lam = np.concatenate([[0.05, 0.1j, -0.2], 3 + rng.standard_normal(n - 3)])
    X = np.eye(n) + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    Ap = X @ np.diag(lam) @ np.linalg.inv(X)
    Mi = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    A = Ap @ np.linalg.inv(Mi)
    mv, pc = (lambda v: A @ v), (lambda v: Mi @ v)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    sp = RecycleSpace(k)
    gcrodr(mv, pc, b, sp, tol=1e-15, restart=5, max_iters=5)      # a rough space
    Qx, _ = np.linalg.qr(X[:, :3])
    before = scipy.linalg.svdvals(np.linalg.qr(sp.U)[0].conj().T @ Qx)
    assert before.min() < 0.999                                   # not exact yet
    b2 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    gcrodr(mv, pc, b2, sp, fresh_operator=False, tol=1e-15, restart=n + 1, max_iters=n - k)
    s = scipy.linalg.svdvals(np.linalg.qr(sp.U)[0].conj().T @ Qx)
    assert np.all(s > 1 - 1e-8), s
