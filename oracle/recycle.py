"""Krylov subspace recycling over a sequence of systems: GCRO-DR (oracle).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this module; the product path never does.

Sec. 6 proposes, for the slowly varying systems that the imaging loop solves
one after another, to carry a Krylov subspace from one solve to the next with
GCRO-DR, the method of Parks, de Sturler, Mackey, Johnson and Maiti
(SIAM J. Sci. Comput. 28(5), 2006) that Sec. 6 cites.  This module is that
method, applied to the right-preconditioned operator  Ap = A M^{-1}  of
Sec. 5 with the ORAS preconditioner M^{-1} of Sec. 4, written from the
description of the method:

* A recycled space is a pair (U, C) with  Ap U = C  and  C^H C = I.  The
  solve first removes from the residual its part in range(C) (the minimal
  residual correction over range(U)), then runs Arnoldi for the operator
  (I - C C^H) Ap, which gives  Ap V_j = C B_j + V_{j+1} Hbar_j.
* The least-squares problem over range([U, V_j]) splits: its V part is the
  GMRES problem  min |beta e_1 - Hbar_j y|  and its U part is  -B_j y.
* At the end of every cycle the space is replaced by the k harmonic Ritz
  vectors of Ap with respect to range([U, V_j]) of smallest harmonic Ritz
  value: the eigenvectors of  Gbar^H Gbar z = theta Gbar^H (W^H Vhat) z  with
  W = [C, V_{j+1}], Vhat = [U D, V_j], Gbar = [[D, B_j], [0, Hbar_j]] and D
  the diagonal that scales the columns of U to unit length.  With P the
  selected eigenvectors and  Gbar P = Q R:  C <- W Q,  U <- Vhat P R^{-1}.
  Without a recycled space (the first cycle of the first system) this is
  GMRES(m) followed by the same selection with Gbar = Hbar.
* For a new system (new A and a new ORAS factorisation, Sec. 4-5) the kept
  U is carried over and C is recomputed:  Ap U = Q R,  C <- Q, U <- U R^{-1}.

Readings (the method leaves them open):
* the solution is x = M^{-1} u; the module keeps Ubar = M^{-1} U beside U so
  that no extra preconditioner application is needed in the update
  x += Ubar t (M is fixed within a system);
* a cycle holds m vectors in total: k recycled ones and m - k Arnoldi
  steps (the first cycle without a recycled space runs m steps);
* Arnoldi orthogonalises against C and then against V_j (modified
  Gram-Schmidt), Givens rotations solve the Hessenberg problem as in the
  GMRES oracle; a cycle ends at |g_{j+1}| <= tol ||b|| or after its steps;
  then the true residual b - A x is recomputed and its part in range(C)
  removed at the start of the next cycle;
* the iteration count is the number of Arnoldi steps; the work of carrying
  the space to a new system (k preconditioner applications and products)
  is reported apart;
* harmonic Ritz values of infinite magnitude (a singular right-hand matrix
  of the pencil) are never selected.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .krylov import givens


class RecycleSpace:
    """The recycled subspace carried from one solve to the next: columns of
    U (preconditioned space), Ubar = M^{-1} U and C = A Ubar, with C^H C = I."""

    def __init__(self, k: int):
        self.k = int(k)
        self.U = None
        self.Ubar = None
        self.C = None

    @property
    def dim(self) -> int:
        return 0 if self.U is None else self.U.shape[1]


def _refresh(space, matvec, precond):
    """Carry U over to a new operator: C = Ap U = Q R, C <- Q, U <- U R^{-1}."""
    U = space.U
    Ubar = np.stack([precond(U[:, i]) for i in range(U.shape[1])], axis=1)
    AU = np.stack([matvec(Ubar[:, i]) for i in range(U.shape[1])], axis=1)
    Q, R = np.linalg.qr(AU)
    Ri = np.linalg.inv(R)
    space.C = Q
    space.U = U @ Ri
    space.Ubar = Ubar @ Ri


def harmonic_ritz(G, WV, k):
    """The k eigenvectors of  G^H G z = theta G^H WV z  of smallest |theta|
    (finite theta only) and all the eigenvalues theta."""
    a = G.conj().T @ G
    b = G.conj().T @ WV
    theta, Z = scipy.linalg.eig(a, b)
    mag = np.where(np.isfinite(theta), np.abs(theta), np.inf)
    order = np.argsort(mag, kind="stable")
    return Z[:, order[:k]], theta


def gcrodr(matvec, precond, b, space: RecycleSpace, fresh_operator=True, tol=1e-8, restart=50,
           max_iters=5000, history=None):
    """Solve A x = b, using and then replacing the recycled space.

    fresh_operator: the operator differs from the one the space was made for
    (a new system), so C and Ubar are recomputed first.
    Returns (x, iterations, true relative residual, converged)."""
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    m, k = int(restart), space.k
    if k >= m:
        raise ValueError("the recycled dimension must be below the cycle length")
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0, True
    if space.dim and fresh_operator:
        _refresh(space, matvec, precond)
    r = b.copy()
    iters = 0
    while True:
        kk = space.dim
        if kk:
            # minimal residual correction over range(U): r -= C C^H r
            t = space.C.conj().T @ r
            x = x + space.Ubar @ t
            r = r - space.C @ t
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            rt = np.linalg.norm(b - matvec(x))
            if rt <= tol * bnorm or beta == 0.0:
                return x, iters, rt / bnorm, bool(rt <= tol * bnorm)
        steps = m - kk
        V = np.zeros((steps + 1, n), dtype=np.complex128)
        Z = np.zeros((steps, n), dtype=np.complex128)
        H = np.zeros((steps + 1, steps), dtype=np.complex128)
        Bm = np.zeros((kk, steps), dtype=np.complex128)
        cs = np.zeros(steps)
        sn = np.zeros(steps, dtype=np.complex128)
        g = np.zeros(steps + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        jd = 0
        for j in range(steps):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            w0 = np.linalg.norm(w)
            for i in range(kk):                         # against C
                Bm[i, j] = np.vdot(space.C[:, i], w)
                w = w - Bm[i, j] * space.C[:, i]
            for i in range(j + 1):                      # against V_j
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] <= 1e-14 * w0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            iters += 1
            jd = j + 1
            # the least-squares state: a rotated copy of H's column j
            hc = H[: j + 2, j].copy()
            for i in range(j):
                t_ = cs[i] * hc[i] + sn[i] * hc[i + 1]
                hc[i + 1] = -np.conj(sn[i]) * hc[i] + cs[i] * hc[i + 1]
                hc[i] = t_
            cs[j], sn[j] = givens(hc[j], hc[j + 1])
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            if j == 0:
                Rt = np.zeros((steps, steps), dtype=np.complex128)
            hc[j] = cs[j] * hc[j] + sn[j] * hc[j + 1]
            Rt[: j + 1, j] = hc[: j + 1]
            if history is not None:
                history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or breakdown or iters >= max_iters:
                break
        y = scipy.linalg.solve_triangular(Rt[:jd, :jd], g[:jd])
        x = x + y @ Z[:jd]
        if kk:
            x = x - space.Ubar @ (Bm[:, :jd] @ y)
        # new recycled space from this cycle (deflated restarting)
        _deflate(space, kk, jd, V, Z, H, Bm)
        r = b - matvec(x)
        rn = np.linalg.norm(r)
        if rn <= tol * bnorm:
            return x, iters, rn / bnorm, True
        if iters >= max_iters or not np.isfinite(rn):
            return x, iters, rn / bnorm, False


def cycle_matrices(space: RecycleSpace, kk, jd, V, H, Bm):
    """Gbar and W^H Vhat of a cycle with kk recycled vectors and jd steps."""
    s = kk + jd
    G = np.zeros((s + 1, s), dtype=np.complex128)
    WV = np.zeros((s + 1, s), dtype=np.complex128)
    if kk:
        d = 1.0 / np.linalg.norm(space.U, axis=0)
        G[:kk, :kk] = np.diag(d)
        G[:kk, kk:] = Bm[:, :jd]
        UD = space.U * d
        WV[:kk, :kk] = space.C.conj().T @ UD
        WV[kk:, :kk] = V[: jd + 1].conj() @ UD
    G[kk:, kk:] = H[: jd + 1, :jd]
    WV[kk:kk + jd, kk:] = np.eye(jd)
    return G, WV


def _deflate(space: RecycleSpace, kk, jd, V, Z, H, Bm):
    s = kk + jd
    knew = min(space.k, s)
    if knew == 0:
        return
    G, WV = cycle_matrices(space, kk, jd, V, H, Bm)
    P, _ = harmonic_ritz(G, WV, knew)
    Q, R = np.linalg.qr(G @ P)
    PR = P @ np.linalg.inv(R)
    Wb = V[: jd + 1].T
    if kk:
        d = 1.0 / np.linalg.norm(space.U, axis=0)
        C = np.concatenate([space.C, Wb], axis=1) @ Q
        U = (space.U * d) @ PR[:kk] + V[:jd].T @ PR[kk:]
        Ubar = (space.Ubar * d) @ PR[:kk] + Z[:jd].T @ PR[kk:]
    else:
        C = Wb @ Q
        U = V[:jd].T @ PR
        Ubar = Z[:jd].T @ PR
    space.C, space.U, space.Ubar = C, U, Ubar


# ---------------------------------------------------------------------------
# Block GCRO-DR: the same recycling for a block of right-hand sides
# ---------------------------------------------------------------------------
# Sec. 6 names the combination of block and recycling strategies (a "Block
# GCRO-DR" method) for the many transmitting antennas of the imaging loop.
# This is GCRO-DR above with a block Krylov space (the block FGMRES oracle of
# krylov.py) in place of the single-vector one:
# * a cycle removes from the block residual its part in range(C), then runs
#   block Arnoldi for (I - C C^H) Ap from the QR of that residual,
#   Ap Z_j = C B_j + [V_0 .. V_{j+1}] Hbar_j, each block orthogonalised against
#   C and then the previous blocks (block modified Gram-Schmidt) and
#   factorised by Householder QR;
# * the least squares over range([U, V]) splits as in GCRO-DR: the V part is
#   the block GMRES problem min ||E1 S0 - Hbar Y||_F, the U part is -B Y;
# * the deflated restart takes the k harmonic Ritz vectors of Ap with respect
#   to range([U, V_j]) of smallest harmonic Ritz value, with Gbar =
#   [[D, B], [0, Hbar]] of size (kk + (j+1) p) x (kk + j p);
# * the cycle length `restart` counts vectors: (restart - kk) // p block steps
#   (restart // p without a recycled space), at least one;
# * iterations count block steps; the space is carried to a new operator as
#   in GCRO-DR.
# With p = 1 this is GCRO-DR (the tests check it).

def _householder_qr(W):
    from .krylov import householder_qr
    return householder_qr(W)


def block_gcrodr(matvec_block, precond_block, B, space: RecycleSpace, fresh_operator=True, tol=1e-8, restart=50,
                 max_iters=5000, history=None):
    """Solve A X = B (columns of B), using and then replacing the recycled space.

    Returns (X, block steps, true relative residual per column, converged)."""
    B = np.asarray(B, dtype=np.complex128)
    n, p = B.shape
    m, k = int(restart), space.k
    if k >= m:
        raise ValueError("the recycled dimension must be below the cycle length")
    X = np.zeros_like(B)
    bn = np.linalg.norm(B, axis=0)
    if np.any(bn == 0.0):
        raise ValueError("block GCRO-DR needs non-zero right-hand sides")
    if space.dim and fresh_operator:
        _refresh(space, lambda v: matvec_block(v[:, None])[:, 0], lambda v: precond_block(v[:, None])[:, 0])
    R = B.copy()
    steps = 0
    while True:
        kk = space.dim
        if kk:
            T = space.C.conj().T @ R
            X = X + space.Ubar @ T
            R = R - space.C @ T
        if np.all(np.linalg.norm(R, axis=0) <= tol * bn):
            rt = np.linalg.norm(B - matvec_block(X), axis=0) / bn
            if np.all(rt <= tol):
                return X, steps, rt, True
        nb = max(1, (m - kk) // p)
        V1, S0 = _householder_qr(R)
        Vs, Zs = [V1], []
        H = np.zeros(((nb + 1) * p, nb * p), dtype=np.complex128)
        Bm = np.zeros((kk, nb * p), dtype=np.complex128)
        E = np.zeros(((nb + 1) * p, p), dtype=np.complex128)
        E[:p, :] = S0
        jd = 0
        for j in range(nb):
            Zj = precond_block(Vs[j])
            Zs.append(Zj)
            W = matvec_block(Zj)
            if kk:                                   # against C
                Bj = space.C.conj().T @ W
                Bm[:, j * p:(j + 1) * p] = Bj
                W = W - space.C @ Bj
            for i in range(j + 1):                   # against the previous blocks
                Hij = Vs[i].conj().T @ W
                H[i * p:(i + 1) * p, j * p:(j + 1) * p] = Hij
                W = W - Vs[i] @ Hij
            Q, Rr = _householder_qr(W)
            H[(j + 1) * p:(j + 2) * p, j * p:(j + 1) * p] = Rr
            Vs.append(Q)
            steps += 1
            jd = j + 1
            Hk = H[:(jd + 1) * p, :jd * p]
            Qh, _ = np.linalg.qr(Hk, mode="complete")
            G = Qh.conj().T @ E[:(jd + 1) * p, :]
            est = np.linalg.norm(G[jd * p:, :], axis=0)
            if history is not None:
                history.append(est / bn)
            if np.all(est <= tol * bn) or steps >= max_iters:
                break
        Hk = H[:(jd + 1) * p, :jd * p]
        Qh, Rh = np.linalg.qr(Hk, mode="reduced")
        Y = np.linalg.solve(Rh, Qh.conj().T @ E[:(jd + 1) * p, :])
        Zcat = np.concatenate(Zs[:jd], axis=1)
        X = X + Zcat @ Y
        if kk:
            X = X - space.Ubar @ (Bm[:, :jd * p] @ Y)
        Vcat = np.concatenate(Vs[:jd + 1], axis=1)
        _deflate_block(space, kk, jd * p, Vcat, Zcat, Hk, Bm[:, :jd * p])
        R = B - matvec_block(X)
        rt = np.linalg.norm(R, axis=0) / bn
        if np.all(rt <= tol):
            return X, steps, rt, True
        if steps >= max_iters or not np.all(np.isfinite(rt)):
            return X, steps, rt, False


def _deflate_block(space: RecycleSpace, kk, q, Vcat, Zcat, Hbar, Bm):
    """The deflated restart of a block cycle: q = j p Krylov vectors, Vcat
    [n, q + p], Zcat [n, q], Hbar [(q + p), q], Bm [kk, q]."""
    p = Vcat.shape[1] - q
    s = kk + q
    knew = min(space.k, s)
    if knew == 0:
        return
    G = np.zeros((s + p, s), dtype=np.complex128)
    WV = np.zeros((s + p, s), dtype=np.complex128)
    if kk:
        d = 1.0 / np.linalg.norm(space.U, axis=0)
        G[:kk, :kk] = np.diag(d)
        G[:kk, kk:] = Bm
        UD = space.U * d
        WV[:kk, :kk] = space.C.conj().T @ UD
        WV[kk:, :kk] = Vcat.conj().T @ UD
    G[kk:, kk:] = Hbar
    WV[kk:kk + q, kk:] = np.eye(q)
    P, _ = harmonic_ritz(G, WV, knew)
    Qg, Rg = np.linalg.qr(G @ P)
    PR = P @ np.linalg.inv(Rg)
    if kk:
        d = 1.0 / np.linalg.norm(space.U, axis=0)
        C = np.concatenate([space.C, Vcat], axis=1) @ Qg
        U = (space.U * d) @ PR[:kk] + Vcat[:, :q] @ PR[kk:]
        Ubar = (space.Ubar * d) @ PR[:kk] + Zcat @ PR[kk:]
    else:
        C = Vcat @ Qg
        U = Vcat[:, :q] @ PR
        Ubar = Zcat @ PR
    space.C, space.U, space.Ubar = C, U, Ubar
