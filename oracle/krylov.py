"""Right-preconditioned flexible GMRES, single and multiple right-hand sides (oracle).

Sec. 5 solves every system with GMRES preconditioned by ORAS and, for several
right-hand sides, "pseudo-block" GMRES: the per-right-hand-side operations
are fused but each right-hand side keeps its own Krylov space.  Block GMRES
(one shared block Krylov space) is the variant Sec. 6 lists as future work.

Readings (the paper names none of these):
* right preconditioning, x0 = 0, restart length m (default 50);
* Arnoldi with modified Gram-Schmidt and the Hermitian inner product
  sum conj(u_i) v_i; Hessenberg least squares by complex Givens rotations;
* a cycle ends when the estimate |g_{j+1}| <= tol ||b|| or after m steps;
  then x += Z y and the true residual ||b - A x|| / ||b|| is recomputed;
  the solve has converged when that true relative residual is <= tol;
* the iteration count is the total number of Arnoldi steps.

Pins: Givens rotations annihilate; GMRES on a matrix with k distinct
eigenvalues stops after k steps; restarted and preconditioned runs reach the
direct solution; block GMRES reaches the direct solutions of every column.
Parity unpinned: the iteration counts on the chamber and cube workloads (the
paper prints none for this method on these inputs).
"""
from __future__ import annotations

import numpy as np


def givens(a: complex, b: complex):
    """(c, s) with c real: [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    nu = np.hypot(abs(a), abs(b))
    c = abs(a) / nu
    s = (a / abs(a)) * np.conj(b) / nu
    return c, s


def fgmres(matvec, precond, b, tol=1e-8, restart=50, max_iters=5000, history=None):
    """Returns (x, iterations, true relative residual, converged)."""
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0, True
    r = b.copy()
    beta = bnorm
    iters = 0
    while True:
        m = restart
        V = np.zeros((m + 1, n), dtype=np.complex128)
        Z = np.zeros((m, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        j_done = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            w0 = np.linalg.norm(w)
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] <= 1e-14 * w0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                          # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            j_done = j + 1
            if history is not None:
                history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or breakdown or iters >= max_iters:
                break
        y = np.zeros(j_done, dtype=np.complex128)
        for i in range(j_done - 1, -1, -1):            # back substitution
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:]) / H[i, i]
        x = x + y @ Z[:j_done]
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            return x, iters, beta / bnorm, True
        if iters >= max_iters:
            return x, iters, beta / bnorm, False


def pseudo_block_fgmres(matvec, precond, B, tol=1e-8, restart=50, max_iters=5000):
    """Each column runs its own FGMRES; the fused execution does not change the
    arithmetic of any column, so the reference runs them one after another."""
    out = [fgmres(matvec, precond, B[:, c], tol, restart, max_iters) for c in range(B.shape[1])]
    X = np.stack([o[0] for o in out], axis=1)
    return X, [o[1] for o in out], [o[2] for o in out], [o[3] for o in out]


def householder_qr(W):
    """Thin QR of a tall complex matrix by Householder reflections: W = Q R."""
    W = np.array(W, dtype=np.complex128)
    n, p = W.shape
    Q = np.eye(n, p, dtype=np.complex128)
    vs = []
    R = W.copy()
    for k in range(p):
        x = R[k:, k].copy()
        alpha = np.linalg.norm(x)
        if alpha == 0.0:
            vs.append(None)
            continue
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        v = x.copy()
        v[0] += phase * alpha
        v /= np.linalg.norm(v)
        R[k:, k:] -= 2.0 * np.outer(v, np.conj(v) @ R[k:, k:])
        vs.append(v)
    for k in range(p - 1, -1, -1):
        v = vs[k]
        if v is None:
            continue
        Q[k:, :] -= 2.0 * np.outer(v, np.conj(v) @ Q[k:, :])
    return Q, np.triu(R[:p, :])


def block_fgmres(matvec_block, precond_block, B, tol=1e-8, restart=50, max_iters=5000):
    """Block flexible GMRES(m) over one shared block Krylov space.

    R0 = V_1 S0 (Householder QR); block Arnoldi with block modified
    Gram-Schmidt and a QR of each new block; the block Hessenberg least
    squares min ||E1 S0 - H Y||_F is solved with Householder QR of H;
    per-column residual estimates come from the transformed right-hand side.
    A cycle ends when every column's estimate is <= tol ||b_k|| or after m
    block steps; the true residuals are then recomputed.  The count is the
    number of block steps.  Returns (X, block steps, relres per column, ok).
    """
    B = np.asarray(B, dtype=np.complex128)
    n, p = B.shape
    X = np.zeros_like(B)
    bn = np.linalg.norm(B, axis=0)
    bn[bn == 0] = 1.0
    R = B.copy()
    steps = 0
    while True:
        m = restart
        V1, S0 = householder_qr(R)
        Vs = [V1]
        Zs = []
        H = np.zeros(((m + 1) * p, m * p), dtype=np.complex128)
        E = np.zeros(((m + 1) * p, p), dtype=np.complex128)
        E[:p, :] = S0
        jd = 0
        for j in range(m):
            Zj = precond_block(Vs[j])
            Zs.append(Zj)
            W = matvec_block(Zj)
            for i in range(j + 1):
                Hij = np.conj(Vs[i].T) @ W
                H[i * p:(i + 1) * p, j * p:(j + 1) * p] = Hij
                W = W - Vs[i] @ Hij
            Q, Rr = householder_qr(W)
            H[(j + 1) * p:(j + 2) * p, j * p:(j + 1) * p] = Rr
            Vs.append(Q)
            steps += 1
            jd = j + 1
            # least squares on the current block Hessenberg
            Hk = H[:(jd + 1) * p, :jd * p]
            Ek = E[:(jd + 1) * p, :]
            Qh, Rh = np.linalg.qr(Hk, mode="complete")
            G = np.conj(Qh.T) @ Ek
            est = np.linalg.norm(G[jd * p:, :], axis=0)
            if np.all(est <= tol * bn) or steps >= max_iters:
                break
        Hk = H[:(jd + 1) * p, :jd * p]
        Ek = E[:(jd + 1) * p, :]
        Qh, Rh = np.linalg.qr(Hk, mode="reduced")
        Y = np.linalg.solve(Rh, np.conj(Qh.T) @ Ek)
        Zcat = np.concatenate(Zs[:jd], axis=1)
        X = X + Zcat @ Y
        R = B - matvec_block(X)
        rel = np.linalg.norm(R, axis=0) / bn
        if np.all(rel <= tol):
            return X, steps, rel, True
        if steps >= max_iters:
            return X, steps, rel, False
