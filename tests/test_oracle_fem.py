"""Pins of the oracle's discretisation against what the mathematics fixes.

Each test checks the oracle with something other than the oracle itself:
closed-form counts, textbook closed forms, pointwise quadrature of the
generators written from their definition, finite differences, exact
reproduction of fields that lie in the discrete space, and the curl-curl
kernel.
"""
import itertools
import math

import numpy as np
import pytest

from oracle.assemble import Discretization, face_geometry
from oracle.basis import Basis, LOCAL_EDGES, LOCAL_FACES, element_mass_stiffness, face_matrix
from paper_1605_04521_amd import gen


def kuhn_counts(n):
    """V, E, F, T of an n^3 Kuhn grid from Euler's formula V - E + F - T = 1."""
    T = 6 * n ** 3
    V = (n + 1) ** 3
    F = (4 * T + 12 * n * n) // 2          # each interior face shared by 2 tets; 12 n^2 boundary
    E = V + F - T - 1
    return V, E, F, T


def dofs_closed_form(n, r):
    V, E, F, T = kuhn_counts(n)
    return r * E + r * (r - 1) * F + r * (r - 1) * (r - 2) // 2 * T


def make_disc(mesh, r, eps=1.0 + 0.1j, k0=2 * math.pi):
    e = np.full(len(mesh.tets), eps, dtype=np.complex128)
    return Discretization(mesh.xyz, mesh.tets, e, mesh.bfaces, mesh.bface_kind, k0, r)


# --------------------------------------------------------------------------
# counts
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 4])
def test_entity_counts_match_euler(n):
    V, E, F, T = kuhn_counts(n)
    d = make_disc(gen.unit_cube(n), 1)
    assert len(d.topo.edges) == E
    assert len(d.topo.faces) == F
    assert d.topo.n_tets == T
    assert len(d.topo.boundary_face_ids) == 12 * n * n


@pytest.mark.parametrize("r", [1, 2, 3])
def test_dof_counts(r):
    # 8^3 grid: the closed form gives 4,184 / 21,424 / 60,936 unknowns; the
    # oracle's numbering must produce the closed-form count
    assert dofs_closed_form(8, r) == {1: 4184, 2: 21424, 3: 60936}[r]
    d = make_disc(gen.unit_cube(4), r)
    assert d.ndof == dofs_closed_form(4, r)
    assert {1: 604, 2: 2936, 3: 8148}[r] == d.ndof


def brute_nnz(mesh, r):
    """Structural non-zeros by brute force over entity pairs sharing a tet."""
    per = {0: r, 1: r * (r - 1), 2: r * (r - 1) * (r - 2) // 2}
    pairs = set()
    for t in mesh.tets.tolist():
        t = sorted(t)
        ents = [(0, tuple(e)) for e in itertools.combinations(t, 2)]
        ents += [(1, tuple(f)) for f in itertools.combinations(t, 3)]
        ents += [(2, tuple(t))]
        ents = [e for e in ents if per[e[0]] > 0]
        for a in ents:
            for b in ents:
                pairs.add((a, b))
    return sum(per[a[0]] * per[b[0]] for a, b in pairs)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_nnz_brute_force(r):
    mesh = gen.unit_cube(3)
    d = make_disc(mesh, r)
    rp, ci = d.pattern()
    assert rp[-1] == brute_nnz(mesh, r)


@pytest.mark.slow
def test_nnz_cube8():
    # structural non-zeros of the 8^3 grid, r = 1, 2, 3: the brute-force count
    # over entity pairs sharing an element (61,784 / 872,288 / 4,952,088)
    mesh = gen.unit_cube(8)
    for r in (1, 2, 3):
        expect = brute_nnz(mesh, r)
        d = make_disc(mesh, r)
        assert d.pattern()[0][-1] == expect


def test_pec_elimination_count():
    """Chamber: lateral wall + bottom metallic.  The metallic surface is an open
    box (a disc topologically), V_s - E_s + F_s = 1, with F_s = 10 n^2
    triangles; all its edge and face unknowns are removed."""
    n = 3
    for r in (1, 2, 3):
        mesh = gen.chamber_cylinder(n)
        d = make_disc(mesh, r, eps=44 + 20j, k0=gen.K0_1GHZ)
        Fs = 10 * n * n
        Vs = (n + 1) ** 3 - (n - 1) ** 2 * n
        Es = Vs + Fs - 1
        assert int(d.dofs.pec_face.sum()) == Fs
        assert int(d.dofs.pec_edge.sum()) == Es
        assert d.ndof == dofs_closed_form(n, r) - (r * Es + r * (r - 1) * Fs)


# --------------------------------------------------------------------------
# generators
# --------------------------------------------------------------------------

def random_tet(rng):
    while True:
        X = rng.standard_normal((4, 3))
        Mx = np.hstack([X, np.ones((4, 1))])
        if abs(np.linalg.det(Mx)) > 0.3:
            C = np.linalg.inv(Mx)
            return X, C[:3, :].T.copy(), abs(np.linalg.det(Mx)) / 6.0


def all_generators_values(r, lam, grads):
    """Every lambda^k w^e, |k| = r-1, all 6 edges (the redundant family)."""
    vals = []
    for i, j in LOCAL_EDGES:
        w = lam[i] * grads[j] - lam[j] * grads[i]
        for k in itertools.product(range(r), repeat=4):
            if sum(k) == r - 1:
                vals.append(np.prod([lam[m] ** k[m] for m in range(4)]) * w)
    return np.array(vals)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_generator_subset_is_a_basis(r):
    rng = np.random.default_rng(1)
    X, grads, vol = random_tet(rng)
    b = Basis(r)
    dim = r * (r + 2) * (r + 3) // 2
    assert b.nloc == dim
    rows_all, rows_kept = [], []
    for _ in range(4 * dim):
        lam = rng.dirichlet(np.ones(4))
        rows_all.append(all_generators_values(r, lam, grads).T)    # [3, nall]
        rows_kept.append(b.eval_phi(lam, grads).T)                 # [3, nloc]
    A_all = np.concatenate(rows_all)
    A_kept = np.concatenate(rows_kept)
    s_all = np.linalg.svd(A_all, compute_uv=False)
    s_kept = np.linalg.svd(A_kept, compute_uv=False)
    rank_all = int(np.sum(s_all > 1e-10 * s_all[0]))
    assert rank_all == dim                        # span of the redundant family
    assert s_kept[-1] > 1e-6 * s_kept[0]          # kept subset independent
    s_both = np.linalg.svd(np.hstack([A_all, A_kept]), compute_uv=False)
    assert int(np.sum(s_both > 1e-10 * s_both[0])) == dim   # same space


@pytest.mark.parametrize("r", [1, 2, 3])
def test_curl_matches_finite_differences(r):
    rng = np.random.default_rng(2)
    X, grads, vol = random_tet(rng)
    b = Basis(r)
    Mx = np.hstack([X, np.ones((4, 1))])
    C = np.linalg.inv(Mx)
    lam_of = lambda x: np.append(x, 1.0) @ C
    x0 = rng.dirichlet(np.ones(4)) @ X
    h = 1e-5
    J = np.zeros((b.nloc, 3, 3))     # J[p, comp, dir]
    for k in range(3):
        e = np.zeros(3); e[k] = h
        J[:, :, k] = (b.eval_phi(lam_of(x0 + e), grads) - b.eval_phi(lam_of(x0 - e), grads)) / (2 * h)
    curl_fd = np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], axis=1)
    assert np.allclose(b.eval_curl(lam_of(x0), grads), curl_fd, atol=1e-7)


def tet_rule(q):
    """Collapsed Gauss-Legendre rule on the reference simplex (test copy)."""
    g, w = np.polynomial.legendre.leggauss(q)
    g = 0.5 * (g + 1); w = 0.5 * w
    pts, wts = [], []
    for a, wa in zip(g, w):
        for bb, wb in zip(g, w):
            for c, wc in zip(g, w):
                l1, l2, l3 = a, bb * (1 - a), c * (1 - a) * (1 - bb)
                pts.append([1 - l1 - l2 - l3, l1, l2, l3])
                wts.append(6 * wa * wb * wc * (1 - a) ** 2 * (1 - bb))
    return np.array(pts), np.array(wts)


def test_tet_rule_textbook_moments():
    pts, wts = tet_rule(4)
    assert np.isclose(wts.sum(), 1.0)
    assert np.allclose(wts @ pts, 0.25)                      # int lambda_i = |T|/4
    assert np.allclose(wts @ pts ** 2, 0.1)                  # int lambda_i^2 = |T|/10
    assert np.isclose(wts @ (pts[:, 0] * pts[:, 1]), 0.05)   # int lambda_i lambda_j = |T|/20


@pytest.mark.parametrize("r", [1, 2, 3])
def test_element_matrices_vs_pointwise_quadrature(r):
    rng = np.random.default_rng(3)
    X, grads, vol = random_tet(rng)
    b = Basis(r)
    M, K = element_mass_stiffness(b, grads[None], np.array([vol]))
    pts, wts = tet_rule(r + 2)
    Mq = np.zeros((b.nloc, b.nloc)); Kq = np.zeros_like(Mq)
    for lam, w in zip(pts, wts):
        P = b.eval_phi(lam, grads)
        Cc = b.eval_curl(lam, grads)
        Mq += w * vol * P @ P.T
        Kq += w * vol * Cc @ Cc.T
    assert np.allclose(M[0], Mq, rtol=1e-12, atol=1e-12 * np.abs(Mq).max())
    assert np.allclose(K[0], Kq, rtol=1e-12, atol=1e-12 * np.abs(Kq).max())
    assert np.linalg.eigvalsh(0.5 * (M[0] + M[0].T)).min() > 0          # SPD
    assert np.linalg.eigvalsh(0.5 * (K[0] + K[0].T)).min() > -1e-10 * np.abs(K[0]).max()


def test_lowest_order_closed_forms():
    """r=1: K_T = 4|T| (g_a x g_b).(g_c x g_d); M_T from int l_i l_j = |T|(1+d_ij)/20."""
    rng = np.random.default_rng(4)
    X, g, vol = random_tet(rng)
    b = Basis(1)
    M, K = element_mass_stiffness(b, g[None], np.array([vol]))
    mm = lambda i, j: vol * (1 + (i == j)) / 20.0
    for p, (a, bb) in enumerate(LOCAL_EDGES):
        for q, (c, d) in enumerate(LOCAL_EDGES):
            k = 4 * vol * np.dot(np.cross(g[a], g[bb]), np.cross(g[c], g[d]))
            m = (mm(a, c) * g[bb] @ g[d] - mm(a, d) * g[bb] @ g[c]
                 - mm(bb, c) * g[a] @ g[d] + mm(bb, d) * g[a] @ g[c])
            assert np.isclose(K[0, p, q], k, rtol=1e-13, atol=1e-13)
            assert np.isclose(M[0, p, q], m, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_face_matrix_vs_tangential_quadrature(r):
    rng = np.random.default_rng(5)
    X, grads, vol = random_tet(rng)
    b = Basis(r)
    g, w = np.polynomial.legendre.leggauss(r + 2)
    g = 0.5 * (g + 1); w = 0.5 * w
    for lf, fv in enumerate(LOCAL_FACES):
        opp = ({0, 1, 2, 3} - set(fv)).pop()
        P = X[list(fv)]
        nrm = np.cross(P[1] - P[0], P[2] - P[0])
        area = 0.5 * np.linalg.norm(nrm)
        nrm /= np.linalg.norm(nrm)
        B = face_matrix(b, lf, grads, nrm, area)
        Bq = np.zeros_like(B)
        for xi, wx in zip(g, w):
            for eta, we in zip(g, w):
                lam = np.zeros(4)
                lam[list(fv)] = (1 - xi, xi * (1 - eta), xi * eta)
                Ph = b.eval_phi(lam, grads)
                Pt = Ph - np.outer(Ph @ nrm, nrm)
                Pt[~b.face_mask[lf]] = 0.0
                Bq += 2 * area * wx * we * xi * Pt @ Pt.T
        assert np.allclose(B, Bq, rtol=1e-12, atol=1e-12 * np.abs(Bq).max())
        # generators off the face have no tangential trace on it
        lam = np.zeros(4); lam[list(fv)] = rng.dirichlet(np.ones(3))
        Ph = b.eval_phi(lam, grads)
        Pt = Ph - np.outer(Ph @ nrm, nrm)
        assert np.abs(Pt[~b.face_mask[lf]]).max() < 1e-12


# --------------------------------------------------------------------------
# global operator
# --------------------------------------------------------------------------

def test_discrete_gradients_in_curl_kernel_r1():
    """k0 = 0: A = K; the edge-vertex incidence G (oriented low -> high) has K G = 0."""
    mesh = gen.unit_cube(3)
    d = make_disc(mesh, 1, k0=0.0)
    A = d.global_matrix()
    E = d.topo.edges
    G = np.zeros((len(E), d.topo.n_vertices))
    G[np.arange(len(E)), E[:, 0]] = -1.0
    G[np.arange(len(E)), E[:, 1]] = 1.0
    KG = A @ G
    assert np.abs(KG).max() < 1e-12 * abs(A).max()


@pytest.mark.parametrize("r", [2, 3])
def test_polynomial_gradients_conforming_and_in_kernel(r):
    """grad q, deg q <= r, lies in the degree-r space: fit it per element,
    check that shared unknowns agree between elements (tangential conformity
    and orientation), and that the global curl-curl matrix annihilates it."""
    mesh = gen.unit_cube(2)
    d = make_disc(mesh, r, k0=0.0)
    rng = np.random.default_rng(6)
    coef = rng.standard_normal(20)

    def grad_q(x):
        # q = sum of monomials x^a y^b z^c, a+b+c <= r (random coefficients)
        out = np.zeros(3)
        i = 0
        for a in range(r + 1):
            for bb in range(r + 1 - a):
                for c in range(r + 1 - a - bb):
                    if i >= len(coef):
                        break
                    cc = coef[i]; i += 1
                    if a: out[0] += cc * a * x[0] ** (a - 1) * x[1] ** bb * x[2] ** c
                    if bb: out[1] += cc * bb * x[0] ** a * x[1] ** (bb - 1) * x[2] ** c
                    if c: out[2] += cc * c * x[0] ** a * x[1] ** bb * x[2] ** (c - 1)
        return out

    u = np.full(d.ndof, np.nan)
    for t in range(d.topo.n_tets):
        rows, rhs = [], []
        for _ in range(3 * d.basis.nloc):
            lam = rng.dirichlet(np.ones(4))
            rows.append(d.basis.eval_phi(lam, d.grads[t]))
            rhs.append(grad_q(d.point(t, lam)))
        Amat = np.concatenate([p.T for p in rows])
        bvec = np.concatenate(rhs)
        c, *_ = np.linalg.lstsq(Amat, bvec, rcond=None)
        assert np.linalg.norm(Amat @ c - bvec) < 1e-10 * np.linalg.norm(bvec)
        for p, gd in enumerate(d.dofs.tet_dofs[t]):
            if np.isnan(u[gd]):
                u[gd] = c[p]
            else:
                assert abs(u[gd] - c[p]) < 1e-9 * (1 + abs(c[p]))
    A = d.global_matrix()
    assert np.linalg.norm(A @ u) < 1e-10 * abs(A).max() * np.linalg.norm(u)


def test_global_matrix_symmetric():
    d = make_disc(gen.unit_cube(2), 2)
    A = d.global_matrix()
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
