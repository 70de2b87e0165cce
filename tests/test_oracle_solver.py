"""Pins of the oracle's solver stages: Galerkin exactness, plane-wave
convergence, direct solves, ORAS special cases, partition of unity,
reciprocity and the Krylov kernels."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.assemble import Discretization
from oracle.krylov import block_fgmres, fgmres, givens
from oracle.schwarz import ORAS, build_subdomains
from oracle.solve import OracleSolver
from paper_1605_04521_amd import gen


def make_disc(mesh, r, eps=1.0 + 0.1j, k0=2 * math.pi):
    e = np.full(len(mesh.tets), eps, dtype=np.complex128)
    return Discretization(mesh.xyz, mesh.tets, e, mesh.bfaces, mesh.bface_kind, k0, r)


class PolyField:
    """E(x) = a + B x + Q(x), Q_i = sum_jk C[i,j,k] x_j x_k (C symmetric in j,k)."""

    def __init__(self, rng, degree):
        cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
        self.a = cplx(3)
        self.B = cplx(3, 3) if degree >= 1 else np.zeros((3, 3))
        C = cplx(3, 3, 3) if degree >= 2 else np.zeros((3, 3, 3))
        self.C = 0.5 * (C + np.transpose(C, (0, 2, 1)))

    def __call__(self, x):
        return self.a + self.B @ x + np.einsum("ijk,j,k->i", self.C, x, x)

    def jac(self, x):              # J[i,j] = d E_i / d x_j
        return self.B + 2 * np.einsum("ijk,k->ij", self.C, x)

    def curl(self, x):
        J = self.jac(x)
        return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])

    def curlcurl(self):            # grad(div E) - lap E, constant
        C = self.C
        return np.array([2 * np.einsum("iim->", C[:, :, m:m + 1]) - 2 * np.einsum("jj->", C[m])
                         for m in range(3)])


@pytest.mark.parametrize("r", [1, 2, 3])
def test_galerkin_exactness(r):
    """A field of degree <= r-1 lies in the discrete space; with the matching
    volume source f = curl curl E - kappa^2 E and impedance data
    g = (curl E) x n - i beta E_t the discrete solution is E itself."""
    mesh = gen.unit_cube(2)
    eps = 1.3 + 0.2j
    d = make_disc(mesh, r, eps=eps, k0=3.0)
    E = PolyField(np.random.default_rng(10 + r), r - 1)
    kap2 = d.k0 ** 2 * eps
    f = lambda x, t: E.curlcurl() - kap2 * E(x)
    g = lambda x, n, beta, t: np.cross(E.curl(x), n) - 1j * beta * np.cross(n, np.cross(E(x), n))
    b = d.rhs_volume(f) + d.rhs_boundary(g)
    A = d.global_matrix()
    u = spla.spsolve(A.tocsc(), b)
    err, ref = d.l2_error(u, lambda x, t: E(x))
    assert err < 1e-10 * ref
    # the same through ORAS + FGMRES on 8 overlapping subdomains
    part, nsub = gen.box_partition(mesh, 1)
    P = ORAS(d, part, nsub, 1)
    x, it, rr, ok = fgmres(lambda v: A @ v, P.apply, b, tol=1e-12)
    assert ok and rr <= 1e-12
    assert np.linalg.norm(x - u) < 1e-9 * np.linalg.norm(u)


def planewave_error(n, r):
    prob = gen.cube_planewave_problem(n=n, degree=r, box=max(1, n // 2))
    m = prob.mesh
    d = Discretization(m.xyz, m.tets, prob.eps, m.bfaces, m.bface_kind, prob.k0, r)
    src = prob.sources[0]
    A = d.global_matrix()
    u = spla.spsolve(A.tocsc(), d.rhs(src))
    p, dd = np.asarray(src.pol), np.asarray(src.dir)
    kap = prob.k0 * np.sqrt(prob.eps[0])
    err, ref = d.l2_error(u, lambda x, t: p * np.exp(1j * kap * (dd @ x)))
    return err / ref


@pytest.mark.slow
@pytest.mark.parametrize("r,ns", [(1, (4, 8)), (2, (2, 4)), (3, (2, 4))])
def test_planewave_convergence_order(r, ns):
    """E = p exp(i kappa d.x), kappa = k0 sqrt(eps), solves eq. (1) exactly; the
    L2 error of the degree-r solution decays like h^r."""
    e0, e1 = planewave_error(ns[0], r), planewave_error(ns[1], r)
    slope = math.log(e0 / e1, 2)
    assert e1 < e0
    assert slope > r - 0.35, (e0, e1, slope)


@pytest.mark.parametrize("n", [1, 2])
def test_dense_direct_solve_tiny(n):
    prob = gen.cube_planewave_problem(n=n, degree=2, box=1)
    s = OracleSolver.from_problem(prob)
    b = s.rhs(prob.sources[0])
    xd = np.linalg.solve(s.A.toarray(), b)
    x, it, rr, ok = s.solve(b, tol=1e-12)
    assert ok
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_one_subdomain_is_a_direct_solve():
    """N_sub = 1: A_1 = A and D_1 = I, so M^{-1} = A^{-1}: one iteration."""
    prob = gen.cube_planewave_problem(n=3, degree=2)
    prob.part[:] = 0
    prob.n_sub = 1
    s = OracleSolver.from_problem(prob)
    x, it, rr, ok = s.solve(s.rhs(prob.sources[0]))
    assert ok and it == 1


@pytest.mark.parametrize("overlap", [1, 2])
def test_partition_of_unity(overlap):
    """sum_s R_s^T D_s R_s = I: every unknown has weight 1 in exactly one
    subdomain, which contains it."""
    prob = gen.chamber_problem(n=4, degree=2, n_sub=5, overlap=overlap)
    m = prob.mesh
    d = Discretization(m.xyz, m.tets, prob.eps, m.bfaces, m.bface_kind, prob.k0, 2)
    subs = build_subdomains(d, prob.part, prob.n_sub, overlap)
    acc = np.zeros(d.ndof)
    cover = np.zeros(d.ndof)
    for s in subs:
        assert np.all(np.diff(s.dofs) > 0)
        acc[s.dofs] += s.pou
        cover[s.dofs] += 1
    assert np.array_equal(acc, np.ones(d.ndof))
    assert cover.min() >= 1 and cover.max() > 1


def test_reciprocity():
    """A = A^T (bilinear form) gives b2^T A^{-1} b1 = b1^T A^{-1} b2."""
    prob = gen.chamber_problem(n=4, degree=2, n_sub=4, overlap=1, n_sources=2)
    s = OracleSolver.from_problem(prob)
    b1, b2 = s.rhs(prob.sources[0]), s.rhs(prob.sources[1])
    x1, *_ = s.solve(b1, tol=1e-11)
    x2, *_ = s.solve(b2, tol=1e-11)
    assert abs(b2 @ x1 - b1 @ x2) <= 1e-8 * abs(b2 @ x1)


def test_oras_not_slower_than_oas():
    """Sec. 4: dropping D_s (OAS) converges more slowly than ORAS."""
    prob = gen.cube_planewave_problem(n=8, degree=1)
    so = OracleSolver.from_problem(prob, "oras")
    sa = OracleSolver.from_problem(prob, "oas")
    b = so.rhs(prob.sources[0])
    _, it_oras, _, ok1 = so.solve(b)
    _, it_oas, _, _ = sa.solve(b, max_iters=400)
    assert ok1 and it_oras <= it_oas


def brute_force_local_sizes(mesh, part, n_sub, layers):
    """Local unknown counts of r = 1 (no metallic faces): edges of the
    elements of each overlapping subdomain, by brute force over vertex sets."""
    tets = [tuple(sorted(t)) for t in mesh.tets.tolist()]
    by_face = {}
    for i, t in enumerate(tets):
        for f in ((t[0], t[1], t[2]), (t[0], t[1], t[3]), (t[0], t[2], t[3]), (t[1], t[2], t[3])):
            by_face.setdefault(f, []).append(i)
    sizes = []
    for s in range(n_sub):
        inside = {i for i in range(len(tets)) if part[i] == s}
        for _ in range(layers):
            grown = set(inside)
            for i in inside:
                t = tets[i]
                for f in ((t[0], t[1], t[2]), (t[0], t[1], t[3]), (t[0], t[2], t[3]), (t[1], t[2], t[3])):
                    grown.update(by_face[f])
            inside = grown
        edges = {(t[a], t[b]) for i in inside for t in [tets[i]] for a in range(4) for b in range(a + 1, 4)}
        sizes.append(len(edges))
    return sizes


def test_small_cube_counts_and_subdomains():
    """8^3 cube, 2x2x2 boxes, one face layer: 4,184 unknowns (Euler's formula),
    61,784 non-zeros and 796 local unknowns in every subdomain (brute-force
    counts over vertex sets, independent of the oracle's entity tables)."""
    prob = gen.cube_planewave_problem()
    s = OracleSolver.from_problem(prob)
    n = 8
    T, V = 6 * n ** 3, (n + 1) ** 3
    F = (4 * T + 12 * n * n) // 2
    assert s.ndof == V + F - T - 1 == 4184
    pairs = set()
    for t in prob.mesh.tets.tolist():
        t = sorted(t)
        es = [(t[a], t[b]) for a in range(4) for b in range(a + 1, 4)]
        pairs.update((e1, e2) for e1 in es for e2 in es)
    assert s.A.nnz == len(pairs) == 61784
    sizes = brute_force_local_sizes(prob.mesh, prob.part, prob.n_sub, prob.overlap)
    assert [len(x.dofs) for x in s.prec.subs] == sizes == [796] * 8


# --------------------------------------------------------------------------
# Krylov kernels
# --------------------------------------------------------------------------

def test_givens_annihilates():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s = givens(a, b)
        assert abs(-np.conj(s) * a + c * b) < 1e-14
        assert abs(abs(c * a + s * b) - np.hypot(abs(a), abs(b))) < 1e-14
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-14


def matrix_with_k_eigenvalues(n, k, seed):
    rng = np.random.default_rng(seed)
    lam = (rng.standard_normal(k) + 1j * rng.standard_normal(k)) + 3.0
    diag = lam[np.arange(n) % k]
    S = np.eye(n) + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    return S @ np.diag(diag) @ np.linalg.inv(S)


def test_fgmres_minimal_polynomial():
    """GMRES ends after as many steps as the degree of the minimal polynomial."""
    A = matrix_with_k_eigenvalues(40, 5, 1)
    b = np.random.default_rng(2).standard_normal(40) + 0j
    x, it, rr, ok = fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-10)
    assert ok and it == 5
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-8 * np.linalg.norm(x)


def test_fgmres_restart_and_preconditioner():
    A = matrix_with_k_eigenvalues(40, 12, 3)
    b = np.random.default_rng(4).standard_normal(40) + 1j
    x, it, rr, ok = fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-10, restart=4, max_iters=2000)
    assert ok and it > 12
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)
    Ainv = np.linalg.inv(A)
    x, it, rr, ok = fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-10)
    assert ok and it == 1


def test_block_fgmres():
    A = matrix_with_k_eigenvalues(40, 5, 5)
    B = np.random.default_rng(6).standard_normal((40, 3)) + 0j
    X, steps, rel, ok = block_fgmres(lambda V: A @ V, lambda V: V, B, tol=1e-10)
    assert ok and steps <= 5
    assert np.linalg.norm(X - np.linalg.solve(A, B)) < 1e-8 * np.linalg.norm(X)
    A = matrix_with_k_eigenvalues(40, 14, 7)
    X, steps, rel, ok = block_fgmres(lambda V: A @ V, lambda V: V, B, tol=1e-10, restart=3)
    assert ok and np.all(rel <= 1e-10)
    assert np.linalg.norm(A @ X - B) <= 1e-9 * np.linalg.norm(B)


@pytest.mark.parametrize("variant", ["oras", "ras", "oras_mult"])
def test_variants_are_partitions_of_unity(variant):
    """sum_s R_s^T D_s R_s = I for the Boolean (ORAS, RAS) and the
    multiplicity (ORAS_MULT) weights: the preconditioner maps a vector that
    every local solve reproduces exactly (A_s = I) to itself.  Checked with
    the weights the oracle's application uses."""
    prob = gen.chamber_problem(n=4, degree=2, n_sub=5, overlap=2)
    s = OracleSolver.from_problem(prob, variant)
    acc = np.zeros(s.ndof)
    for sub in s.prec.subs:
        acc[sub.dofs] += s.prec.weights(sub)
    assert np.allclose(acc, 1.0, rtol=0, atol=1e-15)
    if variant == "oras_mult":
        w = np.concatenate([s.prec.weights(sub) for sub in s.prec.subs])
        assert w.min() < 1.0   # some unknowns lie in several subdomains


@pytest.mark.parametrize("variant", ["ras", "oras_mult"])
def test_variant_one_subdomain_is_a_direct_solve(variant):
    """One subdomain: R_1 = I, D_1 = I and A_1 = A for every variant (no
    interface), so one iteration solves the system."""
    prob = gen.cube_planewave_problem(n=3, degree=2)
    prob.part[:] = 0
    prob.n_sub = 1
    s = OracleSolver.from_problem(prob, variant)
    x, it, rr, ok = s.solve(s.rhs(prob.sources[0]))
    assert ok and it == 1


def test_ras_local_matrix_is_principal_submatrix():
    """RAS: A_s = R_s A R_s^T, i.e. the global matrix restricted to the
    subdomain's unknowns, entry by entry (checked against the dense A)."""
    prob = gen.chamber_problem(n=3, degree=1, n_sub=3, overlap=1)
    s = OracleSolver.from_problem(prob, "ras")
    Ad = s.A.toarray()
    for sub in s.prec.subs:
        assert np.array_equal(sub.A.toarray(), Ad[np.ix_(sub.dofs, sub.dofs)])
