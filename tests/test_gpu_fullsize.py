"""Parity at the benchmark's full size and launch configuration (synthetic
chamber, O-grid 22 x 11 x 27 cells, r=2, 1,477,926 unknowns, 3,465
block-aligned 2 x 2 x 3-cell subdomains, 2 face layers), on outputs the
oracle can compute piece by piece: every value of the global matrix, the
right-hand side, one SpMV, the ORAS application (one column, FP64; 32 columns,
FP32 factors) restricted to the unknowns owned by a sample of subdomains (each
checked against the oracle's own local matrix and sparse LU for that
subdomain), and the true residual of a full FP64 solve."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import scipy.sparse.linalg as spla

from oracle.assemble import Discretization
from oracle.schwarz import Subdomain, grow_overlap, local_matrix, owners
from paper_1605_04521_amd import _lib as B
from paper_1605_04521_amd import gen
from paper_1605_04521_amd.api import Layout, Problem

pytestmark = pytest.mark.gpu

N_GRID = int(os.environ.get("MXW_FULL_N", "22"))
N_Z = int(os.environ.get("MXW_FULL_NZ", "27"))
N_SUB = tuple(int(q) for q in os.environ.get("MXW_FULL_NSUB", "2x2x3").split("x"))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_subdomain(d, part, own, s, layers):
    tets = grow_overlap(d, part, s, layers)
    in_s = np.zeros(d.topo.n_tets, dtype=bool)
    in_s[tets] = True
    dd = d.dofs.tet_dofs[tets].ravel()
    dofs = np.unique(dd[dd >= 0])
    iface = []
    for t in tets:
        for lf, f in enumerate(d.topo.tet_faces[t]):
            other = [u for u in d.topo.face_tets[f] if u >= 0 and u != t]
            if other and not in_s[other[0]]:
                iface.append((int(t), lf, d.k0 * np.sqrt(d.eps[t].real)))
    return Subdomain(s, tets, dofs, (own[dofs] == s).astype(np.uint8), iface)


@pytest.fixture(scope="module")
def full():
    prob = gen.chamber_problem(n=N_GRID, nz=N_Z, degree=2, n_sub=N_SUB, overlap=2, n_sources=32)
    say(f"[gpu] full-size chamber n={N_GRID} nz={N_Z} blocks={N_SUB}: oracle setup")
    m = prob.mesh
    d = Discretization(m.xyz, m.tets, prob.eps, m.bfaces, m.bface_kind, prob.k0, prob.degree)
    A = d.global_matrix()
    return prob, d, A


def test_full_matrix_rhs_spmv(full):
    prob, d, A = full
    say("[gpu] full-size matrix / rhs / spmv")
    P = Problem.from_problem(prob, defer_factor=True)
    assert P.ndof == d.ndof
    vals = P.matrix_values()
    assert np.abs(vals - A.data).max() <= 1e-12 * np.abs(A.data).max()
    b = P.rhs(prob.sources[:1]).cpu().numpy()[0]
    bo = d.rhs(prob.sources[0])
    assert np.abs(b - bo).max() <= 1e-12 * np.abs(bo).max()
    rng = np.random.default_rng(7)
    x = rng.standard_normal(d.ndof) + 1j * rng.standard_normal(d.ndof)
    y = P.apply_A(torch.from_numpy(x[None]).cuda()).cpu().numpy()[0]
    assert np.linalg.norm(y - A @ x) <= 1e-13 * np.linalg.norm(A @ x)
    P.close()


def check_sampled(prob, d, A, z, v, rng, tol, label):
    own = owners(d, prob.part)
    picks = list(rng.choice(prob.n_sub, size=6, replace=False)) + [0, prob.n_sub - 1]
    lay = Layout.from_problem(prob)
    for s in picks:
        sub = oracle_subdomain(d, prob.part, own, int(s), prob.overlap)
        dofs, pou = lay.subdomain(int(s))
        assert np.array_equal(dofs, sub.dofs) and np.array_equal(pou, sub.pou), s
        lu = spla.splu(local_matrix(d, sub))
        o = sub.pou == 1
        for c in range(v.shape[0]):
            y = lu.solve(v[c][sub.dofs])
            err = np.linalg.norm(z[c][sub.dofs[o]] - y[o]) / np.linalg.norm(y[o])
            assert err <= tol, (s, c, err)
        say(f"   {label} subdomain {s}: n_s={len(sub.dofs)} owned={int(o.sum())} last rel err {err:.2e}")


def test_full_oras_sampled_subdomains(full):
    prob, d, A = full
    say("[gpu] full-size ORAS application (FP64, one column), sampled subdomains")
    P = Problem.from_problem(prob)
    rng = np.random.default_rng(8)
    v = rng.standard_normal((1, d.ndof)) + 1j * rng.standard_normal((1, d.ndof))
    z = P.apply_prec(torch.from_numpy(v).cuda()).cpu().numpy()
    check_sampled(prob, d, A, z, v, rng, 1e-9, "fp64")
    P.close()


def test_full_oras_32_columns_mixed(full):
    """The multi-column kernel in the configuration of the batched benchmark
    (32 columns, FP32 factors) against the FP64 oracle: FP32 rounding of the
    factors and of the solve, checked at 1e-4 relative per owned block."""
    prob, d, A = full
    say("[gpu] full-size ORAS application (FP32 factors, 32 columns), sampled subdomains")
    P = Problem.from_problem(prob, precision=B.MXW_MIXED)
    rng = np.random.default_rng(9)
    v = rng.standard_normal((32, d.ndof)) + 1j * rng.standard_normal((32, d.ndof))
    z = P.apply_prec(torch.from_numpy(v).cuda()).cpu().numpy()
    check_sampled(prob, d, A, z, v[:4], rng, 1e-4, "mixed")
    P.close()


def test_full_solve_true_residual(full):
    """The benchmark's solve (FP64, one dipole): the true relative residual,
    recomputed with the oracle's matrix and right-hand side, is below 1e-8."""
    prob, d, A = full
    say("[gpu] full-size FGMRES + ORAS solve (FP64, 1 dipole)")
    P = Problem.from_problem(prob)
    x, it, rr, st = P.solve(prob.sources[:1])
    x = x.cpu().numpy()[0]
    b = d.rhs(prob.sources[0])
    true_rr = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    say(f"   iterations {it[0]} reported {rr[0]:.3e} true {true_rr:.3e}")
    assert rr[0] <= 1e-8 and true_rr <= 1.01e-8
    P.close()


def test_full_block_mixed_restart30(full):
    """Block FGMRES(30) on the batched benchmark's 32 dipoles with FP32 factors:
    the residual block becomes numerically low-rank over the restarts, and the
    Cholesky QR of a cycle's first block met floored pivots; it once ended in
    non-finite values (MXW_EBREAKDOWN at the first step of the 12th cycle).
    It must converge, with the true residuals of two sources recomputed with
    the oracle's matrix and right-hand sides."""
    prob, d, A = full
    say("[gpu] full-size block FGMRES(30), 32 dipoles, FP32 factors")
    P = Problem.from_problem(prob, precision=B.MXW_MIXED)
    x, it, rr, st = P.solve(prob.sources, krylov=B.MXW_KRYLOV_BLOCK, restart=30, max_iters=1200)
    say(f"   block steps {it[0]}, max relres {rr.max():.2e}")
    assert st == B.MXW_OK and np.all(rr <= 1e-8)
    x = x.cpu().numpy()
    for c in (0, 17):
        b = d.rhs(prob.sources[c])
        assert np.linalg.norm(b - A @ x[c]) <= 1.01e-8 * np.linalg.norm(b), c
    P.close()
