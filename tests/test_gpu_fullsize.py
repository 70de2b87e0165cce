"""Parity at the benchmark's full size (synthetic chamber, r=2, 1,470,500
unknowns, RCB subdomains, 2 face layers), on outputs the oracle can compute
piece by piece: every value of the global matrix, the right-hand side, one
SpMV, and the ORAS application restricted to the unknowns owned by a sample
of subdomains (each checked against the oracle's own local matrix and sparse
LU for that subdomain)."""
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

N_GRID = int(os.environ.get("MXW_FULL_N", "34"))
N_SUB = int(os.environ.get("MXW_FULL_NSUB", "2500"))


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
    prob = gen.chamber_problem(n=N_GRID, degree=2, n_sub=N_SUB, overlap=2)
    say(f"[gpu] full-size chamber n={N_GRID} n_sub={N_SUB}: oracle setup")
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


def test_full_oras_sampled_subdomains(full):
    prob, d, A = full
    say("[gpu] full-size ORAS application, sampled subdomains")
    P = Problem.from_problem(prob)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(d.ndof) + 1j * rng.standard_normal(d.ndof)
    z = P.apply_prec(torch.from_numpy(v[None]).cuda()).cpu().numpy()[0]
    own = owners(d, prob.part)
    picks = list(rng.choice(prob.n_sub, size=6, replace=False)) + [0, prob.n_sub - 1]
    lay = Layout.from_problem(prob)
    for s in picks:
        sub = oracle_subdomain(d, prob.part, own, int(s), prob.overlap)
        dofs, pou = lay.subdomain(int(s))
        assert np.array_equal(dofs, sub.dofs) and np.array_equal(pou, sub.pou), s
        y = spla.splu(local_matrix(d, sub)).solve(v[sub.dofs])
        o = sub.pou == 1
        err = np.linalg.norm(z[sub.dofs[o]] - y[o]) / np.linalg.norm(y[o])
        say(f"   subdomain {s}: n_s={len(sub.dofs)} owned={int(o.sum())} rel err {err:.2e}")
        assert err <= 1e-9, s
    P.close()
