"""High-order Nedelec generators on a tetrahedron (oracle).

Sec. 3 defines the Whitney edge function of an oriented edge e = {n_i, n_j}
as w^e = lambda_i grad(lambda_j) - lambda_j grad(lambda_i) and the degree-r
generators as lambda^k w^e for every edge e and every multi-index k of weight
r-1.  These generators are linearly dependent for r > 1; the paper defers the
choice of an independent subset to other work.  The subset used here (the
same one the GPU library uses, implemented separately there) is, for a tet
with vertices ordered by global id a<b<c<d:

* edge (x<y): lambda_x^{k_x} lambda_y^{k_y} w^{xy}, k_x + k_y = r-1, listed
  with k_x = r-1, ..., 0 (r per edge);
* face (x<y<z), r >= 2: lambda^k w^{xy} with k on {x,y,z}, |k| = r-1, k_z >= 1,
  then lambda^k w^{xz} with k_y >= 1; within each, (k_x,k_y,k_z) in
  descending lexicographic order (r(r-1) per face; the generators on edge
  (y,z) are the ones dropped);
* volume, r = 3: lambda_c lambda_d w^{ab}, lambda_b lambda_d w^{ac},
  lambda_b lambda_c w^{ad} (3 per tet).

That gives 6, 20, 45 functions per tet for r = 1, 2, 3, the dimension
r(r+2)(r+3)/2 of the degree-r Nedelec space.

Local vertices 0..3 are the tet's vertices sorted by global id, so local
order equals global order and every generator is oriented low -> high.
Integrals of barycentric monomials use the exact formula
  int_T lambda^alpha = 6 |T| alpha! / (|alpha| + 3)!,
  int_F lambda^alpha = 2 |F| alpha! / (|alpha| + 2)!   (alpha on F's vertices).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from math import factorial

import numpy as np

LOCAL_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
LOCAL_FACES = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
CROSS_PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


@dataclass(frozen=True)
class Generator:
    kind: int          # 0 edge, 1 face, 2 volume
    entity: int        # local edge index, local face index, or 0
    sub: int           # index within the entity
    edge: tuple        # (i, j) local vertices, i < j
    k: tuple           # multi-index (k0, k1, k2, k3), weight r-1


def _weights(verts, total):
    """All multi-indices of weight `total` supported on `verts`, descending lex."""
    out = []
    for combo in itertools.product(range(total, -1, -1), repeat=len(verts)):
        if sum(combo) == total:
            k = [0, 0, 0, 0]
            for v, c in zip(verts, combo):
                k[v] = c
            out.append((tuple(combo), tuple(k)))
    out.sort(key=lambda t: t[0], reverse=True)
    return [k for _, k in out]


def generators(r: int) -> list:
    gens = []
    for le, (i, j) in enumerate(LOCAL_EDGES):
        for s, k in enumerate(_weights((i, j), r - 1)):
            gens.append(Generator(0, le, s, (i, j), k))
    if r >= 2:
        for lf, (x, y, z) in enumerate(LOCAL_FACES):
            s = 0
            for e, opp in (((x, y), z), ((x, z), y)):
                for k in _weights((x, y, z), r - 1):
                    if k[opp] >= 1:
                        gens.append(Generator(1, lf, s, e, k))
                        s += 1
    if r == 3:
        for s, (e, pq) in enumerate((((0, 1), (2, 3)), ((0, 2), (1, 3)), ((0, 3), (1, 2)))):
            k = [0, 0, 0, 0]
            k[pq[0]] = 1
            k[pq[1]] = 1
            gens.append(Generator(2, 0, s, e, tuple(k)))
    return gens


def _add(a, b):
    return tuple(x + y for x, y in zip(a, b))


def _unit(m):
    e = [0, 0, 0, 0]
    e[m] = 1
    return tuple(e)


def phi_terms(g: Generator):
    """phi = lambda^k (lambda_i grad l_j - lambda_j grad l_i) as (coef, alpha, m)."""
    i, j = g.edge
    return [(1.0, _add(g.k, _unit(i)), j), (-1.0, _add(g.k, _unit(j)), i)]


def curl_terms(g: Generator):
    """curl phi as (coef, beta, (u,v)) meaning coef lambda^beta grad l_u x grad l_v.

    curl(f w) = grad f x w + f curl w with curl w^{ij} = 2 grad l_i x grad l_j
    and grad lambda^k = sum_m k_m lambda^{k - e_m} grad l_m.
    """
    i, j = g.edge
    raw = [(2.0, g.k, (i, j))]
    for m in range(4):
        km = g.k[m]
        if km == 0:
            continue
        base = list(g.k)
        base[m] -= 1
        base = tuple(base)
        raw.append((float(km), _add(base, _unit(i)), (m, j)))     # grad l_m x lambda_i grad l_j
        raw.append((-float(km), _add(base, _unit(j)), (m, i)))    # - grad l_m x lambda_j grad l_i
    out = []
    for c, beta, (u, v) in raw:
        if u == v:
            continue
        if u > v:
            u, v, c = v, u, -c
        out.append((c, beta, (u, v)))
    return out


def _int_tet(alpha):
    """int_T lambda^alpha / |T|."""
    num = 6 * np.prod([factorial(a) for a in alpha])
    return num / factorial(sum(alpha) + 3)


def _int_face(alpha):
    """int_F lambda^alpha / |F| (alpha supported on the face)."""
    num = 2 * np.prod([factorial(a) for a in alpha])
    return num / factorial(sum(alpha) + 2)


class Basis:
    """Generators of degree r with reference tensors for exact integration."""

    def __init__(self, r: int):
        if r not in (1, 2, 3):
            raise ValueError("degree must be 1, 2 or 3")
        self.r = r
        self.gens = generators(r)
        self.nloc = len(self.gens)
        n = self.nloc
        pt = [phi_terms(g) for g in self.gens]
        ct = [curl_terms(g) for g in self.gens]
        # M_T[p,q] = |T| sum_{u,v} WM[p,q,u,v] (grad l_u . grad l_v)
        WM = np.zeros((n, n, 4, 4))
        for p in range(n):
            for q in range(n):
                for c1, a1, m1 in pt[p]:
                    for c2, a2, m2 in pt[q]:
                        WM[p, q, m1, m2] += c1 * c2 * _int_tet(_add(a1, a2))
        # K_T[p,q] = |T| sum_{a,b} WK[p,q,a,b] (X_a . X_b), X_a = grad l_u x grad l_v
        WK = np.zeros((n, n, 6, 6))
        for p in range(n):
            for q in range(n):
                for c1, b1, uv1 in ct[p]:
                    for c2, b2, uv2 in ct[q]:
                        WK[p, q, CROSS_PAIRS.index(uv1), CROSS_PAIRS.index(uv2)] += \
                            c1 * c2 * _int_tet(_add(b1, b2))
        # face tensors: only generators whose edge and multi-index lie in the face
        WB = np.zeros((4, n, n, 4, 4))
        self.face_mask = np.zeros((4, n), dtype=bool)
        for lf, fv in enumerate(LOCAL_FACES):
            opp = ({0, 1, 2, 3} - set(fv)).pop()
            for p, g in enumerate(self.gens):
                self.face_mask[lf, p] = (opp not in g.edge) and g.k[opp] == 0
            for p in range(n):
                if not self.face_mask[lf, p]:
                    continue
                for q in range(n):
                    if not self.face_mask[lf, q]:
                        continue
                    for c1, a1, m1 in pt[p]:
                        for c2, a2, m2 in pt[q]:
                            WB[lf, p, q, m1, m2] += c1 * c2 * _int_face(_add(a1, a2))
        self.WM, self.WK, self.WB = WM, WK, WB

    # ---- pointwise evaluation, written directly from the definitions --------

    def eval_phi(self, lam, grads):
        """Values of all generators at a point: [nloc,3]."""
        out = np.zeros((self.nloc, 3))
        for p, g in enumerate(self.gens):
            i, j = g.edge
            w = lam[i] * grads[j] - lam[j] * grads[i]
            out[p] = np.prod([lam[m] ** g.k[m] for m in range(4)]) * w
        return out

    def eval_curl(self, lam, grads):
        """Curls of all generators at a point: [nloc,3]."""
        out = np.zeros((self.nloc, 3))
        for p, g in enumerate(self.gens):
            i, j = g.edge
            w = lam[i] * grads[j] - lam[j] * grads[i]
            mono = np.prod([lam[m] ** g.k[m] for m in range(4)])
            grad_mono = np.zeros(3)
            for m in range(4):
                if g.k[m] > 0:
                    rest = np.prod([lam[q] ** (g.k[q] - (q == m)) for q in range(4)])
                    grad_mono += g.k[m] * rest * grads[m]
            out[p] = np.cross(grad_mono, w) + 2.0 * mono * np.cross(grads[i], grads[j])
        return out


def cross_products(grads):
    """X[t,a] = grad l_u x grad l_v for the 6 ordered pairs (u<v): [T,6,3]."""
    return np.stack([np.cross(grads[:, u], grads[:, v]) for u, v in CROSS_PAIRS], axis=1)


def element_mass_stiffness(basis: Basis, grads, vol):
    """Exact M_T = int phi.phi and K_T = int curl phi . curl phi, [T,n,n] each."""
    G = np.einsum("tui,tvi->tuv", grads, grads)
    X = cross_products(grads)
    C = np.einsum("tai,tbi->tab", X, X)
    M = vol[:, None, None] * np.einsum("pquv,tuv->tpq", basis.WM, G)
    K = vol[:, None, None] * np.einsum("pqab,tab->tpq", basis.WK, C)
    return M, K


def face_matrix(basis: Basis, lf: int, grads_t, normal, area):
    """B_F[p,q] = int_F phi_p.phi_q - (phi_p.n)(phi_q.n) over the tet's generators.

    Rows and columns of generators not living on face lf are zero.
    """
    G = grads_t @ grads_t.T
    gn = grads_t @ normal
    GF = G - np.outer(gn, gn)
    return area * np.einsum("pquv,uv->pq", basis.WB[lf], GF)
