"""Overlapping decomposition and the ORAS preconditioner (oracle).

Sec. 4: M^{-1} = sum_s R_s^T D_s A_s^{-1} R_s, where R_s is the Boolean
restriction to the ordered unknown subset N_s of the overlapping subdomain
Omega_s, D_s a diagonal partition of unity with sum_s R_s^T D_s R_s = I, and
A_s the subdomain matrix with the impedance condition
(curl E) x n - i w~ n x (E x n) on the artificial interfaces (exp(-i w t)
convention), w~ = k0 sqrt(Re eps) of the element inside Omega_s that owns
the interface face.

Readings of what Sec. 4 leaves open:

* overlap: Omega_s^0 = elements with part == s; each layer adds every
  element sharing a face with the current set;
* N_s: the sorted global unknowns of all entities of all elements of Omega_s;
* D_s: Boolean; an unknown belongs to the subdomain with the smallest core
  id among the elements containing its entity (weight 1 there, 0 elsewhere);
* A_s: element matrices of Omega_s, the original impedance terms on faces of
  Omega_s on the outer boundary, and the transmission term on interface
  faces (faces of Omega_s whose neighbour element is outside Omega_s);
* local solves: sparse LU of A_s (scipy's SuperLU), an exact A_s^{-1}.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import Discretization, local_face_index


class Subdomain:
    def __init__(self, sid, tets, dofs, pou, iface):
        self.sid = sid
        self.tets = tets          # sorted element ids of Omega_s
        self.dofs = dofs          # N_s, sorted global unknowns
        self.pou = pou            # D_s diagonal, 0/1 uint8
        self.iface = iface        # list of (tet, local face, w~)
        self.A = None
        self.lu = None


def grow_overlap(disc: Discretization, part, s: int, layers: int):
    topo = disc.topo
    inside = np.asarray(part) == s
    for _ in range(layers):
        add = inside.copy()
        for t in np.nonzero(inside)[0]:
            for f in topo.tet_faces[t]:
                for u in topo.face_tets[f]:
                    if u >= 0:
                        add[u] = True
        inside = add
    return np.nonzero(inside)[0]


def owners(disc: Discretization, part):
    """owner(i) = min core id over the elements containing unknown i's entity."""
    own = np.full(disc.ndof, np.iinfo(np.int64).max, dtype=np.int64)
    td = disc.dofs.tet_dofs
    for t in range(len(td)):
        for d in td[t]:
            if d >= 0 and part[t] < own[d]:
                own[d] = part[t]
    return own


def build_subdomains(disc: Discretization, part, n_sub: int, layers: int):
    part = np.asarray(part, dtype=np.int64)
    own = owners(disc, part)
    topo = disc.topo
    subs = []
    for s in range(n_sub):
        tets = grow_overlap(disc, part, s, layers)
        in_s = np.zeros(topo.n_tets, dtype=bool)
        in_s[tets] = True
        d = disc.dofs.tet_dofs[tets].ravel()
        dofs = np.unique(d[d >= 0])
        pou = (own[dofs] == s).astype(np.uint8)
        iface = []
        for t in tets:
            for lf, f in enumerate(topo.tet_faces[t]):
                other = [u for u in topo.face_tets[f] if u >= 0 and u != t]
                if other and not in_s[other[0]]:
                    iface.append((int(t), lf, disc.k0 * np.sqrt(disc.eps[t].real)))
        subs.append(Subdomain(s, tets, dofs, pou, iface))
    return subs


def local_matrix(disc: Discretization, sub: Subdomain, dirichlet: bool = False):
    """A_s on N_s (dense index positions given by searchsorted into N_s)."""
    td = disc.dofs.tet_dofs
    n = disc.basis.nloc
    in_s = np.zeros(disc.topo.n_tets, dtype=bool)
    in_s[sub.tets] = True
    R, C, V = [], [], []

    def add(t, mat):
        g = td[t]
        rows = np.repeat(g, n)
        cols = np.tile(g, n)
        ok = (rows >= 0) & (cols >= 0)
        R.append(rows[ok]); C.append(cols[ok]); V.append(mat.ravel()[ok])

    for t in sub.tets:
        add(t, disc.AT[t])
    for t, lf, beta in disc.imp_faces:
        if in_s[t]:
            add(t, -1j * beta * disc.face_B(t, lf))
    if not dirichlet:
        for t, lf, wt in sub.iface:
            add(t, -1j * wt * disc.face_B(t, lf))
    rows = np.searchsorted(sub.dofs, np.concatenate(R))
    cols = np.searchsorted(sub.dofs, np.concatenate(C))
    ns = len(sub.dofs)
    return sp.coo_matrix((np.concatenate(V), (rows, cols)), shape=(ns, ns)).tocsc()


class ORAS:
    """z = sum_s R_s^T D_s A_s^{-1} R_s v (variant='oras'); 'oas' drops D_s;
    'ras' uses A_s = R_s A R_s^T (Dirichlet transmission) with D_s;
    'oras_mult' keeps the Robin A_s and takes the partition of unity by
    multiplicity, D_s = diag(1 / number of subdomains containing the unknown)
    (Sec. 4 allows any D_s with sum_s R_s^T D_s R_s = I)."""

    def __init__(self, disc: Discretization, part, n_sub: int, layers: int, variant: str = "oras",
                 A=None):
        self.disc = disc
        self.variant = variant
        self.subs = build_subdomains(disc, part, n_sub, layers)
        for sub in self.subs:
            if variant == "ras":
                sub.A = A[sub.dofs][:, sub.dofs].tocsc()
            else:
                sub.A = local_matrix(disc, sub)
            sub.lu = spla.splu(sub.A)
        if variant == "oras_mult":
            mult = np.zeros(disc.ndof)
            for sub in self.subs:
                mult[sub.dofs] += 1.0
            for sub in self.subs:
                sub.weight = 1.0 / mult[sub.dofs]

    def weights(self, sub):
        """The diagonal of D_s."""
        if self.variant == "oas":
            return np.ones(len(sub.dofs))
        if self.variant == "oras_mult":
            return sub.weight
        return sub.pou.astype(np.float64)

    def apply(self, v):
        """z = M^{-1} v; v is one vector [n] or several columns [n, k] (the
        columns are handed to each local solve together)."""
        z = np.zeros(v.shape, dtype=np.complex128)
        for sub in self.subs:
            y = sub.lu.solve(np.asarray(v[sub.dofs], dtype=np.complex128))
            w = self.weights(sub)
            z[sub.dofs] += w[:, None] * y if y.ndim == 2 else w * y
        return z
