"""Mesh entities and the global ordered unknown set (oracle).

Sec. 3 attaches the degrees of freedom of Nedelec elements to oriented
mesh entities (edges for r=1; edges, faces and, for r=3, the tetrahedron
itself for the high-order generators).  Sec. 4 needs "an ordered set of the
unknowns of the whole domain"; the ordering used here is:

* edges = distinct vertex pairs (a<b), numbered in lexicographic order;
* faces = distinct vertex triples (a<b<c), numbered lexicographically;
* tetrahedra keep their input order;
* unknowns: all edge unknowns (edge order, then the order within the edge),
  then all face unknowns, then all volume unknowns;
* unknowns on entities lying in a metallic face (E x n = 0, eq. (2)) are
  removed, the others keep their relative order.

Every edge generator is oriented from its lower to its higher global vertex
id.
"""
from __future__ import annotations

import numpy as np

from .basis import Basis

PEC = 0
IMPEDANCE = 1


class Topology:
    """Edges, faces, boundary faces and element-to-entity maps of a tet mesh."""

    def __init__(self, xyz: np.ndarray, tets: np.ndarray):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        tets = np.asarray(tets, dtype=np.int64)
        # vertices of each tet sorted by global id: local vertex 0 is the
        # lowest global id, so each local edge (i<j) is globally oriented i->j
        self.tets = np.sort(tets, axis=1)
        T = len(self.tets)
        self.n_tets = T
        self.n_vertices = len(self.xyz)

        ledges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
        lfaces = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
        self.local_edges = ledges
        self.local_faces = lfaces

        # --- edges: unique sorted pairs in lexicographic order
        ev = np.stack([self.tets[:, list(e)] for e in ledges], axis=1)       # [T,6,2]
        flat = ev.reshape(-1, 2)
        self.edges, inv = np.unique(flat, axis=0, return_inverse=True)
        self.tet_edges = inv.reshape(T, 6)

        # --- faces: unique sorted triples in lexicographic order
        fv = np.stack([self.tets[:, list(f)] for f in lfaces], axis=1)       # [T,4,3]
        flat = fv.reshape(-1, 3)
        self.faces, inv = np.unique(flat, axis=0, return_inverse=True)
        self.tet_faces = inv.reshape(T, 4)

        # --- face -> adjacent tets (one or two); boundary faces have one
        cnt = np.bincount(self.tet_faces.ravel(), minlength=len(self.faces))
        self.face_ntets = cnt
        self.boundary_face_ids = np.nonzero(cnt == 1)[0]
        # neighbour across each local face (-1 on the boundary)
        owner = np.full((len(self.faces), 2), -1, dtype=np.int64)
        for t in range(T):
            for lf in range(4):
                f = self.tet_faces[t, lf]
                if owner[f, 0] < 0:
                    owner[f, 0] = t
                else:
                    owner[f, 1] = t
        self.face_tets = owner

    def geometry(self, t: int):
        """Barycentric gradients (rows) and volume of tet t (sorted vertex order)."""
        X = self.xyz[self.tets[t]]
        Mx = np.hstack([X, np.ones((4, 1))])
        C = np.linalg.inv(Mx)
        return C[:3, :].T.copy(), abs(np.linalg.det(Mx)) / 6.0

    def all_geometry(self):
        """Vectorised barycentric gradients [T,4,3] and volumes [T]."""
        X = self.xyz[self.tets]                               # [T,4,3]
        Mx = np.concatenate([X, np.ones((self.n_tets, 4, 1))], axis=2)
        C = np.linalg.inv(Mx)                                 # [T,4,4]
        grads = np.transpose(C[:, :3, :], (0, 2, 1))          # grad lambda_i = C[:3,i]
        vol = np.abs(np.linalg.det(Mx)) / 6.0
        return grads, vol


class DofMap:
    """Global unknown numbering for degree r on a Topology (see module doc)."""

    def __init__(self, topo: Topology, basis: Basis, bfaces: np.ndarray, bface_kind: np.ndarray):
        self.topo = topo
        self.basis = basis
        r = basis.r
        ne, nf, nt = len(topo.edges), len(topo.faces), topo.n_tets
        self.per_edge = r
        self.per_face = r * (r - 1)
        self.per_tet = r * (r - 1) * (r - 2) // 2

        # boundary faces given by the caller must be exactly the faces with one tet
        bsorted = np.sort(np.asarray(bfaces, dtype=np.int64), axis=1)
        fidx = {tuple(f): i for i, f in enumerate(topo.faces.tolist())}
        self.bface_ids = np.array([fidx[tuple(f)] for f in bsorted.tolist()], dtype=np.int64)
        if sorted(self.bface_ids.tolist()) != sorted(topo.boundary_face_ids.tolist()):
            raise ValueError("boundary faces differ from the faces with one tetrahedron")
        self.bface_kind = np.asarray(bface_kind, dtype=np.int64)

        # entities lying on metallic faces
        pec_face = np.zeros(nf, dtype=bool)
        pec_face[self.bface_ids[self.bface_kind == PEC]] = True
        eidx = {tuple(e): i for i, e in enumerate(topo.edges.tolist())}
        pec_edge = np.zeros(ne, dtype=bool)
        for f in np.nonzero(pec_face)[0]:
            a, b, c = topo.faces[f]
            for e in ((a, b), (a, c), (b, c)):
                pec_edge[eidx[e]] = True
        self.pec_edge = pec_edge
        self.pec_face = pec_face

        # full numbering (before elimination): entity kind / id / local index
        kinds, ids, locs = [], [], []
        for e in range(ne):
            for l in range(self.per_edge):
                kinds.append(0); ids.append(e); locs.append(l)
        for f in range(nf):
            for l in range(self.per_face):
                kinds.append(1); ids.append(f); locs.append(l)
        for t in range(nt):
            for l in range(self.per_tet):
                kinds.append(2); ids.append(t); locs.append(l)
        kinds = np.array(kinds, dtype=np.int64)
        ids = np.array(ids, dtype=np.int64)
        locs = np.array(locs, dtype=np.int64)
        keep = np.ones(len(kinds), dtype=bool)
        is_e = kinds == 0
        is_f = kinds == 1
        keep[is_e] = ~pec_edge[ids[is_e]]
        keep[is_f] = ~pec_face[ids[is_f]]
        self.n_full = len(kinds)
        self.full_to_dof = np.full(len(kinds), -1, dtype=np.int64)
        self.full_to_dof[keep] = np.arange(keep.sum())
        self.ent_kind = kinds[keep]
        self.ent_id = ids[keep]
        self.ent_local = locs[keep]
        self.ndof = int(keep.sum())
        self.edge_base = 0
        self.face_base = ne * self.per_edge
        self.tet_base = self.face_base + nf * self.per_face

        # element -> global unknowns, in the basis' local generator order
        self.tet_dofs = self._tet_dofs()

    def _tet_dofs(self):
        topo, b = self.topo, self.basis
        T = topo.n_tets
        out = np.empty((T, b.nloc), dtype=np.int64)
        for p, g in enumerate(b.gens):
            if g.kind == 0:
                full = self.edge_base + topo.tet_edges[:, g.entity] * self.per_edge + g.sub
            elif g.kind == 1:
                full = self.face_base + topo.tet_faces[:, g.entity] * self.per_face + g.sub
            else:
                full = self.tet_base + np.arange(T) * self.per_tet + g.sub
            out[:, p] = self.full_to_dof[full]
        return out
