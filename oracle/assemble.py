"""Global matrix, right-hand sides and field evaluation (oracle).

Time convention exp(-i w t) (the complex conjugate of the paper's Sec. 2):
a lossy medium has Im(eps) > 0 and the impedance condition reads
(curl E) x n - i beta n x (E x n) = g.  Integrating eq. (1) by parts against
a test field v gives the bilinear (not sesquilinear) form of Sec. 2,
  int curl E . curl v - k0^2 eps E . v - i beta int_Gamma E_t . v_t
    = int_Gamma g . v,
so the matrix is A = K - k0^2 M_eps - i beta B, complex symmetric.

beta on an impedance face is k0 sqrt(Re eps) of the adjacent element (the
dissipation-free wavenumber of Sec. 2; the paper ties beta to its waveguide
ports, which these synthetic workloads do not have).

Boundary integrals of non-polynomial data use a collapsed (Duffy) product
Gauss-Legendre rule on the triangle with q = r + 3 points per direction:
  mu1 = xi (1 - eta), mu2 = xi eta, mu0 = 1 - xi, weight 2|F| w_xi w_eta xi.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import Basis, LOCAL_FACES, element_mass_stiffness, face_matrix
from .mesh import DofMap, IMPEDANCE, Topology

SRC_DIPOLE = 0
SRC_PLANEWAVE = 1
SRC_PORT = 2


def face_geometry(topo: Topology, t: int, lf: int):
    """Outward unit normal and area of local face lf of tet t."""
    verts = topo.tets[t]
    fv = LOCAL_FACES[lf]
    opp = ({0, 1, 2, 3} - set(fv)).pop()
    P = topo.xyz[verts[list(fv)]]
    nrm = np.cross(P[1] - P[0], P[2] - P[0])
    area = 0.5 * np.linalg.norm(nrm)
    nrm = nrm / np.linalg.norm(nrm)
    if np.dot(topo.xyz[verts[opp]] - P[0], nrm) > 0:
        nrm = -nrm
    return nrm, area


def local_face_index(topo: Topology, t: int, face_id: int) -> int:
    return int(np.nonzero(topo.tet_faces[t] == face_id)[0][0])


class Discretization:
    """Everything the global system needs: topology, unknowns, element data."""

    def __init__(self, xyz, tets, eps, bfaces, bface_kind, k0: float, degree: int):
        self.topo = Topology(xyz, tets)
        self.basis = Basis(degree)
        self.dofs = DofMap(self.topo, self.basis, bfaces, bface_kind)
        self.eps = np.asarray(eps, dtype=np.complex128)
        self.k0 = float(k0)
        self.grads, self.vol = self.topo.all_geometry()
        M, K = element_mass_stiffness(self.basis, self.grads, self.vol)
        self.M, self.K = M, K
        # element matrices A_T = K_T - k0^2 eps_T M_T
        self.AT = K - (self.k0 ** 2) * self.eps[:, None, None] * M
        # impedance boundary faces: (tet, local face, beta)
        self.imp_faces = []
        for f, kind in zip(self.dofs.bface_ids, self.dofs.bface_kind):
            if kind != IMPEDANCE:
                continue
            t = int(self.topo.face_tets[f, 0])
            lf = local_face_index(self.topo, t, f)
            beta = self.k0 * np.sqrt(self.eps[t].real)
            self.imp_faces.append((t, lf, beta))

    @property
    def ndof(self):
        return self.dofs.ndof

    def face_B(self, t: int, lf: int):
        nrm, area = face_geometry(self.topo, t, lf)
        return face_matrix(self.basis, lf, self.grads[t], nrm, area)

    # ------------------------------------------------------------------
    def pattern(self):
        """Structural pattern: (i,j) co-occurring in one tet, columns ascending."""
        td = self.dofs.tet_dofs
        n = td.shape[1]
        rows = np.repeat(td, n, axis=1).ravel()
        cols = np.tile(td, (1, n)).ravel()
        ok = (rows >= 0) & (cols >= 0)
        P = sp.csr_matrix((np.ones(ok.sum()), (rows[ok], cols[ok])), shape=(self.ndof, self.ndof))
        P.sum_duplicates()
        P.sort_indices()
        return P.indptr.astype(np.int64), P.indices.astype(np.int64)

    def global_matrix(self):
        """A = sum_T A_T - sum_{impedance F} i beta_F B_F, CSR with the structural pattern."""
        td = self.dofs.tet_dofs
        n = td.shape[1]
        rows = np.repeat(td, n, axis=1).ravel()
        cols = np.tile(td, (1, n)).ravel()
        vals = self.AT.reshape(len(td), -1).ravel().astype(np.complex128)
        R, Cc, V = [rows], [cols], [vals]
        for t, lf, beta in self.imp_faces:
            B = self.face_B(t, lf)
            R.append(np.repeat(td[t], n))
            Cc.append(np.tile(td[t], n))
            V.append((-1j * beta * B).ravel())
        rows = np.concatenate(R)
        cols = np.concatenate(Cc)
        vals = np.concatenate(V)
        ok = (rows >= 0) & (cols >= 0)
        A = sp.coo_matrix((vals[ok], (rows[ok], cols[ok])), shape=(self.ndof, self.ndof)).tocsr()
        A.sum_duplicates()
        A.sort_indices()
        # make the stored pattern exactly the structural one (keep explicit zeros)
        rp, ci = self.pattern()
        if not (np.array_equal(A.indptr, rp) and np.array_equal(A.indices, ci)):
            Z = sp.csr_matrix((np.zeros(len(ci), dtype=np.complex128), ci, rp), shape=A.shape)
            A = (A + Z).tocsr()
            A.sort_indices()
            assert np.array_equal(A.indptr, rp) and np.array_equal(A.indices, ci)
        return A

    # ------------------------------------------------------------------
    def barycentric(self, t: int, x):
        verts = self.topo.tets[t]
        X = self.topo.xyz[verts]
        return np.linalg.solve(np.hstack([X, np.ones((4, 1))]).T, np.append(x, 1.0))

    def locate(self, x):
        """Lowest-index tet whose barycentric coordinates at x are all >= -1e-12."""
        X = self.topo.xyz[self.topo.tets]
        Mx = np.concatenate([X, np.ones((len(X), 4, 1))], axis=2)
        lam = np.linalg.solve(np.transpose(Mx, (0, 2, 1)), np.broadcast_to(np.append(x, 1.0), (len(X), 4))[..., None])[..., 0]
        inside = np.nonzero(np.all(lam >= -1e-12, axis=1))[0]
        if len(inside) == 0:
            raise ValueError("source point outside the mesh")
        return int(inside[0])

    def rhs_dipole(self, pos, pol):
        """b_i = p . phi_i(x_s) (point dipole; the constant i w mu0 is dropped)."""
        t = self.locate(np.asarray(pos, dtype=np.float64))
        lam = self.barycentric(t, pos)
        vals = self.basis.eval_phi(lam, self.grads[t]) @ np.asarray(pol, dtype=np.complex128)
        b = np.zeros(self.ndof, dtype=np.complex128)
        for p, d in enumerate(self.dofs.tet_dofs[t]):
            if d >= 0:
                b[d] += vals[p]
        return b

    def face_points(self, t: int, lf: int, q: int):
        """Collapsed Gauss-Legendre points on face lf of tet t: (lam[4] list, weights)."""
        g, w = np.polynomial.legendre.leggauss(q)
        g = 0.5 * (g + 1.0)
        w = 0.5 * w
        nrm, area = face_geometry(self.topo, t, lf)
        fv = LOCAL_FACES[lf]
        pts, wts = [], []
        for xi, wx in zip(g, w):
            for eta, we in zip(g, w):
                mu = (1.0 - xi, xi * (1.0 - eta), xi * eta)
                lam = np.zeros(4)
                for v, m in zip(fv, mu):
                    lam[v] = m
                pts.append(lam)
                wts.append(2.0 * area * wx * we * xi)
        return pts, np.array(wts), nrm

    def tet_points(self, t: int, q: int):
        """Collapsed (Stroud) product Gauss-Legendre points inside tet t."""
        g, w = np.polynomial.legendre.leggauss(q)
        g = 0.5 * (g + 1.0)
        w = 0.5 * w
        pts, wts = [], []
        for a, wa in zip(g, w):
            for b, wb in zip(g, w):
                for c, wc in zip(g, w):
                    l1 = a
                    l2 = b * (1.0 - a)
                    l3 = c * (1.0 - a) * (1.0 - b)
                    lam = np.array([1.0 - l1 - l2 - l3, l1, l2, l3])
                    pts.append(lam)
                    wts.append(6.0 * self.vol[t] * wa * wb * wc * (1.0 - a) ** 2 * (1.0 - b))
        return pts, np.array(wts)

    def point(self, t: int, lam):
        return lam @ self.topo.xyz[self.topo.tets[t]]

    def rhs_boundary(self, gfun, q=None, faces=None):
        """b_i = int_{impedance faces} g . phi_i; gfun(x, n, beta, t) -> complex 3-vector.
        faces: a subset of imp_faces (default all)."""
        q = q if q is not None else self.basis.r + 3
        b = np.zeros(self.ndof, dtype=np.complex128)
        for t, lf, beta in (self.imp_faces if faces is None else faces):
            pts, wts, nrm = self.face_points(t, lf, q)
            loc = np.zeros(self.basis.nloc, dtype=np.complex128)
            for lam, wq in zip(pts, wts):
                x = self.point(t, lam)
                phi = self.basis.eval_phi(lam, self.grads[t])
                phi[~self.basis.face_mask[lf]] = 0.0
                loc += wq * (phi @ gfun(x, nrm, beta, t))
            for p, d in enumerate(self.dofs.tet_dofs[t]):
                if d >= 0:
                    b[d] += loc[p]
        return b

    def rhs_volume(self, ffun, q=None):
        """b_i = int_Omega f . phi_i (used only by self-tests)."""
        q = q if q is not None else self.basis.r + 3
        b = np.zeros(self.ndof, dtype=np.complex128)
        for t in range(self.topo.n_tets):
            pts, wts = self.tet_points(t, q)
            loc = np.zeros(self.basis.nloc, dtype=np.complex128)
            for lam, wq in zip(pts, wts):
                x = self.point(t, lam)
                loc += wq * (self.basis.eval_phi(lam, self.grads[t]) @ ffun(x, t))
            for p, d in enumerate(self.dofs.tet_dofs[t]):
                if d >= 0:
                    b[d] += loc[p]
        return b

    def kappa(self, t: int):
        """Complex wavenumber k0 sqrt(eps) of tet t (principal root, Im >= 0)."""
        return self.k0 * np.sqrt(self.eps[t])

    def rhs_planewave(self, pol, direction):
        """Impedance data g of the incident wave E = p exp(i kappa d.x).

        kappa = k0 sqrt(eps) makes E an exact solution of eq. (1) in a
        homogeneous medium; g = (curl E) x n - i beta n x (E x n) with
        curl E = i kappa d x E.
        """
        p = np.asarray(pol, dtype=np.complex128)
        d = np.asarray(direction, dtype=np.float64)

        def g(x, n, beta, t):
            kap = self.kappa(t)
            E = p * np.exp(1j * kap * (d @ x))
            curlE = 1j * kap * np.cross(d, E)
            return np.cross(curlE, n) - 1j * beta * np.cross(n, np.cross(E, n))

        return self.rhs_boundary(g)

    def rhs(self, src):
        if src.kind == SRC_DIPOLE:
            return self.rhs_dipole(src.pos, src.pol)
        if src.kind == SRC_PLANEWAVE:
            return self.rhs_planewave(src.pol, src.dir)
        if src.kind == SRC_PORT:
            from .ports import rhs_port
            return rhs_port(self, src)
        raise ValueError("unknown source kind")

    # ------------------------------------------------------------------
    def field(self, u, t: int, lam):
        """E_h at barycentric point lam of tet t."""
        coef = np.array([u[d] if d >= 0 else 0.0 for d in self.dofs.tet_dofs[t]], dtype=np.complex128)
        return coef @ self.basis.eval_phi(lam, self.grads[t])

    def l2_error(self, u, efun, q=None):
        """(int |E_h - E|^2)^(1/2) and (int |E|^2)^(1/2) by tet quadrature."""
        q = q if q is not None else self.basis.r + 3
        err = ref = 0.0
        for t in range(self.topo.n_tets):
            pts, wts = self.tet_points(t, q)
            for lam, wq in zip(pts, wts):
                x = self.point(t, lam)
                e = efun(x, t)
                d = self.field(u, t, lam) - e
                err += wq * np.real(np.vdot(d, d))
                ref += wq * np.real(np.vdot(e, e))
        return np.sqrt(err), np.sqrt(ref)
