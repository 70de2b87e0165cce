"""End-to-end forward solve (oracle): mesh + eps + k0 + sources + r + partition
-> E coefficients, iteration counts, true relative residuals.

The steps follow the paper's order: discretise (Sec. 2-3), build the
overlapping decomposition and ORAS (Sec. 4), solve each right-hand side with
preconditioned GMRES (Sec. 5).
"""
from __future__ import annotations

import numpy as np

from .assemble import Discretization
from .krylov import block_fgmres, fgmres
from .schwarz import ORAS


class OracleSolver:
    def __init__(self, xyz, tets, eps, bfaces, bface_kind, part, n_sub, overlap, k0, degree,
                 variant="oras"):
        self.disc = Discretization(xyz, tets, eps, bfaces, bface_kind, k0, degree)
        self.A = self.disc.global_matrix()
        self.part = np.asarray(part)
        self.n_sub = int(n_sub)
        self.overlap = int(overlap)
        self.prec = ORAS(self.disc, self.part, self.n_sub, self.overlap, variant, A=self.A)

    @classmethod
    def from_problem(cls, prob, variant="oras"):
        m = prob.mesh
        return cls(m.xyz, m.tets, prob.eps, m.bfaces, m.bface_kind, prob.part, prob.n_sub,
                   prob.overlap, prob.k0, prob.degree, variant)

    @property
    def ndof(self):
        return self.disc.ndof

    def rhs(self, src):
        return self.disc.rhs(src)

    def solve(self, b, tol=1e-8, restart=50, max_iters=5000):
        return fgmres(lambda v: self.A @ v, self.prec.apply, b, tol, restart, max_iters)

    def solve_block(self, B, tol=1e-8, restart=50, max_iters=5000):
        mv = lambda V: self.A @ V
        pc = self.prec.apply
        return block_fgmres(mv, pc, B, tol, restart, max_iters)
