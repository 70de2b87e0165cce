"""Python front end of libmxw: host layouts and device problems.

PyTorch provides device memory and the stream; every computation runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as B


class Layout:
    """Host-side setup: unknown numbering, CSR pattern, subdomains (no GPU)."""

    def __init__(self, desc: B.Desc):
        self.desc = desc
        h = C.c_void_p()
        B.check(B.lib().mxw_layout_create(C.byref(desc.c), C.byref(h)))
        self.h = h

    @classmethod
    def from_problem(cls, prob, **kw):
        return cls(B.Desc.from_problem(prob, **kw))

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and self.h.value:
                B.lib().mxw_layout_destroy(self.h)
                self.h = None
        except (TypeError, AttributeError):
            pass   # interpreter shutdown: the module's globals are already gone

    def info(self) -> B.LayoutInfo:
        i = B.LayoutInfo()
        B.check(B.lib().mxw_layout_get_info(self.h, C.byref(i)))
        return i

    def dofs(self):
        n = self.info().ndof
        k = np.empty(n, np.int8)
        e = np.empty(n, np.int64)
        l = np.empty(n, np.int16)
        B.check(B.lib().mxw_export_dofs(self.h, k.ctypes.data, e.ctypes.data, l.ctypes.data))
        return k, e, l

    def pattern(self):
        i = self.info()
        rp = np.empty(i.ndof + 1, np.int64)
        ci = np.empty(i.nnz, np.int32)
        B.check(B.lib().mxw_export_pattern(self.h, rp.ctypes.data, ci.ctypes.data))
        return rp, ci

    def subdomain(self, s: int):
        n = C.c_int64()
        B.check(B.lib().mxw_export_subdomain(self.h, s, C.byref(n), None, None))
        d = np.empty(n.value, np.int64)
        w = np.empty(n.value, np.uint8)
        B.check(B.lib().mxw_export_subdomain(self.h, s, C.byref(n), d.ctypes.data, w.ctypes.data))
        return d, w

    def footprint(self, precision=B.MXW_FP64, nrhs=1, restart=50) -> int:
        out = C.c_uint64()
        opts = B.solve_opts(restart=restart)
        B.check(B.lib().mxw_layout_footprint(self.h, precision, nrhs, C.byref(opts), C.byref(out)))
        return out.value


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Problem:
    """Device operator: assembled A, local matrices, batched LU factors."""

    def __init__(self, desc: B.Desc = None, hbm_budget: int = 0, defer_factor: bool = False, layout=None,
                 eps=None, k0: float = -1.0, precision=B.MXW_FP64, variant=B.MXW_PREC_ORAS):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required for mxw.Problem")
        self.desc = desc
        self.layout = layout
        h = C.c_void_p()
        if layout is None:
            st = B.lib().mxw_problem_create(C.byref(desc.c), _stream(), hbm_budget, int(defer_factor), C.byref(h))
        else:
            e = None
            if eps is not None:
                e = np.asarray(eps, dtype=np.complex128)
                self._eps = np.ascontiguousarray(np.stack([e.real, e.imag], axis=1))
                e = self._eps.ctypes.data
            st = B.lib().mxw_problem_create_from_layout(layout.h, e, float(k0), int(precision), int(variant),
                                                        _stream(), hbm_budget, int(defer_factor), C.byref(h))
        self.h = h
        self.create_status = st
        if st != B.MXW_OK and not (st == B.MXW_ESINGULAR and h.value):
            B.check(st)
        self._info = self.info()

    @classmethod
    def from_layout(cls, layout, eps=None, k0=-1.0, precision=B.MXW_FP64, variant=B.MXW_PREC_ORAS, **kw):
        """Problem on an existing layout's mesh and partition with a new medium."""
        return cls(layout=layout, eps=eps, k0=k0, precision=precision, variant=variant, **kw)

    def set_medium(self, eps=None, k0: float = -1.0):
        """New permittivity (and optionally k0): re-assemble and re-factorise in place."""
        e = None
        if eps is not None:
            e = np.asarray(eps, dtype=np.complex128)
            self._eps = np.ascontiguousarray(np.stack([e.real, e.imag], axis=1))
            e = self._eps.ctypes.data
        return B.check(B.lib().mxw_problem_set_medium(self.h, e, float(k0), _stream()),
                       (B.MXW_OK, B.MXW_ESINGULAR))

    def close(self):
        """Release the device memory now (instead of at garbage collection)."""
        if getattr(self, "h", None) is not None and self.h.value:
            B.lib().mxw_problem_destroy(self.h)
            self.h = None

    @classmethod
    def from_problem(cls, prob, precision=B.MXW_FP64, variant=B.MXW_PREC_ORAS, **kw):
        return cls(B.Desc.from_problem(prob, precision, variant), **kw)

    def __del__(self):
        try:
            self.close()
        except (TypeError, AttributeError):
            pass   # interpreter shutdown: the module's globals are already gone

    def info(self) -> B.LayoutInfo:
        i = B.LayoutInfo()
        B.check(B.lib().mxw_problem_get_info(self.h, C.byref(i)))
        return i

    @property
    def ndof(self) -> int:
        return self._info.ndof

    def factor(self):
        return B.check(B.lib().mxw_problem_factor(self.h, _stream()))

    def matrix_values(self) -> np.ndarray:
        v = np.empty(self._info.nnz, np.complex128)
        B.check(B.lib().mxw_problem_export_matrix(self.h, v.ctypes.data))
        return v

    def local_matrix(self, s: int, n_s: int) -> np.ndarray:
        a = np.empty((n_s, n_s), np.complex128, order="F")
        B.check(B.lib().mxw_problem_export_local(self.h, s, a.ctypes.data))
        return a

    def rhs(self, sources):
        import torch
        b = torch.empty((len(sources), self.ndof), dtype=torch.complex128, device="cuda")
        src = B.make_sources(sources)
        B.check(B.lib().mxw_problem_rhs(self.h, len(sources), src, b.data_ptr(), _stream()))
        return b

    def apply_A(self, x):
        import torch
        x = x.contiguous()
        y = torch.empty_like(x)
        B.check(B.lib().mxw_problem_apply_A(self.h, x.shape[0], x.data_ptr(), y.data_ptr(), _stream()))
        return y

    def apply_prec(self, v):
        import torch
        v = v.contiguous()
        z = torch.empty_like(v)
        B.check(B.lib().mxw_problem_apply_prec(self.h, v.shape[0], v.data_ptr(), z.data_ptr(), _stream()))
        return z

    def solve_rhs(self, b, tol=1e-8, restart=50, max_iters=5000, krylov=B.MXW_KRYLOV_PSEUDOBLOCK,
                  use_graph=0, allow_notconv=False):
        import torch
        b = b.contiguous()
        nrhs = b.shape[0]
        x = torch.empty_like(b)
        it = np.zeros(nrhs, np.int32)
        rr = np.zeros(nrhs, np.float64)
        opts = B.solve_opts(tol, restart, max_iters, krylov, use_graph)
        st = B.lib().mxw_solve_rhs(self.h, nrhs, b.data_ptr(), C.byref(opts), _stream(), x.data_ptr(),
                                   it.ctypes.data, rr.ctypes.data)
        allowed = (B.MXW_OK, B.MXW_ENOTCONV, B.MXW_EBREAKDOWN) if allow_notconv else (B.MXW_OK,)
        status = B.check(st, allowed)
        return x, it, rr, status

    def smatrix(self, ports, X):
        """S[i, j] (eq. (5)) of the fields X [nsol][ndof] on the ports."""
        import torch
        X = X.contiguous()
        S = torch.empty((len(ports), X.shape[0]), dtype=torch.complex128, device="cuda")
        src = B.make_sources(ports)
        B.check(B.lib().mxw_smatrix(self.h, len(ports), src, X.shape[0], X.data_ptr(), _stream(), S.data_ptr()))
        return S

    def solve_recycle(self, b, k: int = 10, tol=1e-8, restart=50, max_iters=5000, allow_notconv=False):
        """GCRO-DR solves of the columns of b one after another, with the
        problem's recycled space of k vectors carried between them (and to
        later calls, also across set_medium)."""
        import torch
        b = b.contiguous()
        nrhs = b.shape[0]
        x = torch.empty_like(b)
        it = np.zeros(nrhs, np.int32)
        rr = np.zeros(nrhs, np.float64)
        opts = B.solve_opts(tol, restart, max_iters)
        st = B.lib().mxw_solve_recycle(self.h, nrhs, b.data_ptr(), C.byref(opts), k, _stream(), x.data_ptr(),
                                       it.ctypes.data, rr.ctypes.data)
        allowed = (B.MXW_OK, B.MXW_ENOTCONV, B.MXW_EBREAKDOWN) if allow_notconv else (B.MXW_OK,)
        status = B.check(st, allowed)
        return x, it, rr, status

    def recycle_reset(self):
        B.check(B.lib().mxw_recycle_reset(self.h))

    def recycle_space(self):
        """(U, Ubar, C) of the recycled space as device tensors [dim][ndof]."""
        import torch
        d = C.c_int32()
        B.check(B.lib().mxw_recycle_export(self.h, C.byref(d), None, None, None, _stream()))
        U, Ub, Cm = (torch.empty((d.value, self.ndof), dtype=torch.complex128, device="cuda") for _ in range(3))
        B.check(B.lib().mxw_recycle_export(self.h, C.byref(d), U.data_ptr(), Ub.data_ptr(), Cm.data_ptr(),
                                           _stream()))
        return U, Ub, Cm

    def recycle_stats(self) -> dict:
        r, d, f = C.c_int64(), C.c_int64(), C.c_int64()
        B.check(B.lib().mxw_recycle_stats(self.h, C.byref(r), C.byref(d), C.byref(f)))
        return {"refreshes": r.value, "deflations": d.value, "failures": f.value}

    def tune(self, nrhs: int = 1) -> dict:
        """Time the SpMV lanes-per-row and multi-column k slice choices on this
        problem and keep the fastest for later calls."""
        t = B.Tuning()
        B.check(B.lib().mxw_problem_tune(self.h, nrhs, _stream(), C.byref(t)))
        return {"spmv_group": t.spmv_group, "multi_ku": t.multi_ku, "spmv_ms": list(t.spmv_ms),
                "multi_ms": list(t.multi_ms), "lu_ku": t.lu_ku, "lu_ms": list(t.lu_ms),
                "multi_rows": t.multi_rows, "multi_tall_ms": t.multi_tall_ms}

    def set_tiles(self, spmv_group: int = 0, multi_ku: int = 0, lu_ku: int = 0, multi_rows: int = 0):
        B.check(B.lib().mxw_problem_set_tiles(self.h, spmv_group, multi_ku, lu_ku, multi_rows))

    def history(self, col: int = 0) -> np.ndarray:
        """Relative residual estimates of every Arnoldi step of the last solve."""
        n = C.c_int32()
        B.check(B.lib().mxw_solve_history(self.h, col, None, 0, C.byref(n)))
        out = np.empty(n.value, np.float64)
        B.check(B.lib().mxw_solve_history(self.h, col, out.ctypes.data, n.value, C.byref(n)))
        return out

    def solve(self, sources, **kw):
        b = self.rhs(sources)
        return self.solve_rhs(b, **kw)


def timing(enabled: bool = True):
    B.check(B.lib().mxw_set_timing(int(enabled)))


def kernel_time(name: str):
    t = C.c_double()
    n = C.c_int64()
    B.check(B.lib().mxw_get_timing(name.encode(), C.byref(t), C.byref(n)))
    return t.value, n.value


def reset_timing():
    B.check(B.lib().mxw_reset_timing())
