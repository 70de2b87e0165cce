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

    def footprint(self, precision=B.MXW_FP64, nrhs=1, restart=50, krylov=B.MXW_KRYLOV_PSEUDOBLOCK,
                  variant=B.MXW_PREC_ORAS, with_layout_copy=True) -> int:
        """Device bytes of one problem on this layout that solves nrhs sources
        (its operator, factors, workspaces and solve temporaries), plus the
        layout's shared device copy if with_layout_copy."""
        out = C.c_uint64()
        opts = B.solve_opts(restart=restart, krylov=krylov)
        B.check(B.lib().mxw_layout_footprint(self.h, precision, variant, nrhs, C.byref(opts),
                                             int(bool(with_layout_copy)), C.byref(out)))
        return out.value


def footprint(desc: B.Desc, nrhs=1, restart=50, krylov=B.MXW_KRYLOV_PSEUDOBLOCK) -> int:
    """Device bytes of a problem described by desc alone (layout copy included)."""
    out = C.c_uint64()
    opts = B.solve_opts(restart=restart, krylov=krylov)
    B.check(B.lib().mxw_footprint(C.byref(desc.c), nrhs, C.byref(opts), C.byref(out)))
    return out.value


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """Device-memory context of the library: every device allocation of the
    problems made with it goes through PyTorch's caching allocator (allocator
    "torch", the default) or hipMalloc ("hip"), counted against an HBM budget
    (bytes, 0 = none)."""

    def __init__(self, budget: int = 0, device=None, allocator: str = "torch"):
        import torch
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = dev
        if allocator == "torch":
            def _alloc(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
                except Exception:          # out of memory: the library reports MXW_ENOMEM
                    return None

            def _free(ptr, user):
                torch.cuda.caching_allocator_delete(int(ptr))
            self._alloc, self._free = B.ALLOC_FN(_alloc), B.FREE_FN(_free)
        elif allocator == "hip":
            self._alloc, self._free = B.ALLOC_FN(), B.FREE_FN()
        else:
            raise ValueError("allocator must be 'torch' or 'hip'")
        h = C.c_void_p()
        B.check(B.lib().mxw_ctx_create(dev, int(budget), self._alloc, self._free, None, C.byref(h)))
        self.h = h

    def usage(self, reset_peak: bool = False) -> dict:
        u, p, n = C.c_uint64(), C.c_uint64(), C.c_int64()
        B.check(B.lib().mxw_ctx_usage(self.h, C.byref(u), C.byref(p), C.byref(n), int(reset_peak)))
        return {"in_use": u.value, "peak": p.value, "live": n.value}

    def close(self):
        """Releases the context (MxwError MXW_EBUSY while memory is still held)."""
        if getattr(self, "h", None) is not None and self.h.value:
            B.check(B.lib().mxw_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and self.h.value:
                if B.lib().mxw_ctx_destroy(self.h) == B.MXW_OK:
                    self.h = None
        except (TypeError, AttributeError):
            pass


_default_ctx = None


def default_context() -> Context:
    """The context of problems created without one (PyTorch's allocator, no budget)."""
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


class Ticket:
    """A forward solve running on a library worker thread (mxw_solve_async)."""

    def __init__(self, problem, h, x, it, rr, src):
        self.problem, self.h, self.x, self.it, self.rr, self._src = problem, h, x, it, rr, src
        self.status = None

    def done(self) -> bool:
        d = C.c_int32()
        B.check(B.lib().mxw_ticket_poll(self.h, C.byref(d)))
        return bool(d.value)

    def wait(self, allow_notconv=False):
        """(x, iterations, relres, status) once the solve has finished."""
        if self.status is None:
            self.status = B.lib().mxw_ticket_wait(self.h)
            if self.status != B.MXW_OK:
                self._msg = B.lib().mxw_last_error().decode()
            B.lib().mxw_ticket_destroy(self.h)
            self.h = None
        allowed = (B.MXW_OK, B.MXW_ENOTCONV, B.MXW_EBREAKDOWN) if allow_notconv else (B.MXW_OK,)
        if self.status not in allowed:
            raise B.MxwError(self.status, getattr(self, "_msg", ""))
        return self.x, self.it, self.rr, self.status

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                B.lib().mxw_ticket_destroy(self.h)
                self.h = None
        except (TypeError, AttributeError):
            pass


class Problem:
    """Device operator: assembled A, local matrices, batched LU factors."""

    def __init__(self, desc: B.Desc = None, defer_factor: bool = False, layout=None,
                 eps=None, k0: float = -1.0, precision=B.MXW_FP64, variant=B.MXW_PREC_ORAS, ctx: Context = None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required for mxw.Problem")
        self.desc = desc
        self.layout = layout
        self.ctx = ctx if ctx is not None else default_context()
        if layout is not None:
            # the layout's device copy may be allocated through this context
            layout._contexts = getattr(layout, "_contexts", []) + [self.ctx]
        h = C.c_void_p()
        if layout is None:
            st = B.lib().mxw_problem_create(self.ctx.h, C.byref(desc.c), _stream(), int(defer_factor), C.byref(h))
        else:
            e = None
            if eps is not None:
                e = np.asarray(eps, dtype=np.complex128)
                self._eps = np.ascontiguousarray(np.stack([e.real, e.imag], axis=1))
                e = self._eps.ctypes.data
            st = B.lib().mxw_problem_create_from_layout(self.ctx.h, layout.h, e, float(k0), int(precision),
                                                        int(variant), _stream(), int(defer_factor), C.byref(h))
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

    def rhs_noalloc(self, sources, out=None):
        """The same right-hand sides through the entry point that allocates no
        device memory (its face integrals go to the library's fixed buffer);
        out: an existing [nsrc][ndof] complex128 tensor to fill."""
        import torch
        b = out if out is not None else torch.empty((len(sources), self.ndof), dtype=torch.complex128,
                                                     device="cuda")
        src = B.make_sources(sources)
        B.check(B.lib().mxw_problem_rhs_noalloc(self.h, len(sources), src, b.data_ptr(), _stream()))
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

    def solve_recycle(self, b, k: int = 10, tol=1e-8, restart=50, max_iters=5000, allow_notconv=False,
                      block=False):
        """GCRO-DR solves of the columns of b one after another, with the
        problem's recycled space of k vectors carried between them (and to
        later calls, also across set_medium).  block=True: Block GCRO-DR, the
        2..16 columns solved together in one block space (iterations are
        block steps)."""
        import torch
        b = b.contiguous()
        nrhs = b.shape[0]
        x = torch.empty_like(b)
        it = np.zeros(nrhs, np.int32)
        rr = np.zeros(nrhs, np.float64)
        opts = B.solve_opts(tol, restart, max_iters,
                            krylov=B.MXW_KRYLOV_BLOCK if block else B.MXW_KRYLOV_PSEUDOBLOCK)
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
                "multi_rows": t.multi_rows, "multi_tall_ms": t.multi_tall_ms, "lu_launch": t.lu_launch,
                "lu_launch_ms": list(t.lu_launch_ms)}

    def set_tiles(self, spmv_group: int = 0, multi_ku: int = 0, lu_ku: int = 0, multi_rows: int = 0,
                  lu_launch: int = 0):
        B.check(B.lib().mxw_problem_set_tiles(self.h, spmv_group, multi_ku, lu_ku, multi_rows, lu_launch))

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

    def solve_host(self, sources, tol=1e-8, restart=50, max_iters=5000, krylov=B.MXW_KRYLOV_PSEUDOBLOCK,
                   use_graph=0, allow_notconv=False):
        """mxw_solve with the E field returned in host memory (the library
        stages the right-hand sides and the solution on the device itself)."""
        E = np.empty((len(sources), self.ndof), np.complex128)
        it = np.zeros(len(sources), np.int32)
        rr = np.zeros(len(sources), np.float64)
        src = B.make_sources(sources)
        opts = B.solve_opts(tol, restart, max_iters, krylov, use_graph)
        st = B.lib().mxw_solve(self.h, len(sources), src, C.byref(opts), _stream(), E.ctypes.data, 0,
                               it.ctypes.data, rr.ctypes.data)
        allowed = (B.MXW_OK, B.MXW_ENOTCONV, B.MXW_EBREAKDOWN) if allow_notconv else (B.MXW_OK,)
        return E, it, rr, B.check(st, allowed)

    def solve_async(self, sources, tol=1e-8, restart=50, max_iters=5000, krylov=B.MXW_KRYLOV_PSEUDOBLOCK,
                    use_graph=0, stream=None) -> Ticket:
        """Starts the forward solves of the sources on a library worker thread
        driving `stream` (a torch.cuda.Stream; default: the current stream);
        returns a Ticket."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        x = torch.empty((len(sources), self.ndof), dtype=torch.complex128, device="cuda")
        it = np.zeros(len(sources), np.int32)
        rr = np.zeros(len(sources), np.float64)
        src = B.make_sources(sources)
        opts = B.solve_opts(tol, restart, max_iters, krylov, use_graph)
        h = C.c_void_p()
        # x is made on torch's current stream; the worker's stream waits for it
        st.wait_stream(torch.cuda.current_stream())
        B.check(B.lib().mxw_solve_async(self.h, len(sources), src, C.byref(opts), C.c_void_p(st.cuda_stream),
                                        x.data_ptr(), 1, it.ctypes.data, rr.ctypes.data, C.byref(h)))
        return Ticket(self, h, x, it, rr, src)

    def forget_factors(self):
        """The next set_medium factorises every subdomain again."""
        B.check(B.lib().mxw_problem_forget_factors(self.h))

    def factor_stats(self) -> dict:
        """Subdomains re-factorised by the last medium change; totals over the changes."""
        a, b, c = C.c_int32(), C.c_int64(), C.c_int64()
        B.check(B.lib().mxw_problem_factor_stats(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return {"refactored_last": a.value, "refactored_total": b.value, "kept_total": c.value}

    def device_bytes(self) -> int:
        """Device bytes the problem holds now (not the layout's shared copy)."""
        out = C.c_uint64()
        B.check(B.lib().mxw_problem_device_bytes(self.h, C.byref(out)))
        return out.value


def timing(enabled: bool = True):
    B.check(B.lib().mxw_set_timing(int(enabled)))


def kernel_time(name: str):
    t = C.c_double()
    n = C.c_int64()
    B.check(B.lib().mxw_get_timing(name.encode(), C.byref(t), C.byref(n)))
    return t.value, n.value


def reset_timing():
    B.check(B.lib().mxw_reset_timing())
