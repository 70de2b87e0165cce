"""ctypes binding of libmxw.so (argument marshalling only).

Every step of the solver runs inside the library; this module converts
numpy arrays / torch tensors into the C structures of include/mxw.h and
checks status codes.  It raises if the shared library is missing: there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmxw.so")

MXW_OK = 0
MXW_EINVAL = -1
MXW_ENOMEM = -2
MXW_ENOTCONV = -3
MXW_ESINGULAR = -4
MXW_EBREAKDOWN = -5
MXW_EDEVICE = -6
MXW_EBUSY = -7
STATUS_NAMES = {0: "MXW_OK", -1: "MXW_EINVAL", -2: "MXW_ENOMEM", -3: "MXW_ENOTCONV",
                -4: "MXW_ESINGULAR", -5: "MXW_EBREAKDOWN", -6: "MXW_EDEVICE", -7: "MXW_EBUSY"}

MXW_FP64 = 0
MXW_MIXED = 1
MXW_KRYLOV_PSEUDOBLOCK = 0
MXW_KRYLOV_BLOCK = 1
MXW_PREC_ORAS = 0
MXW_PREC_OAS = 1
MXW_PREC_RAS = 2
MXW_PREC_ORAS_MULT = 3


class MxwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ProblemDesc(C.Structure):
    _fields_ = [
        ("n_vertices", C.c_int64), ("xyz", C.c_void_p),
        ("n_tets", C.c_int64), ("tets", C.c_void_p),
        ("eps", C.c_void_p),
        ("n_bfaces", C.c_int64), ("bfaces", C.c_void_p), ("bface_kind", C.c_void_p),
        ("part", C.c_void_p), ("n_sub", C.c_int32), ("overlap_layers", C.c_int32),
        ("k0", C.c_double), ("degree", C.c_int32), ("precision", C.c_int32),
        ("prec_variant", C.c_int32), ("reserved", C.c_int32),
    ]


class Source(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("reserved", C.c_int32),
        ("pos", C.c_double * 3), ("pol_re", C.c_double * 3), ("pol_im", C.c_double * 3),
        ("dir", C.c_double * 3),
    ]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iters", C.c_int32),
                ("krylov", C.c_int32), ("use_graph", C.c_int32)]


class LayoutInfo(C.Structure):
    _fields_ = [("ndof", C.c_int64), ("nnz", C.c_int64), ("n_sub", C.c_int32), ("nloc", C.c_int32),
                ("sum_ns", C.c_int64), ("max_ns", C.c_int64), ("sum_ns2", C.c_double),
                ("sum_ns3", C.c_double), ("n_iface", C.c_int64), ("n_imp_faces", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("spmv_group", C.c_int32), ("multi_ku", C.c_int32), ("spmv_ms", C.c_double * 4),
                ("multi_ms", C.c_double * 2), ("lu_ku", C.c_int32), ("multi_rows", C.c_int32),
                ("lu_ms", C.c_double * 2), ("multi_tall_ms", C.c_double), ("lu_launch", C.c_int32),
                ("reserved", C.c_int32), ("lu_launch_ms", C.c_double * 2)]


# device-memory provider of a context (see mxw_ctx_create)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None

_SIGS = {
    "mxw_last_error": (C.c_char_p, []),
    "mxw_layout_create": (C.c_int32, [C.POINTER(ProblemDesc), C.POINTER(C.c_void_p)]),
    "mxw_layout_destroy": (None, [C.c_void_p]),
    "mxw_layout_get_info": (C.c_int32, [C.c_void_p, C.POINTER(LayoutInfo)]),
    "mxw_export_dofs": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mxw_export_pattern": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mxw_export_subdomain": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "mxw_ctx_create": (C.c_int32, [C.c_int32, C.c_uint64, ALLOC_FN, FREE_FN, C.c_void_p, C.POINTER(C.c_void_p)]),
    "mxw_ctx_destroy": (C.c_int32, [C.c_void_p]),
    "mxw_ctx_usage": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_int64),
                                  C.c_int32]),
    "mxw_layout_footprint": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(SolveOpts),
                                         C.c_int32, C.POINTER(C.c_uint64)]),
    "mxw_footprint": (C.c_int32, [C.POINTER(ProblemDesc), C.c_int32, C.POINTER(SolveOpts), C.POINTER(C.c_uint64)]),
    "mxw_problem_create": (C.c_int32, [C.c_void_p, C.POINTER(ProblemDesc), C.c_void_p, C.c_int32,
                                       C.POINTER(C.c_void_p)]),
    "mxw_problem_create_from_layout": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                                   C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "mxw_solve_async": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Source), C.POINTER(SolveOpts), C.c_void_p,
                                    C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "mxw_ticket_poll": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mxw_ticket_wait": (C.c_int32, [C.c_void_p]),
    "mxw_ticket_destroy": (None, [C.c_void_p]),
    "mxw_problem_device_bytes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "mxw_problem_forget_factors": (C.c_int32, [C.c_void_p]),
    "mxw_problem_factor_stats": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                             C.POINTER(C.c_int64)]),
    "mxw_problem_set_medium": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "mxw_problem_destroy": (None, [C.c_void_p]),
    "mxw_problem_get_info": (C.c_int32, [C.c_void_p, C.POINTER(LayoutInfo)]),
    "mxw_problem_factor": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "mxw_problem_export_matrix": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "mxw_problem_export_local": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mxw_problem_rhs": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Source), C.c_void_p, C.c_void_p]),
    "mxw_problem_rhs_noalloc": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Source), C.c_void_p, C.c_void_p]),
    "mxw_problem_apply_A": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mxw_problem_apply_prec": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mxw_solve": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Source), C.POINTER(SolveOpts), C.c_void_p,
                              C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "mxw_solve_rhs": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(SolveOpts), C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]),
    "mxw_solve_history": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "mxw_problem_tune": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(Tuning)]),
    "mxw_problem_set_tiles": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "mxw_smatrix": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Source), C.c_int32, C.c_void_p, C.c_void_p,
                                C.c_void_p]),
    "mxw_solve_recycle": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(SolveOpts), C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mxw_recycle_reset": (C.c_int32, [C.c_void_p]),
    "mxw_recycle_export": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "mxw_recycle_stats": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]),
    "mxw_set_timing": (C.c_int32, [C.c_int32]),
    "mxw_get_timing": (C.c_int32, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "mxw_reset_timing": (C.c_int32, []),
}


def lib():
    """Load libmxw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1605_04521_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status, allowed=(MXW_OK,)):
    if status not in allowed:
        raise MxwError(status, lib().mxw_last_error().decode())
    return status


def ptr(a) -> int:
    """Address of a contiguous numpy array or torch tensor."""
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


class Desc:
    """Owns the numpy buffers behind a ProblemDesc."""

    def __init__(self, xyz, tets, eps, bfaces, bface_kind, part, n_sub, overlap, k0, degree,
                 precision=MXW_FP64, variant=MXW_PREC_ORAS):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        e = np.asarray(eps, dtype=np.complex128)
        self.eps = np.ascontiguousarray(np.stack([e.real, e.imag], axis=1))
        self.bfaces = np.ascontiguousarray(bfaces, dtype=np.int32)
        self.bface_kind = np.ascontiguousarray(bface_kind, dtype=np.int8)
        self.part = np.ascontiguousarray(part, dtype=np.int32)
        self.c = ProblemDesc(
            n_vertices=len(self.xyz), xyz=self.xyz.ctypes.data, n_tets=len(self.tets),
            tets=self.tets.ctypes.data, eps=self.eps.ctypes.data, n_bfaces=len(self.bfaces),
            bfaces=self.bfaces.ctypes.data, bface_kind=self.bface_kind.ctypes.data,
            part=self.part.ctypes.data, n_sub=int(n_sub), overlap_layers=int(overlap), k0=float(k0),
            degree=int(degree), precision=int(precision), prec_variant=int(variant), reserved=0)

    @classmethod
    def from_problem(cls, prob, precision=MXW_FP64, variant=MXW_PREC_ORAS):
        m = prob.mesh
        return cls(m.xyz, m.tets, prob.eps, m.bfaces, m.bface_kind, prob.part, prob.n_sub,
                   prob.overlap, prob.k0, prob.degree, precision, variant)


def make_sources(srcs):
    arr = (Source * len(srcs))()
    for s, src in zip(arr, srcs):
        s.kind = int(src.kind)
        pol = np.asarray(src.pol, dtype=np.complex128)
        for q in range(3):
            s.pos[q] = float(src.pos[q])
            s.pol_re[q] = float(pol[q].real)
            s.pol_im[q] = float(pol[q].imag)
            s.dir[q] = float(src.dir[q])
    return arr


def solve_opts(tol=1e-8, restart=50, max_iters=5000, krylov=MXW_KRYLOV_PSEUDOBLOCK, use_graph=0):
    return SolveOpts(tol=tol, restart=restart, max_iters=max_iters, krylov=krylov, use_graph=use_graph)
