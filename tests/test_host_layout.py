"""Host-side setup of the library (no GPU): the C ABI loads and exports every
declared entry point; unknown numbering, sparsity pattern, overlapping
subdomains and partition of unity agree bit for bit with the oracle; invalid
inputs are rejected with a message."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.assemble import Discretization
from oracle.schwarz import build_subdomains
from paper_1605_04521_amd import _lib as B
from paper_1605_04521_amd import gen
from paper_1605_04521_amd.api import Layout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "mxw.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mxw_[A-Za-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    # every binding signature refers to a declared symbol
    for s in B._SIGS:
        assert s in syms, s


def oracle_setup(prob):
    m = prob.mesh
    d = Discretization(m.xyz, m.tets, prob.eps, m.bfaces, m.bface_kind, prob.k0, prob.degree)
    subs = build_subdomains(d, prob.part, prob.n_sub, prob.overlap)
    return d, subs


CASES = [
    ("cube8_r1", lambda: gen.cube_planewave_problem(n=8, degree=1)),
    ("cube3_r2_ov2", lambda: gen.cube_planewave_problem(n=3, degree=2, box=2, overlap=2)),
    ("cube2_r3", lambda: gen.cube_planewave_problem(n=2, degree=3, box=1)),
    ("chamber5_r2", lambda: gen.chamber_problem(n=5, degree=2, n_sub=7, overlap=2)),
    ("chamber4_r3", lambda: gen.chamber_problem(n=4, degree=3, n_sub=5, overlap=1)),
    ("chamber4_r1_ov0", lambda: gen.chamber_problem(n=4, degree=1, n_sub=3, overlap=0)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_layout_matches_oracle_bitwise(name, make):
    prob = make()
    d, subs = oracle_setup(prob)
    lay = Layout.from_problem(prob)
    info = lay.info()
    assert info.ndof == d.ndof
    k, e, l = lay.dofs()
    assert np.array_equal(k, d.dofs.ent_kind)
    assert np.array_equal(e, d.dofs.ent_id)
    assert np.array_equal(l, d.dofs.ent_local)
    rp, ci = lay.pattern()
    orp, oci = d.pattern()
    assert np.array_equal(rp, orp)
    assert np.array_equal(ci, oci)
    assert info.n_sub == len(subs)
    for s, sub in enumerate(subs):
        dofs, pou = lay.subdomain(s)
        assert np.array_equal(dofs, sub.dofs), s
        assert np.array_equal(pou, sub.pou), s
    assert info.sum_ns == sum(len(s.dofs) for s in subs)
    assert info.max_ns == max(len(s.dofs) for s in subs)
    assert info.n_iface == sum(len(s.iface) for s in subs)
    assert info.n_imp_faces == len(d.imp_faces)


def test_cube8_reference_sizes():
    lay = Layout.from_problem(gen.cube_planewave_problem())
    i = lay.info()
    assert (i.ndof, i.nnz, i.n_sub, i.max_ns, i.sum_ns) == (4184, 61784, 8, 796, 8 * 796)


def test_footprint_grows_with_rhs_and_precision():
    lay = Layout.from_problem(gen.chamber_problem(n=4, degree=2, n_sub=4, overlap=1))
    f1 = lay.footprint(B.MXW_FP64, 1)
    f32 = lay.footprint(B.MXW_FP64, 32)
    fm = lay.footprint(B.MXW_MIXED, 1)
    assert f32 > f1 > fm > 0
    # a block solve adds its workspace; the layout copy is counted once
    fb = lay.footprint(B.MXW_FP64, 32, krylov=B.MXW_KRYLOV_BLOCK)
    assert fb > f32
    assert 0 < f1 - lay.footprint(B.MXW_FP64, 1, with_layout_copy=False) < f1
    # the standalone call (builds the layout itself) agrees with the layout's
    prob = gen.chamber_problem(n=4, degree=2, n_sub=4, overlap=1)
    from paper_1605_04521_amd.api import footprint
    assert footprint(B.Desc.from_problem(prob, precision=B.MXW_FP64), 32) == f32
    assert footprint(B.Desc.from_problem(prob, precision=B.MXW_MIXED), 1) == fm
    # the gathered variants keep every local solution of a solve
    assert lay.footprint(B.MXW_FP64, 1, variant=B.MXW_PREC_OAS) > f1


def _desc_variant(**changes):
    prob = gen.cube_planewave_problem(n=2, degree=1, box=1)
    m = prob.mesh
    args = dict(xyz=m.xyz, tets=m.tets, eps=prob.eps, bfaces=m.bfaces, bface_kind=m.bface_kind,
                part=prob.part, n_sub=prob.n_sub, overlap=prob.overlap, k0=prob.k0, degree=prob.degree)
    args.update(changes)
    return B.Desc(**args)


@pytest.mark.parametrize("change,msg", [
    (dict(degree=4), "degree"),
    (dict(n_sub=0), "n_sub"),
    (dict(overlap=-1), "overlap"),
    (dict(k0=float("nan")), "k0"),
    (dict(eps=np.full(48, np.nan + 0j)), "permittivity"),
])
def test_invalid_inputs_rejected(change, msg):
    desc = _desc_variant(**change)
    h = C.c_void_p()
    st = B.lib().mxw_layout_create(C.byref(desc.c), C.byref(h))
    assert st == B.MXW_EINVAL
    assert msg in B.lib().mxw_last_error().decode()


def test_invalid_mesh_data_rejected():
    prob = gen.cube_planewave_problem(n=2, degree=1, box=1)
    m = prob.mesh
    # a boundary face missing
    desc = _desc_variant(bfaces=m.bfaces[1:], bface_kind=m.bface_kind[1:])
    h = C.c_void_p()
    assert B.lib().mxw_layout_create(C.byref(desc.c), C.byref(h)) == B.MXW_EINVAL
    assert "boundary faces" in B.lib().mxw_last_error().decode()
    # vertex id out of range
    bad = m.tets.copy()
    bad[3, 2] = 10 ** 6
    desc = _desc_variant(tets=bad)
    assert B.lib().mxw_layout_create(C.byref(desc.c), C.byref(h)) == B.MXW_EINVAL
    # partition id out of range
    part = prob.part.copy()
    part[0] = 99
    desc = _desc_variant(part=part)
    assert B.lib().mxw_layout_create(C.byref(desc.c), C.byref(h)) == B.MXW_EINVAL
    assert "part" in B.lib().mxw_last_error().decode()
    # degenerate element
    xyz = m.xyz.copy()
    t = m.tets[0]
    xyz[t[3]] = xyz[t[0]] + 0.5 * (xyz[t[1]] - xyz[t[0]])
    desc = _desc_variant(xyz=xyz)
    assert B.lib().mxw_layout_create(C.byref(desc.c), C.byref(h)) == B.MXW_EINVAL
