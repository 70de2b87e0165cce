"""The library's host-side setup (unknown numbering, CSR pattern, overlapping
subdomains and their partition of unity, Sec. 3-4) built on its own with g++
under the address and undefined-behaviour sanitizers, run on the parity
meshes, on degenerate but valid inputs (no overlap, empty subdomains, every
boundary face metallic, one element) and on malformed meshes.  Every run must
end without a sanitizer report; a valid mesh must give exactly the numbering,
pattern and subdomains the shipped library exports, and a malformed one the
same status and message the shipped library returns."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1605_04521_amd import _lib as B
from paper_1605_04521_amd import gen
from paper_1605_04521_amd.api import Layout

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1605_04521_amd", "csrc")
DRIVER = os.path.join(HERE, "host", "layout_check.cpp")

SAN_ENV = {
    "ASAN_OPTIONS": "halt_on_error=1:abort_on_error=0:detect_leaks=1:exitcode=23",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
}


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not installed")
    out = str(tmp_path_factory.mktemp("san") / "layout_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           DRIVER, os.path.join(CSRC, "layout.cpp"), os.path.join(CSRC, "basis.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def run_checker(exe, d: B.Desc, tmp):
    """Write the descriptor's arrays, run the sanitized build, read back what
    it wrote: (status, message, arrays or None)."""
    c = d.c
    os.makedirs(tmp, exist_ok=True)
    with open(os.path.join(tmp, "meta.txt"), "w") as f:
        f.write(f"{c.n_vertices} {c.n_tets} {c.n_bfaces} {c.n_sub} {c.overlap_layers} {c.degree} "
                f"{c.precision} {c.prec_variant}\n")
    np.array([c.k0], np.float64).tofile(os.path.join(tmp, "k0.bin"))
    for name, arr in (("xyz", d.xyz), ("tets", d.tets), ("eps", d.eps), ("bfaces", d.bfaces),
                      ("bkind", d.bface_kind), ("part", d.part)):
        np.ascontiguousarray(arr).tofile(os.path.join(tmp, name + ".bin"))
    env = dict(os.environ, **SAN_ENV)
    r = subprocess.run([exe, tmp], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        r.stderr[-4000:]
    with open(os.path.join(tmp, "status.txt")) as f:
        status = int(f.readline())
        msg = f.readline().rstrip("\n")
    if status != B.MXW_OK:
        return status, msg, None

    def rd(name, dt):
        return np.fromfile(os.path.join(tmp, name + ".bin"), dtype=dt)

    with open(os.path.join(tmp, "info.txt")) as f:
        info = [int(x) for x in f.read().split()]
    arrays = {
        "info": info,
        "rowptr": rd("rowptr", np.int64), "cols": rd("cols", np.int32),
        "ent_kind": rd("ent_kind", np.int8), "ent_id": rd("ent_id", np.int64),
        "ent_local": rd("ent_local", np.int16),
        "sub_ptr": rd("sub_ptr", np.int64), "sub_dofs": rd("sub_dofs", np.int32),
        "sub_pou": rd("sub_pou", np.uint8),
        "imp_tet": rd("imp_tet", np.int32), "sub_face_tet": rd("sub_face_tet", np.int32),
        "imp_beta": rd("imp_beta", np.float64), "sub_face_coef": rd("sub_face_coef", np.float64),
    }
    return status, msg, arrays


def compare_with_library(d: B.Desc, a):
    lay = Layout(d)
    i = lay.info()
    ndof, nnz, n_sub, sum_ns, max_ns, n_iface, nloc = a["info"]
    assert (ndof, nnz, n_sub, sum_ns, max_ns, n_iface, nloc) == \
        (i.ndof, i.nnz, i.n_sub, i.sum_ns, i.max_ns, i.n_iface, i.nloc)
    rp, ci = lay.pattern()
    assert np.array_equal(rp, a["rowptr"]) and np.array_equal(ci, a["cols"])
    k, e, l = lay.dofs()
    assert np.array_equal(k, a["ent_kind"]) and np.array_equal(e, a["ent_id"])
    assert np.array_equal(l, a["ent_local"])
    sp = a["sub_ptr"]
    assert len(sp) == n_sub + 1 and sp[-1] == sum_ns
    for s in range(n_sub):
        dofs, pou = lay.subdomain(s)
        assert np.array_equal(dofs, a["sub_dofs"][sp[s]:sp[s + 1]]), s
        assert np.array_equal(pou, a["sub_pou"][sp[s]:sp[s + 1]]), s
    # face coefficients: k0 sqrt(Re eps) of the element owning each face
    # (the impedance coefficient of eq. (2) and the transmission one of Sec. 4)
    k0 = float(d.c.k0)
    wn = k0 * np.sqrt(np.maximum(d.eps[:, 0], 0.0))
    assert len(a["imp_beta"]) == len(a["imp_tet"]) == i.n_imp_faces
    assert np.array_equal(a["imp_beta"], wn[a["imp_tet"]])
    assert np.array_equal(a["sub_face_coef"], wn[a["sub_face_tet"]])


def _desc(prob, **kw):
    return B.Desc.from_problem(prob, **kw)


VALID = {
    "cube8_r1": lambda: _desc(gen.cube_planewave_problem(n=8, degree=1)),
    "cube4_r2": lambda: _desc(gen.cube_planewave_problem(n=4, degree=2, box=2)),
    "cube3_r3": lambda: _desc(gen.cube_planewave_problem(n=3, degree=3, box=2, overlap=1)),
    "chamber6_r2": lambda: _desc(gen.chamber_problem(n=6, degree=2, n_sub=9, overlap=2)),
    "chamber5_r3_mixed": lambda: _desc(gen.chamber_problem(n=5, degree=3, n_sub=6, overlap=1),
                                       precision=B.MXW_MIXED),
    "chamber6_r2_ras": lambda: _desc(gen.chamber_problem(n=6, degree=2, n_sub=9, overlap=2),
                                     variant=B.MXW_PREC_RAS),
    "chamber6_r1_mult": lambda: _desc(gen.chamber_problem(n=6, degree=1, n_sub=9, overlap=3),
                                      variant=B.MXW_PREC_ORAS_MULT),
    "cube4_r2_no_overlap": lambda: _desc(gen.cube_planewave_problem(n=4, degree=2, box=2, overlap=0)),
}


def _cube(n=2, degree=1, **kw):
    return _desc(gen.cube_planewave_problem(n=n, degree=degree, box=1 if n < 2 else 2, **kw))


def _rebuild(d: B.Desc, **over):
    """A copy of the descriptor with some arrays or scalars replaced."""
    c = d.c
    f = dict(xyz=d.xyz.copy(), tets=d.tets.copy(), eps=d.eps[:, 0] + 1j * d.eps[:, 1],
             bfaces=d.bfaces.copy(), bface_kind=d.bface_kind.copy(), part=d.part.copy(),
             n_sub=c.n_sub, overlap=c.overlap_layers, k0=c.k0, degree=c.degree,
             precision=c.precision, variant=c.prec_variant)
    f.update(over)
    return B.Desc(**f)


def _empty_subdomains():
    d = _cube(3, 2)
    return _rebuild(d, part=np.zeros_like(d.part), n_sub=3)


def _all_metallic():
    d = _cube(3, 1)
    return _rebuild(d, bface_kind=np.full_like(d.bface_kind, gen.BC_PEC))


def _one_element():
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    tets = np.array([[0, 1, 2, 3]])
    bfaces = np.array([[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]])
    return B.Desc(xyz, tets, np.array([2.0 + 0.5j]), bfaces, np.full(4, gen.BC_IMPEDANCE), np.zeros(1),
                  1, 1, 3.0, 3)


DEGENERATE = {
    "empty_subdomains": _empty_subdomains,
    "all_metallic": _all_metallic,
    "one_element": _one_element,
}


@pytest.mark.parametrize("name", list(VALID) + list(DEGENERATE))
def test_sanitized_layout_matches_library(checker, tmp_path, name):
    d = (VALID.get(name) or DEGENERATE[name])()
    status, msg, arrays = run_checker(checker, d, str(tmp_path / name))
    assert status == B.MXW_OK, msg
    compare_with_library(d, arrays)


def _bad(name):
    d = _cube(2, 1)
    nv, nt = len(d.xyz), len(d.tets)
    t, b, x, p = d.tets.copy(), d.bfaces.copy(), d.xyz.copy(), d.part.copy()
    if name == "vertex_id_too_large":
        t[3, 2] = nv
        return _rebuild(d, tets=t)
    if name == "vertex_id_negative":
        t[0, 0] = -1
        return _rebuild(d, tets=t)
    if name == "repeated_vertex":
        t[1, 1] = t[1, 0]
        return _rebuild(d, tets=t)
    if name == "coincident_vertices":
        x[t[0, 3]] = x[t[0, 0]]
        return _rebuild(d, xyz=x)
    if name == "nan_coordinate":
        x[5, 1] = np.nan
        return _rebuild(d, xyz=x)
    if name == "nan_permittivity":
        e = d.eps[:, 0] + 1j * d.eps[:, 1]
        e[2] = complex(np.nan, 0.0)
        return _rebuild(d, eps=e)
    if name == "infinite_k0":
        return _rebuild(d, k0=np.inf)
    if name == "negative_k0":
        return _rebuild(d, k0=-1.0)
    if name == "part_too_large":
        p[0] = d.c.n_sub
        return _rebuild(d, part=p)
    if name == "part_negative":
        p[nt - 1] = -1
        return _rebuild(d, part=p)
    if name == "degree_0":
        return _rebuild(d, degree=0)
    if name == "degree_4":
        return _rebuild(d, degree=4)
    if name == "no_subdomains":
        return _rebuild(d, n_sub=0)
    if name == "negative_overlap":
        return _rebuild(d, overlap=-1)
    if name == "unknown_precision":
        return _rebuild(d, precision=7)
    if name == "unknown_variant":
        return _rebuild(d, variant=9)
    if name == "boundary_face_missing":
        return _rebuild(d, bfaces=b[:-1], bface_kind=d.bface_kind[:-1])
    if name == "boundary_face_twice":
        b[-1] = b[0]
        return _rebuild(d, bfaces=b)
    if name == "interior_face_as_boundary":
        # a face of element 0 that no boundary face lists is interior
        listed = {tuple(sorted(f)) for f in b.tolist()}
        v = t[0].tolist()
        inner = next(f for f in ([v[0], v[1], v[2]], [v[0], v[1], v[3]], [v[0], v[2], v[3]],
                                 [v[1], v[2], v[3]]) if tuple(sorted(f)) not in listed)
        b[0] = inner
        return _rebuild(d, bfaces=b)
    if name == "boundary_face_ids_out_of_range":
        b[0] = [nv, nv + 1, nv + 7]
        return _rebuild(d, bfaces=b)
    if name == "unknown_boundary_kind":
        k = d.bface_kind.copy()
        k[0] = 5
        return _rebuild(d, bface_kind=k)
    if name == "no_elements":
        return B.Desc(x, np.zeros((0, 4), np.int32), np.zeros(0, complex), np.zeros((0, 3), np.int32),
                      np.zeros(0, np.int8), np.zeros(0, np.int32), 1, 1, 1.0, 1)
    if name == "element_three_times_on_a_face":
        return _rebuild(d, tets=np.vstack([t, t[:1]]), part=np.append(p, 0),
                        eps=np.append(d.eps[:, 0] + 1j * d.eps[:, 1], 1.0))
    raise KeyError(name)


BAD = ["vertex_id_too_large", "vertex_id_negative", "repeated_vertex", "coincident_vertices",
       "nan_coordinate", "nan_permittivity", "infinite_k0", "negative_k0", "part_too_large",
       "part_negative", "degree_0", "degree_4", "no_subdomains", "negative_overlap",
       "unknown_precision", "unknown_variant", "boundary_face_missing", "boundary_face_twice",
       "interior_face_as_boundary", "boundary_face_ids_out_of_range", "unknown_boundary_kind",
       "no_elements", "element_three_times_on_a_face"]


@pytest.mark.parametrize("name", BAD)
def test_sanitized_layout_rejects_malformed_mesh(checker, tmp_path, name):
    d = _bad(name)
    status, msg, _ = run_checker(checker, d, str(tmp_path / name))
    assert status == B.MXW_EINVAL, (status, msg)
    with pytest.raises(B.MxwError) as ei:
        Layout(d)
    assert ei.value.status == status and str(ei.value) == f"MXW_EINVAL: {msg}"
