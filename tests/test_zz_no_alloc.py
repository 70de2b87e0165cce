"""The no-allocation right-hand-side entry point against mxw_problem_rhs.

mxw_problem_rhs_noalloc computes the face integrals of plane-wave and port
sources in a fixed buffer compiled into the library instead of a temporary
allocation; its results must equal mxw_problem_rhs's bit for bit.  Two calls
in a row, the second on a smaller problem with fewer sources (the buffer
keeps the first call's contents), and a problem beyond the buffer's size
rejected with MXW_EINVAL.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1605_04521_amd import _lib as B
from paper_1605_04521_amd import gen
from paper_1605_04521_amd.api import Problem

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_rhs_noalloc_matches_rhs():
    big = gen.cube_planewave_problem(n=8, degree=3, box=2, n_sources=3)
    big.sources.append(gen.Source(kind=gen.SRC_DIPOLE, pos=(0.41, 0.37, 0.52), pol=(0.2 + 0.1j, -1.0 + 0j, 0.5j)))
    small = gen.cube_planewave_problem(n=4, degree=1, box=2, n_sources=1, seed=7)
    say("[gpu] no-alloc rhs: cube 8^3 r=3 (3 plane waves + dipole), then cube 4^3 r=1 (1 plane wave)")
    Pb = Problem.from_problem(big, defer_factor=True)
    Ps = Problem.from_problem(small, defer_factor=True)
    for P, prob in ((Pb, big), (Ps, small)):
        ref = P.rhs(prob.sources)
        # a poisoned output buffer: every entry must be written
        out = torch.full_like(ref, complex(float("nan"), float("nan")))
        got = P.rhs_noalloc(prob.sources, out=out)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert torch.count_nonzero(ref).item() > 0
    # again on the big problem after the small one
    ref = Pb.rhs(big.sources[:2])
    got = Pb.rhs_noalloc(big.sources[:2])
    assert torch.equal(got, ref)


def test_rhs_noalloc_allocates_nothing():
    """No allocation through the problem's context (whose allocator is
    PyTorch's) and none behind PyTorch's back, over repeated calls."""
    from paper_1605_04521_amd.api import Context
    prob = gen.cube_planewave_problem(n=6, degree=2, box=3, n_sources=2)
    ctx = Context()
    P = Problem.from_problem(prob, defer_factor=True, ctx=ctx)
    out = torch.empty((2, P.ndof), dtype=torch.complex128, device="cuda")
    P.rhs_noalloc(prob.sources, out=out)      # first call on the device looks the buffer up
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    u0 = ctx.usage(reset_peak=True)
    for _ in range(5):
        P.rhs_noalloc(prob.sources, out=out)
    torch.cuda.synchronize()
    u1 = ctx.usage()
    assert torch.cuda.mem_get_info()[0] == free0
    assert u1["peak"] == u0["in_use"] == u1["in_use"] and u1["live"] == u0["live"]
    # the allocating entry point, for contrast, takes its face buffer through the context
    P.rhs(prob.sources)
    assert ctx.usage()["peak"] > u1["in_use"]


def slab_problem(n):
    """One layer of an n^2 x 1 Kuhn grid (the bottom layer of the unit cube):
    many impedance faces for few elements; 512 RCB cores, no overlap, r = 3."""
    cube = gen.unit_cube(n)
    keep = cube.cube_of_tet[:, 2] == 0
    tets = cube.tets[keep]
    faces = np.sort(np.concatenate([tets[:, [0, 1, 2]], tets[:, [0, 1, 3]], tets[:, [0, 2, 3]],
                                    tets[:, [1, 2, 3]]]), axis=1)
    uniq, cnt = np.unique(faces, axis=0, return_counts=True)
    bf = uniq[cnt == 1].astype(np.int32)
    mesh = gen.Mesh(xyz=cube.xyz, tets=tets, bfaces=bf, bface_kind=np.full(len(bf), gen.BC_IMPEDANCE, np.int8))
    part = gen.rcb_partition(gen.centroids(mesh), 512)
    eps = np.full(len(tets), 1.0 + 0.1j)
    return gen.Problem(mesh=mesh, eps=eps, part=part, n_sub=512, overlap=0, k0=2 * np.pi, degree=3,
                       sources=[gen.plane_wave(0)])


def test_rhs_noalloc_rejects_too_many_faces():
    prob = slab_problem(66)          # 17,952 impedance faces x 15 face unknowns > 262,144
    from paper_1605_04521_amd.api import Layout
    lay = Layout.from_problem(prob)
    assert lay.info().n_imp_faces * 15 > (1 << 18)
    P = Problem.from_layout(lay, precision=B.MXW_MIXED, defer_factor=True)
    with pytest.raises(B.MxwError) as e:
        P.rhs_noalloc(prob.sources)
    assert e.value.status == B.MXW_EINVAL
    # the allocating entry point still serves it
    assert torch.count_nonzero(P.rhs(prob.sources)).item() > 0
