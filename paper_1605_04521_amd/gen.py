"""Seeded synthetic inputs: meshes, permittivity maps, partitions and sources.

This module produces problem *inputs* only (geometry, material data, the
core partition and source descriptions).  It performs none of the method's
arithmetic: no entity extraction, no basis functions, no assembly, no
solves.  Both the library binding and the CPU reference take its output.

Workload shapes follow the paper's imaging chamber (Sec. 1, Fig. 1: a
metallic cylinder filled with a lossy matching medium, Sec. 5.1 for the
medium values) and the unit-cube plane-wave problem used for validation.

Time convention: fields vary as exp(-i w t), so a lossy medium has
Im(eps) > 0.  The paper writes exp(+i w t) and Im(eps) < 0; every value
here is the complex conjugate of the paper's.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

BC_PEC = 0
BC_IMPEDANCE = 1
SRC_DIPOLE = 0
SRC_PLANEWAVE = 1
SRC_PORT = 2

# speed of light (m/s); chamber wavenumber at 1 GHz in 1/m
C0 = 299792458.0
K0_1GHZ = 2.0 * math.pi * 1.0e9 / C0


@dataclass
class Mesh:
    xyz: np.ndarray          # float64 [V,3]
    tets: np.ndarray         # int32 [T,4]
    bfaces: np.ndarray       # int32 [Fb,3], vertex ids ascending
    bface_kind: np.ndarray   # int8 [Fb]
    grid_n: int = 0          # cubes per side of the underlying Kuhn grid
    cube_of_tet: np.ndarray = field(default=None, repr=False)  # int32 [T,3]


@dataclass
class Source:
    kind: int
    pos: tuple = (0.0, 0.0, 0.0)
    pol: tuple = (0j, 0j, 0j)       # complex polarisation / dipole moment; port: half-height vector
    dir: tuple = (0.0, 0.0, 0.0)    # plane-wave propagation direction; port: half-width vector


@dataclass
class Problem:
    mesh: Mesh
    eps: np.ndarray          # complex128 [T]
    part: np.ndarray         # int32 [T]
    n_sub: int
    overlap: int
    k0: float
    degree: int
    sources: list
    name: str = ""


# --------------------------------------------------------------------------
# Kuhn-split structured grids
# --------------------------------------------------------------------------

_PERMS = list(itertools.permutations(range(3)))
_UNIT = np.eye(3, dtype=np.int64)


def _kuhn_topology(n: int):
    """Vertex grid (n+1)^3 and the 6 Kuhn tets of each of the n^3 cubes.

    Vertex (i,j,k) has id i + (n+1)(j + (n+1)k).  Cube (i,j,k) is split into
    the tets {v, v+e_a, v+e_a+e_b, v+(1,1,1)} for each permutation (a,b,c)
    of the axes, in itertools order.  Tet id = 6*(i + n(j + n k)) + perm.
    """
    m = n + 1
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cube = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)   # i fastest
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    gidx = lambda p: p[:, 0] + m * (p[:, 1] + m * p[:, 2])
    for q, (a, b, _) in enumerate(_PERMS):
        p0 = cube
        p1 = cube + _UNIT[a]
        p2 = p1 + _UNIT[b]
        p3 = cube + 1
        tets[:, q, 0] = gidx(p0)
        tets[:, q, 1] = gidx(p1)
        tets[:, q, 2] = gidx(p2)
        tets[:, q, 3] = gidx(p3)
    cube_of_tet = np.repeat(cube, 6, axis=0)
    return tets.reshape(-1, 4), cube_of_tet


def _grid_boundary_faces(n: int, tets: np.ndarray, kind_of_plane):
    """Faces of the Kuhn tets lying in one of the 6 planes of the index box.

    kind_of_plane(axis, side) -> BC kind.  Classification uses integer grid
    coordinates only.
    """
    m = n + 1
    ijk = np.stack([tets % m, (tets // m) % m, tets // (m * m)], axis=2)  # [T,4,3]
    faces, kinds = [], []
    for drop in range(4):
        keep = [c for c in range(4) if c != drop]
        fv = tets[:, keep]
        fijk = ijk[:, keep, :]
        for axis in range(3):
            for side, val in ((0, 0), (1, n)):
                on = np.all(fijk[:, :, axis] == val, axis=1)
                if on.any():
                    faces.append(np.sort(fv[on], axis=1))
                    kinds.append(np.full(on.sum(), kind_of_plane(axis, side), dtype=np.int8))
    faces = np.concatenate(faces)
    kinds = np.concatenate(kinds)
    order = np.lexsort((faces[:, 2], faces[:, 1], faces[:, 0]))
    return faces[order].astype(np.int32), kinds[order]


def unit_cube(n: int, bc: int = BC_IMPEDANCE) -> Mesh:
    """[0,1]^3 as an n^3 Kuhn grid; every boundary face gets kind `bc`."""
    tets, cube = _kuhn_topology(n)
    m = n + 1
    g = np.arange(m) / n
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    bf, bk = _grid_boundary_faces(n, tets, lambda a, s: bc)
    return Mesh(xyz=xyz, tets=tets.astype(np.int32), bfaces=bf, bface_kind=bk,
                grid_n=n, cube_of_tet=cube.astype(np.int32))


def waveguide(n: int, a: float, b: float, length: float, cells=None) -> Mesh:
    """Rectangular waveguide section [0,a] x [0,b] x [0,length] as a Kuhn grid
    of n^3 cells (stretched per axis): metallic (PEC) side walls, impedance
    faces at z = 0 and z = length (the two ports)."""
    tets, cube = _kuhn_topology(n)
    m = n + 1
    g = np.arange(m) / n
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([a * x.ravel(), b * y.ravel(), length * z.ravel()], axis=1)
    bf, bk = _grid_boundary_faces(n, tets, lambda ax, side: BC_IMPEDANCE if ax == 2 else BC_PEC)
    return Mesh(xyz=xyz, tets=tets.astype(np.int32), bfaces=bf, bface_kind=bk,
                grid_n=n, cube_of_tet=cube.astype(np.int32))


def port(center, half_width, half_height) -> Source:
    """Rectangular port: centre, half the wide side (the TE10 profile varies
    along it) and half the narrow side (the direction of E)."""
    return Source(kind=SRC_PORT, pos=tuple(float(v) for v in center),
                  pol=tuple(complex(v) for v in half_height), dir=tuple(float(v) for v in half_width))


def top_ports(count: int, radius: float = 0.15, height: float = 0.28, ring: float = 0.09,
              width: float = 0.04, narrow: float = 0.02) -> list:
    """count rectangular ports on the chamber's flat top (z = height), centred
    on a ring, wide side tangential: synthetic stand-ins for the chamber's
    waveguide ports (the real ones open into the lateral wall)."""
    out = []
    for q in range(count):
        t = 2.0 * math.pi * q / count
        c = (ring * math.cos(t), ring * math.sin(t), height)
        hw = (-0.5 * width * math.sin(t), 0.5 * width * math.cos(t), 0.0)
        hh = (0.5 * narrow * math.cos(t), 0.5 * narrow * math.sin(t), 0.0)
        out.append(port(c, hw, hh))
    return out


def chamber_cylinder(n: int, radius: float = 0.15, height: float = 0.28, shape: str = "cylinder") -> Mesh:
    """Cylindrical chamber: Kuhn grid on [-1,1]^2 x [0,1] mapped to a cylinder.

    (u,v) -> R (u sqrt(1 - v^2/2), v sqrt(1 - u^2/2)), w -> H w; straight-sided
    tets.  Lateral wall and bottom are metallic (PEC), the top is an
    impedance boundary (Sec. 2: metallic bottom, impedance top).
    """
    tets, cube = _kuhn_topology(n)
    m = n + 1
    g = np.arange(m)
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    u = -1.0 + 2.0 * ii.ravel() / n
    v = -1.0 + 2.0 * jj.ravel() / n
    w = kk.ravel() / n
    if shape == "cylinder":
        x = radius * u * np.sqrt(1.0 - 0.5 * v * v)
        y = radius * v * np.sqrt(1.0 - 0.5 * u * u)
    elif shape == "box":          # square cross-section [-R,R]^2 (no mapping)
        x = radius * u
        y = radius * v
    else:
        raise ValueError("shape must be 'cylinder' or 'box'")
    xyz = np.stack([x, y, height * w], axis=1)

    def kind(axis, side):
        if axis == 2 and side == 1:
            return BC_IMPEDANCE
        return BC_PEC

    bf, bk = _grid_boundary_faces(n, tets, kind)
    return Mesh(xyz=xyz, tets=tets.astype(np.int32), bfaces=bf, bface_kind=bk,
                grid_n=n, cube_of_tet=cube.astype(np.int32))


def _kuhn_block(vid: np.ndarray) -> np.ndarray:
    """Kuhn split of a structured block; vid[a,b,c] = global vertex id."""
    na, nb, nc = (d - 1 for d in vid.shape)
    A, Bb, Cc = np.meshgrid(np.arange(na), np.arange(nb), np.arange(nc), indexing="ij")
    A, Bb, Cc = A.ravel(), Bb.ravel(), Cc.ravel()
    out = np.empty((len(A), 6, 4), dtype=np.int64)
    for q, (x, y, _) in enumerate(_PERMS):
        p0 = np.stack([A, Bb, Cc], axis=1)
        p1 = p0 + _UNIT[x]
        p2 = p1 + _UNIT[y]
        p3 = p0 + 1
        for c, p in enumerate((p0, p1, p2, p3)):
            out[:, q, c] = vid[p[:, 0], p[:, 1], p[:, 2]]
    return out.reshape(-1, 4)


def _block_faces(vid: np.ndarray, tets: np.ndarray, axis: int, side: int) -> np.ndarray:
    """Faces of the block's Kuhn tets lying on its face axis=0 (side 0) or axis=max (side 1)."""
    val = 0 if side == 0 else vid.shape[axis] - 1
    on = np.zeros(vid.max() + 1, dtype=bool)
    sl = [slice(None)] * 3
    sl[axis] = val
    on[vid[tuple(sl)].ravel()] = True
    out = []
    for drop in range(4):
        keep = [c for c in range(4) if c != drop]
        fv = tets[:, keep]
        sel = np.all(on[fv], axis=1)
        out.append(np.sort(fv[sel], axis=1))
    return np.concatenate(out)


def chamber_ogrid(nc: int, nr: int, nz: int, radius: float = 0.15, height: float = 0.28,
                  inner: float = 0.5) -> Mesh:
    """Cylindrical chamber as a 5-block O-grid, each block Kuhn-split.

    Centre block: the square |x|,|y| <= inner*R with nc x nc cells.  Four outer
    blocks join the square's sides to the circle of radius R: nr radial x nc
    tangential cells, points blended linearly from the square side to the arc.
    nz layers in height.  Local axes are oriented so that every face shared by
    two blocks gets the same diagonal from both sides (a conforming mesh).
    Lateral wall and bottom are metallic (PEC), the top is an impedance face.
    No grid corner lies on the circle, so no element degenerates there.
    """
    a = inner * radius
    zc = height * np.arange(nz + 1) / nz
    tt = -1.0 + 2.0 * np.arange(nc + 1) / nc
    ss = np.arange(nr + 1) / nr
    pts, blocks = [], []

    def add(X, Y):
        """X, Y: [n0+1, n1+1] planar coordinates; returns local vertex ids [n0+1,n1+1,nz+1]."""
        base = sum(len(p) for p in pts)
        n0, n1 = X.shape
        P = np.empty((n0, n1, nz + 1, 3))
        P[..., 0] = X[:, :, None]
        P[..., 1] = Y[:, :, None]
        P[..., 2] = zc[None, None, :]
        pts.append(P.reshape(-1, 3))
        return base + np.arange(n0 * n1 * (nz + 1)).reshape(n0, n1, nz + 1)

    # centre: axes (x, y, z)
    U, V = np.meshgrid(tt, tt, indexing="ij")
    blocks.append(("centre", add(a * U, a * V)))
    S, T = np.meshgrid(ss, tt, indexing="ij")           # [radial, tangential]
    th = T * np.pi / 4
    specs = {  # inner point (on the square) and outer point (on the circle)
        "right": ((a + 0 * T, a * T), (radius * np.cos(th), radius * np.sin(th))),
        "top": ((a * T, a + 0 * T), (radius * np.sin(th), radius * np.cos(th))),
        "left": ((-a + 0 * T, a * T), (-radius * np.cos(th), radius * np.sin(th))),
        "bottom": ((a * T, -a + 0 * T), (radius * np.sin(th), -radius * np.cos(th))),
    }
    for name, ((xi, yi), (xo, yo)) in specs.items():
        blocks.append((name, add((1 - S) * xi + S * xo, (1 - S) * yi + S * yo)))
    xyz_all = np.concatenate(pts)
    key = np.round(xyz_all / (radius * 1e-9)).astype(np.int64)
    uniq, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.ravel()
    # renumber merged vertices in order of first appearance
    order = np.argsort(first)
    rank = np.empty_like(order)
    rank[order] = np.arange(len(order))
    gid = rank[inv]
    xyz = xyz_all[first[order]]
    tets, faces, kinds, cells = [], [], [], []
    for bi, (name, vid) in enumerate(blocks):
        g = gid[vid]
        tb = _kuhn_block(g)
        tets.append(tb)
        na, nb, ncz = (d - 1 for d in vid.shape)
        A, Bb, Cc = np.meshgrid(np.arange(na), np.arange(nb), np.arange(ncz), indexing="ij")
        cl = np.stack([np.full(A.size, bi), A.ravel(), Bb.ravel(), Cc.ravel()], axis=1)
        cells.append(np.repeat(cl, 6, axis=0))
        bot = _block_faces(g, tb, 2, 0)
        top = _block_faces(g, tb, 2, 1)
        faces += [bot, top]
        kinds += [np.full(len(bot), BC_PEC, np.int8), np.full(len(top), BC_IMPEDANCE, np.int8)]
        if name != "centre":
            wall = _block_faces(g, tb, 0, 1)
            faces.append(wall)
            kinds.append(np.full(len(wall), BC_PEC, np.int8))
    tets = np.concatenate(tets)
    faces = np.concatenate(faces)
    kinds = np.concatenate(kinds)
    o = np.lexsort((faces[:, 2], faces[:, 1], faces[:, 0]))
    return Mesh(xyz=xyz, tets=tets.astype(np.int32), bfaces=faces[o].astype(np.int32),
                bface_kind=kinds[o], grid_n=0, cube_of_tet=np.concatenate(cells).astype(np.int32))


def ogrid_block_partition(mesh: Mesh, ba: int, bb: int, bc: int) -> tuple[np.ndarray, int]:
    """Core subdomains of an O-grid mesh: boxes of ba x bb x bc cells in each
    block's own (radial or x, tangential or y, z) index space."""
    cl = mesh.cube_of_tet
    blk = cl[:, 0]
    key = np.stack([blk, cl[:, 1] // ba, cl[:, 2] // bb, cl[:, 3] // bc], axis=1)
    _, part = np.unique(key, axis=0, return_inverse=True)
    part = part.ravel().astype(np.int32)
    return part, int(part.max()) + 1


def centroids(mesh: Mesh) -> np.ndarray:
    return mesh.xyz[mesh.tets].mean(axis=1)


# --------------------------------------------------------------------------
# permittivity maps
# --------------------------------------------------------------------------

EPS_MATCHING = 44.0 + 20.0j   # matching medium, Sec. 5.1 (conjugated)
EPS_HEAD = 40.0 + 15.0j


def chamber_eps(mesh: Mesh, seed: int):
    """Background medium, a seeded ellipsoidal head and one spherical inclusion.

    The inclusion changes the head permittivity by +-20 % (sign from the
    seed), mimicking the two stroke types of the introduction.
    Returns (eps[T], description dict).
    """
    rng = np.random.default_rng(seed)
    c = centroids(mesh)
    centre = np.array([0.0, 0.0, 0.14]) + rng.uniform(-0.01, 0.01, 3)
    axes = np.array([0.08, 0.10, 0.09])
    theta = rng.uniform(0.0, 2.0 * math.pi)
    ct, st = math.cos(theta), math.sin(theta)
    rot = np.array([[ct, -st, 0.0], [st, ct, 0.0], [0.0, 0.0, 1.0]])
    loc = (c - centre) @ rot              # coordinates in the head frame
    in_head = np.sum((loc / axes) ** 2, axis=1) <= 1.0
    r_inc = rng.uniform(0.01, 0.02)
    # inclusion centre: inside the head, at most half-way to its surface
    off = rng.uniform(-0.5, 0.5, 3) * (axes - r_inc)
    inc_centre = centre + rot @ off
    in_inc = np.sum((c - inc_centre) ** 2, axis=1) <= r_inc ** 2
    sign = 1.0 if rng.uniform() < 0.5 else -1.0
    eps = np.full(len(c), EPS_MATCHING, dtype=np.complex128)
    eps[in_head] = EPS_HEAD
    eps[in_inc & in_head] = EPS_HEAD * (1.0 + 0.2 * sign)
    info = dict(head_centre=centre, head_theta=theta, inc_centre=inc_centre,
                inc_radius=r_inc, inc_sign=sign)
    return eps, info


# --------------------------------------------------------------------------
# partitions
# --------------------------------------------------------------------------

def box_partition(mesh: Mesh, box: int) -> tuple[np.ndarray, int]:
    """Core subdomain = box of box^3 grid cubes; id in lexicographic box order."""
    n = mesh.grid_n
    nb = -(-n // box)
    b = mesh.cube_of_tet // box
    part = b[:, 0] + nb * (b[:, 1] + nb * b[:, 2])
    return part.astype(np.int32), nb ** 3


def rcb_partition(points: np.ndarray, n_sub: int, weights=None) -> np.ndarray:
    """Recursive coordinate bisection of element centroids into n_sub parts.

    Each split cuts the longest bounding-box axis; elements are ordered by
    (coordinate, element id) and divided in proportion to the number of
    leaves on each side.  Deterministic.
    """
    npts = len(points)
    part = np.empty(npts, dtype=np.int32)
    ids = np.arange(npts)
    stack = [(ids, 0, n_sub)]
    while stack:
        sel, first, cnt = stack.pop()
        if cnt == 1:
            part[sel] = first
            continue
        p = points[sel]
        axis = int(np.argmax(p.max(axis=0) - p.min(axis=0)))
        order = np.lexsort((sel, p[:, axis]))
        left = cnt // 2
        cut = int(round(len(sel) * left / cnt))
        stack.append((sel[order[:cut]], first, left))
        stack.append((sel[order[cut:]], first + left, cnt - left))
    return part


# --------------------------------------------------------------------------
# sources
# --------------------------------------------------------------------------

def plane_wave(seed: int) -> Source:
    """Plane wave with seeded unit direction d and unit polarisation p _|_ d."""
    rng = np.random.default_rng(seed)
    g1 = rng.standard_normal(3)
    u = rng.standard_normal(3)
    d = g1 / np.linalg.norm(g1)
    p = u - (u @ d) * d
    p /= np.linalg.norm(p)
    return Source(kind=SRC_PLANEWAVE, pol=tuple(complex(x) for x in p), dir=tuple(d))


def ring_dipoles(count: int = 32, radius: float = 0.14, z: float = 0.196,
                 first: int = 0, stride: int = 1) -> list:
    """z-polarised point dipoles at angles 2 pi (m + 1/2)/count on a ring."""
    out = []
    for m in range(first, count, stride):
        phi = 2.0 * math.pi * (m + 0.5) / count
        out.append(Source(kind=SRC_DIPOLE,
                          pos=(radius * math.cos(phi), radius * math.sin(phi), z),
                          pol=(0j, 0j, 1.0 + 0j)))
    return out


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def cube_planewave_problem(n: int = 8, degree: int = 1, box: int = 4, overlap: int = 1,
                           eps=1.0 + 0.1j, k0: float = 2.0 * math.pi, seed: int = 0,
                           n_sources: int = 1) -> Problem:
    """Unit cube, homogeneous eps, impedance everywhere, plane-wave source(s).

    Default: 8^3 cubes, r=1, 2x2x2 box subdomains, one face-layer overlap,
    eps = 1+0.1i, k0 = 2 pi (one free-space wavelength per side).
    """
    mesh = unit_cube(n)
    eps_t = np.full(len(mesh.tets), eps, dtype=np.complex128)
    part, n_sub = box_partition(mesh, box)
    srcs = [plane_wave(seed + s) for s in range(n_sources)]
    return Problem(mesh=mesh, eps=eps_t, part=part, n_sub=n_sub, overlap=overlap,
                   k0=k0, degree=degree, sources=srcs,
                   name=f"cube n={n} r={degree} box={box} ov={overlap}")


def chamber_problem(n: int = 22, degree: int = 2, n_sub=(2, 2, 3), overlap: int = 2,
                    seed: int = 0, n_sources: int = 1, ring_z: float = 0.196, shape: str = "cylinder",
                    nr: int = None, nz: int = None) -> Problem:
    """Synthetic imaging chamber (cylinder R=0.15 m, H=0.28 m) at 1 GHz.

    shape "cylinder": 5-block O-grid with n cells along the centre square's
    side, nr radial cells (default n//2) and nz layers (default n);
    the default 22/11/27 gives 1,477,926 degree-2 unknowns.  "mapped" and
    "box": single-block n^3 Kuhn grids (square mapped to the disc, or a
    square cross-section).  Background eps = 44+20i, seeded head ellipsoid
    eps = 40+15i and a +-20 % spherical inclusion.  n_sub: an int gives an
    RCB core partition into that many parts; a tuple (a, b, c) gives O-grid
    block-aligned cores of a x b x c cells.  z-polarised dipoles on the ring
    of radius 0.14 m.
    """
    if shape == "cylinder":
        nr = nr if nr is not None else max(1, n // 2)
        nz = nz if nz is not None else n
        mesh = chamber_ogrid(n, nr, nz)
        tag = f"ogrid {n}x{nr}x{nz}"
    else:
        mesh = chamber_cylinder(n, shape=shape)
        tag = f"{shape} {n}^3"
    eps, _ = chamber_eps(mesh, seed)
    if isinstance(n_sub, tuple):       # (ba, bb, bc) block-aligned boxes of an O-grid
        part, n_sub = ogrid_block_partition(mesh, *n_sub)
    else:
        part = rcb_partition(centroids(mesh), n_sub)
    srcs = ring_dipoles(32, 0.14, ring_z)[:n_sources] if n_sources <= 32 else \
        [s for z in (0.028, 0.084, 0.140, 0.196, 0.252) for s in ring_dipoles(32, 0.14, z)][:n_sources]
    return Problem(mesh=mesh, eps=eps, part=part, n_sub=n_sub, overlap=overlap,
                   k0=K0_1GHZ, degree=degree, sources=srcs,
                   name=f"chamber {tag} r={degree} nsub={n_sub} ov={overlap}")
