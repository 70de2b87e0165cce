"""Pins of the port oracle (TE10 excitation, eq. (3); S-matrix, eq. (5)):
a straight waveguide section whose exact field is known in closed form,
reciprocity of the discrete S-matrix, the mode norm and the port's faces."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.assemble import Discretization
from oracle.ports import beta10, port_faces, port_weights, smatrix
from paper_1605_04521_amd import gen

A_W, B_W, LEN, K0 = 1.0, 0.5, 1.5, 5.0


def guide_ports():
    return [gen.port((A_W / 2, B_W / 2, 0.0), (A_W / 2, 0, 0), (0, B_W / 2, 0)),
            gen.port((A_W / 2, B_W / 2, LEN), (A_W / 2, 0, 0), (0, B_W / 2, 0))]


def guide_disc(n, r):
    mesh = gen.waveguide(n, A_W, B_W, LEN)
    eps = np.ones(len(mesh.tets), dtype=np.complex128)
    return Discretization(mesh.xyz, mesh.tets, eps, mesh.bfaces, mesh.bface_kind, K0, r)


def exact_profile():
    """E = f(z) sin(pi x / a) y with f'' + beta10^2 f = 0, the excitation
    -f'(0) - i beta f(0) = -i (beta10 + beta) at z = 0 and the homogeneous
    impedance condition f'(L) - i beta f(L) = 0 at z = L; beta = k0 (eps = 1)."""
    bt = K0
    b10 = np.sqrt(K0 ** 2 - (np.pi / A_W) ** 2)
    e = np.exp(1j * b10 * LEN)
    M = np.array([[-1j * b10 - 1j * bt, 1j * b10 - 1j * bt],
                  [(1j * b10 - 1j * bt) * e, (-1j * b10 - 1j * bt) / e]])
    A, B = np.linalg.solve(M, [-1j * (b10 + bt), 0.0])
    return lambda z: A * np.exp(1j * b10 * z) + B * np.exp(-1j * b10 * z)


def solved_smatrix(n, r):
    d = guide_disc(n, r)
    ports = guide_ports()
    Am = d.global_matrix().tocsc()
    X = np.stack([spla.spsolve(Am, d.rhs(p)) for p in ports], axis=1)
    return smatrix(d, X, ports)


def test_waveguide_closed_form():
    """S_11 = conj(f(0)) and S_21 = conj(f(L)) for the exact field; the error
    falls with h and with the degree r."""
    f = exact_profile()
    ex = np.array([np.conj(f(0.0)), np.conj(f(LEN))])
    err = {}
    for n, r in [(4, 2), (6, 2), (4, 3)]:
        S = solved_smatrix(n, r)
        err[(n, r)] = np.abs(S[:, 0] - ex).max()
    assert err[(4, 2)] < 3e-2
    assert err[(6, 2)] < err[(4, 2)] / 3.0
    assert err[(4, 3)] < 1e-3


def test_reciprocity():
    """Identical ports and a symmetric matrix: S_12 = S_21."""
    S = solved_smatrix(4, 1)
    assert abs(S[0, 1] - S[1, 0]) <= 1e-12 * abs(S[1, 0])


def test_mode_norm_and_port_faces():
    """int |E^0|^2 = a b / 2 up to the face quadrature's error; the port at
    z = 0 is the whole end of the guide (2 n^2 triangles)."""
    d = guide_disc(4, 2)
    p0 = guide_ports()[0]
    assert len(port_faces(d, p0)) == 2 * 4 ** 2
    _, nrm = port_weights(d, p0)
    assert abs(nrm - A_W * B_W / 2) <= 1e-6 * A_W * B_W
    # a port on a quarter of the end: only the faces inside it
    q = gen.port((A_W / 4, B_W / 4, 0.0), (A_W / 4, 0, 0), (0, B_W / 4, 0))
    assert len(port_faces(d, q)) == 2 * 2 ** 2


def test_port_rhs_is_the_scaled_mode_weight():
    """On a homogeneous port g = -i (beta10 + beta) E^0, so b = -i (beta10 +
    beta) w with w the mode weights."""
    d = guide_disc(3, 2)
    p0 = guide_ports()[0]
    w, _ = port_weights(d, p0)
    b = d.rhs(p0)
    fac = -1j * (beta10(K0, A_W) + K0)
    assert np.linalg.norm(b - fac * w) <= 1e-13 * np.linalg.norm(b)
