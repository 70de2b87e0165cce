"""Waveguide ports: TE10 excitation (eq. (3)) and the S-matrix (eq. (5)) (oracle).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this module; the product path never does.

Sec. 2 excites the chamber through the port of one waveguide with the
impedance data g_j built from the TE10 fundamental mode E_j^0 of that
waveguide (eq. (3)), the other ports carrying the same impedance condition
without data (eq. (4)); Sec. 5 compares with measurements through the
S-matrix, the projection of the field on each port's mode normalised by the
mode's own norm on that port (eq. (5)).

Readings (the chamber's ports are not available, so the ports here are
synthetic):
* a port is a rectangle on an impedance part of the boundary, given by its
  centre c, half its wide side (unit vector u, width a) and half its narrow
  side (unit vector v, height b); its faces are the impedance faces whose
  centroid lies in the rectangle (within 1e-9 (a + b) of its plane);
* the mode on the port plane is E^0 = sin(pi ((x - c).u + a/2) / a) v, and
  it propagates into the domain as exp(i beta10 w), w the distance from the
  port along the inward normal, beta10 = sqrt(beta^2 - (pi/a)^2) with beta
  the face's impedance wave number (R2: k0 sqrt(Re eps)); below cut-off
  beta10 = 0;
* with the exp(-i w t) convention of the rest of the code the impedance
  condition reads (curl E) x n - i beta E_t = g, and for the incoming mode
  (curl E^0) x n = -i beta10 E^0_t on the port, so g = -i (beta10 + beta) E^0;
* the S-matrix integrals use the same face quadrature as the right-hand
  sides (R11): S_ij = sum_k conj(x_j[k]) w_i[k] / d_i with
  w_i[k] = int_{Gamma_i} phi_k . E_i^0 and d_i = int_{Gamma_i} |E_i^0|^2
  (the basis functions are real, so conj(E_j) = sum_k conj(x_j[k]) phi_k).
"""
from __future__ import annotations

import numpy as np

from .basis import LOCAL_FACES


def frame(src):
    """(c, u, v, a, b) of a port source (pos = centre, dir = half width,
    pol = half height)."""
    c = np.asarray(src.pos, dtype=np.float64)
    hw = np.asarray(src.dir, dtype=np.float64)
    hh = np.real(np.asarray(src.pol, dtype=np.complex128))
    a, b = 2.0 * np.linalg.norm(hw), 2.0 * np.linalg.norm(hh)
    return c, hw / np.linalg.norm(hw), hh / np.linalg.norm(hh), a, b


def port_faces(disc, src):
    """The impedance faces (t, lf, beta) of the port."""
    c, u, v, a, b = frame(src)
    nrm = np.cross(u, v)
    tol = 1e-9 * (a + b)
    out = []
    for t, lf, beta in disc.imp_faces:
        lam = np.full(4, 1.0 / 3.0)
        lam[[q for q in range(4) if q not in LOCAL_FACES[lf]]] = 0.0
        x = disc.point(t, lam) - c
        if abs(x @ nrm) <= tol and abs(x @ u) <= 0.5 * a + tol and abs(x @ v) <= 0.5 * b + tol:
            out.append((t, lf, beta))
    return out


def mode(src):
    """E^0(x) on the port plane."""
    c, u, v, a, b = frame(src)
    return lambda x: np.sin(np.pi * ((x - c) @ u + 0.5 * a) / a) * v


def beta10(beta, a):
    return np.sqrt(max(beta * beta - (np.pi / a) ** 2, 0.0))


def rhs_port(disc, src):
    """b_k = int_{Gamma} g . phi_k with g = -i (beta10 + beta) E^0 (eq. (3))."""
    _, _, _, a, _ = frame(src)
    E0 = mode(src)
    g = lambda x, n, beta, t: -1j * (beta10(beta, a) + beta) * E0(x)
    return disc.rhs_boundary(g, faces=port_faces(disc, src))


def port_weights(disc, src):
    """w_k = int_{Gamma} phi_k . E^0 and d = int_{Gamma} |E^0|^2."""
    E0 = mode(src)
    faces = port_faces(disc, src)
    w = disc.rhs_boundary(lambda x, n, beta, t: E0(x).astype(np.complex128), faces=faces)
    d = 0.0
    q = disc.basis.r + 3
    for t, lf, beta in faces:
        pts, wts, _ = disc.face_points(t, lf, q)
        for lam, wq in zip(pts, wts):
            e = E0(disc.point(t, lam))
            d += wq * float(e @ e)
    return w, d


def smatrix(disc, X, ports):
    """S[i, j] (eq. (5)) for the fields X[:, j] and the ports' modes."""
    S = np.zeros((len(ports), X.shape[1]), dtype=np.complex128)
    for i, p in enumerate(ports):
        w, d = port_weights(disc, p)
        S[i] = (X.conj().T @ w) / d
    return S
