"""Oracle: the inter-element coupling predictors of Sec. II-E, from a port
impedance matrix.

TEST INFRASTRUCTURE ONLY (see oracle/mom.py).  Plain definitions, written from
the equations:

* xi_Z (eq. (predZ)): |Z_p,cj| / |Z_p,cc| for the border element j nearest to the
  center element c; the unapproximated form takes the maximum over the border
  (the expression just before eq. (predZ)); the bound of eq. (badpred) is the
  sum of |Z_p,cn| over the border.
* C_n (eq. (amitayPred)): the Fourier coefficients of the center element's
  active reflection coefficient along the E-plane cut, Gamma_a(psi) =
  sum_j S_cj exp(j n_j psi) with n_j the column offset of element j from the
  center column (psi_y = 0, uniform amplitudes), C_n = (1/2 pi) int Gamma_a(psi)
  exp(-j n psi) dpsi over [-pi, pi], evaluated with the Q-point trapezoid rule
  (exact for Q >= nx: Gamma_a is a trigonometric polynomial of degree < nx).
  Eq. (amitayPredTheta) is the same integral with the ARC sampled at the scan
  angles theta = asin(psi / (k d)); sampling psi uniformly is sampling those.
* xi_S (eq. (predS)): an idealised scattering matrix S_ideal on the lattice
  (diagonal S_cc, off-diagonal S_1 (rho/1)^a exp(-j k (r - d1)): the nearest-
  neighbour coupling S_1 at lattice distance 1 and physical distance d1 = dx,
  decaying as the element distance rho to the power a (a = -2 for an infinite
  planar array) with the free-space phase of the extra path), converted by
  eq. (S2Z), and |[Z_ideal]_cj| / |Z_p,cc| for the border element j nearest c.

Readings where the paper is silent: the border E_B of an nx x ny array is its
outer ring (the elements that growing from (nx-2) x (ny-2) adds; an axis of
extent 1 contributes no border); "nearest" is the smallest physical distance,
ties broken by the smallest element index; the element distance rho between two
elements is the Euclidean distance of their lattice indices; S_1 is the
coupling of the center element to its +x neighbour.
"""
from __future__ import annotations

import numpy as np

from . import mom


def border_elements(lat) -> np.ndarray:
    """Element indices of the outer ring (e = iy*nx + ix)."""
    iy, ix = np.divmod(np.arange(lat.nx * lat.ny), lat.nx)
    on = np.zeros(lat.nx * lat.ny, dtype=bool)
    if lat.nx > 1:
        on |= (ix == 0) | (ix == lat.nx - 1)
    if lat.ny > 1:
        on |= (iy == 0) | (iy == lat.ny - 1)
    return np.nonzero(on)[0]


def nearest_border(lat, c: int) -> int:
    """The border element nearest to c (not c itself); ties: smallest index."""
    xy = mom.element_xy(lat)
    B = np.array([e for e in border_elements(lat) if e != c])
    if B.size == 0:
        raise ValueError("the array has no border element other than the center")
    d = np.hypot(xy[B, 0] - xy[c, 0], xy[B, 1] - xy[c, 1])
    return int(B[np.flatnonzero(d == d.min())[0]])


def xi_z(Zp: np.ndarray, lat, center=None) -> dict:
    """Eq. (predZ) and its maximum form; eq. (badpred)'s border sum (ohm)."""
    c = mom.center_element(lat) if center is None else center
    j = nearest_border(lat, c)
    B = np.array([e for e in border_elements(lat) if e != c])
    zcc = abs(Zp[c, c])
    return {
        "nearest": j,
        "xi_z": abs(Zp[c, j]) / zcc,
        "xi_z_max": max(abs(Zp[c, e]) for e in B) / zcc,
        "border_sum": float(sum(abs(Zp[c, e]) for e in B)),
    }


def eplane_arc(S: np.ndarray, lat, psi, center=None) -> np.ndarray:
    """Gamma_a(psi) = sum_j S_cj exp(j (ix_j - ix_c) psi): uniform amplitudes,
    progressive phase psi between columns, none between rows."""
    c = mom.center_element(lat) if center is None else center
    ix = np.arange(lat.nx * lat.ny) % lat.nx
    n = ix - ix[c]
    psi = np.atleast_1d(np.asarray(psi, dtype=float))
    return np.array([np.sum(S[c, :] * np.exp(1j * n * p)) for p in psi])


def column_coupling(S: np.ndarray, lat, nq: int, center=None):
    """C_n of eq. (amitayPred) for n = -ix_c .. nx-1-ix_c by the nq-point
    trapezoid rule over psi in [-pi, pi); returns (n, C_n, psi, Gamma_a(psi))."""
    c = mom.center_element(lat) if center is None else center
    ixc = c % lat.nx
    psi = -np.pi + 2.0 * np.pi * np.arange(nq) / nq
    g = eplane_arc(S, lat, psi, c)
    n = np.arange(-ixc, lat.nx - ixc)
    C = np.array([np.mean(g * np.exp(-1j * k * psi)) for k in n])
    return n, C, psi, g


def ideal_s(lat, s: float, s_cc: complex, s_1: complex, decay: float = -2.0) -> np.ndarray:
    """S_ideal on the lattice (P x P)."""
    k = mom.wavenumber(s)
    P = lat.nx * lat.ny
    iy, ix = np.divmod(np.arange(P), lat.nx)
    xy = mom.element_xy(lat)
    S = np.empty((P, P), dtype=np.complex128)
    for a in range(P):
        for b in range(P):
            if a == b:
                S[a, b] = s_cc
            else:
                rho = np.hypot(ix[a] - ix[b], iy[a] - iy[b])
                r = np.hypot(xy[a, 0] - xy[b, 0], xy[a, 1] - xy[b, 1])
                S[a, b] = s_1 * rho ** decay * np.exp(-1j * k * (r - lat.dx))
    return S


def xi_s(lat, s: float, s_cc: complex, s_1: complex, zp_cc: complex, z0: float = 50.0, decay: float = -2.0,
         center=None) -> float:
    """Eq. (predS): |[z0 (1 + S_ideal)(1 - S_ideal)^{-1}]_cj| / |Z_p,cc|."""
    c = mom.center_element(lat) if center is None else center
    j = nearest_border(lat, c)
    Zi = mom.z_from_s(ideal_s(lat, s, s_cc, s_1, decay), z0)
    return abs(Zi[c, j]) / abs(zp_cc)


def center_couplings(S: np.ndarray, lat, center=None):
    """(S_cc, S_1): the center element's reflection and its coupling to the +x
    neighbour, the two numbers S_ideal is built from."""
    c = mom.center_element(lat) if center is None else center
    return S[c, c], S[c, c + 1]
