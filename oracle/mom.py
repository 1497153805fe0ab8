"""Oracle: plain CPU FP64 reference for the finite-array port quantities.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the GPU
path (no kernels, headers, tables or helpers); the only common module is the
seeded input description in ``paper_2608_17844_amd.workloads``.

What it computes is the plain definition of the solver's result, which the
Toeplitz/FFT/Krylov machinery reaches up to rounding and iteration tolerance:

* the dense impedance matrix Z from absolute positions (``fill.c``; the element
  is the thin-wire dipole of the benchmark workloads because the paper gives no
  fill formulas for its RWG elements);
* the all-port multi-RHS system Z I = V with one unit delta-gap excitation per
  port (Sec. II-D, eq. (eqProb), one feed per element, F = 1), solved by LAPACK
  LU (zgetrf/zgetrs);
* the port admittance from the port-basis currents, the open-circuit port
  impedance Z_p = Y_p^{-1} (eq. (passZ), read as the inverse of the
  short-circuit admittance that delta-gap excitation yields);
* the scattering matrix S from eq. (S2Z) solved for S;
* the active impedance of the center element (eqs. (actZ), (actZmat)) for
  phased port currents, its active reflection coefficient (eq. (ARC)) and the
  wave-excited variant built from the phased S-sum of Sec. II-E.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import scipy.linalg as sla

ETA0 = 376.730313668          # free-space wave impedance, ohm
HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "_fill.so")
_lib_handle = None


def build(force: bool = False) -> str:
    """Compile fill.c into _fill.so with gcc/OpenMP (plain -O2, no fast-math)."""
    src = os.path.join(HERE, "fill.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _lib_handle
    if _lib_handle is None:
        build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_fill_dense.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, dp]
        lib.oracle_fill_dense.restype = ctypes.c_int
        lib.oracle_fill_entries.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_int, i64p, i64p, ctypes.c_int64, dp]
        lib.oracle_fill_entries.restype = ctypes.c_int
        lib.oracle_gl4.argtypes = [dp, dp]
        lib.oracle_gl4.restype = None
        _lib_handle = lib
    return _lib_handle


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------- geometry

def gl4_rule():
    """The four-point Gauss-Legendre nodes/weights on [-1, 1] used by the fill."""
    x = np.zeros(4)
    w = np.zeros(4)
    _lib().oracle_gl4(_dptr(x), _dptr(w))
    return x, w


def wavenumber(s: float) -> float:
    """k = 2 pi s in units of 1/lambda0 (s = f/f0)."""
    return 2.0 * np.pi * s


def n_elements(lat) -> int:
    return lat.nx * lat.ny


def n_unknowns(lat, dip) -> int:
    return lat.nx * lat.ny * dip.nbases


def element_xy(lat) -> np.ndarray:
    """(P, 2) positions; element e = iy*nx + ix (x is the fastest lattice index)."""
    iy, ix = np.divmod(np.arange(lat.nx * lat.ny), lat.nx)
    return np.stack([ix * lat.dx, iy * lat.dy], axis=1)


def port_basis(dip) -> int:
    """The port is the center rooftop of each element (z = 0)."""
    return (dip.nbases - 1) // 2


def port_unknown(lat, dip, e) -> np.ndarray:
    return np.asarray(e) * dip.nbases + port_basis(dip)


def center_element(lat) -> int:
    """c = (floor(nx/2), floor(ny/2))."""
    return (lat.ny // 2) * lat.nx + lat.nx // 2


def _check(lat, dip, s):
    if dip.nbases < 1 or dip.nbases % 2 == 0:
        raise ValueError("nbases must be odd and >= 1")
    if lat.nx < 1 or lat.ny < 1 or dip.radius <= 0 or dip.length <= 0 or s <= 0:
        raise ValueError("invalid geometry or frequency")


# --------------------------------------------------------------------------- fill

def fill_dense(lat, dip, s: float, kernel_mode: int = 0, eta: float = ETA0) -> np.ndarray:
    """Dense Z (N x N complex128), every entry from absolute positions."""
    _check(lat, dip, s)
    N = n_unknowns(lat, dip)
    Z = np.empty((N, N), dtype=np.complex128)
    rc = _lib().oracle_fill_dense(lat.nx, lat.ny, lat.dx, lat.dy, dip.length, dip.radius, dip.nbases,
                                  wavenumber(s), eta, kernel_mode, _dptr(Z.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle_fill_dense failed (%d)" % rc)
    return Z


def fill_entries(lat, dip, s: float, rows, cols, kernel_mode: int = 0, eta: float = ETA0) -> np.ndarray:
    """Selected entries Z[rows[i], cols[i]] of the same dense matrix."""
    _check(lat, dip, s)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.shape, dtype=np.complex128)
    rc = _lib().oracle_fill_entries(lat.nx, lat.ny, lat.dx, lat.dy, dip.length, dip.radius, dip.nbases,
                                    wavenumber(s), eta, kernel_mode,
                                    rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    rows.size, _dptr(out.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle_fill_entries failed (%d)" % rc)
    return out


def block(Z: np.ndarray, lat, dip, e_row: int, e_col: int) -> np.ndarray:
    """The M x M interaction block between elements e_row (test) and e_col (source)."""
    M = dip.nbases
    return Z[e_row * M:(e_row + 1) * M, e_col * M:(e_col + 1) * M]


# --------------------------------------------------------------------------- excitation and solve

def excitation(lat, dip, ports: Optional[Sequence[int]] = None) -> np.ndarray:
    """Unit delta-gap at the port basis of each listed element: V[:, j] = e_{n(port j)}."""
    P = n_elements(lat)
    ports = np.arange(P) if ports is None else np.asarray(ports)
    V = np.zeros((n_unknowns(lat, dip), len(ports)), dtype=np.complex128)
    V[port_unknown(lat, dip, ports), np.arange(len(ports))] = 1.0
    return V


def solve_lu(Z: np.ndarray, V: np.ndarray, overwrite: bool = False) -> np.ndarray:
    """I = Z^{-1} V by LAPACK LU with partial pivoting."""
    lu, piv = sla.lu_factor(Z, overwrite_a=overwrite, check_finite=False)
    return sla.lu_solve((lu, piv), V, check_finite=False)


# --------------------------------------------------------------------------- port quantities

def port_admittance(I: np.ndarray, lat, dip) -> np.ndarray:
    """Y_p[i, j] = current at port i for a unit voltage at port j (others shorted)."""
    return I[port_unknown(lat, dip, np.arange(n_elements(lat))), :]


def port_impedance(Yp: np.ndarray) -> np.ndarray:
    """Open-circuit port impedance Z_p = Y_p^{-1}."""
    return sla.inv(Yp)


def s_matrix(Zp: np.ndarray, z0: float = 50.0) -> np.ndarray:
    """S from eq. (S2Z) solved for S: S = (Z_p - z0 I)(Z_p + z0 I)^{-1}."""
    n = Zp.shape[0]
    E = np.eye(n)
    # X (Zp + z0) = (Zp - z0)  <=>  (Zp + z0)^T X^T = (Zp - z0)^T
    return sla.solve((Zp + z0 * E).T, (Zp - z0 * E).T).T


def z_from_s(S: np.ndarray, z0: float = 50.0) -> np.ndarray:
    """Eq. (S2Z): Z_p = z0 (I + S)(I - S)^{-1}."""
    n = S.shape[0]
    E = np.eye(n)
    return z0 * sla.solve((E - S).T, (E + S).T).T


def scan_phases(lat, s: float, theta, phi) -> np.ndarray:
    """Progressive port phases that point the main beam at (theta, phi) (Sec. II-E:
    the scan angle is the direction the excitation steers the beam to).

    The fill's kernel is e^{-jkR}/(4 pi R) (time factor e^{+j omega t}); far from
    the array a source at rho_e then contributes with phase exp(+j k rhat.rho_e),
    so the contributions add in phase at rhat(theta, phi) when
    I_e = exp(-j k (x_e u + y_e v)), u = sin(th)cos(ph), v = sin(th)sin(ph).
    The paper's printed exp(+j n psi) is the same excitation written with the
    opposite time factor.  Shape (P, nscan)."""
    k = wavenumber(s)
    xy = element_xy(lat)
    u = np.sin(theta) * np.cos(phi)
    v = np.sin(theta) * np.sin(phi)
    return np.exp(-1j * k * (np.outer(xy[:, 0], u) + np.outer(xy[:, 1], v)))


def active_impedance(Zp: np.ndarray, lat, s: float, theta, phi, center: Optional[int] = None) -> np.ndarray:
    """Eq. (actZ) at the center element: Z_a,c = (1/I_c) sum_j Z_p,cj I_j."""
    c = center_element(lat) if center is None else center
    Ip = scan_phases(lat, s, np.atleast_1d(theta), np.atleast_1d(phi))
    return (Zp[c, :] @ Ip) / Ip[c, :]


def arc(Za: np.ndarray, z0: float = 50.0) -> np.ndarray:
    """Eq. (ARC): Gamma = (Z_a - z0)/(Z_a + z0)."""
    return (Za - z0) / (Za + z0)


def wave_arc(S: np.ndarray, lat, s: float, theta, phi, center: Optional[int] = None) -> np.ndarray:
    """Phased S-sum of Sec. II-E: Gamma_wave,c = sum_e S_ce a_e / a_c with incident
    waves a_e carrying the same progressive phases as the port currents."""
    c = center_element(lat) if center is None else center
    a = scan_phases(lat, s, np.atleast_1d(theta), np.atleast_1d(phi))
    return (S[c, :] @ a) / a[c, :]


# --------------------------------------------------------------------------- end to end

@dataclass
class OracleResult:
    Zp: np.ndarray
    Yp: np.ndarray
    S: np.ndarray
    Za: np.ndarray
    Gamma: np.ndarray
    Gamma_wave: np.ndarray
    times: dict


def solve_array(lat, dip, s: float, theta=(), phi=(), z0: float = 50.0, keep_Z: bool = False):
    """Dense fill -> LU -> Y_p -> Z_p -> S -> scan quantities, with phase timings."""
    t0 = time.perf_counter()
    Z = fill_dense(lat, dip, s)
    t1 = time.perf_counter()
    lu, piv = sla.lu_factor(Z, overwrite_a=not keep_Z, check_finite=False)
    t2 = time.perf_counter()
    I = sla.lu_solve((lu, piv), excitation(lat, dip), check_finite=False)
    t3 = time.perf_counter()
    Yp = port_admittance(I, lat, dip)
    Zp = port_impedance(Yp)
    S = s_matrix(Zp, z0)
    th = np.asarray(theta, dtype=float)
    ph = np.asarray(phi, dtype=float)
    Za = active_impedance(Zp, lat, s, th, ph) if th.size else np.zeros(0, complex)
    G = arc(Za, z0)
    Gw = wave_arc(S, lat, s, th, ph) if th.size else np.zeros(0, complex)
    t4 = time.perf_counter()
    res = OracleResult(Zp, Yp, S, Za, G, Gw, {"fill": t1 - t0, "lu": t2 - t1, "solve": t3 - t2, "extract": t4 - t3})
    if keep_Z:
        res.Z = Z
    return res
