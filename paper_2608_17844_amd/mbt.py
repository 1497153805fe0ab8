"""Thin Python binding of the C ABI in include/mbt.h (argument marshalling only).

Every function here converts numpy arrays / torch tensors to the pointers and
sizes of the C entry point of the same name and checks the returned status.
All arithmetic runs in the HIP library ``libmbt.so`` built in this directory;
if it is missing, loading fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbt.so")

MBT_OK, MBT_EINVAL, MBT_ENOMEM, MBT_ENOCONV, MBT_EDEVICE, MBT_EBUSY, MBT_EBREAKDOWN, MBT_ETIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7
MBT_FP64, MBT_FP32, MBT_BF16, MBT_FP16 = 0, 1, 2, 3
MBT_PC_NORMAL_EQ, MBT_PC_ELEMENT_BLOCK = 0, 1
MBT_FLAG_NO_CACHE = 1
MBT_FLAG_CGS2 = 2
MBT_FLAG_FP32_BASIS = 4
MBT_FLAG_PCG = 8
MBT_FLAG_COCG = 16
STATUS_NAMES = {0: "MBT_OK", -1: "MBT_EINVAL", -2: "MBT_ENOMEM", -3: "MBT_ENOCONV", -4: "MBT_EDEVICE",
                -5: "MBT_EBUSY", -6: "MBT_EBREAKDOWN", -7: "MBT_ETIMEOUT"}


class mbt_dipole(ctypes.Structure):
    _fields_ = [("length", ctypes.c_double), ("radius", ctypes.c_double), ("nbases", ctypes.c_int32)]


class mbt_lattice(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double)]


class mbt_solve_opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("pc", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("tol", ctypes.c_double), ("max_cycles", ctypes.c_int32), ("refine_max", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("rhs_chunk", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class mbt_stats(ctypes.Structure):
    _fields_ = [("nrhs", ctypes.c_int32), ("nconverged", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("outer_steps", ctypes.c_int32), ("iters_min", ctypes.c_int32), ("iters_max", ctypes.c_int32),
                ("iters_total", ctypes.c_int64), ("matvecs", ctypes.c_int64), ("true_relres_max", ctypes.c_double),
                ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double), ("t_extract", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class mbt_predictors(ctypes.Structure):
    _fields_ = [("xi_z", ctypes.c_double), ("xi_z_max", ctypes.c_double), ("border_sum", ctypes.c_double),
                ("nearest", ctypes.c_int32), ("center", ctypes.c_int32), ("s_cc", ctypes.c_double * 2),
                ("s_1", ctypes.c_double * 2)]


class mbt_rwg_mesh(ctypes.Structure):
    _fields_ = [("nvert", ctypes.c_int32), ("vert", ctypes.POINTER(ctypes.c_double)), ("ntri", ctypes.c_int32),
                ("tri", ctypes.POINTER(ctypes.c_int32)), ("nport_edges", ctypes.c_int32),
                ("port_edges", ctypes.POINTER(ctypes.c_int32)), ("port_dir", ctypes.c_double * 2)]


class mbt_request(ctypes.Structure):
    _fields_ = [("elem", mbt_dipole), ("lat", mbt_lattice), ("nfreq", ctypes.c_int32),
                ("freq_ratio", ctypes.POINTER(ctypes.c_double)), ("nscan", ctypes.c_int32),
                ("theta", ctypes.POINTER(ctypes.c_double)), ("phi", ctypes.POINTER(ctypes.c_double)),
                ("z0", ctypes.c_double), ("opts", mbt_solve_opts)]


class mbt_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nfreq", ctypes.c_int32), ("nports", ctypes.c_int32),
                ("nscan", ctypes.c_int32), ("Zp", ctypes.POINTER(ctypes.c_double)),
                ("Za", ctypes.POINTER(ctypes.c_double)), ("Gamma", ctypes.POINTER(ctypes.c_double)),
                ("Gamma_wave", ctypes.POINTER(ctypes.c_double)), ("iters_max", ctypes.POINTER(ctypes.c_int32)),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class MbtError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Load libmbt.so (raises if the HIP library was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmbt.so is not built; run paper_2608_17844_amd/build.py (hipcc, gfx950)")
        # torch provides device memory and streams to callers of the *_dev entry
        # points; loading it first makes the library bind to the same HIP runtime
        # instance, so pointers and streams are valid on both sides.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        S = ctypes.c_int32
        sig = {
            "mbt_default_opts": (None, [ctypes.POINTER(mbt_solve_opts)]),
            "mbt_ctx_create": (S, [ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(_vp)]),
            "mbt_ctx_destroy": (None, [_vp]),
            "mbt_last_error": (ctypes.c_char_p, []),
            "mbt_version": (ctypes.c_char_p, []),
            "mbt_array_create_dipole": (S, [_vp, ctypes.POINTER(mbt_dipole), ctypes.POINTER(mbt_lattice),
                                            ctypes.POINTER(_vp)]),
            "mbt_array_create_blocks": (S, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dp,
                                            ctypes.POINTER(_vp)]),
            "mbt_array_create_margin": (S, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dp, ctypes.c_int32,
                                            _dp, _dp, ctypes.POINTER(_vp)]),
            "mbt_array_create_rwg": (S, [_vp, ctypes.POINTER(mbt_rwg_mesh), ctypes.POINTER(mbt_lattice),
                                         ctypes.POINTER(_vp)]),
            "mbt_scan_solve": (S, [_vp, _vp, ctypes.c_double, ctypes.POINTER(mbt_solve_opts), _dp, _dp, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_int32, _dp, _dp, _dp, _ip, ctypes.POINTER(mbt_stats)]),
            "mbt_array_destroy": (None, [_vp]),
            "mbt_array_info": (S, [_vp, ctypes.POINTER(ctypes.c_int64), _ip, _ip, _ip]),
            "mbt_footprint": (ctypes.c_size_t, [_vp, ctypes.c_int32, ctypes.POINTER(mbt_solve_opts)]),
            "mbt_port_admittance": (S, [_vp, _vp, ctypes.c_double, _ip, ctypes.c_int32,
                                        ctypes.POINTER(mbt_solve_opts), _dp, _ip, ctypes.POINTER(mbt_stats)]),
            "mbt_port_admittance_dev": (S, [_vp, _vp, ctypes.c_double, _ip, ctypes.c_int32,
                                            ctypes.POINTER(mbt_solve_opts), _vp, _vp, _ip,
                                            ctypes.POINTER(mbt_stats)]),
            "mbt_port_impedance": (S, [_vp, _vp, ctypes.c_double, ctypes.POINTER(mbt_solve_opts), _dp,
                                       ctypes.POINTER(mbt_stats)]),
            "mbt_solve": (S, [_vp, _vp, ctypes.c_double, ctypes.POINTER(mbt_solve_opts), _dp, _dp, ctypes.c_int32,
                              ctypes.c_double, _dp, _dp, _dp, _dp, ctypes.POINTER(mbt_stats)]),
            "mbt_active": (S, [_vp, _vp, ctypes.c_double, _dp, ctypes.c_int32, _dp, _dp, ctypes.c_int32,
                               ctypes.c_double, _dp, _dp, _dp]),
            "mbt_server_create": (S, [_vp, ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(_vp)]),
            "mbt_server_submit": (S, [_vp, ctypes.POINTER(mbt_request), ctypes.POINTER(ctypes.c_uint64)]),
            "mbt_server_wait": (S, [_vp, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(ctypes.POINTER(mbt_result))]),
            "mbt_result_free": (None, [ctypes.POINTER(mbt_result)]),
            "mbt_server_clock": (ctypes.c_double, [_vp]),
            "mbt_server_destroy": (None, [_vp]),
            "mbt_dbg_fill_blocks": (S, [_vp, _vp, ctypes.c_double, _dp]),
            "mbt_dbg_matvec": (S, [_vp, _vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _dp, ctypes.c_int32,
                                   _dp]),
            "mbt_dbg_precond_apply": (S, [_vp, _vp, ctypes.c_double, ctypes.c_int32, _dp, ctypes.c_int32, _dp]),
            "mbt_dbg_precond_blocks": (S, [_vp, _vp, ctypes.c_double, ctypes.c_int32, _dp]),
            "mbt_dbg_solve": (S, [_vp, _vp, ctypes.c_double, ctypes.POINTER(mbt_solve_opts), _dp, ctypes.c_int32,
                                  _dp, _ip, ctypes.POINTER(mbt_stats)]),
            "mbt_dbg_inverse": (S, [_vp, _dp, ctypes.c_int32, _dp]),
            "mbt_active_dev_noalloc": (S, [_vp, _vp, ctypes.c_double, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32,
                                           ctypes.c_double, _vp, _vp, _vp, _vp]),
            "mbt_predict": (S, [_vp, ctypes.POINTER(mbt_lattice), _dp, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_int32, ctypes.POINTER(mbt_predictors), _dp, _dp]),
            "mbt_predict_xi_s": (S, [_vp, ctypes.POINTER(mbt_lattice), ctypes.c_double, _dp, _dp, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int32, _dp]),
            "mbt_prof_start": (S, [ctypes.c_int32]),
            "mbt_prof_read": (S, [_dp, ctypes.POINTER(ctypes.c_int64), _dp, _dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> list:
    """Names of every C entry point this binding declares (all must exist in the library)."""
    return [
        "mbt_default_opts", "mbt_ctx_create", "mbt_ctx_destroy", "mbt_last_error", "mbt_version",
        "mbt_array_create_dipole", "mbt_array_create_blocks", "mbt_array_destroy", "mbt_array_info", "mbt_footprint",
        "mbt_port_admittance", "mbt_port_admittance_dev", "mbt_port_impedance", "mbt_solve", "mbt_active",
        "mbt_server_create", "mbt_server_submit", "mbt_server_wait", "mbt_result_free", "mbt_server_clock",
        "mbt_server_destroy", "mbt_dbg_fill_blocks", "mbt_dbg_matvec", "mbt_dbg_precond_apply",
        "mbt_dbg_precond_blocks", "mbt_dbg_solve", "mbt_dbg_inverse", "mbt_prof_start", "mbt_prof_read",
        "mbt_predict", "mbt_predict_xi_s", "mbt_active_dev_noalloc", "mbt_array_create_margin",
        "mbt_array_create_rwg", "mbt_scan_solve",
    ]


def _check(status: int, allow=(MBT_OK,)):
    if status not in allow:
        raise MbtError(status, lib().mbt_last_error().decode())
    return status


def _cd(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _ci(a: np.ndarray):
    return a.ctypes.data_as(_ip)


# ------------------------------------------------------------------ options

def mbt_default_opts(**overrides) -> mbt_solve_opts:
    o = mbt_solve_opts()
    lib().mbt_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------ handles

def mbt_ctx_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = _vp()
    _check(lib().mbt_ctx_create(device, hbm_budget_bytes, ctypes.byref(h)))
    return h.value


def mbt_ctx_destroy(ctx: int) -> None:
    lib().mbt_ctx_destroy(ctx)


def mbt_array_create_dipole(ctx: int, dipole, lattice) -> int:
    d = mbt_dipole(dipole.length, dipole.radius, dipole.nbases)
    l = mbt_lattice(lattice.nx, lattice.ny, lattice.dx, lattice.dy)
    h = _vp()
    _check(lib().mbt_array_create_dipole(ctx, ctypes.byref(d), ctypes.byref(l), ctypes.byref(h)))
    return h.value


def mbt_array_create_blocks(ctx: int, T: np.ndarray) -> int:
    """T of shape (2ny-1, 2nx-1, M, M), complex: the unique lattice blocks."""
    T = np.ascontiguousarray(T, dtype=np.complex128)
    ny, nx = (T.shape[0] + 1) // 2, (T.shape[1] + 1) // 2
    h = _vp()
    _check(lib().mbt_array_create_blocks(ctx, nx, ny, T.shape[2], T.ctypes.data_as(_dp), ctypes.byref(h)))
    return h.value


def mbt_array_create_margin(ctx: int, T: np.ndarray, ZB: np.ndarray, ZC: np.ndarray) -> int:
    """Partitioned array: unique blocks T (2ny-1, 2nx-1, M, M), margin coupling ZB
    (nc x nx*ny*M) and margin block ZC (nc x nc), complex."""
    T = np.ascontiguousarray(T, dtype=np.complex128)
    ny2, nx2, M, _ = T.shape
    ZB = np.ascontiguousarray(ZB, dtype=np.complex128)
    ZC = np.ascontiguousarray(ZC, dtype=np.complex128)
    out = _vp()
    _check(lib().mbt_array_create_margin(ctx, (nx2 + 1) // 2, (ny2 + 1) // 2, M, _cd(T), ZC.shape[0], _cd(ZB), _cd(ZC),
                                         ctypes.byref(out)))
    return out.value


def mbt_array_create_rwg(ctx: int, mesh, lattice) -> int:
    """Array of planar RWG elements; mesh has vertices (nv, 2), triangles (nt, 3),
    port_edges (ne, 2) and port_dir (2,)."""
    v = np.ascontiguousarray(mesh.vertices, dtype=np.float64)
    t = np.ascontiguousarray(mesh.triangles, dtype=np.int32)
    e = np.ascontiguousarray(mesh.port_edges, dtype=np.int32)
    m = mbt_rwg_mesh(v.shape[0], _cd(v), t.shape[0], _ci(t), e.shape[0], _ci(e),
                     (ctypes.c_double * 2)(*[float(x) for x in mesh.port_dir]))
    l = mbt_lattice(lattice.nx, lattice.ny, lattice.dx, lattice.dy)
    h = _vp()
    _check(lib().mbt_array_create_rwg(ctx, ctypes.byref(m), ctypes.byref(l), ctypes.byref(h)))
    return h.value


def mbt_array_destroy(arr: int) -> None:
    lib().mbt_array_destroy(arr)


def mbt_array_info(arr: int) -> dict:
    N = ctypes.c_int64()
    P, gx, gy = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mbt_array_info(arr, ctypes.byref(N), ctypes.byref(P), ctypes.byref(gx), ctypes.byref(gy)))
    return {"N": N.value, "P": P.value, "gx": gx.value, "gy": gy.value}


def mbt_footprint(arr: int, nrhs: int, opts: mbt_solve_opts) -> int:
    return int(lib().mbt_footprint(arr, nrhs, ctypes.byref(opts)))


# ------------------------------------------------------------------ solves

def mbt_port_admittance(ctx: int, arr: int, freq_ratio: float, ports: Optional[Sequence[int]],
                        opts: mbt_solve_opts, allow_noconv: bool = False):
    info = mbt_array_info(arr)
    P = info["P"]
    if ports is None:
        pl, n, pp = None, -1, None
        ncol = P
    else:
        pl = np.ascontiguousarray(ports, dtype=np.int32)
        n, pp, ncol = len(pl), _ci(pl), len(pl)
    Y = np.zeros((P, ncol), dtype=np.complex128, order="F")
    iters = np.zeros(ncol, dtype=np.int32)
    st = mbt_stats()
    allow = (MBT_OK, MBT_ENOCONV) if allow_noconv else (MBT_OK,)
    _check(lib().mbt_port_admittance(ctx, arr, freq_ratio, pp, n, ctypes.byref(opts), _cd(Y),
                                     _ci(iters), ctypes.byref(st)), allow)
    return Y, iters, st.as_dict()


def mbt_port_admittance_dev(ctx: int, arr: int, freq_ratio: float, ports: Optional[Sequence[int]],
                            opts: mbt_solve_opts, Y_dev_ptr: int, stream_ptr: int = 0):
    if ports is None:
        pp, n, ncol = None, -1, mbt_array_info(arr)["P"]
        pl = None
    else:
        pl = np.ascontiguousarray(ports, dtype=np.int32)
        pp, n, ncol = _ci(pl), len(pl), len(pl)
    iters = np.zeros(ncol, dtype=np.int32)
    st = mbt_stats()
    _check(lib().mbt_port_admittance_dev(ctx, arr, freq_ratio, pp, n, ctypes.byref(opts), Y_dev_ptr,
                                         stream_ptr or None, _ci(iters), ctypes.byref(st)))
    return iters, st.as_dict()


def mbt_port_impedance(ctx: int, arr: int, freq_ratio: float, opts: mbt_solve_opts):
    P = mbt_array_info(arr)["P"]
    Zp = np.zeros((P, P), dtype=np.complex128, order="F")
    st = mbt_stats()
    _check(lib().mbt_port_impedance(ctx, arr, freq_ratio, ctypes.byref(opts), _cd(Zp),
                                    ctypes.byref(st)))
    return Zp, st.as_dict()


def mbt_solve(ctx: int, arr: int, freq_ratio: float, opts: mbt_solve_opts, theta, phi, z0: float = 50.0,
              want_zp: bool = True, allow_noconv: bool = False):
    P = mbt_array_info(arr)["P"]
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    ns = th.size
    Zp = np.zeros((P, P), dtype=np.complex128, order="F") if want_zp else None
    Za = np.zeros(max(ns, 1), dtype=np.complex128)
    G = np.zeros(max(ns, 1), dtype=np.complex128)
    Gw = np.zeros(max(ns, 1), dtype=np.complex128)
    st = mbt_stats()
    allow = (MBT_OK, MBT_ENOCONV) if allow_noconv else (MBT_OK,)
    status = _check(lib().mbt_solve(ctx, arr, freq_ratio, ctypes.byref(opts), _cd(th) if ns else None,
                                    _cd(ph) if ns else None, ns, z0,
                                    _cd(Zp) if want_zp else None,
                                    _cd(Za), _cd(G), _cd(Gw),
                                    ctypes.byref(st)), allow)
    return {"Zp": Zp, "Za": Za[:ns], "Gamma": G[:ns], "Gamma_wave": Gw[:ns], "stats": st.as_dict(),
            "status": status}


def mbt_scan_solve(ctx: int, arr: int, freq_ratio: float, opts: mbt_solve_opts, theta, phi, z0: float = 50.0,
                   center: int = -1, want_ip: bool = True, allow_noconv: bool = False):
    """Phased voltage excitation of every gap per scan direction: gap currents Ip
    (P x nscan), the center element's active impedance and ARC."""
    P = mbt_array_info(arr)["P"]
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    ns = th.size
    Ip = np.zeros((P, ns), dtype=np.complex128, order="F") if want_ip else None
    Za = np.zeros(ns, dtype=np.complex128)
    G = np.zeros(ns, dtype=np.complex128)
    it = np.zeros(ns, dtype=np.int32)
    st = mbt_stats()
    allow = (MBT_OK, MBT_ENOCONV) if allow_noconv else (MBT_OK,)
    status = _check(lib().mbt_scan_solve(ctx, arr, freq_ratio, ctypes.byref(opts), _cd(th), _cd(ph), ns, z0, center,
                                         _cd(Ip) if want_ip else None, _cd(Za), _cd(G), _ci(it),
                                         ctypes.byref(st)), allow)
    return {"Ip": Ip, "Za": Za, "Gamma": G, "iters": it, "stats": st.as_dict(), "status": status}


def mbt_active_dev_noalloc(ctx: int, arr: int, freq_ratio: float, Zp_ptr: int, theta_ptr: int, phi_ptr: int,
                           nscan: int, z0: float, Za_ptr: int, Gamma_ptr: int, Gamma_wave_ptr: Optional[int],
                           stream: Optional[int] = None, center: int = -1) -> None:
    """mbt_active on caller-owned device buffers (integer device addresses, e.g.
    torch tensors' data_ptr()) with no device allocation."""
    _check(lib().mbt_active_dev_noalloc(ctx, arr, freq_ratio, Zp_ptr, center, theta_ptr, phi_ptr, nscan, z0, Za_ptr,
                                        Gamma_ptr, Gamma_wave_ptr, stream))


def _lat(lattice) -> mbt_lattice:
    return mbt_lattice(lattice.nx, lattice.ny, lattice.dx, lattice.dy)


def mbt_predict(ctx: int, lattice, Zp: np.ndarray, z0: float = 50.0, nq: int = 0, center: int = -1) -> dict:
    """Coupling predictors of Sec. II-E from Z_p; nq = 0 picks 2 nx nodes."""
    Zf = np.asfortranarray(Zp, dtype=np.complex128)
    nq = nq if nq > 0 else 2 * lattice.nx
    out = mbt_predictors()
    Cn = np.zeros(lattice.nx, dtype=np.complex128)
    G = np.zeros(nq, dtype=np.complex128)
    lat = _lat(lattice)
    _check(lib().mbt_predict(ctx, ctypes.byref(lat), _cd(Zf), center, z0, nq, ctypes.byref(out), _cd(Cn), _cd(G)))
    c = out.center
    ixc = c % lattice.nx
    return {"xi_z": out.xi_z, "xi_z_max": out.xi_z_max, "border_sum": out.border_sum, "nearest": out.nearest,
            "center": c, "s_cc": complex(out.s_cc[0], out.s_cc[1]), "s_1": complex(out.s_1[0], out.s_1[1]),
            "n": np.arange(-ixc, lattice.nx - ixc), "Cn": Cn, "Gamma_psi": G,
            "psi": -np.pi + 2 * np.pi * np.arange(nq) / nq}


def mbt_predict_xi_s(ctx: int, lattice, freq_ratio: float, s_cc: complex, s_1: complex, zp_cc_abs: float,
                     z0: float = 50.0, decay: float = -2.0, center: int = -1) -> float:
    a = np.array([s_cc.real, s_cc.imag])
    b = np.array([s_1.real, s_1.imag])
    out = np.zeros(1)
    lat = _lat(lattice)
    _check(lib().mbt_predict_xi_s(ctx, ctypes.byref(lat), freq_ratio, _cd(a), _cd(b), zp_cc_abs, z0, decay, center,
                                  _cd(out)))
    return float(out[0])


def mbt_active(ctx: int, arr: int, freq_ratio: float, Zp: np.ndarray, theta, phi, z0: float = 50.0,
               center: int = -1):
    Zf = np.asfortranarray(Zp, dtype=np.complex128)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    ns = th.size
    Za = np.zeros(ns, dtype=np.complex128)
    G = np.zeros(ns, dtype=np.complex128)
    Gw = np.zeros(ns, dtype=np.complex128)
    _check(lib().mbt_active(ctx, arr, freq_ratio, _cd(Zf), center, _cd(th), _cd(ph), ns, z0,
                            _cd(Za), _cd(G), _cd(Gw)))
    return Za, G, Gw


# ------------------------------------------------------------------ serving

def mbt_server_create(ctx: int, max_inflight: int = 4, hbm_budget_bytes: int = 0) -> int:
    h = _vp()
    _check(lib().mbt_server_create(ctx, max_inflight, hbm_budget_bytes, ctypes.byref(h)))
    return h.value


def mbt_server_submit(srv: int, dipole, lattice, freq_ratio, theta, phi, opts: mbt_solve_opts,
                      z0: float = 50.0) -> int:
    f = np.ascontiguousarray(np.atleast_1d(freq_ratio), dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    d = mbt_dipole(*dipole) if not isinstance(dipole, mbt_dipole) else dipole
    la = mbt_lattice(*lattice) if not isinstance(lattice, mbt_lattice) else lattice
    req = mbt_request(elem=d, lat=la, nfreq=f.size, freq_ratio=_cd(f), nscan=th.size,
                      theta=_cd(th) if th.size else None, phi=_cd(ph) if th.size else None, z0=z0, opts=opts)
    t = ctypes.c_uint64()
    _check(lib().mbt_server_submit(srv, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def mbt_server_wait(srv: int, ticket: int, timeout_ms: int = -1) -> Optional[dict]:
    """Result of `ticket` as numpy copies (None on MBT_ETIMEOUT); the library result is freed."""
    rp = ctypes.POINTER(mbt_result)()
    st = _check(lib().mbt_server_wait(srv, ticket, timeout_ms, ctypes.byref(rp)), (MBT_OK, MBT_ETIMEOUT))
    if st == MBT_ETIMEOUT:
        return None
    try:
        r = rp.contents
        nf, P, ns = r.nfreq, r.nports, r.nscan

        def cplx(ptr, n):
            return np.ctypeslib.as_array(ptr, shape=(2 * n,)).copy().view(np.complex128)

        out = {"status": r.status, "nfreq": nf, "nports": P, "nscan": ns,
               "Zp": cplx(r.Zp, nf * P * P).reshape(nf, P, P).transpose(0, 2, 1),
               "Za": cplx(r.Za, nf * ns).reshape(nf, ns) if ns else np.zeros((nf, 0), np.complex128),
               "Gamma": cplx(r.Gamma, nf * ns).reshape(nf, ns) if ns else np.zeros((nf, 0), np.complex128),
               "Gamma_wave": cplx(r.Gamma_wave, nf * ns).reshape(nf, ns) if ns else np.zeros((nf, 0), np.complex128),
               "iters_max": np.ctypeslib.as_array(r.iters_max, shape=(nf,)).copy(),
               "t_submit": r.t_submit, "t_start": r.t_start, "t_done": r.t_done}
    finally:
        lib().mbt_result_free(rp)
    return out


def mbt_server_clock(srv: int) -> float:
    return lib().mbt_server_clock(srv)


def mbt_server_destroy(srv: int) -> None:
    lib().mbt_server_destroy(srv)


# ------------------------------------------------------------------ test hooks

def mbt_dbg_fill_blocks(ctx: int, arr: int, freq_ratio: float, lattice, nbases: int) -> np.ndarray:
    noff = (2 * lattice.nx - 1) * (2 * lattice.ny - 1)
    T = np.zeros((noff, nbases, nbases), dtype=np.complex128)
    _check(lib().mbt_dbg_fill_blocks(ctx, arr, freq_ratio, _cd(T)))
    return T.reshape(2 * lattice.ny - 1, 2 * lattice.nx - 1, nbases, nbases)


def mbt_dbg_matvec(ctx: int, arr: int, freq_ratio: float, x: np.ndarray, op: int = 0, prec: int = MBT_FP64):
    xf = np.asfortranarray(x.reshape(x.shape[0], -1), dtype=np.complex128)
    y = np.zeros_like(xf, order="F")
    _check(lib().mbt_dbg_matvec(ctx, arr, freq_ratio, prec, op, _cd(xf), xf.shape[1],
                                _cd(y)))
    return y.reshape(x.shape)


def mbt_dbg_precond_apply(ctx: int, arr: int, freq_ratio: float, x: np.ndarray, pc: int):
    xf = np.asfortranarray(x.reshape(x.shape[0], -1), dtype=np.complex128)
    y = np.zeros_like(xf, order="F")
    _check(lib().mbt_dbg_precond_apply(ctx, arr, freq_ratio, pc, _cd(xf), xf.shape[1],
                                       _cd(y)))
    return y.reshape(x.shape)


def mbt_dbg_precond_blocks(ctx: int, arr: int, freq_ratio: float, pc: int, nblocks: int, nbases: int):
    nb = 1 if pc == MBT_PC_ELEMENT_BLOCK else nblocks
    Pb = np.zeros((nb, nbases, nbases), dtype=np.complex128)
    _check(lib().mbt_dbg_precond_blocks(ctx, arr, freq_ratio, pc, _cd(Pb)))
    return Pb


def mbt_dbg_solve(ctx: int, arr: int, freq_ratio: float, opts: mbt_solve_opts, V: np.ndarray,
                  allow_noconv: bool = False, allow_breakdown: bool = False):
    Vf = np.asfortranarray(V, dtype=np.complex128)
    I = np.zeros_like(Vf, order="F")
    iters = np.zeros(Vf.shape[1], dtype=np.int32)
    st = mbt_stats()
    allow = (MBT_OK, MBT_ENOCONV) if allow_noconv else (MBT_OK,)
    if allow_breakdown:
        allow = allow + (MBT_EBREAKDOWN,)
    status = _check(lib().mbt_dbg_solve(ctx, arr, freq_ratio, ctypes.byref(opts), _cd(Vf), Vf.shape[1],
                                        _cd(I), _ci(iters), ctypes.byref(st)), allow)
    out = st.as_dict()
    out["status"] = status
    return I, iters, out


def mbt_dbg_inverse(ctx: int, A: np.ndarray) -> np.ndarray:
    Af = np.asfortranarray(A, dtype=np.complex128)
    out = np.zeros_like(Af, order="F")
    _check(lib().mbt_dbg_inverse(ctx, _cd(Af), Af.shape[0], _cd(out)))
    return out


# ------------------------------------------------------------------ kernel timing

MBT_K_NONE, MBT_K_ARNOLDI_DOTS, MBT_K_ARNOLDI_UPDATE_DOTS, MBT_K_ARNOLDI_UPDATE_NORM = 0, 1, 2, 3
MBT_K_FFT_FWD, MBT_K_FFT_INV, MBT_K_BIN_PRODUCT, MBT_K_PRECOND_APPLY = 4, 5, 6, 7
KERNEL_NAMES = {1: "arnoldi_dots", 2: "arnoldi_update_dots", 3: "arnoldi_update_norm", 4: "fft_fwd_pad",
                5: "fft_inv_crop", 6: "bin_product", 7: "precond_apply"}


def mbt_prof_start(kernel: int) -> None:
    _check(lib().mbt_prof_start(kernel))


def mbt_prof_read() -> dict:
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    by = ctypes.c_double()
    fl = ctypes.c_double()
    _check(lib().mbt_prof_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by), ctypes.byref(fl)))
    return {"ms": ms.value, "launches": n.value, "bytes": by.value, "flops": fl.value}
