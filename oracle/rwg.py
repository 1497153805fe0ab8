"""Oracle: RWG EFIE fill and port quantities of arrays of planar elements.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code with the GPU
path; the mesh it is given comes from the seeded input descriptions in
``paper_2608_17844_amd.workloads``.

The paper discretises its elements with Rao-Wilton-Glisson (RWG) functions
(Sec. I, Sec. II-B) but prints no fill formulas, quadrature or singularity
rules.  The reading written out here, from the definitions of the RWG basis
(Rao, Wilton and Glisson, IEEE TAP 1982) and of the Galerkin EFIE:

* basis: one function per interior edge of the element's triangle mesh (an edge
  of exactly two triangles), the edges taken in increasing (smaller vertex,
  larger vertex) order.  On the edge's two triangles T+ (the one with the
  smaller triangle index) and T-, f(r) = +-(l / 2A)(r - v) with v the vertex
  opposite the edge, so div f = +-l / A;
* entries, with G = exp(-jkR) / (4 pi R), k = 2 pi s in units of 1/lambda0:
  Z_mn = j k eta <<f_m . f_n, G>> - j (eta / k) <<div f_m, div f_n, G>>;
* quadrature: Radon's seven-point rule (degree 5) on every triangle, test and
  source.  For elements at most one lattice step apart in x and in y (the
  element itself and its eight neighbours) the source integral of the static
  part 1/(4 pi R) is taken in closed form at each test point (the coplanar
  potential integrals of Wilton et al., IEEE TAP 1984) and only the remainder
  (exp(-jkR) - 1) / (4 pi R) by the seven-point rule;
* port: a delta gap across the feed edges: a gap voltage V drives basis m with
  V sign_m l_m, and the gap current is sum_m sign_m l_m I_m, sign_m = +1 when
  the basis's T+ -> T- direction has a positive component along the gap field.

Port quantities then follow eqs. (eqProb), (passZ), (actZ) and (ARC) as in
``mom``; a scan excitation drives the port gaps with the phased voltages
V_e = exp(-j k (x_e u + y_e v)) and the active impedance of the center element
is its gap voltage over its gap current (eq. (actZ) with the port currents that
this excitation produces).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.linalg as sla

from . import mom

ETA0 = mom.ETA0


# --------------------------------------------------------------------------- quadrature

def rule7():
    """Radon's seven-point rule on a triangle, exact for polynomials of degree
    <= 5: barycentric points (7, 3) and weights (7,) summing to 1."""
    r = np.sqrt(15.0)
    a1, a2 = (6.0 - r) / 21.0, (6.0 + r) / 21.0
    w1, w2 = (155.0 - r) / 1200.0, (155.0 + r) / 1200.0
    pts = [(1 / 3, 1 / 3, 1 / 3)]
    wts = [9.0 / 40.0]
    for a, w in ((a1, w1), (a2, w2)):
        b = 1.0 - 2.0 * a
        pts += [(b, a, a), (a, b, a), (a, a, b)]
        wts += [w, w, w]
    return np.array(pts), np.array(wts)


def tri_points(xy: np.ndarray, bary: np.ndarray) -> np.ndarray:
    """Points of a rule on triangles xy (..., 3, 2): shape (..., npts, 2)."""
    return np.einsum("qk,...kd->...qd", bary, xy)


def tri_area(xy: np.ndarray) -> np.ndarray:
    d1 = xy[..., 1, :] - xy[..., 0, :]
    d2 = xy[..., 2, :] - xy[..., 0, :]
    return 0.5 * np.abs(d1[..., 0] * d2[..., 1] - d1[..., 1] * d2[..., 0])


# --------------------------------------------------------------------------- basis

@dataclass
class RwgElement:
    vert: np.ndarray      # (nv, 2)
    tri: np.ndarray       # (nt, 3)
    area: np.ndarray      # (nt,)
    edges: np.ndarray     # (M, 2) vertex pairs, smaller first
    length: np.ndarray    # (M,)
    tplus: np.ndarray     # (M,) triangle index of T+
    tminus: np.ndarray    # (M,)
    vplus: np.ndarray     # (M,) vertex of T+ opposite the edge
    vminus: np.ndarray    # (M,)
    port_bases: np.ndarray   # (np,)
    port_weights: np.ndarray  # (np,) sign_m * l_m

    @property
    def M(self) -> int:
        return len(self.length)


def rwg_element(mesh) -> RwgElement:
    """RWG bases of a planar mesh (see the module docstring for the rules)."""
    vert = np.asarray(mesh.vertices, dtype=np.float64)
    tri = np.asarray(mesh.triangles, dtype=np.int64)
    owners = {}
    for t, (a, b, c) in enumerate(tri):
        for p, q in ((a, b), (b, c), (c, a)):
            owners.setdefault((min(p, q), max(p, q)), []).append(t)
    if any(len(v) > 2 for v in owners.values()):
        raise ValueError("edge shared by more than two triangles")
    edges = sorted(e for e, ts in owners.items() if len(ts) == 2)
    M = len(edges)
    tplus = np.array([min(owners[e]) for e in edges], dtype=np.int64)
    tminus = np.array([max(owners[e]) for e in edges], dtype=np.int64)

    def opposite(t, e):
        (v,) = [v for v in tri[t] if v not in e]
        return v

    vplus = np.array([opposite(t, e) for t, e in zip(tplus, edges)], dtype=np.int64)
    vminus = np.array([opposite(t, e) for t, e in zip(tminus, edges)], dtype=np.int64)
    E = np.array(edges, dtype=np.int64).reshape(M, 2)
    length = np.linalg.norm(vert[E[:, 1]] - vert[E[:, 0]], axis=1)
    area = tri_area(vert[tri])
    cen = vert[tri].mean(axis=1)
    d = np.asarray(mesh.port_dir, dtype=np.float64)
    pb, pw = [], []
    index = {e: m for m, e in enumerate(edges)}
    for a, b in np.asarray(mesh.port_edges):
        m = index[(min(a, b), max(a, b))]
        proj = float((cen[tminus[m]] - cen[tplus[m]]) @ d)
        if proj == 0.0:
            raise ValueError("port edge parallel to the gap field")
        pb.append(m)
        pw.append(np.sign(proj) * length[m])
    return RwgElement(vert, tri, area, E, length, tplus, tminus, vplus, vminus, np.array(pb), np.array(pw))


def basis_value(el: RwgElement, m: int, tri_index: int, r: np.ndarray) -> np.ndarray:
    """f_m at points r (n, 2) of triangle tri_index (zero off its two triangles)."""
    if tri_index == el.tplus[m]:
        return el.length[m] / (2 * el.area[tri_index]) * (r - el.vert[el.vplus[m]])
    if tri_index == el.tminus[m]:
        return -el.length[m] / (2 * el.area[tri_index]) * (r - el.vert[el.vminus[m]])
    return np.zeros_like(r)


# --------------------------------------------------------------------------- static potentials

def static_potentials(xy: np.ndarray, rho: np.ndarray):
    """For triangles xy (n, 3, 2) (or one, (3, 2)) and points rho (q, 2) in their
    plane: S0 = int_T 1/|r' - rho| dS' (n, q) and S1 = int_T (r' - rho)/|r' - rho| dS'
    (n, q, 2), in closed form (Wilton et al. 1984, coplanar case):
      S0 = sum_i P_i ln((R+_i + l+_i)/(R-_i + l-_i)),
      S1 = 1/2 sum_i u_i [P_i^2 ln(...) + l+_i R+_i - l-_i R-_i],
    over the edges i with endpoints p-, p+, unit direction t_i, outward unit
    normal u_i, P_i = (p - rho).u_i, l+-_i = (p+- - rho).t_i, R+-_i = |p+- - rho|."""
    one = xy.ndim == 2
    xy = np.atleast_3d(xy) if not one else xy[None]
    rho = np.atleast_2d(rho)
    n, q = len(xy), len(rho)
    S0 = np.zeros((n, q))
    S1 = np.zeros((n, q, 2))
    cen = xy.mean(axis=1)                                        # (n, 2)
    for i in range(3):
        pm, pp = xy[:, i], xy[:, (i + 1) % 3]                    # (n, 2)
        t = (pp - pm) / np.linalg.norm(pp - pm, axis=1)[:, None]
        u = np.stack([t[:, 1], -t[:, 0]], axis=1)
        u *= np.where(np.einsum("nd,nd->n", pm - cen, u) < 0, -1.0, 1.0)[:, None]
        dm = pm[:, None, :] - rho[None]                          # (n, q, 2)
        dp = pp[:, None, :] - rho[None]
        P = np.einsum("nqd,nd->nq", dm, u)
        lp = np.einsum("nqd,nd->nq", dp, t)
        lm = np.einsum("nqd,nd->nq", dm, t)
        Rp = np.linalg.norm(dp, axis=2)
        Rm = np.linalg.norm(dm, axis=2)
        # ln((R+ + l+)/(R- + l-)), with R + l = P^2/(R - l) where l < 0 (no cancellation)
        both_neg = (lp < 0) & (lm < 0)
        with np.errstate(divide="ignore", invalid="ignore"):
            num = np.where(lp < 0, P * P / (Rp - lp), Rp + lp)
            den = np.where(lm < 0, P * P / (Rm - lm), Rm + lm)
            L = np.log(np.where(both_neg, (Rm - lm) / (Rp - lp), num / den))
            S0 += np.where(P == 0.0, 0.0, P * L)
            S1 += 0.5 * (np.where(P == 0.0, 0.0, P * P * L) + lp * Rp - lm * Rm)[:, :, None] * u[:, None, :]
    return (S0[0], S1[0]) if one else (S0, S1)


# --------------------------------------------------------------------------- triangle-pair integrals

def green(k: float, R: np.ndarray) -> np.ndarray:
    return np.exp(-1j * k * R) / (4 * np.pi * R)


def green_smooth(k: float, R: np.ndarray) -> np.ndarray:
    """(exp(-jkR) - 1)/(4 pi R), with its limit -jk/(4 pi) at R = 0."""
    out = np.full(R.shape, -1j * k / (4 * np.pi), dtype=np.complex128)
    nz = R > 0
    out[nz] = (np.exp(-1j * k * R[nz]) - 1.0) / (4 * np.pi * R[nz])
    return out


def pair_integrals(k: float, test_xy: np.ndarray, src_xy: np.ndarray, near: np.ndarray):
    """For one test triangle (3, 2) and source triangles (n, 3, 2), with c and
    c' the test and source centroids:
    I0 = <<G>>, Ir = <<(r - c) G>> (n, 2), Irp = <<(r' - c') G>> (n, 2),
    Irr = <<(r - c) . (r' - c') G>>, double surface integrals over test x source
    (positions taken from the centroids so that no large coordinate cancels);
    near[j] selects the closed-form static part for source j.  Also returns c (2,)
    and c' (n, 2)."""
    bary, w = rule7()
    ct = test_xy.mean(axis=0)
    cs = src_xy.mean(axis=1)                                          # (n, 2)
    ro_l = tri_points(test_xy - ct, bary)                             # (7, 2) from the test centroid
    rs_l = tri_points(src_xy - cs[:, None, :], bary)                  # (n, 7, 2) from each source centroid
    ro = ro_l + ct
    rs = rs_l + cs[:, None, :]
    wo = w * tri_area(test_xy)                                        # (7,)
    ws = w[None, :] * tri_area(src_xy)[:, None]                       # (n, 7)
    R = np.linalg.norm(ro[None, :, None, :] - rs[:, None, :, :], axis=-1)   # (n, 7o, 7s)
    Gf = np.empty(R.shape, dtype=np.complex128)
    Gf[near] = green_smooth(k, R[near])
    Gf[~near] = green(k, R[~near])
    g0 = np.einsum("nij,nj->ni", Gf, ws)              # inner integral of G at each outer point
    g1 = np.einsum("nij,nj,njd->nid", Gf, ws, rs_l)   # inner integral of (r' - c') G
    jn = np.nonzero(near)[0]
    if len(jn):
        S0, S1 = static_potentials(src_xy[jn], ro)                       # (nn, 7), (nn, 7, 2)
        g0[jn] += S0 / (4 * np.pi)
        # int (r' - c')/R = S1 + (rho - c') S0
        g1[jn] += (S1 + (ro[None] - cs[jn][:, None, :]) * S0[:, :, None]) / (4 * np.pi)
    I0 = g0 @ wo
    Ir = np.einsum("ni,i,id->nd", g0, wo, ro_l)
    Irp = np.einsum("nid,i->nd", g1, wo)
    Irr = np.einsum("nid,i,id->n", g1, wo, ro_l)
    return I0, Ir, Irp, Irr, ct, cs


# --------------------------------------------------------------------------- fill

def element_positions(lat) -> np.ndarray:
    return mom.element_xy(lat)


def _assemble_rows(el: RwgElement, k: float, eta: float, t: int, vt: np.ndarray, ints, src_tri_area,
                   src_vplus, src_vminus, src_tplus, src_tminus, length_n):
    """Rows of the test bases on triangle t (their contributions from this
    triangle only): dict m -> row over the source bases."""
    I0, Ir, Irp, Irr, ct, cs = ints
    At = el.area[t]
    rows = {}
    for m in range(el.M):
        if el.tplus[m] == t:
            sm, vm = 1.0, vt[el.vplus[m]]
        elif el.tminus[m] == t:
            sm, vm = -1.0, vt[el.vminus[m]]
        else:
            continue
        row = np.zeros(len(length_n), dtype=np.complex128)
        am = vm - ct
        for sn, tn, vn in ((1.0, src_tplus, src_vplus), (-1.0, src_tminus, src_vminus)):
            # <<(r - v_m) . (r' - v_n) G>> from the centroid moments
            an = vn - cs[tn]
            A = Irr[tn] - np.einsum("nd,nd->n", an, Ir[tn]) - Irp[tn] @ am + (an @ am) * I0[tn]
            An = src_tri_area[tn]
            row += sm * sn * el.length[m] * length_n * (
                1j * k * eta * A / (4 * At * An) - 1j * (eta / k) * I0[tn] / (At * An))
        rows[m] = row
    return rows


def fill_dense(el: RwgElement, lat, s: float, eta: float = ETA0) -> np.ndarray:
    """Dense Z (N x N, N = nx ny M) from absolute positions; unknown e*M + m."""
    k = mom.wavenumber(s)
    P = lat.nx * lat.ny
    M, nt = el.M, len(el.tri)
    pos = element_positions(lat)
    ixy = np.stack(np.divmod(np.arange(P), lat.nx)[::-1], axis=1)     # (ix, iy)
    txy = el.vert[el.tri]                                               # (nt, 3, 2)
    all_xy = (pos[:, None, None, None, :] + txy[None]).reshape(P * nt, 3, 2)
    all_area = np.tile(el.area, P)
    # source basis data over the whole array
    e_of_n = np.repeat(np.arange(P), M)
    m_of_n = np.tile(np.arange(M), P)
    src_tplus = e_of_n * nt + el.tplus[m_of_n]
    src_tminus = e_of_n * nt + el.tminus[m_of_n]
    src_vplus = el.vert[el.vplus[m_of_n]] + pos[e_of_n]
    src_vminus = el.vert[el.vminus[m_of_n]] + pos[e_of_n]
    length_n = el.length[m_of_n]
    Z = np.zeros((P * M, P * M), dtype=np.complex128)
    for e in range(P):
        near_e = np.repeat(np.max(np.abs(ixy - ixy[e]), axis=1) <= 1, nt)
        vt = el.vert + pos[e]
        for t in range(nt):
            ints = pair_integrals(k, txy[t] + pos[e], all_xy, near_e)
            rows = _assemble_rows(el, k, eta, t, vt, ints, all_area, src_vplus, src_vminus, src_tplus,
                                  src_tminus, length_n)
            for m, row in rows.items():
                Z[e * M + m] += row
    return Z


def z_rows(el: RwgElement, lat, s: float, unknowns, eta: float = ETA0, chunk: int = 256) -> np.ndarray:
    """Rows of the dense Z (len(unknowns) x N) for arrays too large to fill
    whole, from absolute positions exactly as fill_dense computes them (source
    elements taken chunk elements at a time)."""
    k = mom.wavenumber(s)
    P = lat.nx * lat.ny
    M, nt = el.M, len(el.tri)
    pos = element_positions(lat)
    ixy = np.stack(np.divmod(np.arange(P), lat.nx)[::-1], axis=1)
    txy = el.vert[el.tri]
    all_area = np.tile(el.area, P)
    e_of_n = np.repeat(np.arange(P), M)
    m_of_n = np.tile(np.arange(M), P)
    src_tplus = e_of_n * nt + el.tplus[m_of_n]
    src_tminus = e_of_n * nt + el.tminus[m_of_n]
    src_vplus = el.vert[el.vplus[m_of_n]] + pos[e_of_n]
    src_vminus = el.vert[el.vminus[m_of_n]] + pos[e_of_n]
    length_n = el.length[m_of_n]
    out = np.zeros((len(unknowns), P * M), dtype=np.complex128)
    for i, n in enumerate(unknowns):
        e, m = divmod(int(n), M)
        near_e = np.repeat(np.max(np.abs(ixy - ixy[e]), axis=1) <= 1, nt)
        vt = el.vert + pos[e]
        for t in (el.tplus[m], el.tminus[m]):
            parts = []
            for e0 in range(0, P, chunk):
                e1 = min(P, e0 + chunk)
                src = (pos[e0:e1, None, None, :] + txy[None]).reshape((e1 - e0) * nt, 3, 2)
                parts.append(pair_integrals(k, txy[t] + pos[e], src, near_e[e0 * nt:e1 * nt]))
            ints = tuple(np.concatenate([p[j] for p in parts]) for j in range(4)) + (
                parts[0][4], np.concatenate([p[5] for p in parts]))
            rows = _assemble_rows(el, k, eta, t, vt, ints, all_area, src_vplus, src_vminus, src_tplus,
                                  src_tminus, length_n)
            out[i] += rows[m]
    return out


def offset_block(el: RwgElement, lat, s: float, dx: int, dy: int, eta: float = ETA0) -> np.ndarray:
    """The M x M block between a test element and the source element (-dx, -dy)
    lattice steps away (Z[t][s] = T[t - s]), from their absolute positions:
    the test element at lattice index (dx, dy) and the source at the origin."""
    k = mom.wavenumber(s)
    M, nt = el.M, len(el.tri)
    pt = np.array([dx * lat.dx, dy * lat.dy])
    txy = el.vert[el.tri]
    near = np.full(nt, max(abs(dx), abs(dy)) <= 1)
    vt = el.vert + pt
    T = np.zeros((M, M), dtype=np.complex128)
    for t in range(nt):
        ints = pair_integrals(k, txy[t] + pt, txy, near)
        rows = _assemble_rows(el, k, eta, t, vt, ints, el.area, el.vert[el.vplus], el.vert[el.vminus],
                              el.tplus, el.tminus, el.length)
        for m, row in rows.items():
            T[m] += row
    return T


# --------------------------------------------------------------------------- ports and scans

def port_matrix(el: RwgElement, lat) -> np.ndarray:
    """W (N x P): column e holds the gap weights sign_m l_m at element e's port bases."""
    P = lat.nx * lat.ny
    W = np.zeros((P * el.M, P))
    for e in range(P):
        W[e * el.M + el.port_bases, e] = el.port_weights
    return W


def port_admittance(Z: np.ndarray, el: RwgElement, lat) -> np.ndarray:
    """Y_p = W^T Z^{-1} W: gap currents for unit gap voltages (others shorted)."""
    W = port_matrix(el, lat)
    return W.T @ mom.solve_lu(Z, W.astype(np.complex128))


def scan_voltages(lat, s: float, theta, phi) -> np.ndarray:
    """Gap voltages that steer the beam at (theta, phi): the progressive phases of
    ``mom.scan_phases`` applied to the voltages.  Shape (P, nscan)."""
    return mom.scan_phases(lat, s, np.atleast_1d(theta), np.atleast_1d(phi))


def scan_solve(Z: np.ndarray, el: RwgElement, lat, s: float, theta, phi, z0: float = 50.0,
               center: Optional[int] = None):
    """Phased voltage excitation of every gap: currents I = Z^{-1} W V, gap
    currents I_p = W^T I, the center element's active impedance
    Z_a = V_c / I_p,c (eq. (actZ)) and ARC (eq. (ARC)).  Returns (Ip, Za, Gamma)."""
    c = mom.center_element(lat) if center is None else center
    V = scan_voltages(lat, s, theta, phi)
    W = port_matrix(el, lat)
    Ip = W.T @ mom.solve_lu(Z, W @ V)
    Za = V[c] / Ip[c]
    return Ip, Za, mom.arc(Za, z0)


def radiated_power(el: RwgElement, lat, s: float, I: np.ndarray, nth: int = 64, nph: int = 128,
                   eta: float = ETA0) -> float:
    """Power radiated by the surface current sum_n I_n f_n (all elements), from
    its far field integrated over the sphere (Gauss-Legendre in cos(theta),
    trapezoid in phi); the radiation vector uses the seven-point rule on every
    triangle subdivided once into four."""
    k = mom.wavenumber(s)
    P = lat.nx * lat.ny
    pos = element_positions(lat)
    bary, w = rule7()
    # subdivide each triangle into four for the far-field quadrature
    sub = np.array([[[1, 0, 0], [.5, .5, 0], [.5, 0, .5]], [[0, 1, 0], [.5, .5, 0], [0, .5, .5]],
                    [[0, 0, 1], [.5, 0, .5], [0, .5, .5]], [[.5, .5, 0], [0, .5, .5], [.5, 0, .5]]])
    pts, wts, cur = [], [], []
    for e in range(P):
        for t in range(len(el.tri)):
            xy = el.vert[el.tri[t]]
            for sb in sub:
                sxy = sb @ xy
                r = tri_points(sxy, bary)
                J = np.zeros((7, 2), dtype=np.complex128)
                for m in np.nonzero((el.tplus == t) | (el.tminus == t))[0]:
                    J += I[e * el.M + m] * basis_value(el, m, t, r)
                pts.append(r + pos[e])
                wts.append(w * tri_area(sxy))
                cur.append(J)
    pts = np.concatenate(pts)
    wts = np.concatenate(wts)
    cur = np.concatenate(cur)
    xg, wg = np.polynomial.legendre.leggauss(nth)
    ph = 2 * np.pi * np.arange(nph) / nph
    total = 0.0
    for ct, wc in zip(xg, wg):
        st = np.sqrt(1 - ct * ct)
        u = st * np.cos(ph)
        v = st * np.sin(ph)
        phase = np.exp(1j * k * (np.outer(u, pts[:, 0]) + np.outer(v, pts[:, 1])))   # (nph, npts)
        N = phase @ (cur * wts[:, None])                                            # (nph, 2)
        Nth = ct * (N[:, 0] * np.cos(ph) + N[:, 1] * np.sin(ph))
        Nph = -N[:, 0] * np.sin(ph) + N[:, 1] * np.cos(ph)
        total += wc * np.sum(np.abs(Nth) ** 2 + np.abs(Nph) ** 2) * (2 * np.pi / nph)
    return float(k * k * eta / (32 * np.pi ** 2) * total)
