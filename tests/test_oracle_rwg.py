"""Pins of the RWG oracle (oracle/rwg.py) against facts that do not come from it:
polynomial exactness of the quadrature, closed forms and independent polar or
subdivided integration of the static potentials, normal continuity of the RWG
functions, power balance against the far field, the thin-wire equivalent of a
flat strip, translation invariance, reciprocity and passivity."""
from math import factorial

import numpy as np
import pytest
from scipy import integrate

from oracle import mom, rwg
from paper_2608_17844_amd import workloads as W


def _tri(seed=0):
    rng = np.random.default_rng(seed)
    while True:
        xy = rng.uniform(-0.1, 0.1, (3, 2))
        if rwg.tri_area(xy) > 2e-3:
            return xy


def test_rule7_is_exact_to_degree_five_only():
    """Integral of x^a y^b over the unit right triangle is a! b! / (a+b+2)!."""
    bary, w = rwg.rule7()
    assert abs(w.sum() - 1.0) < 1e-15
    pts = rwg.tri_points(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), bary)
    for a in range(6):
        for b in range(6 - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            approx = 0.5 * np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(approx - exact) < 1e-15, (a, b)
    exact6 = factorial(6) / factorial(8)
    assert abs(0.5 * np.sum(w * pts[:, 0] ** 6) - exact6) > 1e-6


def test_static_potential_of_equilateral_triangle_at_centroid():
    """From the centroid each side is at the inradius a/(2 sqrt 3) and subtends
    half-length a/2, which sums to sqrt(3) a ln(2 + sqrt 3); S1 vanishes by symmetry."""
    a = 0.3
    xy = np.array([[0.0, 0.0], [a, 0.0], [a / 2, a * np.sqrt(3) / 2]])
    S0, S1 = rwg.static_potentials(xy, xy.mean(axis=0)[None])
    assert abs(S0[0] - np.sqrt(3) * a * np.log(2 + np.sqrt(3))) < 1e-14
    assert np.abs(S1).max() < 1e-15


def _polar(xy, rho):
    """S0 = int rho_max(phi) dphi and S1 = int e(phi) rho_max(phi)^2 / 2 dphi in polar
    coordinates about an interior point (rho_max: distance to the boundary)."""
    def rmax(ph):
        e = np.array([np.cos(ph), np.sin(ph)])
        best = np.inf
        for i in range(3):
            p, q = xy[i], xy[(i + 1) % 3]
            A = np.array([e, p - q]).T
            if abs(np.linalg.det(A)) < 1e-300:
                continue
            s, t = np.linalg.solve(A, p - rho)
            if s > 0 and -1e-12 <= t <= 1 + 1e-12:
                best = min(best, s)
        return best

    cuts = sorted(np.mod(np.arctan2(*(v - rho)[::-1]), 2 * np.pi) for v in xy)
    edges = [0.0] + cuts + [2 * np.pi]
    S0 = S1x = S1y = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        if hi - lo < 1e-14:
            continue
        S0 += integrate.quad(rmax, lo, hi, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
        S1x += integrate.quad(lambda p: np.cos(p) * rmax(p) ** 2 / 2, lo, hi, epsabs=1e-14, epsrel=1e-13,
                              limit=200)[0]
        S1y += integrate.quad(lambda p: np.sin(p) * rmax(p) ** 2 / 2, lo, hi, epsabs=1e-14, epsrel=1e-13,
                              limit=200)[0]
    return S0, np.array([S1x, S1y])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_static_potentials_inside_match_polar_integration(seed):
    xy = _tri(seed)
    rng = np.random.default_rng(10 + seed)
    bary = rng.dirichlet([1.0, 1.0, 1.0], size=4)
    rho = bary @ xy
    S0, S1 = rwg.static_potentials(xy, rho)
    for q in range(len(rho)):
        p0, p1 = _polar(xy, rho[q])
        assert abs(S0[q] - p0) < 1e-10 * abs(p0)
        assert np.abs(S1[q] - p1).max() < 1e-10 * np.abs(S0[q]) * 0.1


def _subdivided(xy, f, levels=6):
    """The seven-point rule on the triangle cut 4^levels times."""
    tris = [xy]
    for _ in range(levels):
        nxt = []
        for t in tris:
            a, b, c = t
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, c]), np.array([ab, bc, ca])]
        tris = nxt
    T = np.array(tris)
    bary, w = rwg.rule7()
    pts = rwg.tri_points(T, bary).reshape(-1, 2)
    ws = (w[None, :] * rwg.tri_area(T)[:, None]).reshape(-1)
    return f(pts, ws)


def test_static_potentials_outside_match_subdivided_rule():
    """Points outside the triangle, one on the extension of an edge's line (the
    branch where both edge coordinates are negative) and one beside a vertex."""
    xy = _tri(3)
    c = xy.mean(axis=0)
    e = xy[1] - xy[0]
    rho = np.array([c + 0.4 * (xy[0] - c) * 3, xy[0] - 0.5 * e, xy[1] + 0.3 * e, c + np.array([0.25, -0.2])])
    S0, S1 = rwg.static_potentials(xy, rho)
    for q in range(len(rho)):
        def f(p, w):
            R = np.linalg.norm(p - rho[q], axis=1)
            return np.sum(w / R), np.sum(w[:, None] * (p - rho[q]) / R[:, None], axis=0)
        r0, r1 = _subdivided(xy, f)
        assert abs(S0[q] - r0) < 1e-9 * abs(r0), q
        assert np.abs(S1[q] - r1).max() < 1e-9 * abs(r0), q


def test_bowtie_bases_and_normal_continuity():
    """96 RWG functions on 74 triangles; each has unit normal component across its
    edge from both sides (T+ to T-), so the surface charge has no line sources."""
    el = rwg.rwg_element(W.bowtie_mesh())
    assert el.M == 96 and len(el.tri) == 74
    assert len(el.port_bases) == 2 and np.allclose(np.abs(el.port_weights), el.length[el.port_bases])
    cen = el.vert[el.tri].mean(axis=1)
    for m in range(el.M):
        a, b = el.vert[el.edges[m]]
        mid = (a + b) / 2
        t = (b - a) / np.linalg.norm(b - a)
        n = np.array([t[1], -t[0]])
        if (cen[el.tminus[m]] - cen[el.tplus[m]]) @ n < 0:
            n = -n
        fp = rwg.basis_value(el, m, el.tplus[m], mid[None])[0]
        fm = rwg.basis_value(el, m, el.tminus[m], mid[None])[0]
        assert abs(fp @ n - 1.0) < 1e-12 and abs(fm @ n - 1.0) < 1e-12


@pytest.mark.parametrize("nx,drive", [(1, [1.0]), (2, [1.0, 1j])])
def test_power_balance_against_far_field(nx, drive):
    """Input power 1/2 Re(I^H Z I) equals the power of the far field of the same
    currents integrated over the sphere (the real part of Z comes from the smooth
    sin(kR)/R kernel, so a wrong term, sign or factor breaks the balance)."""
    el = rwg.rwg_element(W.bowtie_mesh())
    lat = W.Lattice(nx, 1, 0.5, 0.5)
    Z = rwg.fill_dense(el, lat, 1.0)
    I = mom.solve_lu(Z, rwg.port_matrix(el, lat) @ np.asarray(drive, dtype=np.complex128))
    p_in = 0.5 * np.real(np.vdot(I, Z @ I))
    p_far = rwg.radiated_power(el, lat, 1.0, I)
    assert abs(p_in - p_far) < 2e-4 * p_in


def test_flat_strip_matches_thin_wire_of_quarter_width_radius():
    """A flat strip of width w radiates like a round wire of radius w/4: the
    0.5-wavelength strip (20 cells) against the thin-wire oracle (19 rooftops)."""
    lat = W.Lattice(1, 1, 0.5, 0.5)
    st = rwg.rwg_element(W.strip_mesh(0.5, 0.02, 20, 1))
    zs = 1.0 / rwg.port_admittance(rwg.fill_dense(st, lat, 1.0), st, lat)[0, 0]
    dip = W.Dipole(0.5, 0.005, 19)
    zw = 1.0 / mom.port_admittance(mom.solve_lu(mom.fill_dense(lat, dip, 1.0), mom.excitation(lat, dip)),
                                   lat, dip)[0, 0]
    assert abs(zs - zw) < 0.03 * abs(zw)
    assert 60 < zs.real < 120 and 20 < zs.imag < 60


@pytest.fixture(scope="module")
def array_3x2():
    el = rwg.rwg_element(W.bowtie_mesh())
    lat = W.Lattice(3, 2, 0.5, 0.5)
    return el, lat, rwg.fill_dense(el, lat, 1.0)


def test_translation_invariance_and_offset_blocks(array_3x2):
    el, lat, Z = array_3x2
    M = el.M
    blk = lambda a, b: Z[a * M:(a + 1) * M, b * M:(b + 1) * M]
    assert np.abs(blk(0, 1) - blk(4, 5)).max() < 1e-11 * np.abs(blk(0, 1)).max()
    assert np.abs(blk(1, 3) - blk(2, 4)).max() < 1e-11 * np.abs(blk(1, 3)).max()
    for (a, b) in ((0, 0), (0, 1), (1, 0), (0, 5), (5, 0), (2, 3)):
        d = np.array(divmod(a, lat.nx)[::-1]) - np.array(divmod(b, lat.nx)[::-1])
        T = rwg.offset_block(el, lat, 1.0, int(d[0]), int(d[1]))
        assert np.abs(T - blk(a, b)).max() < 1e-11 * np.abs(blk(a, b)).max(), (a, b)


def test_reciprocity(array_3x2):
    """Blocks two or more steps apart use the same rule on both sides, so
    Z = Z^T to rounding; nearer blocks differ by the one-sided closed-form
    static part, a quadrature-level asymmetry."""
    el, lat, Z = array_3x2
    M = el.M
    blk = lambda a, b: Z[a * M:(a + 1) * M, b * M:(b + 1) * M]
    assert np.abs(blk(0, 2) - blk(2, 0).T).max() < 1e-12 * np.abs(blk(0, 2)).max()
    assert np.abs(blk(0, 1) - blk(1, 0).T).max() < 1e-3 * np.abs(blk(0, 1)).max()
    assert np.abs(Z - Z.T).max() < 2e-3 * np.abs(Z).max()


def test_port_passivity_and_scan_consistency(array_3x2):
    el, lat, Z = array_3x2
    Yp = rwg.port_admittance(Z, el, lat)
    assert np.abs(Yp - Yp.T).max() < 1e-3 * np.abs(Yp).max()
    Zp = mom.port_impedance(Yp)
    assert np.linalg.eigvalsh(0.5 * (Zp + Zp.conj().T)).min() > 0
    S = mom.s_matrix(Zp, 50.0)
    assert np.max(np.sum(np.abs(S) ** 2, axis=0)) < 1.0
    theta, phi = W.scan_angles(4, seed=2, broadside_first=True)
    Ip, Za, G = rwg.scan_solve(Z, el, lat, 1.0, theta, phi)
    V = rwg.scan_voltages(lat, 1.0, theta, phi)
    assert np.abs(Ip - Yp @ V).max() < 1e-9 * np.abs(Ip).max()
    c = mom.center_element(lat)
    assert np.abs(Za - (Zp @ Ip)[c] / Ip[c]).max() < 1e-8 * np.abs(Za).max()


def test_z_rows_equal_dense_rows(array_3x2):
    """Rows computed for arrays too large to fill whole equal the dense fill's."""
    el, lat, Z = array_3x2
    n = [0, 47, 4 * el.M + 50, Z.shape[0] - 1]
    assert np.array_equal(rwg.z_rows(el, lat, 1.0, n, chunk=2), Z[n])
