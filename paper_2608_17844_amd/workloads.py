"""Seeded synthetic workloads: array geometries, frequencies, scan angles and
serving request streams.

This module only describes inputs (sizes, seeds, random draws).  It holds none
of the solver's arithmetic, so the CPU oracle and the GPU path can both draw
their inputs from it without sharing any computation.

Geometry is in units of the wavelength at the reference frequency f0; a
frequency is given as the ratio s = f / f0.
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Dipole:
    """z-directed thin-wire dipole element (lengths in wavelengths at f0)."""
    length: float = 0.5
    radius: float = 0.005
    nbases: int = 15          # rooftop bases per element, odd (center basis is the port)


@dataclass(frozen=True)
class Lattice:
    """Rectangular lattice: element (ix, iy) sits at (ix*dx, iy*dy)."""
    nx: int = 5
    ny: int = 5
    dx: float = 0.5
    dy: float = 0.5


@dataclass
class Workload:
    name: str
    dipole: Dipole
    lattice: Lattice
    freqs: List[float]
    theta: np.ndarray = field(default_factory=lambda: np.zeros(0))
    phi: np.ndarray = field(default_factory=lambda: np.zeros(0))
    z0: float = 50.0
    restart: int = 50
    tol: float = 1e-10

    def describe(self) -> dict:
        return {
            "workload": self.name,
            "nx": self.lattice.nx, "ny": self.lattice.ny,
            "dx": self.lattice.dx, "dy": self.lattice.dy,
            "length": self.dipole.length, "radius": self.dipole.radius,
            "nbases": self.dipole.nbases,
            "unknowns": self.lattice.nx * self.lattice.ny * self.dipole.nbases,
            "ports": self.lattice.nx * self.lattice.ny,
            "freqs": list(self.freqs), "nscan": int(len(self.theta)),
            "restart": self.restart, "tol": self.tol,
        }


def scan_angles(n: int, seed: int = 0, broadside_first: bool = False) -> Tuple[np.ndarray, np.ndarray]:
    """Seeded scan directions: theta ~ U[0, 60 deg], phi ~ U[0, 360 deg), radians."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, np.deg2rad(60.0), size=n)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n)
    if broadside_first:
        th = np.concatenate([[0.0], th])
        ph = np.concatenate([[0.0], ph])
    return th, ph


def cpu_size_5x5() -> Workload:
    """5x5 dipoles, 15 bases, one frequency, broadside plus 10 seeded scans."""
    th, ph = scan_angles(10, seed=0, broadside_first=True)
    return Workload("dipole_5x5_m15", Dipole(0.5, 0.005, 15), Lattice(5, 5, 0.5, 0.5), [1.0], th, ph)


def gpu_size_32x32() -> Workload:
    """32x32 dipoles, 31 bases (N = 31,744), all 1024 ports, 64 seeded scans."""
    th, ph = scan_angles(64, seed=0)
    return Workload("dipole_32x32_m31", Dipole(0.5, 0.005, 31), Lattice(32, 32, 0.5, 0.5), [1.0], th, ph)


def blocks_64x64_m96_shape():
    """The largest single-GPU shape: 64 x 64 elements of 96 bases (N = 393,216),
    FFT grid 128 x 128, 32 port excitations per operator and 5 operators (one
    per frequency; seeds 0..4 of synthetic_blocks): the solver-only variant of
    the bowtie workload.  Returns (nx, ny, M, seeds, ports)."""
    rng = np.random.default_rng(0)
    ports = np.sort(rng.choice(64 * 64, size=32, replace=False)).astype(np.int32)
    return 64, 64, 96, [0, 1, 2, 3, 4], ports


def sweep_5x5_21f() -> Workload:
    """The 5x5 array at 21 frequencies s_i = 0.5 + 0.05 i."""
    th, ph = scan_angles(10, seed=0, broadside_first=True)
    freqs = [0.5 + 0.05 * i for i in range(21)]
    return Workload("dipole_5x5_m15_21f", Dipole(0.5, 0.005, 15), Lattice(5, 5, 0.5, 0.5), freqs, th, ph)


def synthetic_blocks(nx: int, ny: int, nbases: int, seed: int = 0, coupling: float = 0.05) -> np.ndarray:
    """Seeded unique blocks of a block-Toeplitz lattice operator for solver-only
    workloads (caller-given blocks instead of an element fill): T[dy][dx]
    (M x M complex, offsets dy + ny - 1, dx + nx - 1) with the reciprocity of a
    Galerkin operator, T(-d) = T(d)^T, a symmetric self block I (1 + 0.5j) plus
    a small random part, and random coupling blocks whose size decays as 1/|d|.
    Shape (2ny-1, 2nx-1, M, M), complex128."""
    rng = np.random.default_rng(seed)
    M = nbases
    T = np.zeros((2 * ny - 1, 2 * nx - 1, M, M), dtype=np.complex128)
    for dy in range(0, ny):
        for dx in range(-(nx - 1), nx):
            if dy == 0 and dx < 0:
                continue
            G = (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))) / (2.0 * np.sqrt(M))
            if dy == 0 and dx == 0:
                S = 0.1 * (G + G.T) / 2 + (1.0 + 0.5j) * np.eye(M)
                T[ny - 1, nx - 1] = S
            else:
                B = coupling / np.hypot(dx, dy) * G
                T[dy + ny - 1, dx + nx - 1] = B
                T[-dy + ny - 1, -dx + nx - 1] = B.T
    return T


def synthetic_margin(nx: int, ny: int, nbases: int, nmargin: int, seed: int = 0, rank: int = 6,
                     coupling: float = 0.02):
    """Seeded margin blocks of a partitioned array operator [[Z_A, Z_B^T], [Z_B, Z_C]]
    for the block-defined workloads: Z_C (nmargin x nmargin) symmetric, a unit
    diagonal (1 + 0.5j) plus a small random symmetric part; Z_B (nmargin x
    nx*ny*nbases) of low rank `rank` (the element-margin coupling), entries of
    size about `coupling`.  Returns (Z_B, Z_C), complex128."""
    rng = np.random.default_rng(seed)
    NA = nx * ny * nbases
    G = (rng.standard_normal((nmargin, nmargin)) + 1j * rng.standard_normal((nmargin, nmargin))) / (
        2.0 * np.sqrt(nmargin))
    ZC = (1.0 + 0.5j) * np.eye(nmargin) + 0.1 * (G + G.T) / 2
    U = rng.standard_normal((nmargin, rank)) + 1j * rng.standard_normal((nmargin, rank))
    Vt = rng.standard_normal((rank, NA)) + 1j * rng.standard_normal((rank, NA))
    ZB = coupling * (U @ Vt) / (2.0 * rank)
    return ZB, ZC


@dataclass(frozen=True)
class PlanarMesh:
    """Triangle mesh of one planar element in the plane z = 0, in its own frame
    (wavelengths at f0): vertices (nv, 2), triangles (nt, 3) as counterclockwise
    vertex-index triples, the feed-gap edges (ne, 2) as vertex-index pairs, and
    the direction of the gap field in the element plane."""
    vertices: np.ndarray
    triangles: np.ndarray
    port_edges: np.ndarray
    port_dir: Tuple[float, float] = (1.0, 0.0)


def _strip_between(a: List[int], ta: np.ndarray, b: List[int], tb: np.ndarray) -> List[Tuple[int, int, int]]:
    """Triangles joining two node rows (node ids a, b at parameters ta, tb in
    [0, 1] across the strip): walk both rows and always advance on the row whose
    next node comes first."""
    out = []
    i = k = 0
    while i < len(a) - 1 or k < len(b) - 1:
        if k == len(b) - 1 or (i < len(a) - 1 and ta[i + 1] <= tb[k + 1]):
            out.append((a[i], a[i + 1], b[k]))
            i += 1
        else:
            out.append((a[i], b[k + 1], b[k]))
            k += 1
    return out


def _ccw(vert: np.ndarray, tris: List[Tuple[int, int, int]]) -> np.ndarray:
    t = np.array(tris, dtype=np.int32)
    p, q, r = vert[t[:, 0]], vert[t[:, 1]], vert[t[:, 2]]
    cross = (q[:, 0] - p[:, 0]) * (r[:, 1] - p[:, 1]) - (q[:, 1] - p[:, 1]) * (r[:, 0] - p[:, 0])
    t[cross < 0] = t[cross < 0][:, [0, 2, 1]]
    return t


def bowtie_mesh(span: float = 0.45, flare_deg: float = 60.0, feed_width: float = 0.04,
                counts: Tuple[int, ...] = (3, 4, 4, 5, 6, 6)) -> PlanarMesh:
    """Planar bowtie along x: two wings of full flare angle `flare_deg` joined on
    the feed line x = 0 of width `feed_width`, tip to tip `span`.  Each wing is a
    structured mesh of node rows at x_j = +-(span/2) j/s (j = 0..s, s =
    len(counts) - 1) with counts[j] nodes spread evenly over the wing width
    feed_width + 2|x_j| tan(flare/2); row 0 is the shared feed line, whose edges
    are the port.  The default has 74 triangles and 96 interior edges."""
    s = len(counts) - 1
    half = np.tan(np.radians(flare_deg) / 2.0)
    rows = []
    vert = []
    for j in range(-s, s + 1):
        x = 0.5 * span * j / s
        c = counts[abs(j)]
        w = feed_width + 2.0 * abs(x) * half
        ys = np.linspace(-0.5 * w, 0.5 * w, c)
        rows.append(list(range(len(vert), len(vert) + c)))
        vert.extend((x, y) for y in ys)
    vert = np.array(vert, dtype=np.float64)
    tris = []
    for r0, r1 in zip(rows[:-1], rows[1:]):
        tris += _strip_between(r0, np.linspace(0, 1, len(r0)), r1, np.linspace(0, 1, len(r1)))
    feed = rows[s]
    port = np.array([(feed[i], feed[i + 1]) for i in range(len(feed) - 1)], dtype=np.int32)
    return PlanarMesh(vert, _ccw(vert, tris), port, (1.0, 0.0))


def strip_mesh(length: float = 0.5, width: float = 0.02, nseg: int = 20, nacross: int = 1) -> PlanarMesh:
    """Flat strip dipole along x (length x width), nseg cells along (even, so
    that x = 0 is a node row) and nacross across, each cell split by its
    diagonal; the port is the row of edges at x = 0."""
    if nseg % 2:
        raise ValueError("nseg must be even")
    xs = np.linspace(-0.5 * length, 0.5 * length, nseg + 1)
    ys = np.linspace(-0.5 * width, 0.5 * width, nacross + 1)
    vert = np.array([(x, y) for x in xs for y in ys], dtype=np.float64)
    rows = [list(range(i * (nacross + 1), (i + 1) * (nacross + 1))) for i in range(nseg + 1)]
    tris = []
    for r0, r1 in zip(rows[:-1], rows[1:]):
        tris += _strip_between(r0, np.linspace(0, 1, len(r0)), r1, np.linspace(0, 1, len(r1)))
    feed = rows[nseg // 2]
    port = np.array([(feed[i], feed[i + 1]) for i in range(len(feed) - 1)], dtype=np.int32)
    return PlanarMesh(vert, _ccw(vert, tris), port, (1.0, 0.0))


def bowtie_64x64_workload():
    """Largest single-GPU instance: 64 x 64 bowties (96 RWG bases each,
    N = 393,216) on a 0.5-wavelength square lattice, 32 excitations (broadside
    first, then seeded scan directions) at 5 frequencies 0.9-1.3 f0, the band
    around the frequency where the lattice spacing is 0.55 wavelengths."""
    theta, phi = scan_angles(31, seed=5, broadside_first=True)
    return bowtie_mesh(), Lattice(64, 64, 0.5, 0.5), np.linspace(0.9, 1.3, 5), theta, phi


@dataclass
class Request:
    """One serving request: an array, its frequencies and its scan set."""
    rid: int
    arrival: float            # seconds after stream start
    dipole: Dipole
    lattice: Lattice
    freqs: List[float]
    theta: np.ndarray
    phi: np.ndarray
    z0: float = 50.0


def serving_stream(n: int, rate: float, seed: int = 0, nx_range=(8, 48), ny_range=(8, 48),
                   nbases_choices=(15, 31), nfreq_range=(1, 8), nscan_range=(1, 64)) -> List[Request]:
    """Poisson arrivals at `rate` requests/s; each request draws Nx, Ny uniform
    in the given ranges, M from `nbases_choices`, 1-8 frequencies uniform in
    [0.5, 1.5] f0 and 1-64 scan angles."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        ny = int(rng.integers(ny_range[0], ny_range[1] + 1))
        m = int(rng.choice(nbases_choices))
        nf = int(rng.integers(nfreq_range[0], nfreq_range[1] + 1))
        freqs = sorted(float(f) for f in rng.uniform(0.5, 1.5, size=nf))
        ns = int(rng.integers(nscan_range[0], nscan_range[1] + 1))
        th = rng.uniform(0.0, np.deg2rad(60.0), size=ns)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=ns)
        out.append(Request(i, t, Dipole(0.5, 0.005, m), Lattice(nx, ny, 0.5, 0.5), freqs, th, ph))
    return out


def random_vectors(n: int, r: int, seed: int = 0, dtype=np.complex128) -> np.ndarray:
    """Seeded complex Gaussian test vectors, shape (n, r)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))).astype(dtype)


def to_dict(obj) -> dict:
    return asdict(obj)
