"""Independent physics used to pin the oracle (test helper, not part of either
implementation): far-field radiated power of z-directed wire currents.

For line currents I(z') along z on wires at (x_e, y_e), the radiation vector
N_z(theta, phi) = sum_e exp(j k sin(theta)(x_e cos(phi) + y_e sin(phi)))
                  * integral I_e(z') exp(j k z' cos(theta)) dz'
gives E_theta = j k eta sin(theta) N_z exp(-j k r) / (4 pi r), hence
P_rad = k^2 eta / (32 pi^2) * integral sin^2(theta) |N_z|^2 dOmega.
"""
import numpy as np

ETA_FREE_SPACE = 376.730313668


def radiated_power(lat, dip, s, I, eta=ETA_FREE_SPACE, nmu=128, nphi=128):
    k = 2.0 * np.pi * s
    M = dip.nbases
    Ns = M + 1
    D = dip.length / Ns
    I = np.asarray(I).reshape(lat.nx * lat.ny, M)
    # node currents: ends are zero, node p+1 carries basis coefficient p
    nodes = np.zeros((I.shape[0], Ns + 1), dtype=complex)
    nodes[:, 1:Ns] = I
    q, wq = np.polynomial.legendre.leggauss(10)
    u = 0.5 * (1.0 + q)
    wu = 0.5 * wq
    mu, wmu = np.polynomial.legendre.leggauss(nmu)
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    # per-element line integral as a function of mu = cos(theta)
    seg = np.arange(Ns)
    z = -0.5 * dip.length + (seg[:, None] + u[None, :]) * D            # (Ns, 10)
    lin = nodes[:, :-1, None] * (1.0 - u) + nodes[:, 1:, None] * u      # (P, Ns, 10)
    ph_z = np.exp(1j * k * z[None, :, :] * mu[:, None, None])          # (nmu, Ns, 10)
    Fe = np.einsum("psq,msq,q->mp", lin, ph_z, wu) * D                  # (nmu, P)
    iy, ix = np.divmod(np.arange(lat.nx * lat.ny), lat.nx)
    xe, ye = ix * lat.dx, iy * lat.dy
    st = np.sqrt(1.0 - mu ** 2)
    arg = k * st[:, None, None] * (xe[None, None, :] * np.cos(phi)[None, :, None]
                                   + ye[None, None, :] * np.sin(phi)[None, :, None])
    Nz = np.einsum("mfp,mp->mf", np.exp(1j * arg), Fe)                  # (nmu, nphi)
    integrand = (1.0 - mu[:, None] ** 2) * np.abs(Nz) ** 2
    total = np.sum(wmu[:, None] * integrand) * (2.0 * np.pi / nphi)
    return k ** 2 * eta / (32.0 * np.pi ** 2) * total


def distant_field(lat, s, I, theta, phi, r=1.0e5):
    """Array factor of port currents I (P,) evaluated by summing the fill's own
    kernel exp(-j k R)/(4 pi R) over point sources at the element positions,
    with R the exact distance to a point at range r in direction (theta, phi),
    normalised by the single-source value at the origin.  No plane-wave
    approximation: the sign of the progressive phase comes from the kernel."""
    k = 2.0 * np.pi * s
    iy, ix = np.divmod(np.arange(lat.nx * lat.ny), lat.nx)
    xe, ye = ix * lat.dx, iy * lat.dy
    theta = np.atleast_1d(theta)
    phi = np.atleast_1d(phi)
    px = r * np.sin(theta) * np.cos(phi)
    py = r * np.sin(theta) * np.sin(phi)
    pz = r * np.cos(theta)
    R = np.sqrt((px[:, None] - xe[None, :]) ** 2 + (py[:, None] - ye[None, :]) ** 2 + pz[:, None] ** 2)
    g = np.exp(-1j * k * R) / R
    g0 = np.exp(-1j * k * r) / r
    return (g @ np.asarray(I)) / g0
