"""Writes the stored oracle results for the 32x32-dipole workload.

Calls only oracle/ (dense fill from absolute positions, LAPACK LU, extraction)
and the seeded workload description.  The full dense system (N = 31,744,
16 GB complex128) is too large to rebuild inside a test, so a compact subset of
the result is stored in dipole_32x32_m31_reference.npz:

* Zp_center_row, Zp_diag, Zp_samples (rows, cols, values) and the Frobenius
  and max norms of Z_p;
* 16 whole rows of Z_p (the center row and 15 seeded rows);
* a sketch Z_p @ Omega with Omega = random_vectors(1024, 64, seed=7): for a
  complex Gaussian Omega, ||dZ Omega||_F^2 / 128 is an unbiased estimate of
  ||dZ||_F^2 (each column has E|g|^2 = 2), so a test estimates the Frobenius
  error of a computed Z_p from it;
* Yp columns for a handful of ports;
* S center row;
* Za, Gamma, Gamma_wave at the 64 seeded scan angles;
* phase timings of the oracle run (fill, zgetrf, zgetrs of all 1024 port
  columns, extraction), the host it ran on and its thread count.

Usage:  python tests/golden/make_reference.py   (about 10 minutes on 8 cores)
"""
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mom  # noqa: E402
from paper_2608_17844_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dipole_32x32_m31_reference.npz")
SAMPLE_PORTS = [0, 1, 31, 16 * 32 + 16, 16 * 32 + 15, 527, 992, 1023]
SKETCH_SEED = 7
SKETCH_COLS = 64


def main():
    w = W.gpu_size_32x32()
    lat, dip = w.lattice, w.dipole
    t0 = time.time()
    r = mom.solve_array(lat, dip, 1.0, w.theta, w.phi, z0=w.z0)
    t1 = time.time()
    Zp = r.Zp
    c = mom.center_element(lat)
    rng = np.random.default_rng(0)
    rows = rng.integers(0, Zp.shape[0], 4096)
    cols = rng.integers(0, Zp.shape[0], 4096)
    full_rows = np.concatenate([[c], np.sort(rng.choice(np.setdiff1d(np.arange(Zp.shape[0]), [c]), 15,
                                                           replace=False))])
    omega = W.random_vectors(Zp.shape[0], SKETCH_COLS, seed=SKETCH_SEED)
    np.savez_compressed(
        OUT,
        Zp_center_row=Zp[c, :], Zp_diag=np.diag(Zp).copy(),
        Zp_rows=rows, Zp_cols=cols, Zp_samples=Zp[rows, cols],
        Zp_fro=np.linalg.norm(Zp), Zp_max=np.abs(Zp).max(),
        Zp_full_rows=full_rows, Zp_rows_values=Zp[full_rows, :],
        Zp_sketch=Zp @ omega, sketch_seed=SKETCH_SEED,
        Yp_ports=np.array(SAMPLE_PORTS), Yp_cols=r.Yp[:, SAMPLE_PORTS],
        S_center_row=r.S[c, :],
        theta=w.theta, phi=w.phi, Za=r.Za, Gamma=r.Gamma, Gamma_wave=r.Gamma_wave,
        center=c,
        times=np.array([r.times["fill"], r.times["lu"], r.times["solve"], r.times["extract"]]),
        host=np.array(platform.processor() or platform.machine()), cores=os.cpu_count(),
        threads=int(os.environ.get("OPENBLAS_NUM_THREADS", os.cpu_count())),
    )
    print("wrote", OUT, "in %.1f s" % (t1 - t0), r.times)


if __name__ == "__main__":
    main()
