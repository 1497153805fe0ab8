"""Writes the stored oracle results for the 5x5-dipole frequency sweep.

Calls only oracle/ (dense fill from absolute positions, LAPACK LU, extraction)
and the seeded workload description: the 5x5 array of 15-basis dipoles at the
21 frequencies s = 0.5 + 0.05 i, i = 0..20, with the center element's scan
quantities at the workload's scan angles.  Stored per frequency: the full
25 x 25 Z_p, Za, Gamma and Gamma_wave, in dipole_5x5_m15_21f_reference.npz.

Usage:  python tests/golden/make_sweep_reference.py   (under a minute)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mom  # noqa: E402
from paper_2608_17844_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dipole_5x5_m15_21f_reference.npz")


def main():
    w = W.sweep_5x5_21f()
    res = [mom.solve_array(w.lattice, w.dipole, s, w.theta, w.phi, z0=w.z0) for s in w.freqs]
    np.savez_compressed(
        OUT,
        freqs=np.array(w.freqs), theta=w.theta, phi=w.phi,
        Zp=np.stack([r.Zp for r in res]), Za=np.stack([r.Za for r in res]),
        Gamma=np.stack([r.Gamma for r in res]), Gamma_wave=np.stack([r.Gamma_wave for r in res]),
    )
    print("wrote", OUT)


if __name__ == "__main__":
    main()
