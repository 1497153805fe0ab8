"""Oracle for operators given by their unique lattice blocks.

TEST INFRASTRUCTURE ONLY (see oracle/mom.py).  A regular lattice operator is
defined by one M x M block per lattice offset (Sec. II-A: the interaction of
a test element with a source element depends only on their offset d = test -
source).  This module writes out the plain definitions: the dense matrix
assembled block by block, and single entries of Z x as explicit sums over all
source elements, for sizes where the dense matrix does not fit.
"""
from __future__ import annotations

import numpy as np


def dense_from_blocks(T: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """Z[t*M + p, s*M + q] = T[d][p][q], d = (element t) - (element s); element
    e = iy*nx + ix."""
    M = T.shape[-1]
    P = nx * ny
    Z = np.zeros((P * M, P * M), dtype=np.complex128)
    for t in range(P):
        ty, tx = divmod(t, nx)
        for s in range(P):
            sy, sx = divmod(s, nx)
            Z[t * M:(t + 1) * M, s * M:(s + 1) * M] = T[ty - sy + ny - 1, tx - sx + nx - 1]
    return Z


def matvec_entries(T: np.ndarray, nx: int, ny: int, x: np.ndarray, rows) -> np.ndarray:
    """(Z x)[n] for the unknowns n in rows (x of shape (N, R)): the sum over all
    source elements s and bases q of T[t - s][p][q] x[s*M + q], n = t*M + p."""
    M = T.shape[-1]
    P = nx * ny
    R = x.shape[1]
    xs = x.reshape(P, M, R)
    sy, sx = np.divmod(np.arange(P), nx)
    out = np.zeros((len(rows), R), dtype=np.complex128)
    for i, n in enumerate(rows):
        t, p = divmod(int(n), M)
        ty, tx = divmod(t, nx)
        blocks = T[ty - sy + ny - 1, tx - sx + nx - 1, p, :]        # (P, M): row p of every block
        out[i] = np.einsum("sq,sqr->r", blocks, xs)
    return out
