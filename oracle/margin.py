"""Oracle: arrays whose impedance matrix has a non-MBT margin (Sec. II-A
eq. (Zblock)), their normal equations (Sec. II-B eq. (Z2)) and the block
preconditioner of Sec. III-A (eq. (precond)).

TEST INFRASTRUCTURE ONLY (see oracle/mom.py).  Plain definitions:

* Z = [[Z_A, Z_B^T], [Z_B, Z_C]], Z_A the multilevel block-Toeplitz interaction
  of the P = nx*ny elements (N_A = P*M unknowns, assembled from its unique
  blocks), Z_B (N_C x N_A) the element-margin coupling and Z_C (N_C x N_C) the
  margin's own interaction; the margin unknowns follow the element unknowns;
* the all-port system Z I = V with unit delta gaps at the element ports (the
  margin carries no port), solved by LAPACK LU;
* P = blkdiag(P_A, P_C): P_A the diagonal M x M blocks of Z_A^H Z_A (Sec. III-A
  leaves the Z_B^H Z_B part of the upper-left block of eq. (Z2) out of the
  preconditioner), P_C = Z_B^* Z_B^T + Z_C^H Z_C, each Cholesky factorised; the
  normal-equation strategy runs GMRES or PCG on P^{-1} Z^H Z I = P^{-1} Z^H V;
* the element-block fallback P_K = blkdiag(T[0], ..., T[0], Z_C), LU factorised.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import blocks as ob


def dense(T: np.ndarray, nx: int, ny: int, ZB: np.ndarray, ZC: np.ndarray) -> np.ndarray:
    """The whole matrix of eq. (Zblock)."""
    ZA = ob.dense_from_blocks(T, nx, ny)
    return np.block([[ZA, ZB.T], [ZB, ZC]])


def excitation(nx: int, ny: int, M: int, nc: int, ports) -> np.ndarray:
    """Unit delta gap at basis (M-1)/2 of each listed element; zero on the margin."""
    ports = np.asarray(ports)
    V = np.zeros((nx * ny * M + nc, len(ports)), dtype=np.complex128)
    V[ports * M + (M - 1) // 2, np.arange(len(ports))] = 1.0
    return V


def pa_blocks(ZA: np.ndarray, P: int, M: int):
    """Diagonal M x M blocks of Z_A^H Z_A by brute force."""
    return [ZA[:, e * M:(e + 1) * M].conj().T @ ZA[:, e * M:(e + 1) * M] for e in range(P)]


def pc_block(ZB: np.ndarray, ZC: np.ndarray) -> np.ndarray:
    """P_C = Z_B^* Z_B^T + Z_C^H Z_C (eq. (precond))."""
    return ZB.conj() @ ZB.T + ZC.conj().T @ ZC


class MarginSystem:
    """The system a Krylov solver runs on for a margin array.

    'normal_eq':      A = P^{-1} Z^H Z, b = P^{-1} Z^H V, P = blkdiag(P_A, P_C)
    'element_block':  A = P_K^{-1} Z,   b = P_K^{-1} V,   P_K = blkdiag(T[0] ..., Z_C)
    """

    def __init__(self, T: np.ndarray, nx: int, ny: int, ZB: np.ndarray, ZC: np.ndarray, kind: str):
        self.M = T.shape[-1]
        self.P = nx * ny
        self.NA = self.P * self.M
        self.kind = kind
        self.Z = dense(T, nx, ny, ZB, ZC)
        ZA = self.Z[:self.NA, :self.NA]
        if kind == "normal_eq":
            self.fa = [sla.cho_factor(B, lower=True) for B in pa_blocks(ZA, self.P, self.M)]
            self.fc = sla.cho_factor(pc_block(ZB, ZC), lower=True)
            solve = sla.cho_solve
        elif kind == "element_block":
            self.fa = [sla.lu_factor(T[ny - 1, nx - 1])] * self.P
            self.fc = sla.lu_factor(ZC)
            solve = sla.lu_solve
        else:
            raise ValueError(kind)
        self._solve = solve

    def pinv(self, x: np.ndarray) -> np.ndarray:
        y = np.empty_like(x)
        M = self.M
        for e, f in enumerate(self.fa):
            y[e * M:(e + 1) * M] = self._solve(f, x[e * M:(e + 1) * M])
        y[self.NA:] = self._solve(self.fc, x[self.NA:])
        return y

    def apply(self, x: np.ndarray) -> np.ndarray:
        if self.kind == "element_block":
            return self.pinv(self.Z @ x)
        return self.pinv(self.Z.conj().T @ (self.Z @ x))

    def rhs(self, v: np.ndarray) -> np.ndarray:
        if self.kind == "element_block":
            return self.pinv(v)
        return self.pinv(self.Z.conj().T @ v)
