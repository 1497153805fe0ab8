"""Oracle: reference preconditioners and restarted GMRES on the dense matrix.

TEST INFRASTRUCTURE ONLY (see oracle/mom.py).  Used for iteration-count parity
and for the iterative-versus-direct check; the Z_p target itself is always the
LU result of oracle/mom.py.

Preconditioners (Sec. III-A):
* P_K, the block diagonal of Z on the lowest level (the element self blocks),
  each block LU-factorised (the older strategy, Table I first row);
* P_A, the block diagonal of Z^H Z (eq. (precondA)), taken here by brute force
  as the diagonal M x M blocks of the explicit product Z^H Z, each Cholesky
  factorised (P = L L^H); GMRES then runs on P^{-1} Z^H Z I = P^{-1} Z^H V.

PCG (Sec. II-C, the paper's own solver): conjugate gradients on the normal
equations Z^H Z I = Z^H V with the preconditioner P_A, stopped on the relative
residual of the split system of eq. (precond).

COCG (not in the paper; van der Vorst and Melissen, 1990): CG with the bilinear
form on the complex symmetric Z itself, preconditioned by the symmetric P_K.

GMRES(m) (the solver of the "new M1" configuration; the paper relies on
MATLAB's implementation and states none of its details, so this reading fixes
them): x0 = 0, Arnoldi with classical Gram-Schmidt applied twice (CGS2),
complex Givens rotations, stop a cycle as soon as the least-squares residual
|g_{j+1}| <= tol * ||b||, explicit residual recomputed at every restart.  The
verdict is taken on the explicit residual r = b - A x of the restart: converged
when ||r|| <= tol ||b||, or ||r|| <= 2 tol ||b|| after a cycle whose
least-squares residual met the tolerance (the two differ by rounding; a larger
gap means the Arnoldi relation was lost, and the solve restarts from r).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np
import scipy.linalg as sla

from . import mom


# --------------------------------------------------------------------------- preconditioners

def pk_factors(Z: np.ndarray, lat, dip):
    """LU factors of every element self block of Z."""
    P = mom.n_elements(lat)
    return [sla.lu_factor(mom.block(Z, lat, dip, e, e)) for e in range(P)]


def pk_apply(factors, x: np.ndarray, M: int) -> np.ndarray:
    y = np.empty_like(x)
    for e, f in enumerate(factors):
        y[e * M:(e + 1) * M] = sla.lu_solve(f, x[e * M:(e + 1) * M])
    return y


def pa_blocks(Z: np.ndarray, lat, dip) -> List[np.ndarray]:
    """Diagonal M x M blocks of Z^H Z by brute force: P_e = Z[:, cols_e]^H Z[:, cols_e]."""
    M = dip.nbases
    out = []
    for e in range(mom.n_elements(lat)):
        Zc = Z[:, e * M:(e + 1) * M]
        out.append(Zc.conj().T @ Zc)
    return out


def pa_factors(blocks):
    """Cholesky P_e = L L^H of each block (lower factor)."""
    return [sla.cho_factor(B, lower=True) for B in blocks]


def pa_apply(factors, x: np.ndarray, M: int) -> np.ndarray:
    y = np.empty_like(x)
    for e, f in enumerate(factors):
        y[e * M:(e + 1) * M] = sla.cho_solve(f, x[e * M:(e + 1) * M])
    return y


def refined_inverse(B: np.ndarray) -> np.ndarray:
    """Inverse of a small matrix in extended precision (numpy clongdouble, a
    64-bit significand on x86): the FP64 inverse refined by three Newton-Schulz
    steps X <- X (2 I - B X), each of which squares the residual I - B X."""
    Bl = B.astype(np.clongdouble)
    X = np.linalg.inv(B.astype(np.complex128)).astype(np.clongdouble)
    E = np.eye(B.shape[0], dtype=np.clongdouble)
    for _ in range(3):
        X = X @ (2 * E - Bl @ X)
    return X


def block_apply(inv, x: np.ndarray, M: int) -> np.ndarray:
    """y = blockdiag(inv) x with one M x M inverse per element."""
    y = np.empty_like(x)
    for e, X in enumerate(inv):
        y[e * M:(e + 1) * M] = X @ x[e * M:(e + 1) * M]
    return y


class PreconditionedSystem:
    """The system GMRES runs on, for one of the two strategies.

    'element_block':  A = P_K^{-1} Z,        b = P_K^{-1} V
    'normal_eq':      A = P^{-1} Z^H Z,      b = P^{-1} Z^H V

    extended=True runs the same system in numpy's extended precision
    (clongdouble): Z as given, every product and preconditioner block formed
    and applied with a 64-bit significand.  On the normal equations (condition
    number squared) the step at which a Krylov recurrence crosses tol depends
    on the arithmetic itself; the extended run stands in for exact arithmetic.
    """

    def __init__(self, Z: np.ndarray, lat, dip, kind: str, extended: bool = False):
        self.M = dip.nbases
        self.kind = kind
        self.extended = extended
        P = mom.n_elements(lat)
        M = self.M
        if extended:
            Zl = Z.astype(np.clongdouble)
            self.Z = Zl
            if kind == "element_block":
                inv = [refined_inverse(Zl[e * M:(e + 1) * M, e * M:(e + 1) * M]) for e in range(P)]
            elif kind == "normal_eq":
                inv = [refined_inverse(Zl[:, e * M:(e + 1) * M].conj().T @ Zl[:, e * M:(e + 1) * M])
                       for e in range(P)]
            else:
                raise ValueError(kind)
            self.pinv = lambda x: block_apply(inv, x, M)
            return
        self.Z = Z
        if kind == "element_block":
            self.f = pk_factors(Z, lat, dip)
            self.pinv = lambda x: pk_apply(self.f, x, self.M)
        elif kind == "normal_eq":
            self.f = pa_factors(pa_blocks(Z, lat, dip))
            self.pinv = lambda x: pa_apply(self.f, x, self.M)
        else:
            raise ValueError(kind)

    def apply(self, x: np.ndarray) -> np.ndarray:
        if self.kind == "element_block":
            return self.pinv(self.Z @ x)
        return self.pinv(self.Z.conj().T @ (self.Z @ x))

    def rhs(self, v: np.ndarray) -> np.ndarray:
        v = v.astype(self.Z.dtype)
        if self.kind == "element_block":
            return self.pinv(v)
        return self.pinv(self.Z.conj().T @ v)


# --------------------------------------------------------------------------- GMRES

def givens(h1: complex, h2: complex):
    """Complex rotation (c real, s complex) with c*h1 + s*h2 = r, -conj(s)*h1 + c*h2 = 0."""
    if h1 == 0:
        return 0.0, 1.0 + 0j
    t = np.sqrt(abs(h1) ** 2 + abs(h2) ** 2)
    c = abs(h1) / t
    s = (h1 / abs(h1)) * np.conj(h2) / t
    return c, s


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    converged: bool
    cycles: int
    history: List[float] = field(default_factory=list)   # |g_{j+1}| after every iteration
    arnoldi_ratio: List[float] = field(default_factory=list)  # ||w|| after / before orthogonalisation
    restart_residuals: List[float] = field(default_factory=list)


def gmres(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, restart: int = 50,
          tol: float = 1e-10, max_cycles: int = 400) -> GmresResult:
    n = b.shape[0]
    m = restart
    ct = b.dtype                       # complex128, or clongdouble for the extended-precision run
    x = np.zeros(n, dtype=ct)
    bnorm = np.linalg.norm(b)
    res = GmresResult(x, 0, False, 0)
    if bnorm == 0.0:
        res.converged = True
        return res
    r = b.copy()
    beta = np.linalg.norm(r)
    candidate = False
    for cycle in range(max_cycles + 1):
        res.restart_residuals.append(beta)
        if _accept(beta, bnorm, tol, candidate):
            res.converged = True
            break
        if cycle == max_cycles:
            break
        res.cycles = cycle + 1
        V = np.zeros((m + 1, n), dtype=ct)
        H = np.zeros((m + 1, m), dtype=ct)
        cs = np.zeros(m, dtype=bnorm.dtype)
        sn = np.zeros(m, dtype=ct)
        g = np.zeros(m + 1, dtype=ct)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = apply_A(V[j])
            wnorm0 = np.linalg.norm(w)
            # classical Gram-Schmidt, twice
            h = V[:j + 1].conj() @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1].conj() @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                a_, b_ = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a_ + sn[i] * b_
                H[i + 1, j] = -np.conj(sn[i]) * a_ + cs[i] * b_
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            res.iters += 1
            res.history.append(abs(g[j + 1]))
            res.arnoldi_ratio.append(hn / wnorm0 if wnorm0 > 0 else 0.0)
            k = j + 1
            if abs(g[j + 1]) <= tol * bnorm or hn == 0.0:
                break
            V[j + 1] = w / hn
        y = _back_substitute(H[:k, :k], g[:k])
        x = x + V[:k].T @ y
        candidate = abs(g[k]) <= tol * bnorm
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
    res.x = x
    return res


def _back_substitute(Rm: np.ndarray, g: np.ndarray) -> np.ndarray:
    """y = R^{-1} g for upper triangular R (k <= 63), in the dtype of R."""
    k = g.shape[0]
    y = np.zeros(k, dtype=Rm.dtype)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - Rm[i, i + 1:k] @ y[i + 1:k]) / Rm[i, i]
    return y


def _accept(beta: float, bnorm: float, tol: float, candidate: bool) -> bool:
    """Convergence verdict on the explicit residual of a restart."""
    return beta <= tol * bnorm or (candidate and beta <= 2.0 * tol * bnorm)


def _rotate_column(H, cs, sn, g, j):
    """Apply the previous rotations to column j of H, form rotation j, update g."""
    for i in range(j):
        a_, b_ = H[i, j], H[i + 1, j]
        H[i, j] = cs[i] * a_ + sn[i] * b_
        H[i + 1, j] = -np.conj(sn[i]) * a_ + cs[i] * b_
    cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
    H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
    H[j + 1, j] = 0.0
    g[j + 1] = -np.conj(sn[j]) * g[j]
    g[j] = cs[j] * g[j]


def gmres_dcgs2(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, restart: int = 50,
                tol: float = 1e-10, max_cycles: int = 400) -> GmresResult:
    """GMRES(m) with delayed classical Gram-Schmidt reorthogonalisation (DCGS2,
    Swirydowicz, Langou, Ananthan, Yang and Thomas, "Low synchronization
    Gram-Schmidt and GMRES algorithms", Numer. Linear Algebra Appl. 2021).

    The operator is applied to the candidate u_k (the once-projected, not yet
    reorthogonalised or normalised next vector).  One sweep then gives
    s = V^H u, z = V^H w, ||u||^2 and u^H w; the reorthogonalisation of u
    (coefficients s, norm nu = sqrt(||u||^2 - ||s||^2)) completes Hessenberg
    column k-1, and the projection of A v_k = (w - V Hbar s)/nu is obtained from
    z by the Arnoldi relation, so that one update sweep writes both v_k and the
    next candidate.  In exact arithmetic the iterates equal those of CGS2-GMRES;
    the stopping rule and x0 are the same as in gmres()."""
    n = b.shape[0]
    m = restart
    ct = b.dtype                       # complex128, or clongdouble for the extended-precision run
    x = np.zeros(n, dtype=ct)
    bnorm = np.linalg.norm(b)
    res = GmresResult(x, 0, False, 0)
    if bnorm == 0.0:
        res.converged = True
        return res
    r = b.copy()
    beta = np.linalg.norm(r)
    candidate = False
    for cycle in range(max_cycles + 1):
        res.restart_residuals.append(beta)
        if _accept(beta, bnorm, tol, candidate):
            res.converged = True
            break
        if cycle == max_cycles:
            break
        res.cycles = cycle + 1
        V = np.zeros((m + 1, n), dtype=ct)
        Hraw = np.zeros((m + 1, m), dtype=ct)    # unrotated Hessenberg
        Hrot = np.zeros((m + 1, m), dtype=ct)    # rotated copy (upper triangular part used)
        cs = np.zeros(m, dtype=bnorm.dtype)
        sn = np.zeros(m, dtype=ct)
        g = np.zeros(m + 1, dtype=ct)
        u = r / beta
        k = 0
        steps = 0
        av_norm = 1.0     # ||A v_{k-1}||, for the Arnoldi norm ratio diagnostic
        while True:
            w = apply_A(u) if k < m else None
            Vf = V[:k]
            s = Vf.conj() @ u
            alpha = np.vdot(u, u).real
            # nu^2 by Pythagoras: below 1e-12 alpha it has cancelled to rounding
            # noise, the candidate lies in span(V) (breakdown, the cycle ends)
            nu2 = alpha - np.vdot(s, s).real
            nu = np.sqrt(nu2) if nu2 > 1e-12 * alpha else 0.0
            if k == 0:
                g[0] = beta * nu
            else:
                Hraw[:k, k - 1] += s
                Hraw[k, k - 1] = nu
                Hrot[:k + 1, k - 1] = Hraw[:k + 1, k - 1]
                _rotate_column(Hrot, cs, sn, g, k - 1)
                res.iters += 1
                res.history.append(abs(g[k]))
                res.arnoldi_ratio.append(nu / av_norm if av_norm > 0 else 0.0)
                steps = k
                if abs(g[k]) <= tol * bnorm or nu == 0.0 or k == m:
                    break
            z = Vf.conj() @ w
            bet = np.vdot(u, w)
            V[k] = (u - Vf.T @ s) / nu
            t = Hraw[:k + 1, :k] @ s
            h = np.zeros(k + 1, dtype=ct)
            h[:k] = (z - t[:k]) / nu
            h[k] = ((bet - np.vdot(s, z)) / nu - t[k]) / nu
            c = t / nu + h
            u = w / nu - V[:k + 1].T @ c
            Hraw[:k + 1, k] = h
            av_norm = np.linalg.norm(u + V[:k + 1].T @ h)
            k += 1
        y = _back_substitute(Hrot[:steps, :steps], g[:steps])
        x = x + V[:steps].T @ y
        candidate = abs(g[steps]) <= tol * bnorm
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
    res.x = x
    return res


def gmres_all(system: PreconditionedSystem, V: np.ndarray, restart: int = 50, tol: float = 1e-10,
              max_cycles: int = 400, orth: str = "cgs2"):
    """Independent GMRES for every column of V; returns (I, per-RHS results)."""
    solver = gmres if orth == "cgs2" else gmres_dcgs2
    B = system.rhs(V)
    I = np.zeros_like(V)
    results = []
    for j in range(V.shape[1]):
        r = solver(system.apply, B[:, j], restart, tol, max_cycles)
        I[:, j] = r.x
        results.append(r)
    return I, results


# --------------------------------------------------------------------------- PCG

@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: List[float] = field(default_factory=list)   # split-system residual after each iteration


def pcg(apply_N: Callable[[np.ndarray], np.ndarray], apply_Pinv: Callable[[np.ndarray], np.ndarray],
        b: np.ndarray, tol: float = 1e-10, maxit: int = 20000) -> PCGResult:
    """Preconditioned conjugate gradients (Sec. II-C) for N x = b with N Hermitian
    positive definite (Z^H Z) and preconditioner P (P^{-1} applied by apply_Pinv).

    With P = L L^H these are the iterates of plain CG on the split system of
    eq. (precond), L^{-1} N L^{-H} w = L^{-1} b with x = L^{-H} w; the stop test
    is that system's relative residual, ||L^{-1} r|| / ||L^{-1} b|| =
    sqrt(r^H P^{-1} r / b^H P^{-1} b) <= tol, with x0 = 0.
    """
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_Pinv(r)
    p = z.copy()
    rho = np.real(np.vdot(r, z))
    rho0 = rho
    res = PCGResult(x=x, iters=0, converged=(rho0 == 0.0))
    if res.converged:
        return res
    for k in range(1, maxit + 1):
        q = apply_N(p)
        mu = np.real(np.vdot(p, q))
        alpha = rho / mu
        x += alpha * p
        r -= alpha * q
        z = apply_Pinv(r)
        rho_new = np.real(np.vdot(r, z))
        res.iters = k
        rel = np.sqrt(max(rho_new, 0.0) / rho0)
        res.relres.append(rel)
        if rel <= tol:
            res.converged = True
            break
        p = z + (rho_new / rho) * p
        rho = rho_new
    res.x = x
    return res


def pcg_all(Z: np.ndarray, lat, dip, V: np.ndarray, tol: float = 1e-10, maxit: int = 20000,
            extended: bool = False):
    """PCG on the normal equations Z^H Z I = Z^H V with P_A (diagonal blocks of
    Z^H Z, eq. (precondA)) for every column of V; returns (I, per-RHS results).
    extended=True: the same in clongdouble (see PreconditionedSystem)."""
    M = dip.nbases
    if extended:
        sysm = PreconditionedSystem(Z, lat, dip, "normal_eq", extended=True)
        Zx, pinv = sysm.Z, sysm.pinv
    else:
        f = pa_factors(pa_blocks(Z, lat, dip))
        Zx, pinv = Z, (lambda v: pa_apply(f, v, M))
    ZH = Zx.conj().T
    B = ZH @ V.astype(Zx.dtype)
    I = np.zeros_like(V)
    results = []
    for j in range(V.shape[1]):
        r = pcg(lambda v: ZH @ (Zx @ v), pinv, B[:, j], tol, maxit)
        I[:, j] = r.x
        results.append(r)
    return I, results


# --------------------------------------------------------------------------- COCG

@dataclass
class COCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: List[float] = field(default_factory=list)   # ||r|| / ||b|| after each iteration


def cocg(apply_A: Callable[[np.ndarray], np.ndarray], apply_Minv: Callable[[np.ndarray], np.ndarray],
         b: np.ndarray, tol: float = 1e-10, maxit: int = 20000) -> COCGResult:
    """Conjugate orthogonal conjugate gradients (van der Vorst and Melissen,
    IEEE Trans. Magn. 26, 1990) for A x = b with A complex symmetric (A = A^T)
    and a complex symmetric preconditioner M (M^{-1} applied by apply_Minv).

    Not part of the paper: an alternative Krylov solver for the symmetric MoM
    matrix.  It is preconditioned CG with the bilinear form u^T v in place of
    u^H v (for real symmetric positive definite A it is CG itself); x0 = 0,
    stop when ||r|| <= tol ||b||.
    """
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_Minv(r)
    p = z.copy()
    rho = r @ z                      # bilinear: no conjugation
    bn = np.linalg.norm(b)
    res = COCGResult(x=x, iters=0, converged=(bn == 0.0))
    if res.converged:
        return res
    for k in range(1, maxit + 1):
        q = apply_A(p)
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = apply_Minv(r)
        rho_new = r @ z
        res.iters = k
        rel = np.linalg.norm(r) / bn
        res.relres.append(rel)
        if rel <= tol:
            res.converged = True
            break
        p = z + (rho_new / rho) * p
        rho = rho_new
    res.x = x
    return res


def cocg_all(Z: np.ndarray, lat, dip, V: np.ndarray, tol: float = 1e-10, maxit: int = 20000):
    """COCG on Z I = V with the element-block preconditioner P_K for every
    column of V; returns (I, per-RHS results)."""
    M = dip.nbases
    f = pk_factors(Z, lat, dip)
    I = np.zeros_like(V)
    results = []
    for j in range(V.shape[1]):
        r = cocg(lambda v: Z @ v, lambda v: pk_apply(f, v, M), V[:, j], tol, maxit)
        I[:, j] = r.x
        results.append(r)
    return I, results
