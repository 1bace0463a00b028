"""Parareal for the advection-diffusion example of Section 5.1 (P1 elements, fem.py).

Time stepping (Section 5.1: backward Euler for F and G).  One step of size tau that ends at
time t solves
    (M + tau L) w_new = M w + tau F(t),   L = a K + B.
  F on slice s (from T_s = s dT to T_{s+1}, dT = T/N): J steps of dt = dT/J, step j ending at
    t = T_s + (j+1) dt;
  G on slice s: one step of dT ending at T_{s+1}.
The reference solution is the serial fine solution u_{s+1} = F_s(u_s), u_0 the initial value.

Algorithm 1 (sequential CGC, "standard parareal"):
    U^{k+1}_1 = F_0(u_0),  U^{k+1}_{s+1} = G_s(U^{k+1}_s) + F_s(U^k_s) - G_s(U^k_s).
Algorithms 2/3 (diagonalised CGC, Section 3.2).  With the mass matrix the coarse problem of
eq. guodu reads, for the stacked unknown u = (U_1, ..., U_N),
    (C_alpha (x) M + dT I (x) L) u = r,   r_s = (M + dT L) F_s - M z_s,
z_0 = alpha U^k_N, z_s = U^k_s (s >= 1), F_s the fine result of slice s (from u_0 on the
first slice); the forcing of G cancels (it enters b^k and the coarse solve alike).  It is
solved by the three steps of eq. three-steps with M in place of I:
    (a) p = (F_N^* (x) I)(Lambda_alpha (x) I) r,
    (b) (lambda_k M + dT L) q_k = p_k,
    (c) u = (Lambda_alpha^{-1} (x) I)(F_N (x) I) q,
lambda_k, Lambda_alpha and F_N as for the finite-difference problem (cgc.py), F_N applied as
a dense matrix and every shifted system by a sparse LU.  The stop rule is the increment of
parareal.increment; the error against the serial fine solution is recorded per iteration.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import cgc
from .fem import Discretisation


class ADEPropagators:
    """F and G for one sample of the Section 5.1 problem."""

    def __init__(self, disc: Discretisation, a: float, T: float, N: int, J: int):
        self.disc, self.a = disc, float(a)
        self.N, self.J = N, J
        self.dT = T / N
        self.dt = self.dT / J
        self.L = disc.operator(self.a)
        self.fine_lu = spla.splu((disc.M + self.dt * self.L).tocsc())
        self.coarse_lu = spla.splu((disc.M + self.dT * self.L).tocsc())

    def F(self, v: np.ndarray, s: int) -> np.ndarray:
        """J backward-Euler steps of dt over slice s from v."""
        w = np.array(v, dtype=np.float64, copy=True)
        t0 = s * self.dT
        for j in range(self.J):
            t = t0 + (j + 1) * self.dt
            w = self.fine_lu.solve(self.disc.M @ w + self.dt * self.disc.load(self.a, t))
        return w

    def G(self, v: np.ndarray, s: int) -> np.ndarray:
        """One backward-Euler step of dT over slice s from v."""
        t = (s + 1) * self.dT
        return self.coarse_lu.solve(self.disc.M @ np.asarray(v, dtype=np.float64)
                                    + self.dT * self.disc.load(self.a, t))


def serial_fine(props: ADEPropagators, u0: np.ndarray) -> np.ndarray:
    """Reference solution [N, Nx]."""
    out = np.empty((props.N, props.disc.Nx))
    u = np.asarray(u0, dtype=np.float64)
    for s in range(props.N):
        u = props.F(u, s)
        out[s] = u
    return out


def coarse_sweep(props: ADEPropagators, u0: np.ndarray) -> np.ndarray:
    """U_{s+1} = G_s(U_s) from u0 (the coarse initial guess)."""
    out = np.empty((props.N, props.disc.Nx))
    u = np.asarray(u0, dtype=np.float64)
    for s in range(props.N):
        u = props.G(u, s)
        out[s] = u
    return out


class ADEDiagSolver:
    """Steps (a)-(c) for (C_alpha (x) M + dT I (x) L) u = r, one sample; the shifted
    matrices are factorised once each and reused."""

    def __init__(self, props: ADEPropagators, alpha: float):
        N = props.N
        self.props = props
        self.FN = cgc.dft_matrix(N)
        self.Lam = cgc.scaling(N, alpha)
        self.lam = cgc.eigenvalues(N, alpha)
        self.M = props.disc.M.astype(np.complex128)
        self.dTL = (props.dT * props.L).astype(np.complex128)
        self.lu = [None] * N

    def solve(self, r: np.ndarray) -> np.ndarray:
        p = self.FN.conj().T @ (self.Lam[:, None] * r)                          # step (a)
        q = np.empty_like(p)
        for k in range(self.props.N):                                           # step (b)
            if self.lu[k] is None:
                self.lu[k] = spla.splu((self.lam[k] * self.M + self.dTL).tocsc())
            q[k] = self.lu[k].solve(p[k])
        u = (1.0 / self.Lam)[:, None] * (self.FN @ q)                             # step (c)
        scale = max(np.abs(u.real).max(), 1e-300)
        assert np.abs(u.imag).max() <= 1e-8 * scale, "diagonalised CGC lost conjugate symmetry"
        return u.real


def all_at_once_matrix(props: ADEPropagators, alpha: float) -> sp.csr_matrix:
    """C_alpha (x) M + dT I (x) L (for brute-force checks)."""
    N = props.N
    return (sp.kron(sp.csr_matrix(cgc.c_alpha(N, alpha)), props.disc.M)
            + props.dT * sp.kron(sp.identity(N), props.L)).tocsr()


def cgc_rhs(props: ADEPropagators, alpha: float, U: np.ndarray, Fv: np.ndarray) -> np.ndarray:
    """r_s = (M + dT L) F_s - M z_s, z_0 = alpha U_N, z_s = U_s."""
    M = props.disc.M
    A = (M + props.dT * props.L).tocsr()
    z = np.concatenate([alpha * U[-1:], U[:-1]], axis=0)
    return (A @ Fv.T).T - (M @ z.T).T


@dataclasses.dataclass
class ADEHistory:
    iters: int
    deltas: list
    errors: list          # [iteration][slice] |u_s - U^k_s|_inf for k = 0..iters (if ref given)
    U: np.ndarray


def _errors(U, ref):
    return None if ref is None else np.abs(U - ref).max(axis=1)


def parareal_diag(props: ADEPropagators, alpha: float, u0: np.ndarray, U0: np.ndarray,
                  tol: float, max_iter: int, ref: np.ndarray | None = None) -> ADEHistory:
    """Algorithms 2/3 (U0 is the initial guess); tol = 0 runs exactly max_iter iterations."""
    U = np.array(U0, dtype=np.float64, copy=True)
    solver = ADEDiagSolver(props, alpha)
    deltas, errs = [], [_errors(U, ref)]
    k = 0
    while k < max_iter:
        starts = [u0] + [U[s - 1] for s in range(1, props.N)]
        Fv = np.stack([props.F(v, s) for s, v in enumerate(starts)])
        Unew = solver.solve(cgc_rhs(props, alpha, U, Fv))
        den = np.abs(Unew).max()
        delta = float(np.abs(Unew - U).max() / (den if den > 0 else 1.0))
        deltas.append(delta)
        U = Unew
        k += 1
        errs.append(_errors(U, ref))
        if tol > 0 and delta <= tol:
            break
    return ADEHistory(k, deltas, errs if ref is not None else [], U)


def parareal_sequential(props: ADEPropagators, u0: np.ndarray, U0: np.ndarray,
                        tol: float, max_iter: int, ref: np.ndarray | None = None) -> ADEHistory:
    """Algorithm 1; tol = 0 runs exactly max_iter iterations."""
    U = np.array(U0, dtype=np.float64, copy=True)
    deltas, errs = [], [_errors(U, ref)]
    k = 0
    while k < max_iter:
        starts = [u0] + [U[s - 1] for s in range(1, props.N)]
        Fv = [props.F(v, s) for s, v in enumerate(starts)]
        Gold = [props.G(v, s) for s, v in enumerate(starts)]
        Unew = np.empty_like(U)
        prev = np.asarray(u0, dtype=np.float64)
        for s in range(props.N):
            Unew[s] = props.G(prev, s) + Fv[s] - Gold[s]
            prev = Unew[s]
        den = np.abs(Unew).max()
        delta = float(np.abs(Unew - U).max() / (den if den > 0 else 1.0))
        deltas.append(delta)
        U = Unew
        k += 1
        errs.append(_errors(U, ref))
        if tol > 0 and delta <= tol:
            break
    return ADEHistory(k, deltas, errs if ref is not None else [], U)
