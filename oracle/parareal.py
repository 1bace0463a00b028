"""Parareal with sequential CGC (Algorithm 1) and with diagonalised CGC
(Algorithms 2 and 3), for one sample, in FP64.

Algorithm 1: U_0 = u_0; for k = 0, 1, ...
    F_n = F(U_{n-1}^k)                            (step 1, parallel over n)
    U_n^{k+1} = G(U_{n-1}^{k+1}) + F_n - G(U_{n-1}^k)   (step 2, eq. pred_correc)
Algorithm 2 (parallel CGC): step 1 runs F from u_0 on the first slice and from
U_{n-1}^k elsewhere; step 2 solves the coupled coarse problem with
U_0^{k+1} = alpha U_N^{k+1}, which is the all-at-once system of eq.
matrix_NT with b_1 = F_1 - G(alpha U_N^k), b_n = F_n - G(U_{n-1}^k) (the
stacked vector b^k of Section 3.2).  For linear f, r = (I + dT A) b + dT g and
the system is solved by the three diagonalised steps (cgc.diag_solve).
Step 3 (reading of "stopping criterion"): stop when the FP64 increment
delta^{k+1} = max_n |U_n^{k+1} - U_n^k|_inf / max_n |U_n^{k+1}|_inf <= tol,
or at max_iter.  The error against the serial fine solution is recorded
(the per-slice error vectors of Section 5) but never used to stop.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import cgc
from . import operator as op
from .prop import Propagators


@dataclasses.dataclass
class History:
    iters: int
    deltas: list
    iterates: list          # U^k for k = 0..iters ([N, Nx] each), if kept
    converged: bool


def increment(U_new: np.ndarray, U_old: np.ndarray) -> float:
    den = np.abs(U_new).max()
    return float(np.abs(U_new - U_old).max() / (den if den > 0 else 1.0))


def parareal_sequential(props: Propagators, u0: np.ndarray, U0: np.ndarray, n_iter: int) -> list:
    """Algorithm 1 for exactly n_iter iterations; returns [U^0, ..., U^n_iter]."""
    N = U0.shape[0]
    U = np.array(U0, dtype=np.float64, copy=True)
    out = [U.copy()]
    for _ in range(n_iter):
        starts = [u0] + [U[k - 1] for k in range(1, N)]
        Fv = [props.F(s) for s in starts]
        Gold = [props.G(s) for s in starts]
        Unew = np.empty_like(U)
        prev = np.asarray(u0, dtype=np.float64)
        for k in range(N):
            Unew[k] = props.G(prev) + Fv[k] - Gold[k]
            prev = Unew[k]
        U = Unew
        out.append(U.copy())
    return out


def cgc_rhs(props: Propagators, alpha: float, U: np.ndarray, Fv: np.ndarray) -> np.ndarray:
    """r^k = (I + dT A) b^k + dT g with b^k of Section 3.2 (linear flux)."""
    N = U.shape[0]
    A = op.assemble(props.dim, props.n, props.a)
    b = np.empty_like(U)
    b[0] = Fv[0] - props.G(alpha * U[N - 1])
    for k in range(1, N):
        b[k] = Fv[k] - props.G(U[k - 1])
    return b + props.dT * (A @ b.T).T + props.dT * props.g[None, :]


def parareal_diag(props: Propagators, alpha: float, u0: np.ndarray, U0: np.ndarray,
                  tol: float, max_iter: int, keep: bool = False, fixed_iters: int | None = None) -> History:
    """Algorithms 2/3 (the initial guess U0 is an argument)."""
    N = U0.shape[0]
    U = np.array(U0, dtype=np.float64, copy=True)
    its = [U.copy()] if keep else []
    deltas = []
    converged = False
    k = 0
    n_max = fixed_iters if fixed_iters is not None else max_iter
    solver = cgc.DiagSolver(props.dim, props.n, props.a, props.dT, alpha, N)
    while k < n_max:
        starts = [u0] + [U[j - 1] for j in range(1, N)]
        Fv = np.stack([props.F(s) for s in starts])
        r = cgc_rhs(props, alpha, U, Fv)
        Unew = solver.solve(r)
        delta = increment(Unew, U)
        deltas.append(delta)
        U = Unew
        k += 1
        if keep:
            its.append(U.copy())
        if fixed_iters is None and delta <= tol:
            converged = True
            break
    return History(k, deltas, its if keep else [U], converged)


def per_slice_error(U: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """||u_n - U_n||_inf per slice (one sample's term of the Section 5 metrics)."""
    return np.abs(U - ref).max(axis=1)


def relative_error(U: np.ndarray, ref: np.ndarray) -> float:
    return float(np.abs(U - ref).max() / np.abs(ref).max())
