"""Fine and coarse propagators (backward Euler) and the serial fine reference.

Section 3.1: the fine propagator F advances one coarse slice [T_n, T_{n+1}] by
J steps of size dt = dT/J; the coarse propagator G takes one step of size dT.
Section 5 (numerical results) uses backward Euler for both.  For the linear
problem u' = -A u + g one backward-Euler step of size tau is
    (I + tau A) w_new = w + tau g.
The reference solution is the fine solution computed serially over all slices
(remark after the problem statement in Section 2; Section 5).

Solves here are direct: banded Cholesky of the SPD matrix I + tau A (bandwidth
1 in 1D, n in 2D), factorised once per sample and step size.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.linalg import cho_solve_banded, cholesky_banded

from . import operator as op


class BESolver:
    """Direct solver for (I + tau A) x = b for one sample."""

    def __init__(self, dim: int, n: int, a: np.ndarray, tau: float):
        A = op.assemble(dim, n, a)
        Mt = sp.identity(A.shape[0], format="csr") + tau * A
        bw = op.bandwidth(dim, n)
        self.cf = cholesky_banded(op.to_upper_banded(Mt, bw), lower=False)
        self.tau = tau

    def solve(self, b: np.ndarray) -> np.ndarray:
        return cho_solve_banded((self.cf, False), b)


class Propagators:
    """F and G for one sample (Section 3.1), linear diffusion with source g."""

    def __init__(self, dim: int, n: int, a: np.ndarray, T: float, N: int, J: int, forcing: float):
        self.dim, self.n, self.a = dim, n, np.asarray(a, dtype=np.float64)
        self.dT = T / N
        self.dt = self.dT / J
        self.J = J
        self.Nx = n ** dim
        self.g = forcing * np.ones(self.Nx)
        self.fine_solver = BESolver(dim, n, self.a, self.dt)
        self.coarse_solver = BESolver(dim, n, self.a, self.dT)

    def F(self, v: np.ndarray) -> np.ndarray:
        """J backward-Euler steps of size dt from v."""
        w = np.array(v, dtype=np.float64, copy=True)
        for _ in range(self.J):
            w = self.fine_solver.solve(w + self.dt * self.g)
        return w

    def G(self, v: np.ndarray) -> np.ndarray:
        """One backward-Euler step of size dT from v."""
        return self.coarse_solver.solve(np.asarray(v, dtype=np.float64) + self.dT * self.g)


def serial_fine(props: Propagators, u0: np.ndarray, N: int) -> np.ndarray:
    """Reference solution u_n = F(u_{n-1}), n = 1..N; returns [N, Nx]."""
    out = np.empty((N, props.Nx))
    u = np.asarray(u0, dtype=np.float64)
    for k in range(N):
        u = props.F(u)
        out[k] = u
    return out


def coarse_sweep(props: Propagators, u0: np.ndarray, N: int) -> np.ndarray:
    """Sequential coarse solution U_n = G(U_{n-1}) (the COARSE initial guess)."""
    out = np.empty((N, props.Nx))
    u = np.asarray(u0, dtype=np.float64)
    for k in range(N):
        u = props.G(u)
        out[k] = u
    return out
