"""Nonlinear problems of Sections 5.2 and 5.3 and the Newton form of the coarse grid correction
(Section 3.2, eq. Newton, eq. Jac, eq. Newton2).

Semi-discrete problems u' = f(u) (autonomous, so the time argument of f in eq. guodu plays no
role):
  Burgers (Section 5.2): u_t + u u_x = (eps/50) u_xx on (0, 1), u = 0 at both ends; n interior
    nodes x_i = i h, h = 1/(n+1); central differences for u_xx and first-order upwinding for
    the convective term, chosen by the sign of u_i:
        f_i = nu (u_{i+1} - 2 u_i + u_{i-1}) / h^2 - u_i (u_i - u_{i-1}) / h   (u_i >= 0)
        f_i = nu (u_{i+1} - 2 u_i + u_{i-1}) / h^2 - u_i (u_{i+1} - u_i) / h   (u_i < 0)
    nu = eps / 50.  Reading: the paper does not give u_0; u_0(x) = sin(pi x) is taken.
  Allen-Cahn (Section 5.3): u_t - eps u_xx + u^3 - u = 0 on (-1, 1), u(-1) = -1, u(1) = 1;
    nodes x_i = -1 + i h, h = 2/(n+1) (h = 1/128 gives n = 255); central differences,
        f_i = eps (u_{i+1} - 2 u_i + u_{i-1}) / h^2 - (u_i^3 - u_i),
    with the boundary values in the end rows; u_0(x) = 0.53 x + 0.47 sin(-1.5 pi x).
Both Jacobians are tridiagonal; the upwind term is differentiated on the branch chosen at the
evaluation point.

Backward Euler (F: J steps of dt, G: one step of dT) solves w - tau f(w) = v by Newton's
method with the exact Jacobian, started from v; the iteration stops when
|dw|_inf <= newton_tol max(|w|_inf, 1) or after newton_max steps, keeping the last iterate
(reading of "solve"; the paper names no tolerance, and where the upwind branch switches at
u_i = 0 Newton can cycle at rounding level instead of converging).

Coarse grid correction (Algorithm 2 step 2) for nonlinear f.  With b_1 = F_1 - G(alpha U^k_N),
b_n = F_n - G(U^k_{n-1}) the new iterate u = (U_1, .., U_N) solves eq. matrix_NT,
    (C_alpha (x) I) u = dT Ft(u) + b,   Ft(u)_n = f(U_n - b_n),
by the simplified Newton iteration of eq. Newton2 with the averaged Jacobian of eq. Jac,
    Jbar = (1/N) sum_n grad f(U_{n,l} - b_n),
    (C_alpha (x) I - dT I (x) Jbar) u_{l+1} = -dT (I (x) Jbar) u_l + dT Ft(u_l) + b,
each step by the three steps of eq. three-steps with lambda_n I - dT Jbar as the shifted
matrices (dense DFT over slices, banded LU with pivoting per shifted system).  Readings:
u_0 = U^k; stop when |u_{l+1} - u_l|_inf <= newton_tol max(|u_{l+1}|_inf, 1) or after
newton_max_iter steps.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.linalg import solve_banded

from . import cgc


class Burgers:
    """f and its Jacobian for the upwind Burgers discretisation (Section 5.2)."""

    def __init__(self, n: int, eps: float):
        self.n = n
        self.h = 1.0 / (n + 1)
        self.nu = eps / 50.0
        self.x = np.arange(1, n + 1) * self.h

    def initial_value(self) -> np.ndarray:
        return np.sin(np.pi * self.x)

    def f(self, u: np.ndarray) -> np.ndarray:
        h, nu = self.h, self.nu
        up = np.concatenate([[0.0], u, [0.0]])
        lap = (up[2:] - 2 * up[1:-1] + up[:-2]) / h ** 2
        back = (up[1:-1] - up[:-2]) / h
        fwd = (up[2:] - up[1:-1]) / h
        conv = np.where(u >= 0, u * back, u * fwd)
        return nu * lap - conv

    def jacobian(self, u: np.ndarray):
        """(lower, diag, upper): d f_i / d u_{i-1}, d u_i, d u_{i+1} (lower[0], upper[-1] unused)."""
        h, nu = self.h, self.nu
        up = np.concatenate([[0.0], u, [0.0]])
        pos = u >= 0
        lower = np.full(self.n, nu / h ** 2) + np.where(pos, u / h, 0.0)
        upper = np.full(self.n, nu / h ** 2) - np.where(pos, 0.0, u / h)
        diag = -2 * nu / h ** 2 - np.where(pos, (2 * u - up[:-2]) / h, (up[2:] - 2 * u) / h)
        return lower, diag, upper


class AllenCahn:
    """f and its Jacobian for the Allen-Cahn discretisation (Section 5.3)."""

    def __init__(self, n: int, eps: float):
        self.n = n
        self.h = 2.0 / (n + 1)
        self.eps = eps
        self.x = -1.0 + np.arange(1, n + 1) * self.h

    def initial_value(self) -> np.ndarray:
        return 0.53 * self.x + 0.47 * np.sin(-1.5 * np.pi * self.x)

    def f(self, u: np.ndarray) -> np.ndarray:
        up = np.concatenate([[-1.0], u, [1.0]])
        lap = (up[2:] - 2 * up[1:-1] + up[:-2]) / self.h ** 2
        return self.eps * lap - (u ** 3 - u)

    def jacobian(self, u: np.ndarray):
        c = self.eps / self.h ** 2
        return np.full(self.n, c), -2 * c - (3 * u ** 2 - 1), np.full(self.n, c)

    def energy(self, u: np.ndarray) -> float:
        """E_h(u) = (eps/2) sum_cells h ((u_{i+1} - u_i)/h)^2 + h sum_nodes (u_i^2 - 1)^2 / 4."""
        up = np.concatenate([[-1.0], u, [1.0]])
        grad = np.diff(up) / self.h
        return float(0.5 * self.eps * self.h * np.sum(grad ** 2) + self.h * np.sum((u ** 2 - 1) ** 2) / 4)


MODELS = {2: Burgers, 3: AllenCahn}


def tri_solve(lower, diag, upper, rhs):
    """Solve the tridiagonal system (LU with partial pivoting, LAPACK gbsv)."""
    n = len(diag)
    ab = np.zeros((3, n), dtype=np.result_type(lower, diag, upper, rhs))
    ab[0, 1:] = upper[:-1]
    ab[1] = diag
    ab[2, :-1] = lower[1:]
    return solve_banded((1, 1), ab, rhs)


def be_step(prob, v: np.ndarray, tau: float, newton_tol: float, newton_max: int):
    """w - tau f(w) = v by Newton from w = v; returns (w, Newton steps)."""
    w = np.array(v, dtype=np.float64, copy=True)
    for it in range(1, newton_max + 1):
        r = w - tau * prob.f(w) - v
        lo, di, up = prob.jacobian(w)
        dw = tri_solve(-tau * lo, 1.0 - tau * di, -tau * up, -r)
        w = w + dw
        if np.abs(dw).max() <= newton_tol * max(np.abs(w).max(), 1.0):
            return w, it
    return w, newton_max


class NLPropagators:
    """F (J steps of dt) and G (one step of dT) for one sample."""

    def __init__(self, model, n: int, eps: float, T: float, N: int, J: int,
                 newton_tol: float = 1e-13, newton_max: int = 50):
        # model: 2 (Burgers), 3 (Allen-Cahn), or a problem object with n, f, jacobian
        self.prob = MODELS[model](n, eps) if isinstance(model, int) else model
        self.N, self.J = N, J
        self.dT = T / N
        self.dt = self.dT / J
        self.tol, self.max = newton_tol, newton_max

    def F(self, v):
        w = np.asarray(v, dtype=np.float64)
        for _ in range(self.J):
            w, _ = be_step(self.prob, w, self.dt, self.tol, self.max)
        return w

    def G(self, v):
        return be_step(self.prob, np.asarray(v, dtype=np.float64), self.dT, self.tol, self.max)[0]


def serial_fine(P: NLPropagators, u0) -> np.ndarray:
    out = np.empty((P.N, P.prob.n))
    u = np.asarray(u0, dtype=np.float64)
    for s in range(P.N):
        u = P.F(u)
        out[s] = u
    return out


def coarse_sweep(P: NLPropagators, u0) -> np.ndarray:
    out = np.empty((P.N, P.prob.n))
    u = np.asarray(u0, dtype=np.float64)
    for s in range(P.N):
        u = P.G(u)
        out[s] = u
    return out


def cgc_b(P: NLPropagators, alpha: float, U: np.ndarray, Fv: np.ndarray) -> np.ndarray:
    """b^k of Section 3.2: b_1 = F_1 - G(alpha U_N), b_n = F_n - G(U_{n-1})."""
    b = np.empty_like(U)
    b[0] = Fv[0] - P.G(alpha * U[-1])
    for s in range(1, P.N):
        b[s] = Fv[s] - P.G(U[s - 1])
    return b


def all_at_once_residual(P: NLPropagators, alpha: float, u: np.ndarray, b: np.ndarray) -> np.ndarray:
    """(C_alpha (x) I) u - dT Ft(u) - b of eq. matrix_NT."""
    z = np.concatenate([alpha * u[-1:], u[:-1]], axis=0)
    Ft = np.stack([P.prob.f(u[s] - b[s]) for s in range(P.N)])
    return u - z - P.dT * Ft - b


def newton_cgc(P: NLPropagators, alpha: float, U: np.ndarray, b: np.ndarray):
    """eq. Newton2 with the averaged Jacobian, from u_0 = U; returns (u, Newton steps)."""
    N, n, dT = P.N, P.prob.n, P.dT
    FN, Lam, lam = cgc.dft_matrix(N), cgc.scaling(N, alpha), cgc.eigenvalues(N, alpha)
    u = np.array(U, dtype=np.float64, copy=True)
    for it in range(1, P.max + 1):
        jac = [P.prob.jacobian(u[s] - b[s]) for s in range(N)]
        jl = sum(j[0] for j in jac) / N
        jd = sum(j[1] for j in jac) / N
        ju = sum(j[2] for j in jac) / N
        Ft = np.stack([P.prob.f(u[s] - b[s]) for s in range(N)])
        Ju = np.stack([jd * u[s] + jl * np.concatenate([[0.0], u[s, :-1]]) + ju * np.concatenate([u[s, 1:], [0.0]])
                       for s in range(N)])
        r = -dT * Ju + dT * Ft + b
        p = FN.conj().T @ (Lam[:, None] * r)                                       # step (a)
        q = np.stack([tri_solve(-dT * jl + 0j, lam[k] - dT * jd, -dT * ju + 0j, p[k])   # step (b)
                      for k in range(N)])
        unew = ((1.0 / Lam)[:, None] * (FN @ q)).real                               # step (c)
        done = np.abs(unew - u).max() <= P.tol * max(np.abs(unew).max(), 1.0)
        u = unew
        if done:
            return u, it
    return u, P.max


@dataclasses.dataclass
class NLHistory:
    iters: int
    deltas: list
    errors: list
    newton: list
    U: np.ndarray


def _errs(U, ref):
    return None if ref is None else np.abs(U - ref).max(axis=1)


def parareal_diag(P: NLPropagators, alpha: float, u0, U0, tol: float, max_iter: int, ref=None) -> NLHistory:
    """Algorithm 2 for nonlinear f (U0 the initial guess); tol = 0 runs max_iter iterations."""
    U = np.array(U0, dtype=np.float64, copy=True)
    deltas, errs, newton = [], [_errs(U, ref)], []
    k = 0
    while k < max_iter:
        starts = [u0] + [U[s - 1] for s in range(1, P.N)]
        Fv = np.stack([P.F(v) for v in starts])
        b = cgc_b(P, alpha, U, Fv)
        Unew, its = newton_cgc(P, alpha, U, b)
        newton.append(its)
        den = np.abs(Unew).max()
        delta = float(np.abs(Unew - U).max() / (den if den > 0 else 1.0))
        deltas.append(delta)
        U = Unew
        k += 1
        errs.append(_errs(U, ref))
        if tol > 0 and delta <= tol:
            break
    return NLHistory(k, deltas, errs if ref is not None else [], newton, U)


def parareal_sequential(P: NLPropagators, u0, U0, tol: float, max_iter: int, ref=None) -> NLHistory:
    """Algorithm 1 for nonlinear f; tol = 0 runs max_iter iterations."""
    U = np.array(U0, dtype=np.float64, copy=True)
    deltas, errs = [], [_errs(U, ref)]
    k = 0
    while k < max_iter:
        starts = [u0] + [U[s - 1] for s in range(1, P.N)]
        Fv = [P.F(v) for v in starts]
        Gold = [P.G(v) for v in starts]
        Unew = np.empty_like(U)
        prev = np.asarray(u0, dtype=np.float64)
        for s in range(P.N):
            Unew[s] = P.G(prev) + Fv[s] - Gold[s]
            prev = Unew[s]
        den = np.abs(Unew).max()
        delta = float(np.abs(Unew - U).max() / (den if den > 0 else 1.0))
        deltas.append(delta)
        U = Unew
        k += 1
        errs.append(_errs(U, ref))
        if tol > 0 and delta <= tol:
            break
    return NLHistory(k, deltas, errs if ref is not None else [], [], U)


def rho_nonlinear(alpha: float, L: float, dT: float) -> float:
    """rho(alpha) of Theorem 4.3 (one-sided Lipschitz constant L)."""
    x = L * dT
    g = 1.0 / (1.0 + x)
    return max(abs(alpha) * (1.0 + np.exp(-x)) / x, (np.exp(-x) + g) / (1.0 - g))
