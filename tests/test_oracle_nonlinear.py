"""Pins of the oracle's nonlinear problems (Sections 5.2, 5.3) and of the Newton coarse grid
correction with the averaged Jacobian (Section 3.2, eq. Newton2; Theorem 4.3).

Independent checks: the Jacobians against central finite differences (both upwind branches);
consistency of the discrete right-hand sides with the differential operators at first
(upwind) and second (central) order; the backward-Euler Newton residual; small-amplitude
Burgers against the linear heat step; the discrete Allen-Cahn energy decays along the serial
fine solution (the property Section 5.3 checks); the Newton CGC lands on a root of the
all-at-once system of eq. matrix_NT, the same one a full-Jacobian Newton on the dense system
finds; the serial fine solution is the fixed point of Algorithm 2; Algorithm 1 terminates at
k = N; and on a scalar dissipative problem the error contracts by no more than rho(alpha) of
Theorem 4.3 per iteration.
"""
import numpy as np
import pytest

from oracle import nonlinear as nl


def _fd_jacobian(prob, u, eps=1e-6):
    n = len(u)
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = eps
        J[:, j] = (prob.f(u + e) - prob.f(u - e)) / (2 * eps)
    return J


@pytest.mark.parametrize("cls,eps", [(nl.Burgers, 1.7), (nl.AllenCahn, 0.3)])
def test_jacobian_matches_finite_differences(cls, eps):
    n = 12
    prob = cls(n, eps)
    rng = np.random.default_rng(0)
    u = rng.uniform(-0.8, 0.8, n)
    u[np.abs(u) < 0.05] = 0.3          # keep the upwind branch fixed inside the stencil
    lo, di, up = prob.jacobian(u)
    J = np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
    Jfd = _fd_jacobian(prob, u)
    assert np.abs(J - Jfd).max() < 1e-6 * np.abs(J).max()


def test_burgers_consistent_first_order():
    errs = []
    for n in [99, 999]:
        p = nl.Burgers(n, 2.0)
        u = np.sin(np.pi * p.x)
        exact = p.nu * (-np.pi ** 2 * u) - u * np.pi * np.cos(np.pi * p.x)
        errs.append(np.abs(p.f(u) - exact).max())
    assert 7 < errs[0] / errs[1] < 13


def test_allen_cahn_consistent_second_order():
    errs = []
    for n in [63, 127]:
        p = nl.AllenCahn(n, 0.5)
        u = np.sin(np.pi * p.x / 2)
        exact = -0.5 * (np.pi / 2) ** 2 * u - (u ** 3 - u)
        errs.append(np.abs(p.f(u) - exact).max())
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.parametrize("model", [2, 3])
def test_be_step_residual(model):
    prob = nl.MODELS[model](31, 1.0 if model == 2 else 0.2)
    v = prob.initial_value()
    w, its = nl.be_step(prob, v, 0.05, 1e-13, 50)
    assert np.abs(w - 0.05 * prob.f(w) - v).max() < 1e-12
    assert its <= 8


def test_burgers_small_amplitude_is_the_heat_step():
    n, eps, tau = 31, 2.0, 0.01
    p = nl.Burgers(n, eps)
    v = 1e-6 * p.initial_value()
    w, _ = nl.be_step(p, v, tau, 1e-15, 50)
    A = (np.diag(2 * np.ones(n)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)) / p.h ** 2
    lin = np.linalg.solve(np.eye(n) + tau * p.nu * A, v)
    assert np.abs(w - lin).max() < 1e-5 * np.abs(lin).max()


def test_allen_cahn_energy_decays_along_serial_fine():
    P = nl.NLPropagators(3, 63, 0.1, 6.0, 12, 8)
    u0 = P.prob.initial_value()
    U = nl.serial_fine(P, u0)
    E = [P.prob.energy(u0)] + [P.prob.energy(u) for u in U]
    assert all(E[i + 1] <= E[i] + 1e-13 for i in range(len(E) - 1))
    assert E[-1] < E[0]


def _dense_full_newton(P, alpha, U, b):
    """Full-Jacobian Newton on the stacked residual (brute force, tiny sizes)."""
    N, n, dT = P.N, P.prob.n, P.dT
    u = U.copy()
    C = np.eye(N)
    for k in range(1, N):
        C[k, k - 1] = -1.0
    C[0, N - 1] = -alpha
    for _ in range(60):
        R = nl.all_at_once_residual(P, alpha, u, b).reshape(-1)
        Jm = np.kron(C, np.eye(n))
        for s in range(N):
            lo, di, up = P.prob.jacobian(u[s] - b[s])
            Js = np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
            Jm[s * n:(s + 1) * n, s * n:(s + 1) * n] -= dT * Js
        du = np.linalg.solve(Jm, -R).reshape(N, n)
        u = u + du
        if np.abs(du).max() < 1e-14:
            break
    return u


@pytest.mark.parametrize("model,eps", [(2, 1.5), (3, 0.4)])
def test_newton_cgc_solves_the_all_at_once_system(model, eps):
    P = nl.NLPropagators(model, 7, eps, 1.0, 5, 3)
    u0 = P.prob.initial_value()
    rng = np.random.default_rng(1)
    U = nl.coarse_sweep(P, u0) + 0.01 * rng.standard_normal((5, 7))
    Fv = np.stack([P.F(v) for v in [u0] + [U[s - 1] for s in range(1, 5)]])
    alpha = 0.1
    b = nl.cgc_b(P, alpha, U, Fv)
    u, its = nl.newton_cgc(P, alpha, U, b)
    assert its < P.max
    assert np.abs(nl.all_at_once_residual(P, alpha, u, b)).max() < 1e-11
    assert np.abs(u - _dense_full_newton(P, alpha, U, b)).max() < 1e-11


@pytest.mark.parametrize("model,eps", [(2, 1.2), (3, 0.5)])
def test_serial_fine_is_fixed_point_and_alg2_converges(model, eps):
    P = nl.NLPropagators(model, 15, eps, 1.0, 6, 4)
    u0 = P.prob.initial_value()
    ref = nl.serial_fine(P, u0)
    h = nl.parareal_diag(P, 0.1, u0, ref, 0.0, 1)
    assert np.abs(h.U - ref).max() < 1e-11 * np.abs(ref).max()
    h = nl.parareal_diag(P, 0.1, u0, np.zeros_like(ref), 1e-12, 40, ref)
    assert h.iters < 40 and np.abs(h.U - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("model,eps", [(2, 1.2), (3, 0.5)])
def test_alg1_terminates_at_k_equal_N(model, eps):
    P = nl.NLPropagators(model, 15, eps, 1.0, 5, 4)
    u0 = P.prob.initial_value()
    ref = nl.serial_fine(P, u0)
    h = nl.parareal_sequential(P, u0, np.zeros_like(ref), 0.0, 5, ref)
    for k in range(1, 6):
        assert h.errors[k][:k].max() < 1e-12 * np.abs(ref).max()


class _Scalar:
    """u' = -L u - u^3 (one-sided Lipschitz constant L)."""

    def __init__(self, L):
        self.n, self.L = 1, L

    def f(self, u):
        return -self.L * u - u ** 3

    def jacobian(self, u):
        return np.zeros(1), -self.L - 3 * u ** 2, np.zeros(1)


def test_theorem_4_3_contraction_bound():
    L, T, N, alpha = 5.0, 10.0, 10, 0.1
    P = nl.NLPropagators(_Scalar(L), 1, 0.0, T, N, 400)
    u0 = np.array([1.0])
    ref = nl.serial_fine(P, u0)
    h = nl.parareal_diag(P, alpha, u0, np.zeros((N, 1)), 0.0, 6, ref)
    rho = nl.rho_nonlinear(alpha, L, T / N)
    e = [np.abs(x).max() for x in h.errors]
    for k in range(len(e) - 1):
        if e[k] > 1e-13:
            assert e[k + 1] <= rho * e[k] * 1.05, (k, e[k + 1] / e[k], rho)
