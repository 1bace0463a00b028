"""Pins of the oracle's operator and propagators.

Independent checks: consistency of the stencil with -(a u')' on smooth data
(second order), the sine eigenbasis of the constant-coefficient operator, and
the closed form of J backward-Euler steps, F(v) = w* + R^J (v - w*) with
R = (I + dt A)^{-1} and A w* = g, evaluated with dense linear algebra.
"""
import numpy as np
import pytest

from oracle import field, operator as op, prop


def test_stencil_consistency_1d():
    errs = []
    for n in (31, 63, 127):
        h = 1 / (n + 1)
        xf = (np.arange(n + 1) + 0.5) * h
        x = (np.arange(n) + 1) * h
        a = 1 + xf ** 2
        u = np.sin(np.pi * x)
        exact = -(2 * x * np.pi * np.cos(np.pi * x) - (1 + x ** 2) * np.pi ** 2 * np.sin(np.pi * x))
        errs.append(np.abs(op.apply(1, n, a, u) - exact).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5 and errs[2] < 1e-3


def test_stencil_consistency_2d():
    errs = []
    for n in (15, 31, 63):
        h = 1 / (n + 1)
        xf, yf = field.face_coords(2, n)
        a = 1 + xf + 2 * yf
        g = (np.arange(n) + 1) * h
        X, Y = np.meshgrid(g, g, indexing="xy")
        u = (np.sin(np.pi * X) * np.sin(2 * np.pi * Y)).ravel()
        ux = np.pi * np.cos(np.pi * X) * np.sin(2 * np.pi * Y)
        uy = 2 * np.pi * np.sin(np.pi * X) * np.cos(2 * np.pi * Y)
        lap = -(np.pi ** 2 + 4 * np.pi ** 2) * np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
        exact = -((1 + X + 2 * Y) * lap + 1 * ux + 2 * uy)
        errs.append(np.abs(op.apply(2, n, a, u) - exact.ravel()).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


@pytest.mark.parametrize("dim,n", [(1, 9), (2, 5)])
def test_operator_spd_and_sine_eigenbasis(dim, n):
    F = n + 1 if dim == 1 else 2 * n * (n + 1)
    A = op.assemble(dim, n, np.ones(F)).toarray()
    assert np.allclose(A, A.T)
    h = 1 / (n + 1)
    mu1 = 4 / h ** 2 * np.sin(np.arange(1, n + 1) * np.pi * h / 2) ** 2
    ev = np.sort(np.linalg.eigvalsh(A))
    want = np.sort(mu1 if dim == 1 else (mu1[:, None] + mu1[None, :]).ravel())
    assert np.allclose(ev, want, rtol=1e-12)


@pytest.mark.parametrize("dim,n", [(1, 7), (2, 4)])
def test_fine_propagator_closed_form(dim, n):
    rng = np.random.default_rng(3)
    F = n + 1 if dim == 1 else 2 * n * (n + 1)
    a = np.exp(0.5 * rng.standard_normal(F))
    T, N, J, f = 1.0, 4, 6, 1.3
    P = prop.Propagators(dim, n, a, T, N, J, f)
    A = op.assemble(dim, n, a).toarray()
    Nx = A.shape[0]
    R = np.linalg.inv(np.eye(Nx) + P.dt * A)
    wstar = np.linalg.solve(A, f * np.ones(Nx))
    v = rng.standard_normal(Nx)
    want = wstar + np.linalg.matrix_power(R, J) @ (v - wstar)
    assert np.abs(P.F(v) - want).max() <= 1e-13 * np.abs(want).max()
    Rg = np.linalg.inv(np.eye(Nx) + P.dT * A)
    assert np.abs(P.G(v) - (wstar + Rg @ (v - wstar))).max() <= 1e-13 * np.abs(v).max()


def test_fine_propagator_sine_mode_decay():
    n, J = 15, 10
    h = 1 / (n + 1)
    x = (np.arange(n) + 1) * h
    P = prop.Propagators(1, n, np.ones(n + 1), 1.0, 5, J, 0.0)
    k = 3
    mu = 4 / h ** 2 * np.sin(k * np.pi * h / 2) ** 2
    v = np.sin(k * np.pi * x)
    assert np.allclose(P.F(v), v / (1 + P.dt * mu) ** J, rtol=1e-13, atol=1e-16)


def test_serial_fine_is_composition():
    rng = np.random.default_rng(5)
    a = np.exp(rng.standard_normal(8))
    P = prop.Propagators(1, 7, a, 1.0, 3, 4, 1.0)
    ref = prop.serial_fine(P, np.zeros(7), 3)
    assert np.allclose(ref[2], P.F(P.F(P.F(np.zeros(7)))), rtol=0, atol=1e-16)


@pytest.mark.parametrize("dim,n", [(1, 6), (2, 3)])
def test_coarse_sweep_closed_form(dim, n):
    # N backward-Euler steps of size dT from u0: U_s = w* + R_G^s (u0 - w*), R_G = (I + dT A)^{-1},
    # A w* = g (dense matrix powers; independent of the banded solves and of the loop over slices)
    rng = np.random.default_rng(11)
    F = n + 1 if dim == 1 else 2 * n * (n + 1)
    a = np.exp(0.4 * rng.standard_normal(F))
    T, N, J, f = 0.7, 5, 3, 1.7
    P = prop.Propagators(dim, n, a, T, N, J, f)
    A = op.assemble(dim, n, a).toarray()
    Nx = A.shape[0]
    RG = np.linalg.inv(np.eye(Nx) + (T / N) * A)
    wstar = np.linalg.solve(A, f * np.ones(Nx))
    u0 = rng.standard_normal(Nx)
    got = prop.coarse_sweep(P, u0, N)
    assert got.shape == (N, Nx)
    for s in range(N):
        want = wstar + np.linalg.matrix_power(RG, s + 1) @ (u0 - wstar)
        assert np.abs(got[s] - want).max() <= 1e-13 * np.abs(want).max()


def test_coarse_sweep_steady_state_is_fixed():
    # the steady state A w* = g is a fixed point of every coarse step
    rng = np.random.default_rng(12)
    a = np.exp(rng.standard_normal(10))
    P = prop.Propagators(1, 9, a, 1.0, 4, 2, 2.0)
    wstar = np.linalg.solve(op.assemble(1, 9, a).toarray(), 2.0 * np.ones(9))
    got = prop.coarse_sweep(P, wstar, 4)
    assert np.abs(got - wstar[None, :]).max() <= 1e-13 * np.abs(wstar).max()
