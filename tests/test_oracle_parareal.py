"""Pins of the oracle's parareal iterations (Algorithms 1-2, Section 4.1 theory).

Independent checks:
  * Algorithm 1 (sequential CGC) reproduces the serial fine solution at k = N;
  * the serial fine solution is a fixed point of Algorithm 2;
  * Lemma 4.1 holds exactly: e^{k+1} = G^{-1}(G - F) e^k with block matrices
    built from dense (I + dT A)^{-1} and (I + dt A)^{-J};
  * the Gander-Vandewalle bound: |G(z)^{-1}(G(z) - F(z))|_inf <= K_cla(z, J) at alpha = 0,
    and the classical BE/BE factor stays below 1/3 (Section 1);
  * Algorithm 2 converges to the serial fine solution.
"""
import numpy as np
import pytest

from oracle import field, operator as op, parareal, prop, theory


def _problem(dim=1, n=9, N=6, J=5, seed=0, f=1.0):
    rng = np.random.default_rng(seed)
    F = n + 1 if dim == 1 else 2 * n * (n + 1)
    a = np.exp(0.6 * rng.standard_normal(F))
    return prop.Propagators(dim, n, a, 1.0, N, J, f), a


def test_sequential_parareal_terminates_at_k_equal_N():
    P, _ = _problem()
    N = 6
    u0 = np.zeros(P.Nx)
    ref = prop.serial_fine(P, u0, N)
    U0 = np.random.default_rng(1).random((N, P.Nx))
    its = parareal.parareal_sequential(P, u0, U0, N)
    assert np.abs(its[N] - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.abs(its[N - 1] - ref).max() > 1e-12   # not earlier in general


@pytest.mark.parametrize("alpha", [1e-4, 1e-2, 0.3])
def test_serial_fine_is_fixed_point_of_alg2(alpha):
    P, _ = _problem(N=8)
    u0 = np.zeros(P.Nx)
    ref = prop.serial_fine(P, u0, 8)
    h = parareal.parareal_diag(P, alpha, u0, ref, 1e-30, 1, fixed_iters=1)
    assert np.abs(h.iterates[-1] - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("alpha", [1e-2, 0.2])
def test_lemma_4_1_exact_error_recursion(alpha):
    N, J = 5, 4
    P, a = _problem(n=6, N=N, J=J, seed=4)
    A = op.assemble(1, 6, a).toarray()
    Rg = np.linalg.inv(np.eye(6) + P.dT * A)
    RfJ = np.linalg.matrix_power(np.linalg.inv(np.eye(6) + P.dt * A), J)
    E = theory.block_error_operator(Rg, RfJ, N, alpha)
    u0 = np.zeros(6)
    ref = prop.serial_fine(P, u0, N)
    U0 = np.random.default_rng(9).random((N, 6))
    h = parareal.parareal_diag(P, alpha, u0, U0, 0.0, 4, keep=True, fixed_iters=4)
    for k in range(4):
        e_k = (ref - h.iterates[k]).ravel()
        e_k1 = (ref - h.iterates[k + 1]).ravel()
        assert np.abs(e_k1 - E @ e_k).max() <= 1e-12 * max(np.abs(e_k).max(), 1e-300)


def test_scalar_error_operator_bounded_by_kcla_alpha0():
    for J in (2, 8, 32, 64):
        for z in np.logspace(-3, 3, 61):
            M = theory.error_operator(z, 16, J, 0.0)
            assert np.abs(M).sum(1).max() <= theory.k_cla(z, J) * (1 + 1e-12)


def test_kcla_below_one_third_and_sup_values():
    z = np.logspace(-4, 5, 40001)
    sups = [theory.k_cla(z, J).max() for J in (2, 32, 64, 128)]
    assert all(s < 1 / 3 for s in sups)
    assert sups == sorted(sups)
    # derived values (the paper quotes rho ~ 1/3 for BE/BE)
    assert sups[1] == pytest.approx(0.2856, abs=2e-4)
    assert sups[2] == pytest.approx(0.2920, abs=2e-4)


def test_theorem_4_1_alpha_factor_reduces_to_kcla():
    z = np.logspace(-2, 3, 50)
    assert np.allclose(theory.k_alpha(z, 32, 0.0), theory.k_cla(z, 32))
    assert np.all(theory.k_alpha(z, 32, 0.5) >= theory.k_cla(z, 32))


@pytest.mark.parametrize("dim,n", [(1, 15), (2, 6)])
def test_alg2_converges_to_serial_fine(dim, n):
    P, _ = _problem(dim=dim, n=n, N=8, J=8, seed=2)
    u0 = np.zeros(P.Nx)
    ref = prop.serial_fine(P, u0, 8)
    h = parareal.parareal_diag(P, 1e-2, u0, np.zeros((8, P.Nx)), 1e-10, 60)
    assert h.converged
    assert parareal.relative_error(h.iterates[-1], ref) < 1e-9
    # increments decay geometrically with a rate below the classical bound
    d = np.array(h.deltas)
    assert np.all(d[3:] / d[2:-1] < 0.35)


def test_expected_iterations_on_a_geometric_sequence():
    # an error that shrinks by exactly rho per iteration reaches eps after log(eps/e0)/log(rho)
    # iterations (Section 3.3 estimate): e0 = 1, rho = 1/2, eps = 2^-10 gives 10
    assert theory.expected_iterations(2.0 ** -10, 1.0, 0.5) == pytest.approx(10.0, rel=1e-14)
    assert theory.expected_iterations(1e-8, 1e-2, 0.1) == pytest.approx(6.0, rel=1e-14)


def test_expected_iterations_bounds_the_scalar_error_recursion():
    # Lemma 4.1 on the scalar model problem: |e^k|_inf <= |E|_inf^k |e^0|_inf, so the error meets
    # eps no later than the estimate taken with rho = |E|_inf
    N, J, alpha, eps = 16, 32, 1e-2, 1e-10
    for z in (0.3, 3.0, 30.0):
        E = theory.error_operator(z, N, J, alpha)
        rho = np.abs(E).sum(1).max()
        assert rho < 1
        e = np.random.default_rng(3).random(N)
        e0 = np.abs(e).max()
        k = 0
        while np.abs(e).max() > eps:
            e = E @ e
            k += 1
        assert k <= int(np.ceil(theory.expected_iterations(eps, e0, rho)))
