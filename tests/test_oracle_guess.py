"""Pins of the oracle's non-gPC initial guesses (oracle/guess.py).

Independent checks:
  * SplitMix64 reproduces the generator's published first outputs for seed 0, and the
    counter form is a pure function of (seed, entry index);
  * the U(0,1) guess has the moments of the uniform distribution;
  * the continuity defect equals its dense closed form (F(v) = w* + R^J (v - w*)) and
    vanishes on the serial fine solution;
  * the chooser keeps the guess with the smaller defect, the learned one on ties.
"""
import numpy as np
import pytest

from oracle import guess, operator as op, prop


def test_splitmix64_known_answers_seed_0():
    # first four outputs of the SplitMix64 reference generator seeded with 0
    st = (np.arange(1, 5, dtype=np.uint64) * guess.GOLDEN)
    got = [int(x) for x in guess.splitmix64(st)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    u = guess.uniform_counter(0, 0, 4)
    assert u[0] == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53


def test_counter_stream_is_positional():
    whole = guess.uniform_counter(12345, 0, 1000)
    part = guess.uniform_counter(12345, 700, 300)
    assert np.array_equal(whole[700:], part)
    assert not np.array_equal(guess.uniform_counter(12346, 0, 1000), whole)
    g = guess.random_guess(99, 3, 4, 5)
    assert g.shape == (3, 4, 5) and np.array_equal(g.ravel(), guess.uniform_counter(99, 0, 60))


def test_uniform_moments():
    u = guess.uniform_counter(2024, 0, 1_000_000)
    assert u.min() >= 0.0 and u.max() < 1.0
    # mean 1/2 (sd of the estimate 0.000289), variance 1/12 (sd 0.000075): 5 sigma
    assert abs(u.mean() - 0.5) < 5 * 0.000289
    assert abs(u.var() - 1 / 12) < 5 * 0.000075
    # 10 equal bins: chi-square with 9 degrees of freedom far below its 0.999 quantile (27.9)
    cnt = np.bincount((u * 10).astype(int), minlength=10)
    assert ((cnt - 1e5) ** 2 / 1e5).sum() < 27.9


@pytest.mark.parametrize("dim,n", [(1, 7), (2, 3)])
def test_continuity_defect_closed_form(dim, n):
    rng = np.random.default_rng(21)
    F = n + 1 if dim == 1 else 2 * n * (n + 1)
    a = np.exp(0.5 * rng.standard_normal(F))
    T, N, J, f = 1.0, 5, 4, 1.2
    P = prop.Propagators(dim, n, a, T, N, J, f)
    A = op.assemble(dim, n, a).toarray()
    Nx = A.shape[0]
    RJ = np.linalg.matrix_power(np.linalg.inv(np.eye(Nx) + P.dt * A), J)
    wstar = np.linalg.solve(A, f * np.ones(Nx))
    u0 = 0.1 * rng.standard_normal(Nx)
    U0 = rng.random((N, Nx))
    jumps = [wstar + RJ @ ((u0 if s == 0 else U0[s - 1]) - wstar) - U0[s] for s in range(N)]
    want = max(np.abs(j).max() for j in jumps) / np.abs(U0).max()
    assert guess.continuity_defect(P, u0, U0) == pytest.approx(want, rel=1e-12)


def test_continuity_defect_vanishes_on_serial_fine():
    rng = np.random.default_rng(22)
    P = prop.Propagators(1, 15, np.exp(rng.standard_normal(16)), 1.0, 8, 6, 1.0)
    ref = prop.serial_fine(P, np.zeros(15), 8)
    assert guess.continuity_defect(P, np.zeros(15), ref) <= 1e-15
    # a zero guess: the defect is the first slice's F(u0) over the denominator 1
    d0 = guess.continuity_defect(P, np.zeros(15), np.zeros((8, 15)))
    assert d0 == pytest.approx(np.abs(P.F(np.zeros(15))).max(), rel=1e-15)


def test_chooser_keeps_the_smaller_defect():
    rng = np.random.default_rng(23)
    P = prop.Propagators(1, 9, np.exp(rng.standard_normal(10)), 1.0, 4, 4, 1.0)
    u0 = np.zeros(9)
    ref = prop.serial_fine(P, u0, 4)
    bad = ref + 0.1 * rng.standard_normal(ref.shape)
    g, used_f, dl, df = guess.choose_guess(P, u0, bad, ref)
    assert used_f and g is ref and df < dl
    g, used_f, dl, df = guess.choose_guess(P, u0, ref, bad)
    assert not used_f and g is ref and dl < df
    g, used_f, dl, df = guess.choose_guess(P, u0, bad, bad.copy())
    assert not used_f and dl == df            # ties keep the learned guess


def test_chooser_falls_back_from_a_non_finite_learned_guess():
    rng = np.random.default_rng(24)
    P = prop.Propagators(1, 9, np.exp(rng.standard_normal(10)), 1.0, 4, 4, 1.0)
    u0 = np.zeros(9)
    ref = prop.serial_fine(P, u0, 4)
    nan_guess = ref.copy()
    nan_guess[2, 3] = np.nan
    g, used_f, dl, df = guess.choose_guess(P, u0, nan_guess, ref + 1.0)
    assert used_f and np.isnan(dl) and np.isfinite(df)
