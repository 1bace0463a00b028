"""Pins of the oracle's MLP and grid transfer.

Independent checks: central finite differences of the FP64 loss (all six parameter
blocks), a width-1 network worked by hand, the first Adam step's closed form
(-lr * sign(g)), exactness of bfloat16 rounding on representable values and ties,
GELU against its integral definition, and bilinear transfer exact on functions that are
bilinear on both grids' common support, with second-order convergence on smooth ones.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import mlp


def _params(n_in=3, hidden=5, n_out=4, seed=0):
    rng = np.random.default_rng(seed)
    shp = mlp.Params.shapes(n_in, hidden, n_out)
    return mlp.Params(*[rng.standard_normal(s) * 0.5 for s in shp])


def test_finite_difference_gradients():
    p = _params()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((6, 3))
    T = rng.standard_normal((6, 4))
    _, g = mlp.loss_and_grad(p, X, T)
    h = 1e-6
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        A = getattr(p, k)
        num = np.zeros_like(A)
        for idx in np.ndindex(A.shape):
            old = A[idx]
            A[idx] = old + h
            lp = mlp.loss_and_grad(p, X, T)[0]
            A[idx] = old - h
            lm = mlp.loss_and_grad(p, X, T)[0]
            A[idx] = old
            num[idx] = (lp - lm) / (2 * h)
        assert np.abs(num - g[k]).max() <= 1e-7 * max(1.0, np.abs(g[k]).max()), k


def test_width_one_network_by_hand():
    p = mlp.Params(np.array([[2.0]]), np.array([0.5]), np.array([[1.5]]), np.array([-1.0]),
                   np.array([[0.25]]), np.array([0.1]))
    x = 0.3
    pre1 = 2.0 * x + 0.5
    h1 = pre1 * 0.5 * (1 + math.erf(pre1 / math.sqrt(2)))
    pre2 = 1.5 * h1 - 1.0
    h2 = pre2 * 0.5 * (1 + math.erf(pre2 / math.sqrt(2)))
    y = 0.25 * h2 + 0.1
    Y, _ = mlp.forward(p, np.array([[x]]))
    assert Y[0, 0] == pytest.approx(y, rel=1e-15)


def test_first_adam_step_moves_by_lr_sign():
    p = _params()
    rng = np.random.default_rng(2)
    X = rng.standard_normal((6, 3))
    T = rng.standard_normal((6, 4))
    _, g = mlp.loss_and_grad(p, X, T)
    before = {k: getattr(p, k).copy() for k in g}
    m = {k: np.zeros_like(v) for k, v in g.items()}
    v = {k: np.zeros_like(x) for k, x in g.items()}
    mlp.adam_step(p, g, m, v, 1, 1e-3)
    for k in g:
        step = getattr(p, k) - before[k]
        big = np.abs(g[k]) > 1e-6
        assert np.allclose(step[big], -1e-3 * np.sign(g[k][big]), rtol=1e-4)


def test_bf16_rounding():
    # representable values are unchanged; a tie rounds to even
    vals = np.array([1.0, -2.5, 0.0078125, 2.0 ** 100, -3.0 * 2.0 ** -90])
    assert np.all(mlp.bf16_round(vals) == np.float32(vals).astype(np.float64))
    one_plus_half_ulp = 1.0 + 2.0 ** -8          # bf16 ulp at 1 is 2^-7: exact tie
    assert mlp.bf16_round(np.array([one_plus_half_ulp]))[0] == 1.0
    three_halves_ulp = 1.0 + 3 * 2.0 ** -8         # tie between 1+2^-7 and 1+2^-6 -> even (1+2^-6)
    assert mlp.bf16_round(np.array([three_halves_ulp]))[0] == 1.0 + 2.0 ** -6
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.all(np.abs(mlp.bf16_round(x) - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-12))   # unit roundoff 2^-8


def test_gelu_matches_integral_definition():
    for x in (-2.0, -0.3, 0.0, 0.7, 3.0):
        phi = quad(lambda t: math.exp(-t * t / 2) / math.sqrt(2 * math.pi), -np.inf, x)[0]
        assert mlp.gelu(np.array(x)) == pytest.approx(x * phi, abs=1e-12)
        d = (mlp.gelu(np.array(x + 1e-6)) - mlp.gelu(np.array(x - 1e-6))) / 2e-6
        assert mlp.gelu_grad(np.array(x)) == pytest.approx(d, abs=1e-8)


def test_transfer_exact_on_piecewise_linear_and_second_order():
    # f(x, y) = hat-free bilinear product sin-free: x(1-x) is not bilinear; use the fine-grid
    # interpolant of a coarse-grid function: prolong then restrict returns the coarse values
    # exactly when the fine grid contains the coarse nodes (n + 1 = 2 (nc + 1)).
    nc, n = 7, 15
    rng = np.random.default_rng(0)
    Uc = rng.standard_normal(nc * nc)
    assert np.allclose(mlp.restrict(mlp.prolong(Uc, nc, n), n, nc), Uc, atol=1e-14)
    errs = []
    for n in (31, 63, 127):
        h = 1 / (n + 1)
        g = (np.arange(n) + 1) * h
        X, Y = np.meshgrid(g, g, indexing="xy")
        F = (np.sin(np.pi * X) * np.sin(2 * np.pi * Y)).ravel()
        gc = (np.arange(32) + 1) / 33
        Xc, Yc = np.meshgrid(gc, gc, indexing="xy")
        Fc = (np.sin(np.pi * Xc) * np.sin(2 * np.pi * Yc)).ravel()
        errs.append(np.abs(mlp.restrict(F, n, 32) - Fc).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_zscore_hand_computed():
    # three rows: column 0 = (1, 2, 6): mean 3, population variance ((-2)^2 + (-1)^2 + 3^2)/3 = 14/3;
    # column 1 is constant (deviation 0 -> replaced by 1, z = 0); column 2 = (-1, 0, 1): mean 0,
    # population std sqrt(2/3) (a sample std, ddof 1, would be 1)
    Y = np.array([[1.0, 5.0, -1.0], [2.0, 5.0, 0.0], [6.0, 5.0, 1.0]])
    mu, sd, Z = mlp.zscore(Y)
    assert np.allclose(mu, [3.0, 5.0, 0.0], rtol=0, atol=1e-15)
    assert np.allclose(sd, [math.sqrt(14.0 / 3.0), 1.0, math.sqrt(2.0 / 3.0)], rtol=1e-15)
    assert np.allclose(Z[:, 0], np.array([-2.0, -1.0, 3.0]) / math.sqrt(14.0 / 3.0), rtol=1e-15)
    assert np.all(Z[:, 1] == 0.0)
    assert np.allclose(Z[:, 2], np.array([-1.0, 0.0, 1.0]) / math.sqrt(2.0 / 3.0), rtol=1e-15)
    # invariants: every non-constant column of Z has mean 0 and population variance 1
    assert np.allclose(Z.mean(0), 0.0, atol=1e-15)
    assert np.allclose((Z[:, [0, 2]] ** 2).mean(0), 1.0, rtol=1e-14)


def test_zscore_single_row_is_constant():
    mu, sd, Z = mlp.zscore(np.array([[3.0, -4.0]]))
    assert np.all(mu == [3.0, -4.0]) and np.all(sd == 1.0) and np.all(Z == 0.0)
