"""Pins of the oracle's input-field KL (closed-form exponential-covariance eigenpairs).

Independent checks: a Nystrom discretisation of the covariance integral
operator (midpoint rule), the transcendental root equations, L2 normalisation
and orthogonality by quadrature, and Mercer's identity for the pointwise
variance.  None of them reuses the closed-form formulas.
"""
import math

import numpy as np
import pytest

from oracle import field


def nystrom_1d(corr_len, sigma, npts):
    x = (np.arange(npts) + 0.5) / npts
    K = sigma ** 2 * np.exp(-np.abs(x[:, None] - x[None, :]) / corr_len) / npts
    w, V = np.linalg.eigh(K)
    return w[::-1], V[:, ::-1] * math.sqrt(npts), x


@pytest.mark.parametrize("corr_len,sigma", [(0.5, 0.5), (0.3, 1.0), (0.2, 1.0)])
def test_kl_eigenvalues_match_nystrom(corr_len, sigma):
    lam, funcs = field.kl_1d(corr_len, sigma, 8)
    wn, Vn, x = nystrom_1d(corr_len, sigma, 2000)
    assert np.allclose(lam, wn[:8], rtol=2e-5, atol=0)
    for k in range(8):
        phi = funcs[k](x)
        s = np.sign(phi @ Vn[:, k])
        assert np.abs(phi - s * Vn[:, k]).max() < 5e-4


def test_kl_roots_solve_transcendental_equations():
    c = 2.0
    roots = field.kl_roots_1d(0.5, 10)
    ws = [w for w, _ in roots]
    assert all(b > a for a, b in zip(ws, ws[1:]))
    for w, parity in roots:
        if parity == 0:
            assert abs(c - w * math.tan(w / 2)) < 1e-9 * max(1, w)
        else:
            assert abs(w + c * math.tan(w / 2)) < 1e-9 * max(1, w)


def test_kl_values_for_corr_half_sigma_half():
    # corr 0.5, sigma 0.5: these are the closed-form values (not printed in the paper),
    # confirmed here against the Nystrom operator above to 2e-5.
    lam, _ = field.kl_1d(0.5, 0.5, 4)
    assert np.allclose(lam, [0.143664, 0.048868, 0.019631, 0.009945], atol=2e-6)


def test_kl_eigenfunctions_orthonormal():
    _, funcs = field.kl_1d(0.3, 1.0, 6)
    xg, wg = np.polynomial.legendre.leggauss(200)
    x = 0.5 * (xg + 1.0)
    w = 0.5 * wg
    G = np.array([[np.sum(w * funcs[i](x) * funcs[j](x)) for j in range(6)] for i in range(6)])
    assert np.abs(G - np.eye(6)).max() < 1e-12


def test_mercer_pointwise_variance():
    # sum_k lam_k phi_k(x)^2 -> sigma^2 as more modes are kept.
    sigma = 0.7
    lam, funcs = field.kl_1d(0.5, sigma, 400)
    x = np.array([0.1, 0.37, 0.5, 0.9])
    var = sum(lam[k] * funcs[k](x) ** 2 for k in range(400))
    assert np.allclose(var, sigma ** 2, rtol=3e-3)


def test_2d_separable_modes_match_2d_nystrom():
    corr_len, sigma, m = 0.3, 1.0, 40
    g = (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(g, g, indexing="xy")
    P = np.stack([X.ravel(), Y.ravel()], 1)
    K = sigma ** 2 * np.exp(-(np.abs(P[:, None, 0] - P[None, :, 0]) + np.abs(P[:, None, 1] - P[None, :, 1])) / corr_len) / m ** 2
    wn = np.sort(np.linalg.eigvalsh(K))[::-1]
    lam, Phi = field.kl_modes(2, 10, 10, corr_len, sigma)
    assert np.allclose(lam, wn[:10], rtol=1e-2)   # midpoint Nystrom at m = 40 is O(1e-3..1e-2)
    assert np.all(np.diff(lam) <= 0)


def test_2d_tie_break_order():
    lam, _ = field.kl_modes(2, 8, 6, 0.3, 1.0)
    # products (0,1) and (1,0) are bitwise equal and both kept, in order (i=0 first)
    assert lam[1] == lam[2]
    assert lam[4] == lam[5]


def test_face_layout_counts():
    (x,) = field.face_coords(1, 7)
    assert len(x) == 8 and x[0] == pytest.approx(0.5 / 8) and x[-1] == pytest.approx(7.5 / 8)
    x, y = field.face_coords(2, 5)
    assert len(x) == 2 * 5 * 6
    # first x-face of row 0 at (h/2, h); first y-face at (h, h/2)
    h = 1 / 6
    assert (x[0], y[0]) == pytest.approx((h / 2, h))
    assert (x[30], y[30]) == pytest.approx((h, h / 2))


def test_synthesize_log_field_statistics():
    # log a over many draws has covariance sum_k lam_k phi_k(x) phi_k(y).
    lam, Phi = field.kl_modes(1, 15, 4, 0.5, 0.5)
    rng = np.random.default_rng(7)
    xi = rng.standard_normal((20000, 4))
    la = np.log(field.synthesize(lam, Phi, xi))
    emp = np.cov(la.T)
    want = (Phi.T * lam) @ Phi
    assert np.abs(emp - want).max() < 0.01
    assert np.abs(la.mean(0)).max() < 0.01
