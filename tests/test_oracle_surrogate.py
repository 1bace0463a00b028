"""Pins of the oracle's snapshot KL (Section 2.1) and Hermite gPC (Section 2.2).

Independent checks: orthonormality of the KL basis (stated after eq. KLE
basis), the identity zeta_k(xi_j) = sqrt(n_t) e_k^j, exact reconstruction of
the training snapshots, invariance of reconstructions under a uniform inner-
product weight; Gauss-Hermite orthonormality of the basis, the basis count of
eq. complete, exact recovery of polynomial coefficient maps written in
monomials, and invariance of predictions to the single-index order.
"""
import math

import numpy as np
import pytest

from oracle import gpc, snapshot


def _snapshots(n_t=20, L=60, r=6, seed=0):
    rng = np.random.default_rng(seed)
    base = rng.standard_normal((r, L))
    coef = rng.standard_normal((n_t, r)) * np.array([3.0, 2.0, 1.0, 0.5, 0.1, 0.01])[:r]
    return 1.5 + coef @ base


def test_kl_basis_orthonormal_and_coefficients():
    S = _snapshots()
    kl = snapshot.build(S, 1e-14)
    G = kl.basis @ kl.basis.T
    assert np.abs(G - np.eye(kl.n_modes)).max() < 1e-10
    z = snapshot.coefficients(kl, S)
    assert np.allclose(z, math.sqrt(kl.n_t) * kl.evecs, atol=1e-9)
    assert kl.n_modes == 6          # rank of the centred snapshots


def test_kl_reconstructs_training_snapshots():
    S = _snapshots()
    kl = snapshot.build(S, 1e-14)
    rec = snapshot.reconstruct(kl, snapshot.coefficients(kl, S))
    assert np.abs(rec - S).max() < 1e-11 * np.abs(S).max()


def test_kl_truncation_rule():
    S = _snapshots()
    kl = snapshot.build(S, 1e-3)
    w = np.sort(np.linalg.eigvalsh(np.cov(S.T, bias=True)))[::-1]
    frac = np.cumsum(w) / w.sum()
    assert kl.n_modes == int(np.argmax(frac >= 1 - 1e-3) + 1)


def test_kl_projection_invariance_under_weight():
    S = _snapshots()
    kl1 = snapshot.build(S, 1e-14)
    kl2 = snapshot.build(S * 3.0, 1e-14)
    rec1 = snapshot.reconstruct(kl1, snapshot.coefficients(kl1, S[:3]))
    rec2 = snapshot.reconstruct(kl2, snapshot.coefficients(kl2, 3.0 * S[:3])) / 3.0
    assert np.allclose(rec1, rec2, atol=1e-11)


def test_hermite_orthonormal_gauss_quadrature():
    x, w = np.polynomial.hermite_e.hermegauss(20)
    w = w / w.sum()
    H = gpc.hermite_1d(x, 8)
    G = (H * w) @ H.T
    assert np.abs(G - np.eye(9)).max() < 1e-13


@pytest.mark.parametrize("d,p,P", [(4, 3, 35), (10, 3, 286), (20, 3, 1771), (20, 2, 231), (2, 2, 6)])
def test_total_order_counts(d, p, P):
    assert gpc.n_terms(d, p) == P
    idx = gpc.index_set(d, p)
    assert len(idx) == P and len(set(idx)) == P
    assert all(sum(k) <= p for k in idx)
    degs = [sum(k) for k in idx]
    assert degs == sorted(degs)


def test_gpc_exact_recovery_of_polynomial_map():
    rng = np.random.default_rng(1)
    d, p, n_t, L = 3, 3, 60, 40
    xi = rng.standard_normal((n_t, d))

    def field(x):  # degree-3 polynomial in xi, written in monomials
        c1 = 1 + 0.5 * x[:, 0] - x[:, 1] * x[:, 2] + 0.2 * x[:, 0] ** 3
        c2 = x[:, 1] ** 2 - 0.3 * x[:, 2]
        c3 = 0.1 * x[:, 0] * x[:, 1] * x[:, 2]
        return np.stack([c1, c2, c3], 1)

    basis = rng.standard_normal((3, L))
    S = field(xi) @ basis
    kl = snapshot.build(S, 1e-14)
    g = gpc.fit(kl, S, xi, p)
    xt = rng.standard_normal((5, d))
    assert np.abs(gpc.predict(g, xt) - field(xt) @ basis).max() < 1e-10


def test_gpc_prediction_independent_of_index_order():
    rng = np.random.default_rng(2)
    d, p = 2, 3
    xi = rng.standard_normal((30, d))
    S = np.sin(xi[:, :1] * np.linspace(0, 1, 25)[None, :]) + xi[:, 1:2] ** 2
    kl = snapshot.build(S, 1e-12)
    g1 = gpc.fit(kl, S, xi, p)
    g2 = gpc.GPC(list(reversed(g1.idx)), p, None, kl)
    B2 = gpc.design_matrix(xi, g2.idx, p)
    Q, R = np.linalg.qr(B2)
    g2.H = np.linalg.solve(R, Q.T @ snapshot.coefficients(kl, S))
    xt = rng.standard_normal((4, d))
    assert np.allclose(gpc.predict(g1, xt), gpc.predict(g2, xt), atol=1e-11)


def test_gpc_rejects_underdetermined():
    rng = np.random.default_rng(3)
    xi = rng.standard_normal((5, 3))
    S = rng.standard_normal((5, 10))
    kl = snapshot.build(S, 1e-12)
    with pytest.raises(ValueError):
        gpc.fit(kl, S, xi, 3)
