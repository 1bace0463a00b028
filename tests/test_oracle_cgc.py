"""Pins of the oracle's diagonalised coarse grid correction (Section 3.2).

Independent checks: the eigen-decomposition of C_alpha (including a hand
computation at N = 2), the brute-force dense solve of the all-at-once system,
and conjugate symmetry of the transformed right-hand side.
"""
import math

import numpy as np
import pytest

from oracle import cgc


@pytest.mark.parametrize("N,alpha", [(2, 0.3), (8, 1e-2), (16, 1e-4)])
def test_c_alpha_eigendecomposition(N, alpha):
    C = cgc.c_alpha(N, alpha)
    FN = cgc.dft_matrix(N)
    Lam = np.diag(cgc.scaling(N, alpha))
    V = np.linalg.inv(Lam) @ FN
    D = np.diag(cgc.eigenvalues(N, alpha))
    assert np.abs(C @ V - V @ D).max() < 1e-12 * np.abs(V).max()
    # the eigenvalues agree with numpy's
    ev = np.linalg.eigvals(C)
    for lam in np.diag(D):
        assert np.abs(ev - lam).min() < 1e-10


def test_printed_eigenvector_formula_does_not_diagonalise():
    # Reading recorded for Section 3.2: V = Lambda_alpha F_N (as printed) fails.
    N, alpha = 2, 0.3
    C = cgc.c_alpha(N, alpha)
    V = np.diag(cgc.scaling(N, alpha)) @ cgc.dft_matrix(N)
    D = np.diag(cgc.eigenvalues(N, alpha))
    assert np.abs(C @ V - V @ D).max() > 0.1


def test_n2_hand_computation():
    # C = [[1, -a], [-1, 1]]: eigenvalues 1 -/+ sqrt(a), eigenvectors (1, +/- a^{-1/2}).
    a = 0.3
    lam = cgc.eigenvalues(2, a)
    assert np.allclose(lam, [1 - math.sqrt(a), 1 + math.sqrt(a)])
    C = cgc.c_alpha(2, a)
    for s, l in ((1, 1 - math.sqrt(a)), (-1, 1 + math.sqrt(a))):
        v = np.array([1.0, s / math.sqrt(a)])
        assert np.allclose(C @ v, l * v)


@pytest.mark.parametrize("dim,n,N,alpha", [(1, 9, 8, 1e-2), (1, 6, 4, 1e-4), (2, 4, 8, 0.1), (2, 3, 4, 1e-4)])
def test_diag_solve_matches_dense(dim, n, N, alpha):
    rng = np.random.default_rng(11)
    F = n + 1 if dim == 1 else 2 * n * (n + 1)
    a = np.exp(rng.standard_normal(F))
    r = rng.standard_normal((N, n ** dim))
    dT = 1.0 / N
    u = cgc.diag_solve(dim, n, a, dT, alpha, r)
    ud = cgc.dense_solve(dim, n, a, dT, alpha, r)
    # round-off grows like eps * alpha^{-(N-1)/N}
    tol = 200 * np.finfo(float).eps * alpha ** (-(N - 1) / N)
    assert np.abs(u - ud).max() <= tol * np.abs(ud).max()


def test_transformed_rhs_is_conjugate_symmetric():
    N, alpha = 8, 1e-2
    rng = np.random.default_rng(2)
    r = rng.standard_normal((N, 5))
    p = cgc.dft_matrix(N).conj().T @ (cgc.scaling(N, alpha)[:, None] * r)
    for k in range(1, N):
        assert np.allclose(p[k], np.conj(p[N - k]), atol=1e-14)
    lam = cgc.eigenvalues(N, alpha)
    for k in range(1, N):
        assert np.isclose(lam[k], np.conj(lam[N - k]))
