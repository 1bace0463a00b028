"""Convergence theory for the linear case (Section 4.1): scalar model problem.

Backward Euler stability function R(z) = 1 / (1 + z).  For z = dT * mu:
  K_cla(z, J)      = |R(z/J)^J - R(z)| / (1 - |R(z)|)       (eq. er1_condition; also the
                                                               Gander-Vandewalle factor of Section 1)
  K(z, J, alpha)   = max{ |alpha R(z)| (1 + K_cla), K_cla }   (Theorem 4.1)
Lemma 4.1: the parareal error with diagonalised CGC obeys
  e^{k+1} = G^{-1} (G - F) e^k
with the block matrices G (identity diagonal, -R_g below it, -alpha R_g in the
top-right corner) and F (identity diagonal, -R_f^J below it).
Section 3.3: expected iterations k = log(eps / |e^0|) / log(rho).
"""
from __future__ import annotations

import math

import numpy as np


def r_be(z):
    return 1.0 / (1.0 + np.asarray(z, dtype=np.float64))


def k_cla(z, J: int):
    z = np.asarray(z, dtype=np.float64)
    return np.abs(r_be(z / J) ** J - r_be(z)) / (1.0 - np.abs(r_be(z)))


def k_alpha(z, J: int, alpha: float):
    kc = k_cla(z, J)
    return np.maximum(np.abs(alpha * r_be(z)) * (1.0 + kc), kc)


def scalar_G(z: float, N: int, alpha: float) -> np.ndarray:
    G = np.eye(N)
    rg = float(r_be(z))
    for k in range(1, N):
        G[k, k - 1] = -rg
    G[0, N - 1] += -alpha * rg
    return G


def scalar_F(z: float, N: int, J: int) -> np.ndarray:
    F = np.eye(N)
    rf = float(r_be(z / J)) ** J
    for k in range(1, N):
        F[k, k - 1] = -rf
    return F


def error_operator(z: float, N: int, J: int, alpha: float) -> np.ndarray:
    """G(z)^{-1}(G(z) - F(z)) of Lemma 4.1 for one eigenvalue."""
    G = scalar_G(z, N, alpha)
    return np.linalg.solve(G, G - scalar_F(z, N, J))


def block_error_operator(Rg: np.ndarray, RfJ: np.ndarray, N: int, alpha: float) -> np.ndarray:
    """Block G^{-1}(G - F) of Lemma 4.1 for matrices Rg = R_g(dT A), RfJ = R_f^J(dt A)."""
    Nx = Rg.shape[0]
    I = np.eye(Nx)
    G = np.zeros((N * Nx, N * Nx))
    F = np.zeros_like(G)
    for k in range(N):
        G[k * Nx:(k + 1) * Nx, k * Nx:(k + 1) * Nx] = I
        F[k * Nx:(k + 1) * Nx, k * Nx:(k + 1) * Nx] = I
        if k > 0:
            G[k * Nx:(k + 1) * Nx, (k - 1) * Nx:k * Nx] = -Rg
            F[k * Nx:(k + 1) * Nx, (k - 1) * Nx:k * Nx] = -RfJ
    G[0:Nx, (N - 1) * Nx:N * Nx] += -alpha * Rg
    return np.linalg.solve(G, G - F)


def expected_iterations(eps: float, e0: float, rho: float) -> float:
    return math.log(eps / e0) / math.log(rho)
