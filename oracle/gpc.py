"""Generalised polynomial chaos surrogate (Section 2.2; Algorithm 3 steps 3, 5, 6).

Basis: for Gaussian inputs the Wiener-Askey table pairs N(0,1) with Hermite
polynomials; the univariate basis is taken orthonormal under N(0,1)
(probabilists' Hermite He_m / sqrt(m!)), built by the three-term recurrence
    psi_0 = 1, psi_1 = x, psi_{m+1} = (x psi_m - sqrt(m) psi_{m-1}) / sqrt(m+1).
For inputs uniform on [-1, 1] the table pairs U(-1,1) with Legendre polynomials
(the Section 5.1 parameter xi ~ U[2,6] enters as z = (xi - 4)/2); the univariate
basis is orthonormal under the density 1/2 on [-1, 1], psi_m = sqrt(2m+1) P_m,
with Bonnet's recurrence (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}.
Multivariate basis: tensor products over the total-order set
{k : |k|_1 <= p}, of size P = (p + d)! / (p! d!) (eq. complete).  Single-index
order (reading; predictions do not depend on it): degree ascending, then
lexicographic ascending in (k_1, ..., k_d).
Fit: B[j, i] = psi_i(xi_j) (eq. least square A), D = zeta(xi_j) (eq. least
square F), h = argmin |B h - D|_2 (eq. least square problem), solved by
Householder QR (requires n_t >= P and full column rank).
Prediction (Algorithm 3 step 6):
    U^0(xi) = u_bar + sum_i sqrt(lam_i) (sum_j h_{j,i} psi_j(xi)) g_i.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .snapshot import SnapshotKL, coefficients


def hermite_1d(x: np.ndarray, pmax: int) -> np.ndarray:
    """psi_m(x), m = 0..pmax, as rows [pmax+1, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((pmax + 1,) + x.shape)
    out[0] = 1.0
    if pmax >= 1:
        out[1] = x
    for m in range(1, pmax):
        out[m + 1] = (x * out[m] - math.sqrt(m) * out[m - 1]) / math.sqrt(m + 1)
    return out


def legendre_1d(x: np.ndarray, pmax: int) -> np.ndarray:
    """sqrt(2m+1) P_m(x), m = 0..pmax, as rows [pmax+1, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((pmax + 1,) + x.shape)
    P[0] = 1.0
    if pmax >= 1:
        P[1] = x
    for m in range(1, pmax):
        P[m + 1] = ((2 * m + 1) * x * P[m] - m * P[m - 1]) / (m + 1)
    return P * np.sqrt(2.0 * np.arange(pmax + 1) + 1.0).reshape((-1,) + (1,) * x.ndim)


BASES = {"hermite": hermite_1d, "legendre": legendre_1d}


def index_set(d: int, p: int) -> list:
    """Total-order multi-indices, degree ascending then lexicographic ascending."""
    def compositions(total, parts):
        # all tuples of `parts` non-negative integers summing to `total`, lexicographic ascending
        if parts == 1:
            yield (total,)
            return
        for first in range(total + 1):
            for rest in compositions(total - first, parts - 1):
                yield (first,) + rest

    out = []
    for deg in range(p + 1):
        out.extend(compositions(deg, d))
    return out


def n_terms(d: int, p: int) -> int:
    return math.comb(p + d, p)


def design_matrix(xi: np.ndarray, idx: list, p: int, basis: str = "hermite") -> np.ndarray:
    """B[j, i] = prod_l psi_{k_{i,l}}(xi_{j,l})."""
    xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
    H = [BASES[basis](xi[:, l], p) for l in range(xi.shape[1])]
    B = np.ones((xi.shape[0], len(idx)))
    for i, k in enumerate(idx):
        for l, kl in enumerate(k):
            if kl:
                B[:, i] *= H[l][kl]
    return B


@dataclasses.dataclass
class GPC:
    idx: list
    p: int
    H: np.ndarray       # [P, M_Q]
    kl: SnapshotKL
    basis: str = "hermite"


def fit(kl: SnapshotKL, S_train: np.ndarray, xi_train: np.ndarray, p: int,
        basis: str = "hermite") -> GPC:
    d = np.atleast_2d(xi_train).shape[1]
    idx = index_set(d, p)
    B = design_matrix(xi_train, idx, p, basis)
    if B.shape[0] < B.shape[1]:
        raise ValueError("n_t < P: least-squares problem under-determined")
    D = coefficients(kl, S_train)
    Q, R = np.linalg.qr(B, mode="reduced")
    if np.min(np.abs(np.diag(R))) <= 1e-12 * np.max(np.abs(np.diag(R))):
        raise ValueError("design matrix rank-deficient")
    H = np.linalg.solve(R, Q.T @ D)
    return GPC(idx, p, H, kl, basis)


def predict(g: GPC, xi: np.ndarray) -> np.ndarray:
    """U^0(xi) rows [M, L] (Algorithm 3 step 6)."""
    B = design_matrix(xi, g.idx, g.p, g.basis)
    zeta = B @ g.H
    return g.kl.mean[None, :] + (zeta * np.sqrt(g.kl.lam)[None, :]) @ g.kl.basis
