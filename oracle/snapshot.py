"""KL expansion of solution snapshots (Section 2.1; Algorithm 3, offline steps 1, 2, 4).

Snapshots: for every training parameter xi_j the coarse-point states
U(x, T_n), n = 1..N, stacked into one row of S [n_t, L], L = N * Nx.
  mean            u_bar = (1/n_t) sum_j u(xi_j)
  fluctuation     u~_j  = u(xi_j) - u_bar
  covariance      C_nm  = (1/n_t) (u~_n, u~_m)
  eigenpairs      (lam_k, e_k) of C, descending, e_k unit-norm
  basis           g_k   = (lam_k n_t)^{-1/2} sum_j e_k^j u~_j   (eq. KLE basis)
  coefficients    zeta_k(xi) = lam_k^{-1/2} (u~(xi), g_k)      (eq. KLE parameter)
  reconstruction  u ~ u_bar + sum_{k<=M_Q} sqrt(lam_k) zeta_k g_k (eq. KLE Snapshots)
Readings: (., .) is the Euclidean inner product on the stacked vector (a
uniform weight only rescales lam and g and leaves every reconstruction
unchanged).  The truncation rule of Algorithm 3 step 2 is printed with "<=";
it is read as the smallest M_Q whose eigenvalue fraction is >= 1 - eps_KL,
capped at the numerical rank (lam_k > n_t * eps * lam_1), since the centred
snapshot matrix has rank at most n_t - 1.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class SnapshotKL:
    mean: np.ndarray      # [L]
    lam: np.ndarray       # [M_Q] descending
    basis: np.ndarray     # [M_Q, L]  rows g_k
    evecs: np.ndarray     # [n_t, M_Q] e_k as columns
    n_t: int

    @property
    def n_modes(self) -> int:
        return len(self.lam)


def build(S: np.ndarray, eps_kl: float) -> SnapshotKL:
    S = np.asarray(S, dtype=np.float64)
    n_t = S.shape[0]
    mean = S.mean(axis=0)
    St = S - mean[None, :]
    C = (St @ St.T) / n_t
    w, E = np.linalg.eigh(C)
    order = np.argsort(w)[::-1]
    w, E = w[order], E[:, order]
    w = np.maximum(w, 0.0)
    total = w.sum()
    if total <= 0:
        return SnapshotKL(mean, np.zeros(0), np.zeros((0, S.shape[1])), np.zeros((n_t, 0)), n_t)
    frac = np.cumsum(w) / total
    MQ = int(np.searchsorted(frac, 1.0 - eps_kl) + 1)
    rank = int(np.sum(w > n_t * np.finfo(np.float64).eps * w[0]))
    MQ = max(1, min(MQ, rank, n_t))
    lam = w[:MQ]
    E = E[:, :MQ]
    basis = (E.T @ St) / np.sqrt(lam * n_t)[:, None]
    return SnapshotKL(mean, lam, basis, E, n_t)


def coefficients(kl: SnapshotKL, u: np.ndarray) -> np.ndarray:
    """zeta_k(xi) for snapshot rows u [m, L] (eq. KLE parameter)."""
    ut = np.atleast_2d(u) - kl.mean[None, :]
    return (ut @ kl.basis.T) / np.sqrt(kl.lam)[None, :]


def reconstruct(kl: SnapshotKL, zeta: np.ndarray) -> np.ndarray:
    """u_bar + sum_k sqrt(lam_k) zeta_k g_k (eq. KLE Snapshots); zeta [m, M_Q]."""
    return kl.mean[None, :] + (np.atleast_2d(zeta) * np.sqrt(kl.lam)[None, :]) @ kl.basis
