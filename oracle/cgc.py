"""Diagonalised coarse grid correction (Section 3.2).

With backward Euler as G, the parallel CGC of Algorithm 2 amounts to the
all-at-once system (eq. matrix_NT) with the alpha-circulant time matrix
C_alpha (ones on the diagonal, -1 below it, -alpha in the top-right corner).
For the linear flux f(u) = -A u + g the averaged Jacobian of eq. Jac is exact,
so one simplified-Newton step (eq. Newton2) solves it:
    (C_alpha (x) I + dT I (x) A) u = r,   r = (I + dT A) b + dT g.
C_alpha = V diag(lambda_n) V^{-1} with lambda_n = 1 - alpha^{1/N} w^{-(n-1)},
w = exp(2 pi i / N).  Reading of the paper's eigenvector formula: the matrix
printed as V = Lambda_alpha F_N does not diagonalise C_alpha; the one that does
is V = Lambda_alpha^{-1} F_N (Lambda_alpha = diag(alpha^{(n-1)/N})), so the
three steps of eq. three-steps are
    (a) p = (F_N^* (x) I)(Lambda_alpha (x) I) r
    (b) (lambda_n I + dT A) q_n = p_n,  n = 1..N
    (c) u = (Lambda_alpha^{-1} (x) I)(F_N (x) I) q.
Here F_N is applied as a dense N x N matrix (no FFT) and every one of the N
shifted systems is solved by a complex banded (1D) or sparse (2D) LU; no
conjugate symmetry is assumed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.linalg import solve_banded

from . import operator as op


def c_alpha(N: int, alpha: float) -> np.ndarray:
    """The alpha-circulant time matrix of eq. matrix_NT."""
    C = np.eye(N)
    for k in range(1, N):
        C[k, k - 1] = -1.0
    C[0, N - 1] -= alpha
    return C


def dft_matrix(N: int) -> np.ndarray:
    """F_N = N^{-1/2} [w^{jk}], w = exp(2 pi i / N)."""
    j = np.arange(N)
    return np.exp(2j * np.pi * np.outer(j, j) / N) / np.sqrt(N)


def eigenvalues(N: int, alpha: float) -> np.ndarray:
    """lambda_n = 1 - alpha^{1/N} w^{-(n-1)}, n = 1..N."""
    k = np.arange(N)
    return 1.0 - alpha ** (1.0 / N) * np.exp(-2j * np.pi * k / N)


def scaling(N: int, alpha: float) -> np.ndarray:
    """Diagonal of Lambda_alpha: alpha^{(n-1)/N}, n = 1..N."""
    return alpha ** (np.arange(N) / N)


class ShiftedSolver:
    """Solves (lam I + dT A) q = p for one sample, complex lam."""

    def __init__(self, dim: int, n: int, a: np.ndarray, dT: float):
        self.dim, self.n = dim, n
        self.A = op.assemble(dim, n, a).astype(np.complex128)
        self.dT = dT
        self.Nx = self.A.shape[0]

    def solve(self, lam: complex, p: np.ndarray) -> np.ndarray:
        Ms = lam * sp.identity(self.Nx, dtype=np.complex128, format="csr") + self.dT * self.A
        if self.dim == 1:
            return solve_banded((1, 1), op.to_general_banded(Ms.tocsr(), 1), p)
        return spla.splu(Ms.tocsc()).solve(p)


class DiagSolver:
    """Steps (a)-(c) for one sample and one (dT, alpha, N); the N shifted matrices of
    step (b) do not change between parareal iterations of a linear problem, so each is
    factorised once, when first needed, and reused (the same solves, not repeated)."""

    def __init__(self, dim: int, n: int, a: np.ndarray, dT: float, alpha: float, N: int):
        self.N = N
        self.FN = dft_matrix(N)
        self.Lam = scaling(N, alpha)
        self.lam = eigenvalues(N, alpha)
        self.shifted = ShiftedSolver(dim, n, a, dT)
        self.lu = [None] * N

    def _solve_k(self, k: int, p: np.ndarray) -> np.ndarray:
        S = self.shifted
        if S.dim == 1:
            return S.solve(self.lam[k], p)
        if self.lu[k] is None:
            Ms = self.lam[k] * sp.identity(S.Nx, dtype=np.complex128, format="csr") + S.dT * S.A
            self.lu[k] = spla.splu(Ms.tocsc())
        return self.lu[k].solve(p)

    def solve(self, r: np.ndarray) -> np.ndarray:
        """Solve (C_alpha (x) I + dT I (x) A) u = r; r is [N, Nx] real.  Returns the real
        part; the imaginary part is checked to vanish (r real)."""
        assert r.shape[0] == self.N
        p = self.FN.conj().T @ (self.Lam[:, None] * r)                        # step (a)
        q = np.stack([self._solve_k(k, p[k]) for k in range(self.N)])         # step (b)
        u = (1.0 / self.Lam)[:, None] * (self.FN @ q)                           # step (c)
        scale = max(np.abs(u.real).max(), 1e-300)
        assert np.abs(u.imag).max() <= 1e-8 * scale, "diagonalised CGC lost conjugate symmetry"
        return u.real


def diag_solve(dim: int, n: int, a: np.ndarray, dT: float, alpha: float, r: np.ndarray) -> np.ndarray:
    """Steps (a)-(c): solve (C_alpha (x) I + dT I (x) A) u = r; r is [N, Nx] real.

    Returns the real part; the imaginary part is checked to vanish (r real).
    """
    return DiagSolver(dim, n, a, dT, alpha, r.shape[0]).solve(r)


def all_at_once_matrix(dim: int, n: int, a: np.ndarray, dT: float, alpha: float, N: int) -> sp.csr_matrix:
    """C_alpha (x) I_x + dT I_t (x) A as a sparse matrix (for brute-force checks)."""
    A = op.assemble(dim, n, a)
    Nx = A.shape[0]
    return (sp.kron(sp.csr_matrix(c_alpha(N, alpha)), sp.identity(Nx))
            + dT * sp.kron(sp.identity(N), A)).tocsr()


def dense_solve(dim: int, n: int, a: np.ndarray, dT: float, alpha: float, r: np.ndarray) -> np.ndarray:
    """Brute-force solve of the all-at-once system (tiny sizes only)."""
    N = r.shape[0]
    K = all_at_once_matrix(dim, n, a, dT, alpha, N).toarray()
    return np.linalg.solve(K, r.reshape(-1)).reshape(r.shape)
