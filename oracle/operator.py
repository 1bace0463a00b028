"""Finite-difference diffusion operator A(xi) with zero Dirichlet data.

The linear problem class of Section 4.1 (u' + A u = f) with A the discrete
-div(a grad .) on the unit interval / square, h = 1/(n+1):
  1D: (A u)_i = -[a_{i+1/2}(u_{i+1}-u_i) - a_{i-1/2}(u_i-u_{i-1})] / h^2
  2D: the same along x and along y with the face coefficients of each face.
Face layout (see field.face_coords): 1D face f sits between nodes f-1 and f
(0-based nodes, node -1 and n are the boundary); 2D x-face j*(n+1)+f between
(f-1, j) and (f, j); y-face n(n+1) + f*n + i between (i, f-1) and (i, f).
Node (i, j) has unknown index j*n + i (x fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def assemble(dim: int, n: int, a: np.ndarray) -> sp.csr_matrix:
    """Sparse A for one sample's face coefficients a [F]."""
    h2 = (1.0 / (n + 1)) ** 2
    rows, cols, vals = [], [], []
    if dim == 1:
        for i in range(n):
            aw, ae = a[i], a[i + 1]
            rows.append(i); cols.append(i); vals.append((aw + ae) / h2)
            if i > 0:
                rows.append(i); cols.append(i - 1); vals.append(-aw / h2)
            if i < n - 1:
                rows.append(i); cols.append(i + 1); vals.append(-ae / h2)
        return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    off = n * (n + 1)
    for j in range(n):
        for i in range(n):
            p = j * n + i
            aw = a[j * (n + 1) + i]
            ae = a[j * (n + 1) + i + 1]
            as_ = a[off + j * n + i]
            an = a[off + (j + 1) * n + i]
            rows.append(p); cols.append(p); vals.append((aw + ae + as_ + an) / h2)
            if i > 0:
                rows.append(p); cols.append(p - 1); vals.append(-aw / h2)
            if i < n - 1:
                rows.append(p); cols.append(p + 1); vals.append(-ae / h2)
            if j > 0:
                rows.append(p); cols.append(p - n); vals.append(-as_ / h2)
            if j < n - 1:
                rows.append(p); cols.append(p + n); vals.append(-an / h2)
    N = n * n
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def apply(dim: int, n: int, a: np.ndarray, u: np.ndarray) -> np.ndarray:
    """A u via the assembled sparse matrix."""
    return assemble(dim, n, a) @ u


def bandwidth(dim: int, n: int) -> int:
    return 1 if dim == 1 else n


def to_upper_banded(M: sp.spmatrix, bw: int) -> np.ndarray:
    """Upper banded storage (LAPACK 'ab' layout, lower=False) of a symmetric matrix."""
    Md = M.tocoo()
    N = M.shape[0]
    ab = np.zeros((bw + 1, N), dtype=M.dtype)
    for r, c, v in zip(Md.row, Md.col, Md.data):
        if c >= r:
            ab[bw + r - c, c] = v
    return ab


def to_general_banded(M: sp.spmatrix, bw: int) -> np.ndarray:
    """General banded storage for scipy.linalg.solve_banded((bw, bw), ab, b)."""
    Md = M.tocoo()
    N = M.shape[0]
    ab = np.zeros((2 * bw + 1, N), dtype=M.dtype)
    for r, c, v in zip(Md.row, Md.col, Md.data):
        ab[bw + r - c, c] = v
    return ab
