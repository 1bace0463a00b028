"""P1 finite elements for the advection-diffusion example of Section 5.1.

Problem (Section 5.1): on (0,1)^2 with zero Dirichlet data,
    u_t - div(a grad u) + b . grad u = f(x, t; xi),   u(x, 0) = u_0(x),
with a = 0.5 (2 + cos(pi xi)^2) constant in space, b = beta (x2, x1) (beta = 0.1 sin(pi/2)),
    f = exp(-t) [ -s1 s2 + 0.5 pi^2 (2 + cos(pi xi)^2) s1 s2
                  + 0.5 beta pi x2 cos(pi x1) s2 + beta pi x1 s1 cos(2 pi x2) ],
s1 = sin(pi x1), s2 = sin(2 pi x2), u_0 = s1 s2.  Since 0.5 pi^2 (2 + cos^2) = pi^2 a,
    f = exp(-t) (g0(x) + a g1(x)),  g1 = pi^2 s1 s2,
    g0 = -s1 s2 + 0.5 beta pi x2 cos(pi x1) s2 + beta pi x1 s1 cos(2 pi x2).

Readings (the paper names P1 elements and h = 1/20 only):
  * mesh: the uniform grid x = (i h, j h), i, j = 0..n+1, h = 1/(n+1); every cell
    [ih,(i+1)h] x [jh,(j+1)h] is cut by its diagonal from (i, j) to (i+1, j+1) into the
    triangles {(i,j), (i+1,j), (i+1,j+1)} and {(i,j), (i+1,j+1), (i,j+1)};
  * the unknowns are the n^2 interior nodal values, node (i, j) (1-based grid index) at
    position (j-1) n + (i-1), x1 fastest;
  * mass M_ij = int phi_i phi_j, stiffness K_ij = int grad phi_i . grad phi_j and
    advection B_ij = int (b . grad phi_j) phi_i, all integrated exactly (b is linear);
  * load: F_i(t) = sum over all grid nodes j (boundary included) of M_ij f(x_j, t), the
    consistent mass matrix applied to the nodal interpolant of f.
The semi-discrete system is M u' + (a K + B) u = F(t).

Element integrals used (P1 on a triangle T of area |T|, barycentric phi_k):
    int_T phi_i phi_k = |T| (1 + delta_ik) / 12,
    grad phi_k constant on T,
    int_T b phi_i = sum_k b(x_k) |T| (1 + delta_ik) / 12   (b linear, b = sum_k b(x_k) phi_k).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def grid_index(n: int, i: int, j: int) -> int:
    """Index of grid node (i, j), i, j = 0..n+1, in the full (n+2)^2 numbering."""
    return j * (n + 2) + i


def triangles(n: int) -> list:
    """The 2 (n+1)^2 triangles as triples of full-grid node indices (counter-clockwise)."""
    out = []
    for j in range(n + 1):
        for i in range(n + 1):
            p00 = grid_index(n, i, j)
            p10 = grid_index(n, i + 1, j)
            p11 = grid_index(n, i + 1, j + 1)
            p01 = grid_index(n, i, j + 1)
            out.append((p00, p10, p11))
            out.append((p00, p11, p01))
    return out


def coordinates(n: int) -> np.ndarray:
    """[(n+2)^2, 2] node positions of the full grid."""
    h = 1.0 / (n + 1)
    xs = np.arange(n + 2) * h
    X1, X2 = np.meshgrid(xs, xs, indexing="xy")     # X1[j, i] = i h
    return np.stack([X1.reshape(-1), X2.reshape(-1)], axis=1)


def interior(n: int) -> np.ndarray:
    """Full-grid indices of the interior nodes, in unknown order (x1 fastest)."""
    return np.array([grid_index(n, i, j) for j in range(1, n + 1) for i in range(1, n + 1)])


def assemble_full(n: int, beta: float):
    """M, K, B over all (n+2)^2 grid nodes (CSR), by the element loop."""
    X = coordinates(n)
    nn = X.shape[0]
    rows, cols, vm, vk, vb = [], [], [], [], []
    for tri in triangles(n):
        P = X[list(tri)]                                   # [3, 2]
        D = np.array([[1.0, P[0, 0], P[0, 1]],
                      [1.0, P[1, 0], P[1, 1]],
                      [1.0, P[2, 0], P[2, 1]]])
        area = 0.5 * abs(np.linalg.det(D))
        coef = np.linalg.inv(D)                            # phi_k(x) = coef[0,k] + coef[1,k] x1 + coef[2,k] x2
        grads = coef[1:, :].T                              # [3, 2] grad phi_k
        bv = beta * np.stack([P[:, 1], P[:, 0]], axis=1)   # b at the vertices [3, 2]
        for a_ in range(3):
            # int_T b phi_a
            w = np.array([(1.0 + (a_ == k)) for k in range(3)]) * area / 12.0
            bphi = (w[:, None] * bv).sum(axis=0)
            for c_ in range(3):
                rows.append(tri[a_])
                cols.append(tri[c_])
                vm.append(area * (1.0 + (a_ == c_)) / 12.0)
                vk.append(area * float(grads[a_] @ grads[c_]))
                vb.append(float(bphi @ grads[c_]))
    shape = (nn, nn)
    M = sp.coo_matrix((vm, (rows, cols)), shape=shape).tocsr()
    K = sp.coo_matrix((vk, (rows, cols)), shape=shape).tocsr()
    B = sp.coo_matrix((vb, (rows, cols)), shape=shape).tocsr()
    return M, K, B


def assemble(n: int, beta: float):
    """Interior blocks (M, K, B) [n^2, n^2] and the full mass rows Mfull[interior, :]."""
    M, K, B = assemble_full(n, beta)
    idx = interior(n)
    return (M[idx][:, idx].tocsr(), K[idx][:, idx].tocsr(), B[idx][:, idx].tocsr(),
            M[idx].tocsr())


def source_parts(n: int, beta: float):
    """Nodal values of g0 and g1 on the full grid (f = exp(-t) (g0 + a g1))."""
    X = coordinates(n)
    x1, x2 = X[:, 0], X[:, 1]
    s1, s2 = np.sin(np.pi * x1), np.sin(2.0 * np.pi * x2)
    g1 = np.pi ** 2 * s1 * s2
    g0 = (-s1 * s2 + 0.5 * beta * np.pi * x2 * np.cos(np.pi * x1) * s2
          + beta * np.pi * x1 * s1 * np.cos(2.0 * np.pi * x2))
    return g0, g1


def initial_value(n: int) -> np.ndarray:
    """u_0 = sin(pi x1) sin(2 pi x2) at the interior nodes."""
    X = coordinates(n)[interior(n)]
    return np.sin(np.pi * X[:, 0]) * np.sin(2.0 * np.pi * X[:, 1])


def diffusion(xi: np.ndarray) -> np.ndarray:
    """a(xi) = 0.5 (2 + cos(pi xi)^2) (Section 5.1)."""
    return 0.5 * (2.0 + np.cos(np.pi * np.asarray(xi, dtype=np.float64)) ** 2)


class Discretisation:
    """Matrices and load pieces of one grid (shared by every sample)."""

    def __init__(self, n: int, beta: float):
        self.n, self.beta = n, beta
        self.Nx = n * n
        self.M, self.K, self.B, Mrows = assemble(n, beta)
        g0, g1 = source_parts(n, beta)
        self.l0 = Mrows @ g0
        self.l1 = Mrows @ g1
        self.u0 = initial_value(n)

    def operator(self, a: float) -> sp.csr_matrix:
        """L(a) = a K + B."""
        return (a * self.K + self.B).tocsr()

    def load(self, a: float, t: float) -> np.ndarray:
        """F(t) = exp(-t) (l0 + a l1)."""
        return np.exp(-t) * (self.l0 + a * self.l1)
