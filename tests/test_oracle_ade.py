"""Pins of the oracle's P1 finite elements and parareal for the Section 5.1 example.

Independent checks: on the diagonal-cut uniform mesh the P1 stiffness matrix is the
five-point Laplacian and the mass matrix has the known entries h^2/2 and h^2/12; the
mass matrix integrates 1 to the area; div b = 0 makes the exactly integrated advection
matrix skew on the interior and exact on constants and linear functions; the stiffness
matrix passes the patch test; the assembled steady problem converges at second order on
a manufactured solution; the source, split as exp(-t)(g0 + a g1), equals the formula of
Section 5.1 typed as printed; the diagonalised coarse solve equals a dense solve of the
all-at-once system; Algorithm 1 reaches the serial fine solution at k = N exactly and the
serial fine solution is the fixed point of Algorithm 2; J fine steps equal one sparse
solve of the J-step space-time system; the Legendre basis is orthonormal under
Gauss-Legendre quadrature, agrees with numpy's Legendre series, and the gPC fit recovers
a polynomial map exactly.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import ade, fem, gpc, snapshot


@pytest.mark.parametrize("n", [3, 6])
def test_stiffness_is_five_point_laplacian(n):
    M, K, B, _ = fem.assemble(n, 0.1)
    K = K.toarray()
    ref = np.zeros_like(K)
    for j in range(n):
        for i in range(n):
            p = j * n + i
            ref[p, p] = 4.0
            for di, dj in [(-1, 0), (1, 0), (0, -1), (0, 1)]:
                if 0 <= i + di < n and 0 <= j + dj < n:
                    ref[p, (j + dj) * n + i + di] = -1.0
    assert np.abs(K - ref).max() < 1e-12


@pytest.mark.parametrize("n", [3, 6])
def test_mass_entries_and_area(n):
    h = 1.0 / (n + 1)
    Mf, _, _ = fem.assemble_full(n, 0.1)
    assert abs(Mf.sum() - 1.0) < 1e-12
    M = fem.assemble(n, 0.1)[0].toarray()
    for j in range(n):
        for i in range(n):
            p = j * n + i
            assert abs(M[p, p] - h * h / 2) < 1e-15
            for di, dj in [(-1, 0), (1, 0), (0, -1), (0, 1), (1, 1), (-1, -1)]:
                if 0 <= i + di < n and 0 <= j + dj < n:
                    assert abs(M[p, (j + dj) * n + i + di] - h * h / 12) < 1e-15
            for di, dj in [(1, -1), (-1, 1)]:
                if 0 <= i + di < n and 0 <= j + dj < n:
                    assert M[p, (j + dj) * n + i + di] == 0.0


def test_advection_skew_and_exact_on_linears():
    n, beta = 5, 0.37
    Mf, Kf, Bf = fem.assemble_full(n, beta)
    X = fem.coordinates(n)
    idx = fem.interior(n)
    B = Bf[idx][:, idx].toarray()
    assert np.abs(B + B.T).max() < 1e-14
    one = np.ones(X.shape[0])
    assert np.abs(Bf @ one).max() < 1e-14
    # b . grad x1 = beta x2 and b . grad x2 = beta x1 (both linear: the interpolants are exact)
    assert np.abs(Bf @ X[:, 0] - beta * (Mf @ X[:, 1])).max() < 1e-14
    assert np.abs(Bf @ X[:, 1] - beta * (Mf @ X[:, 0])).max() < 1e-14
    # patch test: linear functions are discretely harmonic at interior rows
    lin = 0.3 + 1.7 * X[:, 0] - 0.4 * X[:, 1]
    assert np.abs((Kf @ lin)[idx]).max() < 1e-12


def test_steady_problem_second_order_convergence():
    a, beta = 1.3, 0.1
    errs = []
    for n in [9, 19, 39]:
        Mf, Kf, Bf = fem.assemble_full(n, beta)
        X = fem.coordinates(n)
        idx = fem.interior(n)
        x1, x2 = X[:, 0], X[:, 1]
        u = np.sin(np.pi * x1) * np.sin(np.pi * x2)
        f = (2 * a * np.pi ** 2 * u
             + beta * x2 * np.pi * np.cos(np.pi * x1) * np.sin(np.pi * x2)
             + beta * x1 * np.sin(np.pi * x1) * np.pi * np.cos(np.pi * x2))
        A = (a * Kf + Bf)[idx][:, idx].tocsc()
        uh = spla.spsolve(A, (Mf @ f)[idx])
        errs.append(np.abs(uh - u[idx]).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_source_split_matches_printed_formula():
    n, beta = 4, 0.1 * math.sin(math.pi / 2)
    g0, g1 = fem.source_parts(n, beta)
    X = fem.coordinates(n)
    x1, x2 = X[:, 0], X[:, 1]
    for xi, t in [(2.3, 0.0), (4.9, 0.41), (5.7, 1.0)]:
        a = 0.5 * (2 + math.cos(math.pi * xi) ** 2)
        printed = math.exp(-t) * (
            -np.sin(np.pi * x1) * np.sin(2 * np.pi * x2)
            + 0.5 * np.pi ** 2 * (2 + math.cos(math.pi * xi) ** 2) * np.sin(np.pi * x1) * np.sin(2 * np.pi * x2)
            + 0.05 * np.pi * math.sin(math.pi / 2) * x2 * np.cos(np.pi * x1) * np.sin(2 * np.pi * x2)
            + 0.1 * np.pi * math.sin(math.pi / 2) * x1 * np.sin(np.pi * x1) * np.cos(2 * np.pi * x2))
        assert np.abs(math.exp(-t) * (g0 + a * g1) - printed).max() < 1e-12
        assert abs(fem.diffusion(xi) - a) < 1e-15


def _props(n=4, a=1.2, T=1.0, N=4, J=3, beta=0.1):
    return ade.ADEPropagators(fem.Discretisation(n, beta), a, T, N, J)


def test_fine_steps_equal_space_time_solve():
    p = _props(n=4, J=5)
    d = p.disc
    rng = np.random.default_rng(0)
    v = rng.standard_normal(d.Nx)
    s = 2
    # rows j: (M + dt L) w_{j+1} - M w_j = dt F(t_j+1), w_0 = v
    J, Nx = p.J, d.Nx
    A = sp.lil_matrix((J * Nx, J * Nx))
    rhs = np.zeros(J * Nx)
    Ad = (d.M + p.dt * p.L).toarray()
    Md = d.M.toarray()
    for j in range(J):
        A[j * Nx:(j + 1) * Nx, j * Nx:(j + 1) * Nx] = Ad
        if j > 0:
            A[j * Nx:(j + 1) * Nx, (j - 1) * Nx:j * Nx] = -Md
        rhs[j * Nx:(j + 1) * Nx] = p.dt * d.load(p.a, s * p.dT + (j + 1) * p.dt)
    rhs[:Nx] += Md @ v
    W = spla.spsolve(A.tocsc(), rhs)
    assert np.abs(W[-Nx:] - p.F(v, s)).max() < 1e-13 * max(1.0, np.abs(W).max())


def test_diag_solve_equals_dense_all_at_once():
    p = _props(n=3, N=6)
    alpha = 0.1
    rng = np.random.default_rng(1)
    r = rng.standard_normal((p.N, p.disc.Nx))
    u = ade.ADEDiagSolver(p, alpha).solve(r)
    K = ade.all_at_once_matrix(p, alpha).toarray()
    ref = np.linalg.solve(K, r.reshape(-1)).reshape(r.shape)
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()


def test_alg1_terminates_at_k_equal_N_and_fixed_point_of_alg2():
    p = _props(n=4, N=5, J=4)
    u0 = p.disc.u0
    ref = ade.serial_fine(p, u0)
    U0 = np.zeros_like(ref)
    h1 = ade.parareal_sequential(p, u0, U0, 0.0, p.N, ref)
    assert np.abs(h1.U - ref).max() < 1e-12 * np.abs(ref).max()
    # after k iterations the first k slices are exact (finite termination slice by slice)
    for k in range(1, p.N + 1):
        assert h1.errors[k][:k].max() < 1e-12 * np.abs(ref).max()
    # serial fine is the fixed point of the diagonalised CGC iteration
    h2 = ade.parareal_diag(p, 0.1, u0, ref, 0.0, 1, ref)
    assert np.abs(h2.U - ref).max() < 1e-12 * np.abs(ref).max()
    h3 = ade.parareal_diag(p, 0.1, u0, U0, 1e-13, 60, ref)
    assert h3.iters < 60 and np.abs(h3.U - ref).max() < 1e-11 * np.abs(ref).max()


def test_legendre_orthonormal_and_matches_numpy():
    x, w = np.polynomial.legendre.leggauss(20)
    w = w / 2.0
    P = gpc.legendre_1d(x, 9)
    assert np.abs((P * w) @ P.T - np.eye(10)).max() < 1e-13
    z = np.linspace(-1, 1, 7)
    for m in range(10):
        c = np.zeros(m + 1)
        c[m] = 1.0
        assert np.abs(gpc.legendre_1d(z, 9)[m] - math.sqrt(2 * m + 1) * np.polynomial.legendre.legval(z, c)).max() < 1e-13


def test_legendre_gpc_exact_recovery():
    rng = np.random.default_rng(4)
    z = rng.uniform(-1, 1, (10, 1))
    L = 30
    basis = rng.standard_normal((3, L))

    def field(x):
        x = x[:, 0]
        return np.stack([1 + x - 2 * x ** 3, x ** 2, 0.5 * x ** 4 - x], 1)

    S = field(z) @ basis
    kl = snapshot.build(S, 1e-14)
    g = gpc.fit(kl, S, z, 4, basis="legendre")
    zt = rng.uniform(-1, 1, (6, 1))
    assert np.abs(gpc.predict(g, zt) - field(zt) @ basis).max() < 1e-10
