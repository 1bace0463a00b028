"""Seeded synthetic workloads shared by the CPU oracle and the GPU path.

This module holds problem parameters and random draws only: no step of the
method's arithmetic lives here, so that the oracle and the HIP path can both
take their inputs from it without sharing any computation.

The problem class is the linear parametric diffusion equation
    u' = -A(xi) u + f,  u(0) = u0 = 0,
with A(xi) the finite-difference discretisation of -div(a(x, xi) grad u) on
the unit interval or square with zero Dirichlet data, and log a a truncated
Karhunen-Loeve expansion of a Gaussian field with exponential covariance
(xi_k i.i.d. standard normal).  The parareal method with diagonalised coarse
grid correction (Section 3.2 of the paper) is applied to it, started from a
KL/gPC initial guess (Algorithm 3).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = ["Workload", "CONFIGS", "ModelWorkload", "MODELS", "draw_model_params", "MlpSpec", "MLP_C4", "RaggedSpec", "C3_RAGGED", "draw_xi", "draw_mlp_init", "draw_perms", "get",
           "small_1d", "small_2d"]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dim: int                 # 1 or 2
    n: int                   # interior nodes per dimension, h = 1/(n+1)
    T: float                 # horizon
    N: int                   # coarse slices (power of two)
    J: int                   # fine backward-Euler steps per slice
    alpha: float             # twist parameter of the coarse model, in (0, 1)
    forcing: float           # constant source f
    d: int                   # retained KL terms of the input field
    corr_len: float          # correlation length of the exponential covariance
    sigma: float             # standard deviation of log a
    M: int                   # samples solved in one batch
    precision: str           # "f64" or "f32_refined" (fine path)
    tol: float               # parareal stopping tolerance on the increment
    max_iter: int
    gpc_degree: int          # total degree p of the Hermite gPC surrogate
    n_train: int             # training-set size n_t
    eps_kl: float            # KL truncation tolerance
    seed_train: int
    seed_eval: int

    @property
    def Nx(self) -> int:
        return self.n ** self.dim

    @property
    def n_faces(self) -> int:
        return self.n + 1 if self.dim == 1 else 2 * self.n * (self.n + 1)

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


CONFIGS = {
    # 1D, 127 interior nodes, KL d=4 (corr 0.5, sigma 0.5), N=16, J=32, alpha=1e-2,
    # Hermite gPC degree 3 on 50 training samples, 8 evaluation samples, FP64.
    "c1_1d_n127": Workload("c1_1d_n127", 1, 127, 1.0, 16, 32, 1e-2, 1.0, 4, 0.5, 0.5,
                           8, "f64", 1e-8, 60, 3, 50, 1e-10, 1001, 2001),
    # 2D 128x128, KL d=10 (corr 0.3, sigma 1), N=64, J=64, alpha=1e-4, M=256,
    # FP32 PCG fine path refined to FP64, FP64 coarse correction.
    "c2_2d_n128": Workload("c2_2d_n128", 2, 128, 1.0, 64, 64, 1e-4, 1.0, 10, 0.3, 1.0,
                           256, "f32_refined", 1e-8, 60, 3, 512, 1e-10, 1002, 2002),
    # The c2 problem with the learned initial guess: 4096 training solutions,
    # 512 fresh evaluation samples (gPC degree 3 on the same training set for comparison).
    "c4_2d_n128_mlp": Workload("c4_2d_n128_mlp", 2, 128, 1.0, 64, 64, 1e-4, 1.0, 10, 0.3, 1.0,
                               512, "f32_refined", 1e-8, 60, 3, 4096, 1e-10, 1004, 2004),
    # 2D 512x512, KL d=20 (corr 0.2, sigma 1), N=256, J=128, M=64.
    "c5_2d_n512": Workload("c5_2d_n512", 2, 512, 1.0, 256, 128, 1e-4, 1.0, 20, 0.2, 1.0,
                           64, "f32_refined", 1e-8, 60, 2, 256, 1e-10, 1005, 2005),
}


@dataclasses.dataclass(frozen=True)
class MlpSpec:
    """Learned initial guess: xi [d] -> GELU(hidden) -> GELU(hidden) -> N nc^2 outputs."""
    hidden: int
    nc: int                  # coarse grid (nc x nc interior nodes, H = 1/(nc+1))
    epochs: int
    batch: int
    lr: float
    lr_final: float          # geometric per-epoch decay from lr to lr_final
    seed_init: int
    seed_perm: int


@dataclasses.dataclass(frozen=True)
class RaggedSpec:
    """Uneven batch: per-sample grid size and slice count drawn uniformly."""
    base: Workload           # the shared parameters (n and N are drawn per sample)
    grids: tuple
    slices: tuple


# 1024 samples mixing 64^2, 128^2, 256^2 grids and N in {32, 64, 128}, J = 32, KL d = 10
# (corr 0.3, sigma 1), alpha = 1e-4, f = 1, FP32-refined fine path, coarse-sweep guess.
C3_RAGGED = RaggedSpec(Workload("c3_ragged", 2, 0, 1.0, 0, 32, 1e-4, 1.0, 10, 0.3, 1.0,
                                1024, "f32_refined", 1e-8, 60, 0, 0, 1e-10, 1003, 2003),
                       grids=(64, 128, 256), slices=(32, 64, 128))


MLP_C4 = MlpSpec(hidden=256, nc=32, epochs=1000, batch=64, lr=1e-3, lr_final=1e-5, seed_init=3004, seed_perm=4004)


@dataclasses.dataclass(frozen=True)
class ModelWorkload:
    """One of the Section 5 examples: a scalar random parameter per sample.

    The parameter xi is drawn from `dist` and handed to the solver as the coefficient
    c = coef(xi) (the problem's own parameterisation, part of the input recipe):
      model 1 (advection-diffusion, Section 5.1): xi ~ U[2, 6], c = a = 0.5 (2 + cos(pi xi)^2);
      model 2 (Burgers, Section 5.2): eps ~ U[1, 3], c = eps (viscosity eps / 50);
      model 3 (Allen-Cahn, Section 5.3): eps ~ N(0.53, 0.15^2) truncated to [0.06, 1], c = eps.
    The gPC variable z is xi mapped to [-1, 1] for the uniform laws (Legendre basis) and
    standardised, (eps - 0.53) / 0.15, for the truncated normal (Hermite basis)."""
    name: str
    model: int               # klecgc_model code: 1 ADE_P1, 2 BURGERS, 3 ALLEN_CAHN
    n: int
    T: float
    N: int
    J: int
    alpha: float
    beta: float              # advection scale (model 1)
    M: int                   # evaluation samples
    n_train: int             # training-set size of the snapshot KL (Section 5)
    gpc_degree: int
    eps_kl: float
    err_tol: float           # the error threshold of Section 5 (mean error vs the serial fine solution)
    max_iter: int
    seed_train: int
    seed_eval: int

    @property
    def Nx(self) -> int:
        return self.n * self.n if self.model == 1 else self.n

    def replace(self, **kw) -> "ModelWorkload":
        return dataclasses.replace(self, **kw)


MODELS = {
    # Section 5.1: P1 FEM h = 1/20 (19^2 unknowns), T = 1, dT = 1/24, dt = dT/50, alpha = 0.1,
    # n_t = 10, eps_KL = 1e-10, 1000 samples, beta = 0.1 sin(pi/2).
    "f3_ade_s51": ModelWorkload("f3_ade_s51", 1, 19, 1.0, 24, 50, 0.1, 0.1, 1000, 10, 3, 1e-10, 1e-10, 25,
                                1051, 2051),
    # Section 5.2: Burgers, dx = 1/100 (99 unknowns), T = 2, dT = 2/25, dt = dT/40, n_t = 36,
    # 1000 samples; alpha is not given for the nonlinear examples (reading: 0.1 as in 5.1).
    "f1_burgers_s52": ModelWorkload("f1_burgers_s52", 2, 99, 2.0, 25, 40, 0.1, 0.0, 1000, 36, 4, 1e-10, 1e-10,
                                    25, 1052, 2052),
    # Section 5.3: Allen-Cahn on (-1, 1), dx = 1/128 (255 unknowns), T = 30, dT = 1, dt = dT/48,
    # n_t = 10, 1000 samples, alpha = 0.1 (reading).
    "f1_allen_cahn_s53": ModelWorkload("f1_allen_cahn_s53", 3, 255, 30.0, 30, 48, 0.1, 0.0, 1000, 10, 3, 1e-10,
                                       1e-10, 25, 1053, 2053),
}


def draw_model_params(w: ModelWorkload, M: int, seed: int):
    """(xi [M], coefficient c [M], gPC variable z [M, 1]) for a Section 5 example."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if w.model == 1:
        xi = rng.uniform(2.0, 6.0, size=M)
        return xi, 0.5 * (2.0 + np.cos(np.pi * xi) ** 2), ((xi - 4.0) / 2.0)[:, None]
    if w.model == 2:
        eps = rng.uniform(1.0, 3.0, size=M)
        return eps, eps.copy(), (eps - 2.0)[:, None]
    out = np.empty(0)
    while out.size < M:
        e = 0.53 + 0.15 * rng.standard_normal(2 * M)
        out = np.concatenate([out, e[(e >= 0.06) & (e <= 1.0)]])
    eps = out[:M]
    return eps, eps.copy(), ((eps - 0.53) / 0.15)[:, None]


def get(name: str) -> Workload:
    return CONFIGS[name]


def small_1d(**kw) -> Workload:
    """A small 1D case that the oracle finishes in well under a second."""
    base = Workload("small_1d", 1, 31, 1.0, 8, 8, 1e-2, 1.0, 4, 0.5, 0.5,
                    4, "f64", 1e-8, 60, 2, 30, 1e-10, 11, 21)
    return base.replace(**kw)


def small_2d(**kw) -> Workload:
    """A small 2D case (several tiles plus a ragged tail in every direction)."""
    base = Workload("small_2d", 2, 20, 1.0, 8, 8, 1e-2, 1.0, 6, 0.3, 1.0,
                    3, "f64", 1e-8, 60, 2, 40, 1e-10, 12, 22)
    return base.replace(**kw)


def draw_xi(M: int, d: int, seed: int) -> np.ndarray:
    """xi ~ N(0, I_d), M rows, from a seeded PCG64 generator (FP64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((M, d))


def draw_uniform(shape, seed: int) -> np.ndarray:
    """i.i.d. U(0,1) entries (used for the RANDOM initial guess)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(shape)


def draw_ragged(M: int, seed: int, grids=(64, 128, 256), slices=(32, 64, 128)):
    """Uneven batch: per-sample grid size and slice count, uniform categorical."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.integers(0, len(grids), size=M)
    s = rng.integers(0, len(slices), size=M)
    return np.asarray(grids)[g], np.asarray(slices)[s]


def draw_subset(M: int, k: int, seed: int) -> np.ndarray:
    """k distinct sample indices out of M, ascending (the seeded accuracy subset)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(M, size=k, replace=False))


def draw_normal(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal(shape)


def draw_mlp_init(n_in: int, hidden: int, n_out: int, seed: int) -> np.ndarray:
    """Flat FP32 MLP parameters [W1 b1 W2 b2 W3 b3] (W [in][out] row-major): weights
    i.i.d. U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fi, fo in ((n_in, hidden), (hidden, hidden), (hidden, n_out)):
        b = 1.0 / np.sqrt(fi)
        parts.append(rng.uniform(-b, b, size=fi * fo))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def draw_perms(epochs: int, n: int, seed: int) -> np.ndarray:
    """One random permutation of 0..n-1 per epoch, int32 [epochs][n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32) if epochs else \
        np.zeros((0, n), np.int32)


def describe(w: Workload, M: Optional[int] = None) -> dict:
    d = dataclasses.asdict(w)
    if M is not None:
        d["M"] = M
    return d
