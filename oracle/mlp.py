"""Learned initial guess: a small MLP mapping xi to coarse-restricted coarse-point states.

This replaces the gPC map of Algorithm 3 step 6 by a network trained on solutions the
method itself produces (the learned-initial-guess pattern); it does not change the
parareal iteration.  Plain FP64 NumPy; optionally the rounding points of the BF16
kernels are mirrored (round-to-nearest-even to bfloat16 of the GEMM operands) so that a
GPU result can be compared tightly.

  pre1 = X W1 + b1,  h1 = GELU(pre1)
  pre2 = h1 W2 + b2, h2 = GELU(pre2)
  Y    = h2 W3 + b3
  loss = mean((Y - T)^2)            (targets z-scored per output)
GELU is the exact form x Phi(x).  Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias
correction.  Weight layout: W [in][out] row-major, so X [B][in] @ W.

Restriction / prolongation between the n x n grid (h = 1/(n+1)) and the nc x nc coarse
grid (H = 1/(nc+1)): bilinear interpolation with zero Dirichlet values on the boundary,
evaluated at the other grid's nodes (reading: "coarse-restricted" = point values of the
bilinear interpolant).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import erf

SQRT1_2 = 1.0 / math.sqrt(2.0)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round-to-nearest-even on the float32 bit pattern), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x * SQRT1_2))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x * SQRT1_2)) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


@dataclasses.dataclass
class Params:
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    W3: np.ndarray
    b3: np.ndarray

    def flat(self) -> np.ndarray:
        return np.concatenate([a.ravel() for a in (self.W1, self.b1, self.W2, self.b2, self.W3, self.b3)])

    @staticmethod
    def shapes(n_in, hidden, n_out):
        return [(n_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, n_out), (n_out,)]

    @staticmethod
    def from_flat(v, n_in, hidden, n_out) -> "Params":
        out, o = [], 0
        for s in Params.shapes(n_in, hidden, n_out):
            k = int(np.prod(s))
            out.append(np.array(v[o:o + k], dtype=np.float64).reshape(s))
            o += k
        return Params(*out)


def forward(p: Params, X: np.ndarray, mirror_bf16: bool = False):
    r = bf16_round if mirror_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    Xb = r(X)
    pre1 = Xb @ r(p.W1) + p.b1
    h1 = gelu(pre1)
    h1b = r(h1)
    pre2 = h1b @ r(p.W2) + p.b2
    h2 = gelu(pre2)
    h2b = r(h2)
    Y = h2b @ r(p.W3) + p.b3
    return Y, (Xb, pre1, h1b, pre2, h2b)


def loss_and_grad(p: Params, X: np.ndarray, T: np.ndarray, mirror_bf16: bool = False):
    """MSE loss and its gradient (dict of arrays shaped like the parameters)."""
    r = bf16_round if mirror_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    Y, (Xb, pre1, h1b, pre2, h2b) = forward(p, X, mirror_bf16)
    B, O = Y.shape
    dY = 2.0 * (Y - T) / (B * O)
    loss = float(np.mean((Y - T) ** 2))
    dYb = r(dY)
    g = {}
    g["W3"] = h2b.T @ dYb
    g["b3"] = dY.sum(0)
    dpre2 = (dYb @ r(p.W3).T) * gelu_grad(pre2)
    dpre2b = r(dpre2)
    g["W2"] = h1b.T @ dpre2b
    g["b2"] = dpre2.sum(0)
    dpre1 = (dpre2b @ r(p.W2).T) * gelu_grad(pre1)
    dpre1b = r(dpre1)
    g["W1"] = Xb.T @ dpre1b
    g["b1"] = dpre1.sum(0)
    return loss, g


def adam_step(p: Params, g: dict, m: dict, v: dict, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        setattr(p, k, getattr(p, k) - lr * mh / (np.sqrt(vh) + eps))


def zscore(Y: np.ndarray):
    """Per-output mean and population standard deviation over the rows (a zero
    deviation is replaced by 1) and the z-scored targets."""
    Y = np.asarray(Y, dtype=np.float64)
    mu = Y.mean(0)
    sd = np.sqrt(((Y - mu) ** 2).mean(0))
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd, (Y - mu) / sd


# ---------------------------------------------------------------- grid transfer
def _interp_matrix_1d(n_from: int, n_to: int) -> np.ndarray:
    """Linear interpolation (zero end values) from n_from interior nodes on (0,1) to the
    n_to interior nodes of the other grid; returns [n_to][n_from]."""
    h = 1.0 / (n_from + 1)
    x = (np.arange(n_to) + 1.0) / (n_to + 1)
    M = np.zeros((n_to, n_from))
    for q, xq in enumerate(x):
        s = xq / h - 1.0            # position in units of from-nodes (node i at s = i)
        i0 = int(math.floor(s))
        t = s - i0
        if 0 <= i0 < n_from:
            M[q, i0] += 1.0 - t
        if 0 <= i0 + 1 < n_from:
            M[q, i0 + 1] += t
    return M


def restrict(U: np.ndarray, n: int, nc: int) -> np.ndarray:
    """[..., n*n] (x fastest) -> [..., nc*nc], bilinear point values."""
    R = _interp_matrix_1d(n, nc)
    V = np.asarray(U).reshape(U.shape[:-1] + (n, n))       # [..., y, x]
    W = np.einsum("ab,...bc,dc->...ad", R, V, R)
    return W.reshape(U.shape[:-1] + (nc * nc,))


def prolong(Uc: np.ndarray, nc: int, n: int) -> np.ndarray:
    """[..., nc*nc] -> [..., n*n], bilinear interpolation."""
    P = _interp_matrix_1d(nc, n)
    V = np.asarray(Uc).reshape(Uc.shape[:-1] + (nc, nc))
    W = np.einsum("ab,...bc,dc->...ad", P, V, P)
    return W.reshape(Uc.shape[:-1] + (n * n,))
