"""Input random field: KL expansion of a Gaussian field with exponential covariance.

The paper parameterises random inputs by a truncated KL expansion (Section 2,
separated representation; Section 2.1).  For the input field of the diffusion
coefficient the covariance sigma^2 exp(-|x-y|/l) on [0,1] has closed-form
eigenpairs (Ghanem-Spanos): with c = 1/l and s = x - 1/2,
  even modes: c - w tan(w/2) = 0,  phi = cos(w s) / sqrt(1/2 + sin(w)/(2w))
  odd  modes: w + c tan(w/2) = 0,  phi = sin(w s) / sqrt(1/2 - sin(w)/(2w))
  eigenvalue: sigma^2 * 2c / (w^2 + c^2).
In 2D the covariance is taken separable, sigma^2 exp(-|dx|/l - |dy|/l), so the
eigenpairs are products of 1D ones; modes are ordered by (-lambda, i+j, i).
log a(x, xi) = sum_k sqrt(lambda_k) phi_k(x) xi_k, a = exp(log a), evaluated at
the cell faces of the finite-difference grid (see operator.py for layout).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def kl_roots_1d(corr_len: float, count: int) -> list[tuple[float, int]]:
    """First `count` roots w (ascending) with parity 0 (even) / 1 (odd)."""
    c = 1.0 / corr_len
    out = []
    k = 0
    while len(out) < count:
        lo, hi = k * math.pi, (k + 1) * math.pi
        eps = 1e-13 * max(1.0, hi)
        if k % 2 == 0:   # even: w in (2m pi, 2m pi + pi)
            f = lambda w: c * math.cos(w / 2) - w * math.sin(w / 2)
        else:            # odd: w in ((2m+1)pi, (2m+2)pi)
            f = lambda w: w * math.cos(w / 2) + c * math.sin(w / 2)
        w = brentq(f, lo + eps if k > 0 else 0.0 + 1e-300, hi - eps, xtol=1e-15, rtol=1e-15, maxiter=200)
        out.append((w, k % 2))
        k += 1
    return out


def kl_1d(corr_len: float, sigma: float, count: int):
    """Eigenvalues (descending) and eigenfunction callables of the 1D covariance."""
    c = 1.0 / corr_len
    lam, funcs = [], []
    for w, parity in kl_roots_1d(corr_len, count):
        lam.append(sigma * sigma * 2.0 * c / (w * w + c * c))
        if parity == 0:
            nrm = math.sqrt(0.5 + math.sin(w) / (2.0 * w))
            funcs.append(lambda x, w=w, nrm=nrm: np.cos(w * (np.asarray(x) - 0.5)) / nrm)
        else:
            nrm = math.sqrt(0.5 - math.sin(w) / (2.0 * w))
            funcs.append(lambda x, w=w, nrm=nrm: np.sin(w * (np.asarray(x) - 0.5)) / nrm)
    return np.array(lam), funcs


def face_coords(dim: int, n: int):
    """Coordinates of the faces in the library's face order.

    1D: faces f = 0..n at x = (f + 1/2) h.
    2D: x-faces first, index j*(n+1) + f at ((f+1/2)h, (j+1)h), j = 0..n-1, f = 0..n;
        then y-faces, index n(n+1) + f*n + i at ((i+1)h, (f+1/2)h).
    """
    h = 1.0 / (n + 1)
    if dim == 1:
        return ((np.arange(n + 1) + 0.5) * h,)
    f = np.arange(n + 1)
    i = np.arange(n)
    xf_x = np.tile((f + 0.5) * h, n)
    xf_y = np.repeat((i + 1.0) * h, n + 1)
    yf_x = np.tile((i + 1.0) * h, n + 1)
    yf_y = np.repeat((f + 0.5) * h, n)
    return np.concatenate([xf_x, yf_x]), np.concatenate([xf_y, yf_y])


def kl_modes(dim: int, n: int, d: int, corr_len: float, sigma: float):
    """Return (lambda [d], Phi [d, F]) of the first d KL modes evaluated at faces."""
    if dim == 1:
        lam, funcs = kl_1d(corr_len, sigma, d)
        (x,) = face_coords(1, n)
        return lam, np.stack([f(x) for f in funcs])
    # separable 2D: enough 1D modes that every product among the first d is present
    m1 = d + 1
    lam1, funcs1 = kl_1d(corr_len, 1.0, m1)
    cand = []
    for i in range(m1):
        for j in range(m1):
            cand.append((-(lam1[i] * lam1[j]), i + j, i, j))
    cand.sort()
    x, y = face_coords(2, n)
    lam, rows = [], []
    for negl, _, i, j in cand[:d]:
        lam.append(sigma * sigma * (-negl))
        rows.append(funcs1[i](x) * funcs1[j](y))
    return np.array(lam), np.stack(rows)


def synthesize(lam: np.ndarray, Phi: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """a[m, f] = exp(sum_k sqrt(lam_k) Phi[k, f] xi[m, k])  (FP64)."""
    xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
    out = np.empty((xi.shape[0], Phi.shape[1]))
    for m in range(xi.shape[0]):
        s = np.zeros(Phi.shape[1])
        for k in range(len(lam)):
            s += math.sqrt(lam[k]) * xi[m, k] * Phi[k]
        out[m] = np.exp(s)
    return out
