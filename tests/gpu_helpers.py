"""Helpers shared by the GPU parity tests (inputs from `workloads`, references from `oracle`)."""
from __future__ import annotations

import sys

import numpy as np

import workloads as W
from oracle import field


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def oracle_faces(w: W.Workload, xi: np.ndarray) -> np.ndarray:
    lam, Phi = field.kl_modes(w.dim, w.n, w.d, w.corr_len, w.sigma)
    return field.synthesize(lam, Phi, xi)
