"""Initial guesses of the parareal iteration other than the gPC map.

Algorithm 3 starts parareal from the gPC prediction (step 6); its comparators in Section 5
start from a random guess (the distribution is not stated: read as i.i.d. U(0,1) per entry).
The learned guess replaces the gPC map of step 6 and falls back to it per sample when its
first parareal residual is larger: the residual is read as the continuity defect of the
guess after the fine sweep of iteration 0,
    d(U^0) = max_n |F(U^0_{n-1}) - U^0_n|_inf / max_n |U^0_n|_inf,   U^0_0 := u0,
(the jumps the fine propagator leaves between consecutive slices; 1 replaces a zero
denominator), and the guess with the smaller defect is kept (ties keep the learned guess; a
non-finite learned defect counts as larger than any finite fallback defect).

Random numbers: one counter-based generator, SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): entry i of a guess drawn with seed s
is the SplitMix64 output for the state s + (i + 1) * 0x9E3779B97F4A7C15 (mod 2^64), and its
top 53 bits scaled by 2^-53 give a double in [0, 1).  Entries are numbered row-major over
[M][N][Nx].
"""
from __future__ import annotations

import numpy as np

from .prop import Propagators

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(state: np.ndarray) -> np.ndarray:
    """The SplitMix64 output function applied to (already advanced) 64-bit states."""
    z = np.asarray(state, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform_counter(seed: int, first: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) for entries first .. first+count-1 of the stream of `seed`."""
    i = np.arange(first, first + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed) + (i + np.uint64(1)) * GOLDEN
    return (splitmix64(state) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def random_guess(seed: int, M: int, N: int, Nx: int) -> np.ndarray:
    """The RANDOM initial guess [M][N][Nx]: i.i.d. U(0,1) entries."""
    return uniform_counter(seed, 0, M * N * Nx).reshape(M, N, Nx)


def continuity_defect(props: Propagators, u0: np.ndarray, U0: np.ndarray) -> float:
    """max_n |F(U^0_{n-1}) - U^0_n|_inf / max_n |U^0_n|_inf for one sample's guess [N][Nx]."""
    N = U0.shape[0]
    if not (np.all(np.isfinite(U0)) and np.all(np.isfinite(u0))):
        return float("nan")               # F of a non-finite start is not finite
    jumps = [np.abs(props.F(u0 if n == 0 else U0[n - 1]) - U0[n]).max() for n in range(N)]
    num = float(np.max(jumps))            # NaN propagates
    den = float(np.abs(U0).max())
    return num / (den if den > 0 else 1.0)


def choose_guess(props: Propagators, u0: np.ndarray, U_learned: np.ndarray, U_fallback: np.ndarray):
    """Keep the learned guess unless the fallback's continuity defect is strictly smaller
    (or the learned one is NaN and the fallback's is not).
    Returns (guess, used_fallback, defect_learned, defect_fallback)."""
    d_l = continuity_defect(props, u0, U_learned)
    d_f = continuity_defect(props, u0, U_fallback)
    use_f = bool(d_f < d_l or (np.isnan(d_l) and not np.isnan(d_f)))
    return (U_fallback if use_f else U_learned), use_f, d_l, d_f
