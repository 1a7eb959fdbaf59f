"""Kaiser-Bessel blob profile, FP64 (oracle; test infrastructure only).

The paper's Fourier insertion kernel weights each 2D sample's contribution to
nearby voxels by an interpolation window and lets the weights be either
precomputed or evaluated on the fly (Sect. 4.2, "3D Fourier Reconstruction";
the tuning-space bullets there).  The window named for this path is the
generalised Kaiser-Bessel "blob" of radius a, taper alpha and order m:

    b(d^2) = (1 - d^2/a^2)^(m/2) * I_m(alpha * sqrt(1 - d^2/a^2)) / I_m(alpha)
             for d^2 <= a^2, and 0 beyond,

normalised so that b(0) = 1 (the paper is silent on normalisation; the ratio
G/W does not depend on it).  The precomputed variant is a table of N samples
uniform in d^2, looked up with linear interpolation (default) or truncation.

Only tests/, the smoke check and the benchmark's CPU baseline may import this.
"""
from __future__ import annotations

import math

import numpy as np


def bessel_i(m: int, x) -> np.ndarray:
    """I_m(x) from its power series  sum_j (x/2)^(2j+m) / (j! (j+m)!)  in FP64.

    Terms are added until every remaining term is below 1e-18 of the partial
    sum (31 terms at x = 15 for m = 0)."""
    if m < 0:
        raise ValueError("order must be >= 0")
    x = np.asarray(x, dtype=np.float64)
    half = 0.5 * x
    term = half ** m / math.factorial(m)
    total = np.array(term, dtype=np.float64, copy=True)
    q = half * half
    for j in range(1, 400):
        term = term * q / (j * (j + m))
        total = total + term
        if np.all(term <= 1e-18 * total):
            break
    return total


def kb_profile(d2, a: float, alpha: float, m: int = 0) -> np.ndarray:
    """Exact blob value b(d^2); inclusive cut-off at d^2 = a^2, zero beyond."""
    d2 = np.asarray(d2, dtype=np.float64)
    inside = d2 <= a * a
    s = np.where(inside, np.maximum(1.0 - d2 / (a * a), 0.0), 0.0)
    r = np.sqrt(s)
    val = s ** (0.5 * m) * bessel_i(m, alpha * r) / bessel_i(m, alpha)
    return np.where(inside, val, 0.0)


def kb_table(a: float, alpha: float, m: int, N: int) -> np.ndarray:
    """T[i] = b(i * a^2 / (N-1)), i = 0..N-1 (FP64)."""
    if N < 2:
        raise ValueError("table needs at least 2 entries")
    i = np.arange(N, dtype=np.float64)
    return kb_profile(i * (a * a) / (N - 1), a, alpha, m)


def table_lookup(d2, table: np.ndarray, a: float, lerp: bool = True) -> np.ndarray:
    """Tabulated blob: t = d^2 (N-1)/a^2, i = floor(t), f = t - i;
    lerp -> (1-f) T[i] + f T[min(i+1, N-1)],  trunc -> T[i];  0 for d^2 > a^2."""
    d2 = np.asarray(d2, dtype=np.float64)
    N = table.shape[0]
    inside = d2 <= a * a
    t = np.where(inside, d2 * (N - 1) / (a * a), 0.0)
    i = np.minimum(np.floor(t).astype(np.int64), N - 1)
    f = t - i
    if lerp:
        val = (1.0 - f) * table[i] + f * table[np.minimum(i + 1, N - 1)]
    else:
        val = table[i]
    return np.where(inside, val, 0.0)
