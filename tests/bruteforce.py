"""Brute-force definitions used to pin the oracle (independent of its code).

The multiple-tau correlator of the paper (Section 2.2, Appendix D) is, up to
rounding order, the direct correlation estimate of Eq. (1) applied level by
level to block-averaged copies of the series:

    y0 = x,   y_k[i] = (1/m) * sum_{j<m} y_{k-1}[m i + j]   (incomplete tail dropped)
    C_k(L) = 1/(S_k - L) * sum_{i=L}^{S_k-1} y_k[i] * conj(y_k[i-L])

for lags L = 0..p-1 at level 0 and floor(p/m)..p-1 at levels >= 1, emitted
when S_k > L, at lag time L * m^k.  This module writes that definition out
with numpy; it never calls the oracle.
"""
from __future__ import annotations

import numpy as np


def block_average(y: np.ndarray, m: int) -> np.ndarray:
    """Means of consecutive, non-overlapping groups of m values along axis 0,
    summed in order (first value first)."""
    n = (y.shape[0] // m) * m
    if n == 0:
        return y[:0]
    g = y[:n].reshape((n // m, m) + y.shape[1:])
    acc = g[:, 0].copy()
    for j in range(1, m):
        acc = acc + g[:, j]
    return acc / m


def direct_eq1(y: np.ndarray, L: int):
    """Eq. (1) on one series level: per-channel mean over i of y[i] * conj(y[i-L])."""
    S = y.shape[0]
    if S <= L:
        return None, 0
    prod = y[L:] * np.conj(y[: S - L])
    return prod.sum(axis=0) / (S - L), S - L


def multitau_bruteforce(x: np.ndarray, levels: int, points: int, m: int):
    """x: [S] or [S][n_ch].  Returns (t_steps, C_per_channel [n_out][...], counts),
    in level-major, lag-minor order."""
    y = np.asarray(x)
    ts, cs, ns = [], [], []
    for k in range(levels):
        lag0 = 0 if k == 0 else points // m
        for L in range(lag0, points):
            c, n = direct_eq1(y, L)
            if n > 0:
                ts.append(L * m**k)
                cs.append(c)
                ns.append(n)
        y = block_average(y, m)
    return np.array(ts, dtype=np.float64), np.array(cs), np.array(ns, dtype=np.int64)


def multitau_bruteforce_pair(x: np.ndarray, y: np.ndarray, levels: int, points: int, m: int):
    """The same closed definition for a pair of series (the x, y form of
    Algorithm 1): both are block-averaged level by level and
    C_k(L) = 1/(S_k - L) * sum_{i=L}^{S_k-1} x_k[i] * conj(y_k[i-L])."""
    xs, ys = np.asarray(x), np.asarray(y)
    ts, cs, ns = [], [], []
    for k in range(levels):
        lag0 = 0 if k == 0 else points // m
        S = xs.shape[0]
        for L in range(lag0, points):
            if S > L:
                ts.append(L * m**k)
                cs.append((xs[L:] * np.conj(ys[: S - L])).sum(axis=0) / (S - L))
                ns.append(S - L)
        xs, ys = block_average(xs, m), block_average(ys, m)
    return np.array(ts, dtype=np.float64), np.array(cs), np.array(ns, dtype=np.int64)


def ou_level_expectation(a: float, var: float, k: int, m: int, L: int) -> float:
    """E[C_k(L)] for a stationary AR(1)/OU series with autocorrelation a^|l| and
    variance var, after block averaging over M = m^k samples (derived from the
    covariance of block means; valid for L >= 1 or k = 0):
        var * a^(M L) * a^-(M-1) * ((1 - a^M) / (1 - a))^2 / M^2 ."""
    M = m**k
    if k == 0:
        return var * a**L
    if L == 0:
        # variance of a block mean: (var/M^2) * sum_{j,j'} a^|j-j'|
        s = M + 2.0 * sum((M - d) * a**d for d in range(1, M))
        return var * s / M**2
    g = (1.0 - a**M) / (1.0 - a)
    return var * a ** (M * L - (M - 1)) * g * g / (M * M)
