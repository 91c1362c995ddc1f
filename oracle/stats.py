"""Energy estimator and error bars.  Test infrastructure only.

The paper quotes energies with error bars and the rescaled variance
N var(E_loc) / E^2 (V-score, Sec. 4.3 and its table of operators), without
naming the error-bar method.  Reading used here: the mean is exactly rounded
(math.fsum); the error uses the integrated autocorrelation time
tau_int = 1 + 2 sum_t rho(t) with Sokal's automatic window (c = 5),
cross-checked by Flyvbjerg-Petersen blocking.
"""
from __future__ import annotations

import math

import numpy as np


def fsum_mean(x) -> float:
    x = np.asarray(x, dtype=np.float64).ravel()
    return math.fsum(x) / len(x)


def autocorr(series) -> np.ndarray:
    """Normalised autocorrelation rho(t) of a (T,) or (T, W) series; for many
    walkers the covariances are averaged over walkers.  A series without
    fluctuations (zero variance, e.g. E_loc of an exact eigenstate) has no
    correlations to measure: rho = (1, 0, 0, ...), so tau_int = 1."""
    x = np.asarray(series, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T = x.shape[0]
    d = x - x.mean()
    c = np.array([np.mean(d[: T - t] * d[t:]) for t in range(T)])
    if not c[0] > 0.0:
        rho = np.zeros(T)
        rho[0] = 1.0
        return rho
    return c / c[0]


def tau_int(series, c: float = 5.0) -> float:
    rho = autocorr(series)
    tau = 1.0
    for M in range(1, len(rho)):
        tau = 1.0 + 2.0 * float(np.sum(rho[1:M + 1]))
        if M >= c * tau:
            break
    return max(tau, 1.0)


def blocking_error(x) -> float:
    """Flyvbjerg-Petersen: standard error of the mean of a 1-D series,
    taken at the plateau (max over blocking levels with >= 32 blocks)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    best = 0.0
    while len(x) >= 32:
        n = len(x)
        err = math.sqrt(np.var(x, ddof=1) / n)
        best = max(best, err)
        x = 0.5 * (x[: n // 2 * 2 : 2] + x[1: n // 2 * 2 : 2])
    return best


def energy_estimate(series):
    """series (T, W): mean (exactly rounded), sigma_E from tau_int, tau_int,
    variance of E_loc."""
    x = np.asarray(series, dtype=np.float64)
    T = x.shape[0]
    W = x.shape[1] if x.ndim > 1 else 1
    mean = fsum_mean(x)
    var = float(np.var(x))
    tau = tau_int(x)
    sigma = math.sqrt(var * tau / (T * W))
    return mean, sigma, tau, var


def v_score(var: float, mean: float, N: int) -> float:
    return N * var / (mean * mean)
