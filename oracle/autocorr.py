"""Integrated autocorrelation time (SM S3, "Integrated autocorrelation time").

Oracle code (test infrastructure only).

rho(k) = (<O(t)O(t+k)> - <O>^2) / (<O^2> - <O>^2) and
tau_int = 1/2 + sum_{k>=1} rho(k), the sum cut at a window where rho stops
being significant.  Reading of the window: Sokal's automatic window, the
smallest W with W >= c * tau(W), c = 6.  With several series (replica pairs or
disorder instances) rho(k) is averaged over the series before the window is
chosen.
"""
from __future__ import annotations

import numpy as np


def autocorrelation(series: np.ndarray) -> np.ndarray:
    """Normalised autocorrelation rho(k), k = 0..n-1, of one series."""
    x = np.asarray(series, dtype=np.float64)
    n = x.shape[0]
    x = x - x.mean()
    var = float(np.dot(x, x)) / n
    if var == 0.0:
        out = np.zeros(n)
        out[0] = 1.0
        return out
    rho = np.array([np.dot(x[: n - k], x[k:]) / (n - k) for k in range(n)]) / var
    return rho


def tau_int(series, c: float = 6.0):
    """tau_int of one series (1-D) or the average rho of several (2-D, series x time).
    Returns (tau, window)."""
    s = np.atleast_2d(np.asarray(series, dtype=np.float64))
    rho = np.mean([autocorrelation(r) for r in s], axis=0)
    n = rho.shape[0]
    tau = 0.5
    for W in range(1, n):
        tau += rho[W]
        if W >= c * tau:
            return float(tau), W
    return float(tau), n - 1
