"""Host-side analysis of recorded observables (no part of the proposal itself).

tau_int of the overlap q (SM S3, "Integrated autocorrelation time"):
rho(k) normalised autocorrelation, tau = 1/2 + sum_{k>=1} rho(k), summed up to
Sokal's automatic window (smallest W with W >= 6 tau(W)); with several series
rho is averaged over them first.  Independent samples per second follow the
paper's cost per independent sample t_int = tau_int * t_s: n_pairs / (tau * t_s).
"""
from __future__ import annotations

import numpy as np


def _rho(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    x = x - x.mean()
    v = float(np.dot(x, x)) / n
    if v == 0.0:
        r = np.zeros(n)
        r[0] = 1.0
        return r
    f = np.fft.rfft(x, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n] / np.arange(n, 0, -1)
    return acf / v


def tau_int(series, window_factor: float = 6.0):
    """(tau, window) of one series or of several (rows)."""
    s = np.atleast_2d(np.asarray(series, dtype=np.float64))
    rho = np.mean([_rho(r) for r in s], axis=0)
    tau = 0.5
    for W in range(1, rho.shape[0]):
        tau += rho[W]
        if W >= window_factor * tau:
            return float(tau), W
    return float(tau), rho.shape[0] - 1


def independent_samples_per_second(q_series, seconds_per_sweep: float):
    """n_pairs / (tau_int,q * t_s); q_series is [n_sweeps, n_pairs]."""
    q = np.asarray(q_series)
    tau, W = tau_int(q.T)
    return q.shape[1] / (tau * seconds_per_sweep), tau, W
