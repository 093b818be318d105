"""Pins of the product-side tau_int estimator (paper_2509_23945_amd.analysis),
which turns recorded overlap series into independent samples per second.

* AR(1) series x_t = phi x_{t-1} + noise have rho(k) = phi^k, so
  tau_int = 1/2 + phi/(1-phi) = (1+phi)/(2(1-phi)) (SM S3 definition with the
  1/2 + sum rho convention); the estimate must fall within four standard
  errors of Sokal's variance formula.
* The estimator computes rho by FFT; the oracle's (oracle/autocorr.py) by
  direct lagged sums.  On the same series both must give the same window and
  the same tau to rounding.
* White noise has tau = 1/2; a constant series has rho = (1, 0, 0, ...).
* Independent samples per second = n_pairs / (tau * t_s).
"""
import numpy as np
import pytest

from oracle import autocorr
from paper_2509_23945_amd import analysis


def _ar1(phi, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("phi", [0.5, 0.9, 0.97])
def test_ar1_closed_form(phi):
    exact = (1 + phi) / (2 * (1 - phi))
    series = np.stack([_ar1(phi, 20000, 100 + s) for s in range(4)])
    tau, W = analysis.tau_int(series)
    sigma = exact * np.sqrt(2 * (2 * W + 1) / series.size)
    assert abs(tau - exact) < 4 * sigma, (tau, exact, sigma)


@pytest.mark.parametrize("phi,n,k", [(0.8, 3000, 3), (0.95, 1500, 16), (0.3, 500, 1)])
def test_equals_oracle_on_same_series(phi, n, k):
    series = np.stack([_ar1(phi, n, 7 * s + 1) for s in range(k)])
    tau_a, W_a = analysis.tau_int(series)
    tau_o, W_o = autocorr.tau_int(series)
    assert W_a == W_o
    assert abs(tau_a - tau_o) < 1e-9 * tau_o
    # rho itself, lag by lag
    ra = analysis._rho(series[0])
    ro = autocorr.autocorrelation(series[0])
    assert np.max(np.abs(ra - ro)) < 1e-10


def test_white_noise_and_constant():
    x = np.random.Generator(np.random.PCG64(0)).standard_normal(5000)
    tau, _ = analysis.tau_int(x)
    assert abs(tau - 0.5) < 0.1
    rho = analysis._rho(np.ones(10))
    assert rho[0] == 1.0 and np.all(rho[1:] == 0)


def test_independent_samples_per_second():
    q = np.stack([_ar1(0.9, 4000, 40 + s) for s in range(3)], axis=1)   # [sweeps, pairs]
    indep, tau, W = analysis.independent_samples_per_second(q, 0.05)
    tau_o, W_o = autocorr.tau_int(q.T)
    assert W == W_o and abs(tau - tau_o) < 1e-9 * tau_o
    assert abs(indep - 3 / (tau_o * 0.05)) < 1e-9 * indep
