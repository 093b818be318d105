"""Pin of the tau_int estimator: AR(1) series x_t = phi x_{t-1} + noise have
rho(k) = phi^k, so tau_int = 1/2 + phi/(1-phi) = (1+phi)/(2(1-phi))."""
import numpy as np
import pytest

from oracle import autocorr


def _ar1(phi, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("phi", [0.5, 0.9])
def test_ar1_closed_form(phi):
    exact = (1 + phi) / (2 * (1 - phi))
    series = np.stack([_ar1(phi, 20000, s) for s in range(4)])
    tau, W = autocorr.tau_int(series)
    sigma = exact * np.sqrt(2 * (2 * W + 1) / series.size)
    assert abs(tau - exact) < 4 * sigma


def test_white_noise_and_constant():
    x = np.random.Generator(np.random.PCG64(0)).standard_normal(5000)
    tau, _ = autocorr.tau_int(x)
    assert abs(tau - 0.5) < 0.1
    rho = autocorr.autocorrelation(np.ones(10))
    assert rho[0] == 1.0 and np.all(rho[1:] == 0)
