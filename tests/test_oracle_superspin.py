"""Pins of the general layer model and of the TNMCMC-2 composite update (SM S2.B).

* The general form on a TNMCMC-1 layer gives the pinned oracle's
  environments and log q (bmps / sampler) to rounding.
* A composite layer's energy difference equals the full-lattice energy
  difference (model.energy) of the same two configurations.
* Untruncated (chi = 16 on a 2 x 2 composite layer, 256 configurations):
  log q(a) = -beta E(a) - log Z for every a, E from the full-lattice energy.
* Truncated (chi = 1): sum over all composite configurations of q = 1.
* Exact stationarity of the composite MH kernel on a 2x2x4 lattice.
* Chain averages of TNMCMC-2 sweeps on 2x2x4 against exact enumeration.
"""
import itertools
import math

import numpy as np
import pytest

import bruteforce as bf
import synth
from oracle import autocorr, bmps, chain, layer, model, sampler


def _states4(Ly, Lx):
    for cfg in itertools.product(range(4), repeat=Ly * Lx):
        yield np.array(cfg, dtype=np.int64).reshape(Ly, Lx)


def _with(spins, z0, a):
    t = spins.copy()
    t[z0], t[z0 + 1] = layer.composite_spins(a)
    return t


@pytest.mark.parametrize("d,chi", [(2, 2), (2, 8), (3, 3)])
def test_general_form_reproduces_plain_layer(d, chi):
    J = synth.couplings_gauss(5, 4, 3, 2) if d == 2 else synth.couplings_uniform(5, 4, 3)
    s = synth.spins_random(5, 4, 3, 9, d)
    z, beta = 1, 0.9
    F = model.slice_field(J, s, z, d)
    e1, l1 = bmps.environments(J, F, z, beta, chi, d)
    m = layer.plain_layer(J, s, z, d, F)
    e2, l2 = layer.environments(m, beta, chi)
    assert np.allclose(l1, l2, rtol=1e-13, atol=1e-13)
    for sw in range(3):
        a1, q1, _ = sampler.sample_layer(e1, J, F, z, beta, d, seed=3, chain=1, sweep=sw)
        a2, q2, _ = layer.sample_layer(e2, m, beta, seed=3, chain=1, sweep=sw, z_key=z)
        assert np.array_equal(a1, a2) and abs(q1 - q2) < 1e-11 * max(1.0, abs(q1))
        assert model.slice_energy(J, F, a1, z, d) == layer.layer_energy(m, a1)


@pytest.mark.parametrize("z0", [0, 1, 2])
def test_composite_energy_is_full_lattice_difference(z0):
    J = synth.couplings_gauss(4, 3, 4, 5)
    s = synth.spins_random(4, 3, 4, 6)
    m = layer.composite_layer(J, s, z0)
    rng = np.random.Generator(np.random.PCG64(z0))
    for _ in range(5):
        a = rng.integers(0, 4, size=(3, 4))
        b = rng.integers(0, 4, size=(3, 4))
        lhs = layer.layer_energy(m, a) - layer.layer_energy(m, b)
        rhs = model.energy(J, _with(s, z0, a), 2) - model.energy(J, _with(s, z0, b), 2)
        assert lhs == rhs


@pytest.mark.parametrize("z0", [0, 1, 2])
def test_exact_composite_logq_is_boltzmann(z0):
    J = synth.couplings_pm_j(2, 2, 4, 7)
    s = synth.spins_random(2, 2, 4, 8)
    beta = 0.8
    m = layer.composite_layer(J, s, z0)
    envs, _ = layer.environments(m, beta, 16)
    cfgs = list(_states4(2, 2))
    E = np.array([model.energy(J, _with(s, z0, a), 2) for a in cfgs])
    logz = bf.logsumexp(-beta * E)
    for a, e in zip(cfgs, E):
        _, lq, fault = layer.sample_layer(envs, m, beta, forced=a)
        assert not fault and abs(lq - (-beta * e - logz)) < 1e-11


def test_truncated_composite_q_sums_to_one():
    J = synth.couplings_gauss(3, 2, 4, 11)
    s = synth.spins_random(3, 2, 4, 12)
    m = layer.composite_layer(J, s, 1)
    envs, _ = layer.environments(m, 1.2, 1)
    tot = math.fsum(math.exp(layer.sample_layer(envs, m, 1.2, forced=a)[1]) for a in _states4(2, 3))
    assert abs(tot - 1.0) < 1e-12


@pytest.mark.parametrize("z0", [0, 1, 2])
def test_composite_kernel_is_stationary(z0):
    J = synth.couplings_pm_j(2, 2, 4, 3)
    s = synth.spins_random(2, 2, 4, 13 + z0)
    beta, chi = 1.3, 1
    m = layer.composite_layer(J, s, z0)
    envs, _ = layer.environments(m, beta, chi)
    cfgs = list(_states4(2, 2))
    lq = np.array([layer.sample_layer(envs, m, beta, forced=a)[1] for a in cfgs])
    E = np.array([model.energy(J, _with(s, z0, a), 2) for a in cfgs])
    n = len(cfgs)
    K = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                lr = lq[i] - lq[j] - beta * (E[j] - E[i])
                K[i, j] = math.exp(lq[j]) * math.exp(min(0.0, lr))
        K[i, i] = 1.0 - K[i].sum()
    pi = np.exp(-beta * E - bf.logsumexp(-beta * E))
    assert np.all(K >= -1e-15) and np.max(np.abs(pi @ K - pi)) < 1e-13
    assert float(pi @ (1 - np.diag(K))) < 0.999   # truncated: rejections happen


def test_superspin_chain_averages_match_enumeration():
    Lx, Ly, Lz, beta, chi = 2, 2, 4, 1.0, 1
    J = synth.couplings_pm_j(Lx, Ly, Lz, 3)
    st, E = bf.lattice_states(J, Lx, Ly, Lz, 2)
    w = np.exp(-beta * (E - E.min()))
    w /= w.sum()
    E_exact = float(np.sum(w * E))
    s = synth.spins_random(Lx, Ly, Lz, 31)
    n = 1500
    Es = np.zeros(n)
    acc = 0
    for t in range(n):
        acc += chain.superspin_sweep(J, s, beta, chi, seed=31, chain=0, sweep_index=t)
        Es[t] = model.energy(J, s, 2)
    Es = Es[50:]
    tau, _ = autocorr.tau_int(Es)
    err = math.sqrt(2 * max(tau, 0.5) * np.var(Es) / len(Es))
    assert abs(Es.mean() - E_exact) < 4 * err + 1e-12
    assert acc < 3 * n
