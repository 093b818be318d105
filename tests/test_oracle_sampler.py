"""Pins of the oracle's ancestral sampler and its log q.

* exact regime: log q(s) = -beta E(s) - log Z for every configuration (the
  paper's statement that exact contraction gives exact sampling);
* truncated regime: q is still a normalised distribution (sum over all
  configurations is 1) and teacher forcing reproduces the sampled log q;
* closed forms: beta = 0 is uniform; no in-layer bonds gives a product of
  logistic factors even at chi = 1;
* the draw rule: sampled frequencies follow q."""
import math

import numpy as np
import pytest

import bruteforce as bf
import synth
from oracle import bmps, model, sampler


def _setup(Lx, Ly, d, kind, seed, beta, chi, Lz=3):
    if kind == "pmj":
        J = synth.couplings_pm_j(Lx, Ly, Lz, seed)
    elif kind == "gauss":
        J = synth.couplings_gauss(Lx, Ly, Lz, seed)
    else:
        J = synth.couplings_uniform(Lx, Ly, Lz)
    s = synth.spins_random(Lx, Ly, Lz, seed + 3, d) if kind != "ferro" or Lz > 1 else synth.spins_ordered(Lx, Ly, Lz, d)
    z = Lz // 2
    F = model.slice_field(J, s, z, d)
    envs, ls = bmps.environments(J, F, z, beta, chi, d)
    return J, s, z, F, envs, ls


@pytest.mark.parametrize("Lx,Ly,d,kind", [(3, 3, 2, "pmj"), (4, 3, 2, "gauss"), (2, 4, 2, "pmj"),
                                          (3, 2, 3, "ferro"), (2, 3, 3, "ferro")])
def test_exact_regime_logq_is_boltzmann(Lx, Ly, d, kind):
    beta = 0.9
    J, s, z, F, envs, ls = _setup(Lx, Ly, d, kind, 40, beta, d ** ((Lx + 1) // 2))
    cfgs, E = bf.layer_energies(J, s, z, d)
    logz = bf.logsumexp(-beta * E)
    for a, e in zip(cfgs, E):
        _, lq, fault = sampler.sample_layer(envs, J, F, z, beta, d, forced=np.array(a))
        assert not fault
        assert abs(lq - (-beta * e - logz)) < 1e-12 * max(1.0, abs(logz))


@pytest.mark.parametrize("chi", [1, 2])
@pytest.mark.parametrize("kind", ["pmj", "ferro"])
def test_truncated_q_is_normalised(chi, kind):
    Lx, Ly = 4, 3
    beta = 0.44 if kind == "ferro" else 1.0
    J, s, z, F, envs, ls = _setup(Lx, Ly, 2, kind, 9, beta, chi, Lz=1)
    cfgs, E = bf.layer_energies(J, s, z, 2)
    lqs = np.array([sampler.sample_layer(envs, J, F, z, beta, 2, forced=np.array(a))[1] for a in cfgs])
    assert abs(math.fsum(np.exp(lqs)) - 1.0) < 1e-12
    # the truncation is real: q differs from the Boltzmann distribution
    logp = -beta * E - bf.logsumexp(-beta * E)
    assert np.max(np.abs(lqs - logp)) > 1e-4


def test_forced_path_reproduces_sampled_logq():
    J, s, z, F, envs, ls = _setup(6, 5, 2, "gauss", 2, 1.2, 3)
    for t in range(5):
        a, lq, _ = sampler.sample_layer(envs, J, F, z, 1.2, 2, seed=7, chain=1, sweep=t)
        _, lq2, _ = sampler.sample_layer(envs, J, F, z, 1.2, 2, forced=a)
        assert lq == lq2


def test_beta_zero_logq_uniform():
    for d in (2, 3):
        J, s, z, F, envs, ls = _setup(4, 3, d, "pmj" if d == 2 else "ferro", 1, 0.0, 2)
        a, lq, _ = sampler.sample_layer(envs, J, F, z, 0.0, d, seed=1)
        assert abs(lq + 12 * math.log(d)) < 1e-12


def test_no_in_layer_bonds_logistic_product():
    Lx, Ly, beta = 5, 4, 0.7
    J = synth.couplings_gauss(Lx, Ly, 3, 6)
    J[0] = 0.0
    J[1] = 0.0
    s = synth.spins_random(Lx, Ly, 3, 6)
    F = model.slice_field(J, s, 1, 2)
    envs, _ = bmps.environments(J, F, 1, beta, 1, 2)
    a, lq, _ = sampler.sample_layer(envs, J, F, 1, beta, 2, seed=3)
    ref = 0.0
    for y in range(Ly):
        for x in range(Lx):
            u = a[y, x]
            ref += beta * F[y, x, u] - math.log(math.exp(beta * F[y, x, 0]) + math.exp(beta * F[y, x, 1]))
    assert abs(lq - ref) < 1e-12


def test_sampled_frequencies_follow_q():
    """Chi-square test of 4000 draws of a 3x2 layer against q (truncated, chi=1)."""
    Lx, Ly, beta = 3, 2, 0.8
    J, s, z, F, envs, ls = _setup(Lx, Ly, 2, "pmj", 14, beta, 1, Lz=1)
    cfgs, _ = bf.layer_energies(J, s, z, 2)
    q = np.array([math.exp(sampler.sample_layer(envs, J, F, z, beta, 2, forced=np.array(a))[1]) for a in cfgs])
    counts = np.zeros(len(cfgs))
    index = {tuple(np.array(a).reshape(-1)): i for i, a in enumerate(cfgs)}
    n = 4000
    for t in range(n):
        a, _, _ = sampler.sample_layer(envs, J, F, z, beta, 2, seed=99, chain=0, sweep=t)
        counts[index[tuple(a.reshape(-1))]] += 1
    expected = n * q
    keep = expected > 5
    chi2 = float(np.sum((counts[keep] - expected[keep]) ** 2 / expected[keep]))
    dof = int(keep.sum()) - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof)


def test_clamp_rule():
    p, f = sampler.site_probabilities(np.array([1.0, -1e-3]))
    assert not f and p[1] == pytest.approx(1e-12 / (1 + 1e-12)) and abs(p.sum() - 1) < 1e-15
    p, f = sampler.site_probabilities(np.array([-1.0, -2.0]))
    assert f and np.allclose(p, 0.5)
    p, f = sampler.site_probabilities(np.array([np.nan, 1.0]))
    assert f
    assert sampler.draw(np.array([0.3, 0.7]), 0.29999) == 0
    assert sampler.draw(np.array([0.3, 0.7]), 0.3) == 1
    assert sampler.draw(np.array([0.2, 0.3, 0.5]), 0.49) == 1
    assert sampler.draw(np.array([0.2, 0.3, 0.5]), 0.9999999) == 2
