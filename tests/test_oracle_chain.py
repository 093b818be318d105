"""Pins of the oracle's Metropolis-Hastings step and chain.

* the acceptance rule as a pure function (main text Eq. 1);
* exact contraction gives acceptance 1 (main text, "TNMCMC");
* exact stationarity: on a 2x2x4 lattice with a truncated (chi=1) proposal the
  one-layer transition kernel built from the oracle's own q and MH rule leaves
  the exact conditional Boltzmann distribution invariant (a reversed
  acceptance ratio, a wrong q or a wrong energy sign fails this);
* chain averages on the 2x2x4 lattice agree with exact enumeration."""
import math

import numpy as np
import pytest

import bruteforce as bf
import synth
from oracle import autocorr, bmps, chain, model, sampler


def test_mh_rule_table():
    assert chain.mh_accept(0.0, 0.0, 1.0, -3.0, 0.999999)        # downhill, equal q
    assert chain.mh_accept(-1.0, -2.0, 1.0, 0.5, 0.999999)       # log A = 0.5 > 0
    la = -1.0 - (-0.5) - 2.0 * 0.25                               # = -1.0
    assert chain.mh_accept(-1.0, -0.5, 2.0, 0.25, math.exp(la) * (1 - 1e-12))
    assert not chain.mh_accept(-1.0, -0.5, 2.0, 0.25, math.exp(la) * (1 + 1e-12))
    # orientation: a proposal that q likes more than the current state is penalised
    assert not chain.mh_accept(-10.0, -1.0, 1.0, 0.0, 0.01)
    assert chain.mh_accept(-1.0, -10.0, 1.0, 0.0, 0.99)


def test_exact_regime_accepts_everything():
    """8^3 +-J at beta=0.5 with chi=16 (exact for 8-wide layers): the log acceptance
    ratio vanishes to rounding and every proposal is accepted."""
    J = synth.couplings_pm_j(8, 8, 8, 0)
    s = synth.spins_random(8, 8, 8, 1)
    for z in (0, 3, 7):
        rec = chain.slice_update(J, s, z, 0.5, 16, 2, seed=5, chain=0, sweep=0)
        lr = rec["logq_old"] - rec["logq_new"] - 0.5 * rec["dE"]
        assert abs(lr) < 1e-9
        assert rec["accepted"]


def _kernel(J, spins, z, beta, chi, d, reverse=False):
    """One-layer MH transition matrix K[a, b] over all layer configurations, built
    from the oracle's q (teacher forcing) and its acceptance rule; ``reverse``
    uses the inverse ratio instead (the printed form of Alg. 2)."""
    F = model.slice_field(J, spins, z, d)
    envs, _ = bmps.environments(J, F, z, beta, chi, d)
    Ly, Lx = spins.shape[1:]
    cfgs = list(bf.all_layer_configs(Ly, Lx, d))
    lq = np.array([sampler.sample_layer(envs, J, F, z, beta, d, forced=np.array(a))[1] for a in cfgs])
    Fb = bf.layer_field(J, spins, z, d)
    E = np.array([bf.config_energy(J, Fb, z, a, d) for a in cfgs])
    n = len(cfgs)
    K = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                # probability over u of chain.mh_accept(lq_old, lq_new, beta, dE, u)
                lr = lq[i] - lq[j] - beta * (E[j] - E[i])
                acc = math.exp(min(0.0, -lr if reverse else lr))
                K[i, j] = math.exp(lq[j]) * acc
        K[i, i] = 1.0 - K[i].sum()
    pi = np.exp(-beta * E - bf.logsumexp(-beta * E))
    return K, pi


def test_mh_rule_is_the_kernel_probability():
    """chain.mh_accept(u) is true exactly for u below exp(min(0, log ratio))."""
    for lr in (-3.0, -0.2, 0.0, 1.5):
        A = math.exp(min(0.0, lr))
        assert chain.mh_accept(lr, 0.0, 1.0, 0.0, A * (1 - 1e-9))
        assert not chain.mh_accept(lr, 0.0, 1.0, 0.0, min(A * (1 + 1e-9), 1.0)) or A == 1.0


@pytest.mark.parametrize("z", [0, 1, 3])
def test_exact_stationarity_truncated(z):
    J = synth.couplings_pm_j(2, 2, 4, 3)
    beta, chi = 1.3, 1
    rng = np.random.Generator(np.random.PCG64(z))
    worst_acc = 1.0
    for _ in range(6):
        s = synth.spins_random(2, 2, 4, int(rng.integers(1 << 30)))
        K, pi = _kernel(J, s, z, beta, chi, 2)
        assert np.all(K >= -1e-15)
        assert np.max(np.abs(pi @ K - pi)) < 1e-13
        worst_acc = min(worst_acc, float(pi @ (1 - np.diag(K))))
    # the proposal is inexact, so the test exercises rejections
    assert worst_acc < 0.999


def test_reversed_ratio_breaks_stationarity():
    """Sensitivity: the inverse ratio (printed in Alg. 2) is not stationary."""
    J = synth.couplings_pm_j(2, 2, 4, 3)
    s = synth.spins_random(2, 2, 4, 77)
    K, pi = _kernel(J, s, 1, 1.3, 1, 2)
    assert np.max(np.abs(pi @ K - pi)) < 1e-13
    Kr, _ = _kernel(J, s, 1, 1.3, 1, 2, reverse=True)
    assert np.max(np.abs(pi @ Kr - pi)) > 1e-8      # 5 orders above the rounding level


@pytest.mark.parametrize("chi,seed", [(1, 11), (2, 12)])
def test_chain_averages_match_enumeration(chi, seed):
    Lx, Ly, Lz, beta = 2, 2, 4, 1.0
    J = synth.couplings_pm_j(Lx, Ly, Lz, 3)
    st, E = bf.lattice_states(J, Lx, Ly, Lz, 2)
    w = np.exp(-beta * (E - E.min()))
    w /= w.sum()
    M = np.sum(1 - 2 * st, axis=(1, 2, 3)) / 16.0
    E_exact = float(np.sum(w * E))
    M2_exact = float(np.sum(w * M * M))
    s = synth.spins_random(Lx, Ly, Lz, seed)
    n = 3000
    Es, Ms, acc = chain.run_chain(J, s, beta, chi, 2, n, seed=seed, chain=0)
    Es, Ms = Es[100:], Ms[100:]
    for series, exact in ((Es, E_exact), (Ms * Ms, M2_exact)):
        tau, _ = autocorr.tau_int(series)
        err = math.sqrt(2 * max(tau, 0.5) * np.var(series) / len(series))
        assert abs(series.mean() - exact) < 4 * err + 1e-12
    assert acc <= 4 * n


@pytest.mark.parametrize("direction", [1, 2])
def test_direction_views_keep_the_hamiltonian(direction):
    """The permuted lattice of a slice direction has the same energy as the
    original for every configuration (a wrong coupling component or axis fails),
    its open boundaries stay open, and the spin permutation round-trips."""
    rng = np.random.default_rng(direction)
    J = synth.couplings_gauss(5, 4, 3, 7)
    for d in (2, 3):
        for _ in range(5):
            s = synth.spins_random(5, 4, 3, int(rng.integers(1 << 30)), d)
            Jp, sp = chain.to_direction(J, s, direction)
            assert model.energy(Jp, sp, d) == model.energy(J, s, d)
            assert np.array_equal(chain.from_direction(sp, direction), s)
    Jp, _ = chain.to_direction(J, s, direction)
    assert np.all(Jp[0, :, :, -1] == 0) and np.all(Jp[1, :, -1, :] == 0) and np.all(Jp[2, -1, :, :] == 0)


def test_direction_cycled_chain_matches_enumeration():
    """Sweeps cycling z, y, x slices on 2x2x3 +-J lattices at chi = 1 (truncated):
    averages of E over many chains agree with exact enumeration."""
    Lx, Ly, Lz, beta = 2, 2, 3, 1.0
    devs = []
    for inst in range(24):
        J = synth.couplings_pm_j(Lx, Ly, Lz, 100 + inst)
        s = synth.spins_random(Lx, Ly, Lz, 200 + inst)
        states, En = bf.lattice_states(J, Lx, Ly, Lz, 2)
        w = np.exp(-beta * (En - En.min()))
        w /= w.sum()
        Es = []
        for t in range(90):
            chain.sweep_direction(J, s, beta, 1, 2, t % 3, seed=9, chain=inst, sweep_index=t)
            if t >= 15:
                Es.append(model.energy(J, s, 2))
        devs.append(np.mean(Es) - float(np.sum(w * En)))
    devs = np.array(devs)
    assert abs(devs.mean()) < 4 * devs.std(ddof=1) / math.sqrt(len(devs)) + 1e-12


def test_multi_candidate_update_is_the_chained_kernel():
    """Several candidates per environment: the distribution of the final layer
    after 3 chained candidates from a fixed state equals row `a` of K^3, K the
    exact one-candidate MH kernel (2x2 layer of a 2x2x4 lattice, chi = 1, so
    rejections happen).  Frequencies over 3000 independent sweep counters,
    each within five binomial standard deviations.  A chain that compared
    every candidate with the initial state instead of the current one, or
    reused one uniform stream, has another law and fails."""
    J = synth.couplings_pm_j(2, 2, 4, 3)
    s = synth.spins_random(2, 2, 4, 91)
    z, beta, chi, K = 1, 1.3, 1, 3
    Kmat, pi = _kernel(J, s, z, beta, chi, 2)
    cfgs = [tuple(map(tuple, np.array(a))) for a in bf.all_layer_configs(2, 2, 2)]
    start = cfgs.index(tuple(map(tuple, model.to_states(s[z], 2))))
    want = np.linalg.matrix_power(Kmat, K)[start]
    n = 3000
    counts = np.zeros(len(cfgs))
    for sw in range(n):
        t = s.copy()
        chain.slice_update_multi(J, t, z, beta, chi, 2, K, seed=17, chain=0, sweep=sw)
        counts[cfgs.index(tuple(map(tuple, model.to_states(t[z], 2))))] += 1
    freq = counts / n
    sd = np.sqrt(want * (1 - want) / n)
    assert np.all(np.abs(freq - want) < 5 * sd + 1e-3), (freq, want)
    # the one-candidate form is slice_update itself
    a, b = s.copy(), s.copy()
    r1 = chain.slice_update(J, a, z, beta, chi, 2, seed=17, chain=0, sweep=5)
    r2 = chain.slice_update_multi(J, b, z, beta, chi, 2, 1, seed=17, chain=0, sweep=5)
    assert np.array_equal(a, b) and int(r1["accepted"]) == r2["accepted"]


def test_multi_candidate_chain_averages_match_enumeration():
    Lx, Ly, Lz, beta, chi = 2, 2, 4, 1.0, 1
    J = synth.couplings_pm_j(Lx, Ly, Lz, 3)
    st, E = bf.lattice_states(J, Lx, Ly, Lz, 2)
    w = np.exp(-beta * (E - E.min()))
    w /= w.sum()
    E_exact = float(np.sum(w * E))
    s = synth.spins_random(Lx, Ly, Lz, 21)
    n = 1500
    Es, _, acc = chain.run_chain(J, s, beta, chi, 2, n, seed=21, chain=0, n_candidates=3)
    Es = Es[50:]
    tau, _ = autocorr.tau_int(Es)
    err = math.sqrt(2 * max(tau, 0.5) * np.var(Es) / len(Es))
    assert abs(Es.mean() - E_exact) < 4 * err + 1e-12
    assert acc < 3 * 4 * n
