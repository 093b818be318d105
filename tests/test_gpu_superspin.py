"""TNMCMC-2 (SM S2.B) on the GPU against the oracle's composite-layer update.

* sweeps of superspin composites reproduce the oracle's chain spin for spin
  (Gaussian and +-J couplings, chi = 2, 4 and 8, ragged shapes), with
  identical acceptance counts;
* 64 independent 2x2x4 chains at chi = 1 match exact enumeration of <E> and
  <M^2>;
* 120 seeded random shapes, couplings, temperatures and bond dimensions
  (one sweep each) reproduce the oracle's chain spin for spin;
* on 8^3 at beta = 0.7, TNMCMC-2 chains reproduce the TNMCMC-1 chains'
  averages of E/N and q^2 per instance within statistical error;
* the entry point refuses Potts lattices, chi_max above 8 and one-layer
  lattices.

An earlier build of this path gave wrong truncations from run to run and
faulted the GPU once (6x6x6, chi = 8): the right sweep of a row read the last
left rank from LDS before every wavefront could see thread 0's write of it, so
wavefronts took different branches (with different barrier counts) and
extents.  That read is now ordered by a barrier and clamped into the tiles."""
import math

import numpy as np
import pytest

import bruteforce as bf
import gpu_helpers as gh
import paper_2509_23945_amd as tn
from oracle import chain as ochain

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("Lx,Ly,Lz,kind,beta,chi", [(4, 3, 4, "gauss", 0.9, 2), (5, 4, 5, "pmj", 1.0, 4),
                                                    (6, 6, 6, "pmj", 1.0, 8), (3, 5, 2, "gauss", 1.2, 4),
                                                    (8, 8, 7, "pmj", 0.6, 8)])
def test_superspin_sweeps_match_oracle(Lx, Ly, Lz, kind, beta, chi):
    gh.announce(f"superspin sweeps {Lx}x{Ly}x{Lz} chi={chi}")
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, chi, kind=kind, beta=beta, seed=71, n_chains=2)
    refs = [s.copy() for s in spins]
    for t in range(3):
        st = tn.tnmc_sweep_superspin([lat], 1, sweep_offset=t)
        acc = sum(ochain.superspin_sweep(J[c], refs[c], beta, chi, seed=12345, chain=c, sweep_index=t)
                  for c in range(2))
        assert st["numeric_faults"] == 0 and st["proposed"] == 2 * (Lz - 1)
        assert st["accepted"] == acc
        for c in range(2):
            assert np.array_equal(tn.tnmc_get_spins(lat, c), refs[c]), (t, c)


@pytest.mark.parametrize("block", range(6))
def test_random_composites_match_oracle(block):
    """Seeded draws of shape (Lx, Ly in 2..7, Lz in 2..6), couplings (+-J,
    Gaussian, uniform ferromagnetic), beta in [0.2, 1.6] and chi in {1, 2, 3,
    4, 6, 8}, two chains each: one sweep of composites from a random sweep
    index, spins and acceptance counts equal to the oracle's.  The draws reach
    exact and truncating composites, both Jacobi variants and composites whose
    left ranks pass 64 rows (the 96- and 128-row register QR windows)."""
    rng = np.random.default_rng(4242 + block)
    for k in range(20):
        Lx, Ly, Lz = int(rng.integers(2, 8)), int(rng.integers(2, 8)), int(rng.integers(2, 7))
        kind = str(rng.choice(["pmj", "gauss", "ferro"]))
        beta = float(rng.uniform(0.2, 1.6))
        chi = int(rng.choice([1, 2, 3, 4, 6, 8]))
        sweep = int(rng.integers(0, 1000))
        label = f"random composites block {block} draw {k}: {Lx}x{Ly}x{Lz} {kind} beta={beta:.4f} chi={chi} sweep {sweep}"
        gh.announce(label)
        lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, chi, kind=kind, beta=beta, seed=900 + 41 * block + k,
                                           n_chains=2)
        refs = [s.copy() for s in spins]
        st = tn.tnmc_sweep_superspin([lat], 1, sweep_offset=sweep)
        acc = sum(ochain.superspin_sweep(J[c], refs[c], beta, chi, seed=12345, chain=c, sweep_index=sweep)
                  for c in range(2))
        after = [tn.tnmc_get_spins(lat, c) for c in range(2)]
        tn.tnmc_lattice_free(lat)
        assert st["numeric_faults"] == 0 and st["proposed"] == 2 * (Lz - 1), label
        assert st["accepted"] == acc, label
        for c in range(2):
            assert np.array_equal(after[c], refs[c]), (label, c)


def test_superspin_chain_averages_match_enumeration():
    gh.announce("superspin chain averages 2x2x4")
    Lx, Ly, Lz, beta, n_chains, n_sweeps = 2, 2, 4, 1.0, 64, 300
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, 1, kind="pmj", beta=beta, seed=73, n_chains=n_chains,
                                       record_capacity=n_sweeps)
    st = tn.tnmc_sweep_superspin([lat], n_sweeps, record=True)
    assert st["numeric_faults"] == 0 and st["accepted"] < st["proposed"]
    E, M, _ = tn.tnmc_timeseries(lat)
    devs_E, devs_M2 = [], []
    for c in range(n_chains):
        states, En = bf.lattice_states(J[c], Lx, Ly, Lz, 2)
        w = np.exp(-beta * (En - En.min()))
        w /= w.sum()
        Mn = np.sum(1 - 2 * states, axis=(1, 2, 3)) / 16.0
        devs_E.append(E[30:, c].mean() - float(np.sum(w * En)))
        devs_M2.append((M[30:, c] ** 2).mean() - float(np.sum(w * Mn * Mn)))
    for devs in (np.array(devs_E), np.array(devs_M2)):
        err = devs.std(ddof=1) / math.sqrt(len(devs))
        assert abs(devs.mean()) < 4 * err + 1e-12, (devs.mean(), err)


def test_superspin_chain_reproduces_tnmcmc1_observables():
    """Stationarity of the composite-layer kernel on a lattice too large to
    enumerate: 32 +-J instances x 2 replicas on 8^3 at beta = 0.7 (above the
    glass transition, so chains decorrelate within a few sweeps), TNMCMC-2 at
    chi = 4 against TNMCMC-1 at chi = 8, 400 recorded sweeps each from the
    same states; per instance the averages of E/N and of q^2 over sweeps
    100..399 are compared, and the mean difference over instances must be
    within four standard errors of zero."""
    gh.announce("superspin vs TNMCMC-1 observables 8^3 beta=0.7, 64 chains x 400 sweeps")
    L, beta, n_inst, n_sw = 8, 0.7, 32, 400
    pairs = np.array([[2 * i, 2 * i + 1] for i in range(n_inst)], dtype=np.int32)
    res = []
    for chi, sweep in ((8, tn.tnmc_sweep), (4, tn.tnmc_sweep_superspin)):
        lat = gh.make_lattice(L, L, L, 2, chi, kind="pmj", beta=beta, seed=90, n_chains=2 * n_inst, pairs=pairs,
                              record_capacity=n_sw)[0]
        st = sweep([lat], n_sw, record=True)
        assert st["numeric_faults"] == 0
        E, _, q = tn.tnmc_timeseries(lat)
        tn.tnmc_lattice_free(lat)
        assert E.shape == (n_sw, 2 * n_inst)
        res.append(((E[100:] / L ** 3).mean(axis=0).reshape(n_inst, 2).mean(axis=1), (q[100:] ** 2).mean(axis=0)))
    for name, a, b in zip(("E/N", "q^2"), res[1], res[0]):
        dlt = a - b
        err = dlt.std(ddof=1) / math.sqrt(len(dlt))
        print(f"TNMCMC-2 minus TNMCMC-1, {name}: {dlt.mean():.3e} +- {err:.3e}")
        assert abs(dlt.mean()) < 4 * err + 1e-12, (name, dlt.mean(), err)


def test_superspin_sweeps_are_refused():
    gh.announce("superspin refusals")
    wide = gh.make_lattice(4, 3, 4, 2, 16, kind="gauss", beta=0.9, seed=1)[0]
    potts = gh.make_lattice(4, 4, 4, 3, 4, kind="ferro", beta=0.5, seed=1)[0]
    flat = gh.make_lattice(4, 4, 1, 2, 4, kind="pmj", beta=0.5, seed=1)[0]
    for lat in (wide, potts, flat):
        with pytest.raises(tn.TnmcError) as e:
            tn.tnmc_sweep_superspin([lat], 1)
        assert e.value.status == -5
