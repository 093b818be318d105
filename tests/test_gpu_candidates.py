"""Several candidates per environment (main text, "TNMCMC": a batch of
candidates drawn from the same approximate distribution, one kept) on the GPU
against the oracle's chained independence-MH steps.

* One half-sweep with K candidates: per task, the written-back layer, the
  number of accepted candidates, log q of the initial and final layer and the
  energy change equal the oracle's (FP64 bar).
* Full sweeps with K = 3 reproduce the oracle's chain spin for spin, on an
  Ising and a Potts lattice.
* 64 independent 2x2x4 chains at chi = 1 with K = 3 match exact enumeration
  of <E> and <M^2>."""
import math

import numpy as np
import pytest
import torch

import bruteforce as bf
import gpu_helpers as gh
import paper_2509_23945_amd as tn
from oracle import chain as ochain

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K", [2, 3, 4])
def test_half_sweep_with_candidates_matches_oracle(K):
    gh.announce(f"half-sweep with {K} candidates, 6x5x4 chi=1")
    Lx, Ly, Lz, chi, beta = 6, 5, 4, 1, 1.1
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, chi, kind="gauss", beta=beta, seed=61, n_chains=3,
                                       n_candidates=K)
    tasks = [(c, z) for c in range(3) for z in range(0, Lz, 2)]
    trace = torch.zeros(5 * len(tasks), dtype=torch.float64, device="cuda")
    st = tn.tnmc_half_sweep([lat], 0, 4, trace_ptr=trace.data_ptr())
    torch.cuda.synchronize()
    tr = trace.cpu().numpy().reshape(-1, 5)
    assert st["proposed"] == K * len(tasks) and st["numeric_faults"] == 0
    refs = [s.copy() for s in spins]
    n_acc = 0
    for k, (c, z) in enumerate(tasks):
        rec = ochain.slice_update_multi(J[c], refs[c], z, beta, chi, 2, K, seed=12345, chain=c, sweep=4)
        n_acc += rec["accepted"]
        assert tr[k, 3] == rec["accepted"], (c, z)
        assert gh.logq_close(tr[k, 1], rec["logq_initial"]) and gh.logq_close(tr[k, 0], rec["logq_final"])
        assert tr[k, 2] == rec["dE"]
    assert st["accepted"] == n_acc and 0 < n_acc < K * len(tasks)
    for c in range(3):
        assert np.array_equal(tn.tnmc_get_spins(lat, c), refs[c]), c


@pytest.mark.parametrize("d,kind,chi,beta", [(2, "pmj", 2, 1.0), (3, "ferro", 3, 0.6)])
def test_sweeps_with_candidates_match_oracle(d, kind, chi, beta):
    gh.announce(f"sweeps with 3 candidates d={d}")
    lat, J, spins, _ = gh.make_lattice(5, 4, 5, d, chi, kind=kind, beta=beta, seed=62, n_chains=2, n_candidates=3)
    refs = [s.copy() for s in spins]
    for t in range(3):
        st = tn.tnmc_sweep([lat], 1, sweep_offset=t)
        acc = sum(ochain.sweep(J[c], refs[c], beta, chi, d, seed=12345, chain=c, sweep_index=t, n_candidates=3)
                  for c in range(2))
        assert st["accepted"] == acc and st["proposed"] == 3 * 2 * 5
        for c in range(2):
            assert np.array_equal(tn.tnmc_get_spins(lat, c), refs[c]), (t, c)


def test_candidates_chain_averages_match_enumeration():
    gh.announce("3 candidates, chain averages 2x2x4")
    Lx, Ly, Lz, beta, n_chains, n_sweeps = 2, 2, 4, 1.0, 64, 300
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, 1, kind="pmj", beta=beta, seed=63, n_chains=n_chains,
                                       record_capacity=n_sweeps, n_candidates=3)
    st = tn.tnmc_sweep([lat], n_sweeps, record=True)
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
